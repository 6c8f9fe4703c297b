// C ABI of the batched path (declared in include/sky.h): many independent relations of one
// dimensionality, each a segment of one plan. The skyline rounds of the segmented engine serve
// every relation at once (Sec. 3: each relation is what the paper calls a partition, except
// that no final phase merges them); gres (Def. 2 via Alg. 1) then runs as one persistent search
// over the skyline tuples of every relation. After sky_batch_create, no call reads anything back:
// sky_batch_skylines + sky_batch_gres is a fixed launch sequence a HIP graph can capture.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>

#include "sky_plan.hpp"

using namespace sky;

struct sky_batch {
    sky_plan* plan = nullptr;
    int32_t nbatch = 0, d = 0;
    int64_t total = 0, ld = 0;
    const float* x = nullptr;
    int32_t* dev_status = nullptr;
    int32_t state = 0;             // 1 created, 2 skylines queued
    hipStream_t last_stream = nullptr;  // stream of the last sky_batch_gres
    int64_t cap = 0;               // min(sky_idx capacity of the last sky_batch_skylines, total)
    // workspace after the plan's region, sized for the worst case (every row in a skyline)
    int64_t* dev_count = nullptr;  // the skyline total (int64, sky_idx's count)
    unsigned long long* gtests = nullptr;  // candidate tests of the last gres search
    int32_t* cand_off = nullptr;   // [nbatch + 1] element offsets of every relation's skyline
    int32_t* used = nullptr;       // [2] store slots in use, largest relation's skyline
    int32_t* order = nullptr;      // [nbatch] relations, longest-first
    int32_t* rank_off = nullptr;   // [nbatch + 1]
    int32_t* tord = nullptr;       // [total] targets in longest-first relation order
    int32_t* tseg = nullptr;       // [total] relation of every target
    GresStore store{};
    GresPrepTmp tmp{};
    GresTargets tg{};
    // choices of sky_batch_tune
    int32_t mapping = SKY_GRES_AUTO;
    int32_t near_first = 1;
    int32_t lpt = 1;
    sky_info info{};
    // packed key tables of the gres search (sky_batch_set_keys), caller-owned
    GresKeys keys{};
    int32_t keys_g_max = 0;
};

namespace {

bool valid_offsets(const int64_t* off, int32_t nbatch) {
    if (!off || nbatch < 1 || nbatch > SKY_MAX_CELLS || off[0] != 0) return false;
    for (int32_t j = 0; j < nbatch; ++j)
        if (off[j + 1] < off[j]) return false;
    return off[nbatch] >= 1 && off[nbatch] <= kMaxBuildRows;
}

// Regions after the plan, sized for the worst case: every row a skyline row.
void carve_batch_tail(Carver& c, sky_batch* B, int64_t s, int32_t d, int32_t nbatch) {
    B->dev_count = c.take<int64_t>(8);
    B->gtests = c.take<unsigned long long>(1);
    B->cand_off = c.take<int32_t>((size_t)nbatch + 1);
    B->used = c.take<int32_t>(64);
    B->order = c.take<int32_t>((size_t)nbatch);
    B->rank_off = c.take<int32_t>((size_t)nbatch + 1);
    B->tord = c.take<int32_t>((size_t)s);
    B->tseg = c.take<int32_t>((size_t)s);
    carve_gres_store(c, B->store, s, d, nbatch);
    carve_gres_prep_tmp(c, B->tmp, s);
    carve_gres_targets(c, B->tg, s, d);
}

// candidate slots of the key tables for skylines of up to sky_total tuples over nbatch
// relations: every relation's skyline rounded up to whole tiles, and the padding tile
int64_t key_slots(int64_t sky_total, int32_t nbatch) {
    constexpr int64_t tile = 64;  // candidates per tile of the gres store
    return sky_total + (tile - 1) * nbatch + tile;
}

void carve_batch_keys(Carver& c, GresKeys& k, int64_t sky_total, int32_t nbatch, int32_t g_max) {
    carve_gres_keys_slots(c, k, key_slots(sky_total, nbatch), g_max - 1);
}

size_t tail_bytes(int64_t s, int32_t d, int32_t nbatch) {
    sky_batch tmp;
    Carver c(nullptr, 0);
    carve_batch_tail(c, &tmp, s, d, nbatch);
    return c.used;
}

}  // namespace

extern "C" {

size_t sky_batch_workspace_bytes(const int64_t* offsets, int32_t nbatch, int32_t d) {
    if (d < 1 || d > SKY_MAX_D || !valid_offsets(offsets, nbatch)) return 0;
    const int64_t n = offsets[nbatch];
    const size_t pb = plan_bytes(n, d, kSchemeSegments, nbatch, 0);
    if (pb == 0) return 0;
    return round_up((int64_t)pb, 256) + tail_bytes(n, d, nbatch);
}

sky_status sky_batch_create(const float* x_soa, int32_t d, int64_t ld, const int64_t* offsets,
                            int32_t nbatch, void* ws, size_t ws_bytes, int32_t* dev_status,
                            void* stream, sky_batch** out) {
    if (!out) return SKY_ERR_INVALID_ARG;
    *out = nullptr;
    if (!x_soa || !ws || !dev_status || d < 1 || d > SKY_MAX_D || !valid_offsets(offsets, nbatch))
        return SKY_ERR_INVALID_ARG;
    const int64_t n = offsets[nbatch];
    if (ld < n) return SKY_ERR_INVALID_ARG;
    const size_t need = sky_batch_workspace_bytes(offsets, nbatch, d);
    if (need == 0) return SKY_ERR_INVALID_ARG;
    if (ws_bytes < need) return SKY_ERR_WORKSPACE;
    sky_batch* B = new (std::nothrow) sky_batch();
    if (!B) return SKY_ERR_INVALID_ARG;
    const size_t pb = (size_t)round_up((int64_t)plan_bytes(n, d, kSchemeSegments, nbatch, 0), 256);
    // the plan only: its partition step is queued by every sky_batch_skylines
    sky_status s = plan_build(x_soa, n, d, ld, kSchemeSegments, nbatch, 0, 0, offsets, 0, true, ws, pb,
                              dev_status, (hipStream_t)stream, &B->plan, false);
    if (s != SKY_OK) { delete B; return s; }
    Carver c((char*)ws + pb, ws_bytes - pb);
    carve_batch_tail(c, B, n, d, nbatch);
    if (c.overflow) { sky_plan_destroy(B->plan); delete B; return SKY_ERR_WORKSPACE; }
    B->nbatch = nbatch; B->d = d; B->total = n; B->ld = ld; B->x = x_soa;
    B->dev_status = dev_status;
    B->state = 1;
    int64_t maxp = 0;
    for (int32_t j = 0; j < nbatch; ++j) maxp = std::max(maxp, offsets[j + 1] - offsets[j]);
    B->info.n = n; B->info.d = d; B->info.scheme = SKY_NONE; B->info.p = nbatch;
    B->info.max_partition = maxp; B->info.state = 1;
    *out = B;
    return SKY_OK;
}

sky_status sky_batch_skylines(sky_batch* B, int64_t* sky_idx, int64_t cap, int64_t* sky_off,
                              void* stream) {
    if (!B || !sky_idx || !sky_off || cap < 1) return SKY_ERR_INVALID_ARG;
    if (B->state < 1) return SKY_ERR_STATE;
    hipStream_t st = (hipStream_t)stream;
    sky_plan* P = B->plan;
    // 1. every relation's rows, canonical and along a Hilbert curve, as one segment each
    SKY_TRY(plan_partition(P, st));
    // 2. every relation's skyline: one segment per relation, no final phase
    SKY_TRY(plan_local_phase(P, st));
    // their positions (relation-major, curve order inside each relation), local_flag rewritten
    // to exactly the skylines, and the total
    SKY_TRY(launch_compact_flags(P->local_flag, P->eng.dom, true, (int32_t)P->n, P->final_list,
                                 P->count_tmp + CT_SKY, P->dinfo + D_SKY_COUNT, P->eng.scan_tmp, st,
                                 P->count_tmp + CT_ROWS));
    // 3. ascending rows (SKY_ERR_CAPACITY on the device above cap) and the per-relation offsets
    SKY_TRY(launch_final_output(P->final_list, P->count_tmp + CT_SKY, P->rowid, P->n, P->member_tmp, nullptr,
                                sky_idx, cap, B->dev_count, P->pos_tmp, P->scan_tmp, B->dev_status, st));
    // 4. the candidate store: relation j's skyline in curve order from a 64-aligned slot
    const int64_t c = cap < B->total ? cap : B->total;
    SKY_TRY(launch_batch_store(P->xp, P->ldp, B->d, P->final_list, P->rowid, P->pos_tmp, sky_idx,
                               P->count_tmp + CT_SKY, c, P->seg_off_dev, B->nbatch, sky_off, B->cand_off,
                               B->used, B->store, st));
    P->state = 3;
    B->cap = c;
    B->state = 2;
    B->info.state = 2;
    return SKY_OK;
}

sky_status sky_batch_tune(sky_batch* B, const sky_tune* tune, void* stream) {
    (void)stream;
    if (!B) return SKY_ERR_INVALID_ARG;
    sky_tune t{SKY_GRES_AUTO, 1, 1};
    if (tune) t = *tune;
    if (t.mapping < SKY_GRES_AUTO || t.mapping > SKY_GRES_LEVELS || (t.near_first != 0 && t.near_first != 1) ||
        (t.lpt != 0 && t.lpt != 1))
        return SKY_ERR_INVALID_ARG;
    B->mapping = t.mapping;
    B->near_first = t.near_first;
    B->lpt = t.lpt;
    return SKY_OK;
}

sky_status sky_batch_gres(sky_batch* B, int32_t g_max, int32_t* g_exit, float* gres,
                          void* ev_begin, void* ev_end, void* stream) {
    if (!B || g_max < 2 || g_max > SKY_MAX_G || (!ev_begin) != (!ev_end)) return SKY_ERR_INVALID_ARG;
    if (B->state != 2) return SKY_ERR_STATE;
    B->last_stream = (hipStream_t)stream;
    SKY_TRY(launch_fill_u8(reinterpret_cast<uint8_t*>(B->gtests), sizeof(unsigned long long), 0,
                           (hipStream_t)stream));
    return launch_batch_search(B->store, B->d, B->cap, B->cand_off, B->nbatch, B->used, B->near_first != 0,
                               B->lpt != 0, B->order, B->rank_off, B->tord, B->tseg, B->tg, g_max, B->mapping,
                               g_exit, gres, ev_begin, ev_end, B->gtests, (hipStream_t)stream,
                               B->keys.key && g_max <= B->keys_g_max ? &B->keys : nullptr);
}

size_t sky_batch_keys_bytes(const sky_batch* B, int64_t sky_total, int32_t g_max_keys) {
    if (!B || sky_total < 0 || sky_total > kMaxBuildRows || !key_width(B->d, g_max_keys)) return 0;
    Carver c(nullptr, 0);
    GresKeys k{};
    carve_batch_keys(c, k, sky_total, B->nbatch, g_max_keys);
    return c.used;
}

sky_status sky_batch_set_keys(sky_batch* B, void* ws, size_t ws_bytes, int64_t sky_total, int32_t g_max_keys) {
    if (!B) return SKY_ERR_INVALID_ARG;
    if (!ws) {  // detach
        B->keys = GresKeys{};
        B->keys_g_max = 0;
        return SKY_OK;
    }
    const size_t need = sky_batch_keys_bytes(B, sky_total, g_max_keys);
    if (need == 0) return SKY_ERR_INVALID_ARG;
    if (ws_bytes < need) return SKY_ERR_WORKSPACE;
    Carver c(ws, ws_bytes);
    GresKeys k{};
    carve_batch_keys(c, k, sky_total, B->nbatch, g_max_keys);
    if (c.overflow) return SKY_ERR_WORKSPACE;
    k.used = B->used;
    B->keys = k;
    B->keys_g_max = g_max_keys;
    return SKY_OK;
}

sky_status sky_batch_info(const sky_batch* B, sky_info* out) {
    if (!B || !out) return SKY_ERR_INVALID_ARG;
    *out = B->info;
    if (B->state < 2) return SKY_OK;
    sky_info pi{};
    SKY_TRY(sky_plan_info(B->plan, &pi));  // waits for the last skyline pass
    out->rounds_local = pi.rounds_local;
    out->tests_local = pi.tests_local;
    out->tests_local_max = pi.tests_local_max;  // the costliest relation
    out->rows_kept = pi.rows_kept;
    out->tests_prefilter = pi.tests_prefilter;
    out->local_count = pi.sky_count;
    out->sky_count = pi.sky_count;
    if (B->last_stream) {  // the candidate tests of the last gres search
        unsigned long long gt = 0;
        SKY_HIP(hipMemcpyAsync(&gt, B->gtests, sizeof(gt), hipMemcpyDeviceToHost, B->last_stream));
        SKY_HIP(hipStreamSynchronize(B->last_stream));
        out->tests_gres = (int64_t)gt;
    }
    return SKY_OK;
}

void sky_batch_destroy(sky_batch* B) {
    if (!B) return;
    sky_plan_destroy(B->plan);
    delete B;
}

}  // extern "C"
