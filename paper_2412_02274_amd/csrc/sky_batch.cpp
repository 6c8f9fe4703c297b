// C ABI of the batched path (declared in include/sky.h): many independent relations of one
// dimensionality, each a segment of one plan. The skyline rounds of the segmented engine serve
// every relation at once (Sec. 3: each relation is what the paper calls a partition, except
// that no final phase merges them); gres (Def. 2 via Alg. 1) then runs as one search launch
// over a device table of work items, one workgroup each.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "sky_plan.hpp"

using namespace sky;

struct sky_batch {
    sky_plan* plan = nullptr;
    int32_t nbatch = 0, d = 0;
    int64_t total = 0, ld = 0;
    const float* x = nullptr;
    int32_t* dev_status = nullptr;
    int32_t state = 0;
    // workspace after the plan's region
    char* rest = nullptr;
    size_t rest_bytes = 0;
    int64_t* dev_count = nullptr;
    int32_t* cand_off = nullptr;   // [nbatch + 1] element offsets of every relation's skyline
    GresStore store{};
    GresPrepTmp tmp{};
    GresTargets tg{};
    int32_t* wg_table = nullptr;
    int64_t wg_cap = 0;            // entries available
    // host
    std::vector<int64_t> sky_off;  // [nbatch + 1] after sky_batch_skylines
    int64_t sky_count = 0;
    int32_t max_cnt = 0;
    int32_t n_wg = 0;
    int32_t mapping = SKY_GRES_TILES;
    int32_t near_first = 1;
    const int64_t* sky_idx = nullptr;
    sky_info info{};
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
    B->cand_off = c.take<int32_t>((size_t)nbatch + 1);
    carve_gres_store(c, B->store, s, d, nbatch);
    carve_gres_prep_tmp(c, B->tmp, s);
    carve_gres_targets(c, B->tg, s, d);
    B->wg_cap = s + nbatch;
    B->wg_table = c.take<int32_t>((size_t)(kGresWgEntry * B->wg_cap));
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
    sky_status s = plan_build(x_soa, n, d, ld, kSchemeSegments, nbatch, 0, 0, offsets, ws, pb,
                              dev_status, (hipStream_t)stream, &B->plan);
    if (s != SKY_OK) { delete B; return s; }
    B->rest = (char*)ws + pb;
    B->rest_bytes = ws_bytes - pb;
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
    if (B->state != 1) return SKY_ERR_STATE;
    hipStream_t st = (hipStream_t)stream;
    sky_plan* P = B->plan;
    // 1. every relation's skyline: one segment per relation, no final phase
    SKY_TRY(sky_local_skylines(P, stream));
    // every relation's skyline flags (local_flag rewritten to them), and their count read back
    SKY_TRY(launch_compact_flags(P->local_flag, P->eng.dom, true, (int32_t)P->n, P->final_list,
                                 P->count_tmp + CT_SKY, P->dinfo + D_SKY_COUNT, P->eng.scan_tmp, st));
    P->state = 3;
    sky_info pi{};
    SKY_TRY(sky_plan_info(P, &pi));
    const int64_t S = pi.sky_count;
    B->info.rounds_local = pi.rounds_local;
    B->info.tests_local = pi.tests_local;
    B->info.tests_local_max = pi.tests_local_max;  // the costliest relation
    B->info.local_count = S;
    B->info.sky_count = S;
    if (S > cap) return SKY_ERR_CAPACITY;
    // 2. ascending rows and the per-relation offsets into them
    Carver c(B->rest, B->rest_bytes);
    carve_batch_tail(c, B, S, B->d, B->nbatch);  // sized for the actual skyline
    if (c.overflow) return SKY_ERR_WORKSPACE;
    SKY_TRY(launch_final_output(P->final_list, P->count_tmp + CT_SKY, P->rowid, P->n, P->member_tmp, nullptr,
                                sky_idx, cap, B->dev_count, P->pos_tmp, P->scan_tmp, B->dev_status, st));
    SKY_TRY(launch_batch_offsets(sky_idx, S, P->seg_off_dev, B->nbatch, sky_off, B->cand_off, st));
    B->sky_off.assign((size_t)B->nbatch + 1, 0);
    SKY_HIP(hipMemcpyAsync(B->sky_off.data(), sky_off, sizeof(int64_t) * (size_t)(B->nbatch + 1),
                           hipMemcpyDeviceToHost, st));
    SKY_HIP(hipStreamSynchronize(st));
    if (B->sky_off[B->nbatch] != S) return SKY_ERR_HIP;  // the engine and the output disagree
    // 3. the candidate store: relation j's skyline in curve order from a 64-aligned slot
    std::vector<int32_t> coff((size_t)B->nbatch), cnt((size_t)B->nbatch);
    int64_t slot = 0;
    int32_t max_cnt = 0;
    for (int32_t j = 0; j < B->nbatch; ++j) {
        const int64_t k = B->sky_off[j + 1] - B->sky_off[j];
        if (k < 0) return SKY_ERR_HIP;
        coff[j] = (int32_t)slot;
        cnt[j] = (int32_t)k;
        max_cnt = std::max(max_cnt, (int32_t)k);
        slot += round_up(k, kWave);
    }
    if (slot + kWave > B->store.ccap) return SKY_ERR_HIP;  // never: ccap holds S + 64 (nbatch + 1)
    SKY_HIP(hipMemcpyAsync(B->store.seg_coff, coff.data(), sizeof(int32_t) * coff.size(),
                           hipMemcpyHostToDevice, st));
    SKY_HIP(hipMemcpyAsync(B->store.seg_cnt, cnt.data(), sizeof(int32_t) * cnt.size(),
                           hipMemcpyHostToDevice, st));
    SKY_TRY(launch_gres_prepare_segments(B->x, B->total, B->d, B->ld, sky_idx, S, B->cand_off,
                                         B->nbatch, (int32_t)(slot / kWave), B->store, B->tmp,
                                         B->dev_status, st));
    SKY_HIP(hipStreamSynchronize(st));  // the host tables above go out of scope
    B->sky_count = S;
    B->max_cnt = max_cnt;
    B->sky_idx = sky_idx;
    B->state = 2;
    B->info.state = 2;
    return SKY_OK;
}

sky_status sky_batch_tune(sky_batch* B, const sky_tune* tune, void* stream) {
    if (!B) return SKY_ERR_INVALID_ARG;
    sky_tune t{SKY_GRES_AUTO, 0, 1, 1};
    if (tune) t = *tune;
    if (t.mapping < SKY_GRES_AUTO || t.mapping > SKY_GRES_LEVELS || t.targets_per_wg < 0 ||
        t.targets_per_wg > 4096 || (t.near_first != 0 && t.near_first != 1) || (t.lpt != 0 && t.lpt != 1))
        return SKY_ERR_INVALID_ARG;
    if (B->state < 2) return SKY_ERR_STATE;
    const int32_t per = t.targets_per_wg > 0 ? t.targets_per_wg : 16;
    struct Item { int32_t seg, t0, t1; double cost; };
    std::vector<Item> items;
    for (int32_t j = 0; j < B->nbatch; ++j) {
        const int32_t a = (int32_t)B->sky_off[j], b = (int32_t)B->sky_off[j + 1];
        for (int32_t q = a; q < b; q += per) {
            const int32_t e = std::min(b, q + per);
            // a tuple's search scans up to its relation's whole skyline per level
            items.push_back({j, q, e, (double)(e - q) * (double)(b - a)});
        }
    }
    if ((int64_t)items.size() > B->wg_cap) return SKY_ERR_WORKSPACE;  // never: per >= 1
    if (t.lpt)
        std::stable_sort(items.begin(), items.end(),
                         [](const Item& x, const Item& y) { return x.cost > y.cost; });
    std::vector<int32_t> table(items.size() * kGresWgEntry);
    for (size_t i = 0; i < items.size(); ++i) {
        table[kGresWgEntry * i] = items[i].seg;
        table[kGresWgEntry * i + 1] = items[i].t0;
        table[kGresWgEntry * i + 2] = items[i].t1;
    }
    hipStream_t st = (hipStream_t)stream;
    if (!table.empty()) {
        SKY_HIP(hipMemcpyAsync(B->wg_table, table.data(), sizeof(int32_t) * table.size(),
                               hipMemcpyHostToDevice, st));
        SKY_HIP(hipStreamSynchronize(st));
    }
    B->n_wg = (int32_t)items.size();
    B->mapping = t.mapping;
    B->near_first = t.near_first;
    B->state = 3;
    B->info.state = 3;
    return SKY_OK;
}

sky_status sky_batch_gres(sky_batch* B, int32_t g_max, int32_t* g_exit, float* gres,
                          void* ev_begin, void* ev_end, void* stream) {
    if (!B || g_max < 2 || g_max > SKY_MAX_G || (!ev_begin) != (!ev_end)) return SKY_ERR_INVALID_ARG;
    if (B->state != 3) return SKY_ERR_STATE;
    if (B->sky_count == 0) return SKY_OK;
    hipStream_t st = (hipStream_t)stream;
    // AUTO: by the largest relation's skyline (the launch is shared by all relations)
    const int32_t mapping = B->mapping == SKY_GRES_AUTO ? gres_auto_mapping(B->max_cnt, g_max) : B->mapping;
    SKY_TRY(launch_gres_targets_segments(B->store, B->d, B->sky_count, B->cand_off, B->nbatch,
                                         B->near_first != 0, B->tg, st));
    return launch_gres_search(B->store, B->d, B->max_cnt, B->tg, B->sky_count, nullptr, B->wg_table, B->n_wg,
                              g_max, mapping, g_exit, gres, ev_begin, ev_end, nullptr, st);
}

sky_status sky_batch_info(const sky_batch* B, sky_info* out) {
    if (!B || !out) return SKY_ERR_INVALID_ARG;
    *out = B->info;
    return SKY_OK;
}

void sky_batch_destroy(sky_batch* B) {
    if (!B) return;
    sky_plan_destroy(B->plan);
    delete B;
}

}  // extern "C"
