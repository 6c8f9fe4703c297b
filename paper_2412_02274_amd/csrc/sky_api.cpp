// C ABI of libsky (declared in include/sky.h): argument checks, workspace layout, plans and
// the order of the device steps. All device work is in the .hip files.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <new>

#include "sky_plan.hpp"

using namespace sky;

namespace {

bool valid_d(int32_t d) { return d >= 1 && d <= SKY_MAX_D; }

// m >= 2 minimising |m^e - target| (ties to the smaller m); -1 if no m keeps m^e <= cap
int32_t closest_m(int64_t target, int32_t e, int64_t cap) {
    int32_t best = -1;
    int64_t bestdiff = 0;
    for (int32_t m = 2; m <= 65536; ++m) {
        int64_t v = 1;
        bool over = false;
        for (int32_t i = 0; i < e; ++i) {
            v *= m;
            if (v > (int64_t(1) << 40)) { over = true; break; }
        }
        if (over) break;
        int64_t diff = v > target ? v - target : target - v;
        if (best < 0 || diff < bestdiff) { best = m; bestdiff = diff; }
        if (v > target) break;
    }
    if (best < 0) return -1;
    int64_t v = 1;
    for (int32_t i = 0; i < e; ++i) v *= best;
    return v <= cap ? best : -1;
}

int64_t ipow(int64_t b, int32_t e) {
    int64_t v = 1;
    for (int32_t i = 0; i < e; ++i) v *= b;
    return v;
}

// Resolve scheme -> (p, m); returns SKY_OK or an error.
sky_status resolve_partitions(int64_t n, int32_t d, const sky_params* prm, int32_t* p, int32_t* m) {
    switch (prm->scheme) {
        case SKY_NONE:
            *p = 1; *m = 0;
            return SKY_OK;
        case SKY_GRID: {
            if (prm->target_p < 1) return SKY_ERR_INVALID_ARG;
            int32_t mm = closest_m(prm->target_p, d, SKY_MAX_CELLS);
            if (mm < 0) return SKY_ERR_UNSUPPORTED;
            *m = mm; *p = (int32_t)ipow(mm, d);
            return SKY_OK;
        }
        case SKY_ANGULAR: {
            if (prm->target_p < 1 || d < 2) return SKY_ERR_INVALID_ARG;
            int32_t mm = closest_m(prm->target_p, d - 1, SKY_MAX_CELLS);
            if (mm < 0) return SKY_ERR_UNSUPPORTED;
            *m = mm; *p = (int32_t)ipow(mm, d - 1);
            return SKY_OK;
        }
        case SKY_SLICED:
            if (prm->target_p < 1 || prm->slice_dim < 0 || prm->slice_dim >= d) return SKY_ERR_INVALID_ARG;
            *m = 0;
            *p = (int32_t)(prm->target_p < n ? prm->target_p : n);
            return *p <= SKY_MAX_CELLS ? SKY_OK : SKY_ERR_UNSUPPORTED;
        default:
            return SKY_ERR_INVALID_ARG;
    }
}

// One layout routine serves both sizing (base == nullptr) and carving.
void carve_plan(Carver& c, sky_plan* P, int64_t n, int32_t d, int32_t scheme, int32_t p, int32_t m) {
    const int64_t ldp = round_up(n, 64);
    P->ldp = ldp;
    P->xp = c.take<float>((size_t)(d * ldp));
    P->rowid = c.take<int32_t>((size_t)n);
    P->seg = c.take<int32_t>((size_t)n);
    P->fsum = c.take<float>((size_t)n);
    P->part_off = c.take<int32_t>((size_t)p + 1);
    P->pruned = c.take<uint8_t>((size_t)p);
    P->tan2_dev = c.take<double>((size_t)(scheme == SKY_ANGULAR ? m + 1 : 1));
    P->sel_key = c.take<unsigned long long>((size_t)(scheme == SKY_SLICED ? 3 * p : 1));
    P->sel_i32 = c.take<int32_t>((size_t)(scheme == SKY_SLICED ? slice_select_elems(p) : 1));
    P->seg_off_dev = c.take<int64_t>((size_t)(scheme == kSchemeSegments ? p + 1 : 1));
    P->part_of_row = c.take<int32_t>((size_t)(p > 1 ? n : 1));
    P->pcount = c.take<int32_t>((size_t)p);
    P->kmin = c.take<unsigned long long>((size_t)p * SKY_KILLERS);
    P->krow = c.take<int32_t>((size_t)p * SKY_KILLERS);
    P->kval = c.take<float>((size_t)p * SKY_KILLERS * (size_t)partition_row_stride(d));
    P->alive = c.take<uint8_t>((size_t)n);
    P->blk = c.take<int32_t>((size_t)partition_blocks(n) + 64);
    P->scan_tmp = c.take<int32_t>((size_t)scan_tmp_elems(n));
    P->xa = c.take<float>((size_t)n * (size_t)partition_row_stride(d));
    P->rep_kept = c.take<int32_t>((size_t)SKY_MAX_REPS + 1);
    P->rep_tests = c.take<unsigned long long>(1);
    P->seg_tests = c.take<unsigned long long>((size_t)p);
    P->k0 = c.take<uint32_t>((size_t)n);
    P->v0 = c.take<uint32_t>((size_t)n);
    P->k1 = c.take<uint32_t>((size_t)n);
    P->v1 = c.take<uint32_t>((size_t)n);
    P->radix_tmp = c.take<int32_t>((size_t)radix_tmp_elems(n));
    EngineBuffers& e = P->eng;
    e.hcap = engine_head_capacity(n, p);
    e.tcap = round_up(ceil_div(e.hcap, 64), 64);
    e.w0 = c.take<int32_t>((size_t)n);
    e.w1 = c.take<int32_t>((size_t)n);
    e.head = c.take<int32_t>((size_t)e.hcap);
    e.rest = c.take<int32_t>((size_t)n);
    e.rhb = c.take<int32_t>((size_t)n);
    e.hval = c.take<uint32_t>((size_t)(d * e.hcap));
    e.hlo = c.take<uint32_t>((size_t)(d * e.tcap));
    e.hhi = c.take<uint32_t>((size_t)(d * e.tcap));
    e.seg_min = c.take<uint32_t>((size_t)range_elems(p));
    e.seg_max = c.take<uint32_t>((size_t)range_elems(p));
    e.hist = c.take<int32_t>((size_t)2 * p * kBins);
    e.seg_info = c.take<int32_t>((size_t)2 * p * 8);
    e.dom = c.take<uint8_t>((size_t)n);
    e.tile_off = c.take<int32_t>((size_t)2 * (p + 1));
    e.counters = c.take<int32_t>(48);
    e.tests = c.take<unsigned long long>(3);
    e.work = c.take<int32_t>((size_t)kWorkCounters * kCounterStride);
    e.scan = c.take<int32_t>((size_t)engine_scan_elems(n));
    e.scan_tmp = c.take<int32_t>((size_t)scan_tmp_elems(n));
    P->local_flag = c.take<uint8_t>((size_t)n);
    P->final_flag = c.take<uint8_t>((size_t)n);
    P->member_tmp = c.take<uint8_t>((size_t)n);
    P->final_list = c.take<int32_t>((size_t)n);
    P->pos_tmp = c.take<int32_t>((size_t)n);
    P->count_tmp = c.take<int32_t>(64);
    P->dinfo = c.take<int64_t>(kDinfo);
}

}  // namespace

namespace sky {

size_t plan_bytes(int64_t n, int32_t d, int32_t scheme, int32_t p, int32_t m) {
    if (n < 1 || n > kMaxBuildRows || !valid_d(d) || p < 1) return 0;
    sky_plan tmp;
    Carver c(nullptr, 0);
    carve_plan(c, &tmp, n, d, scheme, p, m);
    return c.used;
}

sky_status plan_partition(sky_plan* P, hipStream_t st) {
    PartitionArgs a{};
    a.x = P->x; a.n = P->n; a.d = P->d; a.ld = P->ld;
    a.scheme = P->scheme; a.p = P->p; a.m = P->m; a.slice_dim = P->slice_dim;
    a.seg_off = P->seg_off_dev;
    a.tan2 = P->tan2_dev;
    a.sel_key = P->sel_key;
    a.sel_i32 = P->sel_i32;
    a.prefilter = P->prefilter;
    a.xp = P->xp; a.ldp = P->ldp; a.rowid = P->rowid; a.seg = P->seg; a.fsum = P->fsum;
    a.n_live = P->count_tmp + CT_ROWS;
    a.part_off = P->part_off; a.pruned = P->pruned;
    a.part_of_row = P->part_of_row;
    a.pcount = P->pcount; a.kmin = P->kmin; a.krow = P->krow; a.kval = P->kval;
    a.alive = P->alive; a.blk = P->blk;
    a.scan_tmp = P->scan_tmp;
    a.k0 = P->k0; a.v0 = P->v0; a.k1 = P->k1; a.v1 = P->v1; a.radix_tmp = P->radix_tmp;
    a.xa = P->xa;
    a.seg_tests = P->seg_tests;
    a.tests = reinterpret_cast<unsigned long long*>(P->dinfo + D_TESTS_FILTER);
    a.smin = P->eng.seg_min; a.smax = P->eng.seg_max;
    // with the prefilter the local phase's first list is every position of the copy
    a.iota_out = P->prefilter ? P->eng.w1 : nullptr;
    // partition statistics (pruned Grid cells and their rows, the largest partition)
    a.stats_out = P->dinfo + D_PRUNED_CELLS;
    a.dev_status = P->dev_status;
    return launch_partition(a, st);
}

sky_status plan_build(const float* x_soa, int64_t n, int32_t d, int64_t ld, int32_t scheme, int32_t p,
                      int32_t m, int32_t slice_dim, const int64_t* seg_off_host, int32_t reps, bool prefilter,
                      void* ws, size_t ws_bytes, int32_t* dev_status, hipStream_t st, sky_plan** out,
                      bool launch) {
    *out = nullptr;
    size_t need = plan_bytes(n, d, scheme, p, m);
    if (need == 0) return SKY_ERR_INVALID_ARG;
    if (ws_bytes < need) return SKY_ERR_WORKSPACE;
    if (scheme == kSchemeSegments && !seg_off_host) return SKY_ERR_INVALID_ARG;
    sky_plan* P = new (std::nothrow) sky_plan();
    if (!P) return SKY_ERR_INVALID_ARG;
    Carver c(ws, ws_bytes);
    carve_plan(c, P, n, d, scheme, p, m);
    if (c.overflow) { delete P; return SKY_ERR_WORKSPACE; }
    P->x = x_soa; P->n = n; P->ld = ld; P->d = d;
    P->scheme = scheme; P->p = p; P->m = m; P->slice_dim = slice_dim;
    P->dev_status = dev_status;
    P->reps = reps;
    P->prefilter = prefilter && reps == 0;
    if (P->scheme == kSchemeSegments) {
        // the caller's host array may go away on return: wait for the copy
        hipError_t e1 = hipMemcpyAsync(P->seg_off_dev, seg_off_host, sizeof(int64_t) * (size_t)(p + 1),
                                       hipMemcpyHostToDevice, st);
        hipError_t e2 = hipStreamSynchronize(st);
        if (e1 != hipSuccess || e2 != hipSuccess) { delete P; return SKY_ERR_HIP; }
    }
    if (launch) {
        sky_status s = plan_partition(P, st);
        if (s != SKY_OK) { delete P; return s; }
    }
    P->state = 1;
    P->info.n = n; P->info.d = d; P->info.scheme = P->scheme; P->info.p = p; P->info.m = m;
    P->info.state = 1;
    *out = P;
    return SKY_OK;
}

}  // namespace sky

extern "C" {

const char* sky_status_string(sky_status s) {
    switch (s) {
        case SKY_OK: return "SKY_OK";
        case SKY_ERR_INVALID_ARG: return "SKY_ERR_INVALID_ARG: invalid argument";
        case SKY_ERR_DOMAIN: return "SKY_ERR_DOMAIN: a value is NaN/inf or outside [0, 1)";
        case SKY_ERR_WORKSPACE: return "SKY_ERR_WORKSPACE: workspace too small";
        case SKY_ERR_CAPACITY: return "SKY_ERR_CAPACITY: output capacity too small";
        case SKY_ERR_HIP: return "SKY_ERR_HIP: HIP runtime error";
        case SKY_ERR_STATE: return "SKY_ERR_STATE: call out of order on a plan";
        case SKY_ERR_UNSUPPORTED: return "SKY_ERR_UNSUPPORTED: outside the implemented limits";
    }
    return "unknown sky_status";
}

int32_t sky_version(void) { return 10000; }

sky_status sky_ingest(const float* x_rows, int64_t n, int32_t d, float* x_soa, int64_t ld,
                      int32_t* dev_status, void* stream) {
    if (n < 0 || !valid_d(d) || ld < n || n > kMaxRows) return SKY_ERR_INVALID_ARG;
    if (n > 0 && (!x_rows || !x_soa || !dev_status)) return SKY_ERR_INVALID_ARG;
    return launch_ingest(x_rows, n, d, x_soa, ld, dev_status, (hipStream_t)stream);
}

sky_status sky_project(const float* x_soa, int64_t n, int32_t d, int64_t ld, const int64_t* rows,
                       int64_t s, int32_t g, float* out_soa, int64_t ld_out, int32_t* dev_status,
                       void* stream) {
    if (s < 0 || s > kMaxRows || !valid_d(d) || g < 1 || g > SKY_MAX_G || ld_out < s) return SKY_ERR_INVALID_ARG;
    if (s == 0) return SKY_OK;
    if (!x_soa || !rows || !out_soa || !dev_status || n < 1 || n > kMaxRows || ld < n) return SKY_ERR_INVALID_ARG;
    return launch_project(x_soa, n, d, ld, rows, s, g, out_soa, ld_out, dev_status, (hipStream_t)stream);
}

sky_status sky_literal_level(const uint8_t* member, int64_t s, int32_t g, int32_t* g_exit, int32_t* nil_left,
                             void* stream) {
    if (s < 0 || s > kMaxRows || g < 1 || g > SKY_MAX_G) return SKY_ERR_INVALID_ARG;
    if (s > 0 && (!g_exit || (g > 1 && !member))) return SKY_ERR_INVALID_ARG;
    return launch_literal_level(member, s, g, g_exit, nil_left, (hipStream_t)stream);
}

size_t sky_build_workspace_bytes(int64_t n, int32_t d, const sky_params* params) {
    if (!params || n < 1 || n > kMaxBuildRows || !valid_d(d) || params->reps < 0 || params->reps > SKY_MAX_REPS)
        return 0;
    int32_t p = 1, m = 0;
    if (resolve_partitions(n, d, params, &p, &m) != SKY_OK) return 0;
    return plan_bytes(n, d, params->scheme, p, m);
}

sky_status sky_build(const float* x_soa, int64_t n, int32_t d, int64_t ld, const sky_params* params,
                     void* ws, size_t ws_bytes, int32_t* dev_status, void* stream, sky_plan** out) {
    if (!out) return SKY_ERR_INVALID_ARG;
    *out = nullptr;
    if (!x_soa || !params || !ws || !dev_status) return SKY_ERR_INVALID_ARG;
    if (n < 1 || n > kMaxBuildRows || !valid_d(d) || ld < n || params->reps < 0 || params->reps > SKY_MAX_REPS ||
        (params->prefilter_off != 0 && params->prefilter_off != 1))
        return SKY_ERR_INVALID_ARG;
    int32_t p = 1, m = 0;
    SKY_TRY(resolve_partitions(n, d, params, &p, &m));
    return plan_build(x_soa, n, d, ld, params->scheme, p, m, params->slice_dim, nullptr, params->reps,
                      params->prefilter_off == 0, ws, ws_bytes, dev_status, (hipStream_t)stream, out, true);
}

sky_status sky_local_skylines(sky_plan* P, void* stream) {
    if (!P) return SKY_ERR_INVALID_ARG;
    if (P->state != 1) return SKY_ERR_STATE;
    SKY_TRY(plan_local_phase(P, (hipStream_t)stream));
    P->state = 2;
    P->info.state = 2;
    return SKY_OK;
}

sky_status sky_merge(sky_plan* P, int64_t* sky_idx, int64_t cap, int64_t* dev_count,
                     uint8_t* member, void* stream) {
    if (!P || !dev_count || cap < 0 || (cap > 0 && !sky_idx)) return SKY_ERR_INVALID_ARG;
    if (P->state != 2) return SKY_ERR_STATE;
    SKY_TRY(plan_final_phase(P, sky_idx, cap, dev_count, member, (hipStream_t)stream));
    P->merge_cap = cap;
    P->state = 3;
    P->info.state = 3;
    return SKY_OK;
}

}  // extern "C"

namespace sky {

sky_status plan_local_phase(sky_plan* P, hipStream_t st) {
    P->last_stream = st;
    const int32_t n = (int32_t)P->n;
    // the local phase's tests per partition (Sec. 4 counts its cost as the largest of them):
    // zeroed here when representatives add to them first, else by the engine run
    // rows of Grid cells pruned by grid dominance take no part (Def. 3)
    const uint8_t* skip = P->scheme == SKY_GRID && P->p > 1 ? P->pruned : nullptr;
    // Representative Filtering (Sec. 3.1): the rows the kept representatives dominate leave
    const uint8_t* keep = nullptr;
    if (P->reps > 0) {
        SKY_TRY(launch_fill_u8(reinterpret_cast<uint8_t*>(P->seg_tests),
                               (int64_t)P->p * (int64_t)sizeof(unsigned long long), 0, st));
        RepArgs ra{};
        ra.fsum = P->fsum; ra.rowid = P->rowid; ra.n = n; ra.d = P->d;
        ra.xp = P->xp; ra.ldp = P->ldp; ra.xa = P->xa; ra.rs = partition_row_stride(P->d);
        ra.k = P->reps;
        ra.k0 = P->k0; ra.v0 = P->v0; ra.k1 = P->k1; ra.v1 = P->v1; ra.radix_tmp = P->radix_tmp;
        ra.kept = P->rep_kept; ra.nkept = P->rep_kept + SKY_MAX_REPS; ra.tests = P->rep_tests;
        ra.seg_of_pos = P->p > 1 ? P->seg : nullptr; ra.seg_tests = P->seg_tests;
        ra.skip_seg = skip;
        ra.keep = P->member_tmp;  // free until sky_merge
        SKY_TRY(launch_representatives(ra, st));
        keep = P->member_tmp;
    }
    // the first round's list: with the prefilter, every position of the copy (it holds only
    // rows of unpruned partitions that no killer row dominates); else every position outside
    // the pruned cells and not filtered out by the representatives
    const int32_t* cnt = P->count_tmp + CT_LIST;
    if (P->prefilter) {
        cnt = P->count_tmp + CT_ROWS;  // (the list itself is written by the build's copy)
    } else {
        SKY_TRY(launch_iota_filtered(skip, P->seg, n, P->eng.w1, P->count_tmp + CT_LIST, P->eng.scan_tmp, st,
                                     keep));
    }
    EngineProblem pb{};
    pb.xp = P->xp; pb.ldp = P->ldp; pb.d = P->d; pb.n_pos = n; pb.fsum = P->fsum;
    pb.seg_of_pos = P->p > 1 ? P->seg : nullptr;
    pb.nseg = P->p;
    pb.seg_tests = P->seg_tests;
    // the prefilter's tests are already in seg_tests (the build zeroed them); representatives
    // add theirs above
    pb.zero_seg_tests = P->reps == 0 && !P->prefilter;
    // the build's copy folded the score range of every partition (of one partition, into the
    // slots); its rows are the first list's unless representatives took some out
    pb.ranges_ready = P->p > 1 || !keep;
    pb.range_slots = P->p == 1;
    pb.extra_tests = reinterpret_cast<const unsigned long long*>(P->dinfo + D_TESTS_FILTER);
    pb.items = P->eng.w1;
    pb.n_items = n;
    pb.n_items_dev = (skip || keep || P->prefilter) ? cnt : nullptr;
    pb.ub_items = n;
    pb.flag_out = P->local_flag;
    pb.out_rounds = P->dinfo + D_ROUNDS_LOCAL;
    pb.out_tests = P->dinfo + D_TESTS_LOCAL;
    pb.out_tests_max = P->dinfo + D_TESTS_LOCAL_MAX;
    pb.ev_begin = P->ev_begin; pb.ev_end = P->ev_end; pb.ev_cap = P->ev_cap; pb.ev_used = &P->ev_used;
    SKY_TRY(run_engine(pb, P->eng, st));
    P->info.events_used = P->ev_used;
    return SKY_OK;
}

sky_status plan_final_phase(sky_plan* P, int64_t* sky_idx, int64_t cap, int64_t* dev_count, uint8_t* member,
                            hipStream_t st) {
    P->last_stream = st;
    const int32_t n = (int32_t)P->n;
    uint8_t* F = P->local_flag;  // per position: in the final skyline (with dom clear)
    if (P->p > 1) {
        // the union of the local skylines, in position order (spatially coherent); local_flag
        // becomes exactly the local skylines
        SKY_TRY(launch_compact_flags(P->local_flag, P->eng.dom, true, n, P->eng.w1, P->count_tmp + CT_UNION,
                                     P->dinfo + D_LOCAL_COUNT, P->eng.scan_tmp, st, P->count_tmp + CT_ROWS));
        EngineProblem pb{};
        pb.xp = P->xp; pb.ldp = P->ldp; pb.d = P->d; pb.n_pos = n; pb.fsum = P->fsum;
        pb.seg_of_pos = nullptr;
        pb.nseg = 1;
        pb.items = P->eng.w1;
        pb.n_items = 0;
        pb.n_items_dev = P->count_tmp + CT_UNION;
        pb.ub_items = n;
        pb.flag_out = P->final_flag;
        pb.out_rounds = P->dinfo + D_ROUNDS_MERGE;
        pb.out_tests = P->dinfo + D_TESTS_MERGE;
        pb.ev_begin = P->ev_begin; pb.ev_end = P->ev_end; pb.ev_cap = P->ev_cap; pb.ev_used = &P->ev_used;
        SKY_TRY(run_engine(pb, P->eng, st));
        P->info.events_used = P->ev_used;
        F = P->final_flag;
    }
    // the skyline's positions in curve order (the gres store of sky_gres reads them), with F
    // rewritten to the skyline itself
    SKY_TRY(launch_compact_flags(F, P->eng.dom, true, n, P->final_list, P->count_tmp + CT_SKY,
                                 P->dinfo + D_SKY_COUNT, P->eng.scan_tmp, st, P->count_tmp + CT_ROWS));
    return launch_final_output(P->final_list, P->count_tmp + CT_SKY, P->rowid, P->n, P->member_tmp, member,
                               sky_idx, cap, dev_count, P->pos_tmp, P->scan_tmp, P->dev_status, st);
}

sky_status check_opts(const sky_gres_opts* opts, int32_t* mapping) {
    *mapping = opts ? opts->mapping : SKY_GRES_AUTO;
    if (*mapping < SKY_GRES_AUTO || *mapping > SKY_GRES_LEVELS) return SKY_ERR_INVALID_ARG;
    if (opts && (opts->reserved != 0 || (!opts->ev_begin) != (!opts->ev_end))) return SKY_ERR_INVALID_ARG;
    return SKY_OK;
}

namespace {

void carve_gres_compute(Carver& c, GresStore& store, GresPrepTmp& tmp, GresTargets& tg, GresKeys& keys,
                        int64_t s, int32_t d, int32_t g_max, bool with_keys) {
    carve_gres_store(c, store, s, d, 1);
    carve_gres_prep_tmp(c, tmp, s);
    carve_gres_targets(c, tg, s, d);
    if (with_keys) carve_gres_keys(c, keys, store, d, g_max);
}

}  // namespace

size_t gres_ws_bytes(int64_t s, int32_t d, int32_t g_max, bool with_keys) {
    if (s < 0 || s > kMaxBuildRows || !valid_d(d) || g_max < 2 || g_max > SKY_MAX_G) return 0;
    Carver c(nullptr, 0);
    GresStore store{};
    GresPrepTmp tmp{};
    GresTargets tg{};
    GresKeys keys{};
    carve_gres_compute(c, store, tmp, tg, keys, s, d, g_max, with_keys);
    return c.used;
}

sky_status gres_compute_ws(const float* x_soa, int64_t n, int32_t d, int64_t ld, const int64_t* sky_idx,
                           int64_t s, int32_t g_max, int32_t* g_exit, float* gres, void* ws, size_t ws_bytes,
                           bool with_keys, int32_t* dev_status, const sky_gres_opts* opts, hipStream_t st) {
    if (s < 0 || s > kMaxBuildRows || !valid_d(d) || g_max < 2 || g_max > SKY_MAX_G) return SKY_ERR_INVALID_ARG;
    if (!dev_status) return SKY_ERR_INVALID_ARG;
    int32_t mapping = 0;
    SKY_TRY(check_opts(opts, &mapping));
    if (s == 0) return SKY_OK;
    if (!x_soa || !sky_idx || n < 1 || n > kMaxRows || ld < n || !ws) return SKY_ERR_INVALID_ARG;
    if (ws_bytes < gres_ws_bytes(s, d, g_max, with_keys)) return SKY_ERR_WORKSPACE;
    Carver c(ws, ws_bytes);
    GresStore store{};
    GresPrepTmp tmp{};
    GresTargets tg{};
    GresKeys keys{};
    carve_gres_compute(c, store, tmp, tg, keys, s, d, g_max, with_keys);
    if (c.overflow) return SKY_ERR_WORKSPACE;
    if (mapping == SKY_GRES_AUTO) mapping = gres_auto_mapping(s, g_max);
    SKY_TRY(launch_gres_prepare(x_soa, n, d, ld, sky_idx, s, store, tmp, dev_status, st));
    SKY_TRY(launch_gres_targets(x_soa, n, d, ld, nullptr, s, s, store, tg, dev_status, st));
    return launch_gres_search(store, d, (int32_t)s, tg, s, nullptr, nullptr, nullptr, g_max, mapping, g_exit, gres,
                              opts ? opts->ev_begin : nullptr, opts ? opts->ev_end : nullptr,
                              opts ? opts->dev_tests : nullptr, st, &keys);
}

}  // namespace sky

extern "C" {

sky_status sky_plan_partitions(const sky_plan* P, int32_t* part, void* stream) {
    if (!P || !part) return SKY_ERR_INVALID_ARG;
    if (P->state < 1) return SKY_ERR_STATE;
    if (P->p == 1)
        return launch_fill_u8(reinterpret_cast<uint8_t*>(part), P->n * (int64_t)sizeof(int32_t), 0,
                              (hipStream_t)stream);
    SKY_HIP(hipMemcpyAsync(part, P->part_of_row, (size_t)P->n * sizeof(int32_t), hipMemcpyDeviceToDevice,
                           (hipStream_t)stream));
    return SKY_OK;
}

sky_status sky_plan_local(const sky_plan* P, uint8_t* local, void* stream) {
    if (!P || !local) return SKY_ERR_INVALID_ARG;
    if (P->state < 2) return SKY_ERR_STATE;
    // before sky_merge the local skylines are the head rows not dominated; sky_merge rewrites
    // local_flag to exactly them (its own phase marks more rows dominated)
    // rows the build did not keep (the prefilter's) are in no local skyline
    SKY_TRY(launch_fill_u8(local, P->n, 0, (hipStream_t)stream));
    return launch_scatter_rows_live(P->local_flag, P->state == 2 ? P->eng.dom : nullptr, P->rowid, P->n,
                                    P->count_tmp + CT_ROWS, local, (hipStream_t)stream);
}

sky_status sky_plan_partition_tests(const sky_plan* P, int64_t* tests, void* stream) {
    if (!P || !tests) return SKY_ERR_INVALID_ARG;
    if (P->state < 2) return SKY_ERR_STATE;
    SKY_HIP(hipMemcpyAsync(tests, P->seg_tests, (size_t)P->p * sizeof(unsigned long long),
                           hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return SKY_OK;
}

sky_status sky_plan_set_events(sky_plan* P, void* const* ev_begin, void* const* ev_end, int32_t cap) {
    if (!P || cap < 0) return SKY_ERR_INVALID_ARG;
    if (cap > 0 && (!ev_begin || !ev_end)) return SKY_ERR_INVALID_ARG;
    P->ev_begin = cap > 0 ? ev_begin : nullptr;
    P->ev_end = cap > 0 ? ev_end : nullptr;
    P->ev_cap = cap;
    P->ev_used = 0;
    P->info.events_used = 0;
    return SKY_OK;
}

sky_status sky_plan_info(const sky_plan* P, sky_info* out) {
    if (!P || !out) return SKY_ERR_INVALID_ARG;
    *out = P->info;
    if (P->state < 2) return SKY_OK;
    // the counters the device wrote, read on the stream of the plan's last call
    int64_t dv[kDinfo];
    int32_t nk = 0, kept = 0;
    unsigned long long rt = 0;
    hipStream_t st = P->last_stream;
    SKY_HIP(hipMemcpyAsync(dv, P->dinfo, sizeof(dv), hipMemcpyDeviceToHost, st));
    SKY_HIP(hipMemcpyAsync(&kept, P->count_tmp + CT_ROWS, sizeof(kept), hipMemcpyDeviceToHost, st));
    if (P->reps > 0) {
        SKY_HIP(hipMemcpyAsync(&nk, P->rep_kept + SKY_MAX_REPS, sizeof(nk), hipMemcpyDeviceToHost, st));
        SKY_HIP(hipMemcpyAsync(&rt, P->rep_tests, sizeof(rt), hipMemcpyDeviceToHost, st));
    }
    SKY_HIP(hipStreamSynchronize(st));
    out->pruned_cells = (int32_t)dv[D_PRUNED_CELLS];
    out->pruned_rows = dv[D_PRUNED_ROWS];
    out->max_partition = dv[D_MAX_PART];
    out->rounds_local = (int32_t)dv[D_ROUNDS_LOCAL];
    out->tests_local = dv[D_TESTS_LOCAL] + (int64_t)rt;
    out->tests_local_max = dv[D_TESTS_LOCAL_MAX];
    out->reps_kept = nk;
    out->rows_kept = kept;
    out->tests_prefilter = dv[D_TESTS_FILTER];
    if (P->state >= 3) {
        out->sky_count = dv[D_SKY_COUNT];
        if (P->p > 1) {
            out->local_count = dv[D_LOCAL_COUNT];
            out->rounds_merge = (int32_t)dv[D_ROUNDS_MERGE];
            out->tests_merge = dv[D_TESTS_MERGE];
        } else {
            out->local_count = dv[D_SKY_COUNT];
        }
    }
    return SKY_OK;
}

void sky_plan_destroy(sky_plan* P) {
    delete P;
}

size_t gres_workspace_bytes(int64_t s, int32_t d, int32_t g_max) {
    return sky::gres_ws_bytes(s, d, g_max, true);
}


sky_status gres_compute(const float* x_soa, int64_t n, int32_t d, int64_t ld, const int64_t* sky_idx,
                        int64_t s, int32_t g_max, int32_t* g_exit, float* gres, void* ws,
                        size_t ws_bytes, int32_t* dev_status, const sky_gres_opts* opts,
                        void* stream) {
    return sky::gres_compute_ws(x_soa, n, d, ld, sky_idx, s, g_max, g_exit, gres, ws, ws_bytes, true,
                                dev_status, opts, (hipStream_t)stream);
}

sky_status sky_gres(sky_plan* P, int32_t g_max, int32_t* g_exit, float* gres, void* ws, size_t ws_bytes,
                    int32_t* dev_status, const sky_gres_opts* opts, void* stream) {
    if (!P || !dev_status || g_max < 2 || g_max > SKY_MAX_G) return SKY_ERR_INVALID_ARG;
    if (P->state != 3) return SKY_ERR_STATE;
    int32_t mapping = 0;
    SKY_TRY(check_opts(opts, &mapping));
    // the skyline size is on the device (count_tmp[CT_SKY]); the workspace holds the largest
    // skyline sky_merge could return in full
    const int64_t cap = P->merge_cap < P->n ? P->merge_cap : P->n;
    const int64_t c = cap > 0 ? cap : 1;
    if (!ws || ws_bytes < gres_workspace_bytes(c, P->d, g_max)) return SKY_ERR_WORKSPACE;
    Carver cv(ws, ws_bytes);
    GresStore store{};
    GresPrepTmp tmp{};
    GresTargets tg{};
    GresKeys keys{};
    carve_gres_compute(cv, store, tmp, tg, keys, c, P->d, g_max, true);
    if (cv.overflow) return SKY_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    P->last_stream = st;
    const int32_t* s_dev = P->count_tmp + CT_SKY;
    // candidates from the partition-contiguous copy at the skyline's positions (ascending, hence
    // curve order inside each partition); pos_tmp maps a row to its index in sky_idx
    // (every candidate is a target: written with the store, no exit yet)
    SKY_TRY(launch_gres_prepare_positions(P->xp, P->ldp, P->d, P->final_list, c, s_dev, P->rowid, P->pos_tmp,
                                          store, dev_status, st, &tg));
    return launch_gres_search(store, P->d, (int32_t)c, tg, c, s_dev, nullptr, nullptr, g_max, mapping, g_exit, gres,
                              opts ? opts->ev_begin : nullptr, opts ? opts->ev_end : nullptr,
                              opts ? opts->dev_tests : nullptr, st, &keys, true);
}

size_t gres_gbar_workspace_bytes(int64_t n) {
    if (n < 0 || n > kMaxRows) return 0;
    Carver c(nullptr, 0);
    GbarBuffers b{};
    carve_gbar(c, b, n);
    return c.used;
}

sky_status gres_gbar(const float* x_soa, int64_t n, int32_t d, int64_t ld, double* ell, int64_t* g_bar,
                     void* ws, size_t ws_bytes, int32_t* dev_status, void* stream) {
    if (n < 0 || n > kMaxRows || !valid_d(d) || !dev_status || (!ell && !g_bar)) return SKY_ERR_INVALID_ARG;
    if (n > 0 && (!x_soa || ld < n)) return SKY_ERR_INVALID_ARG;
    if (!ws || ws_bytes < gres_gbar_workspace_bytes(n)) return SKY_ERR_WORKSPACE;
    Carver c(ws, ws_bytes);
    GbarBuffers b{};
    carve_gbar(c, b, n);
    if (c.overflow) return SKY_ERR_WORKSPACE;
    return launch_gbar(x_soa, n, d, ld, b, ell, g_bar, dev_status, (hipStream_t)stream);
}

size_t gres_prepare_bytes(int64_t s, int32_t d) {
    if (s < 0 || s > kMaxBuildRows || !valid_d(d)) return 0;
    Carver c(nullptr, 0);
    GresStore store{};
    GresPrepTmp tmp{};
    carve_gres_store(c, store, s, d, 1);
    carve_gres_prep_tmp(c, tmp, s);
    return c.used;
}

sky_status gres_prepare(const float* x_soa, int64_t n, int32_t d, int64_t ld, const int64_t* cand_idx,
                        int64_t s, void* prep, size_t prep_bytes, int32_t* dev_status, void* stream) {
    if (s < 0 || s > kMaxBuildRows || !valid_d(d) || !dev_status || !prep) return SKY_ERR_INVALID_ARG;
    if (s > 0 && (!x_soa || !cand_idx || n < 1 || n > kMaxRows || ld < n)) return SKY_ERR_INVALID_ARG;
    if (prep_bytes < gres_prepare_bytes(s, d)) return SKY_ERR_WORKSPACE;
    Carver c(prep, prep_bytes);
    GresStore store{};
    GresPrepTmp tmp{};
    carve_gres_store(c, store, s, d, 1);
    carve_gres_prep_tmp(c, tmp, s);
    if (c.overflow) return SKY_ERR_WORKSPACE;
    return launch_gres_prepare(x_soa, n, d, ld, cand_idx, s, store, tmp, dev_status, (hipStream_t)stream);
}

size_t gres_search_bytes(int64_t nt, int32_t d) {
    // targets are indexed with 32-bit byte offsets inside each attribute column of the target
    // copy, like the rows of a plan
    if (nt < 0 || nt > kMaxBuildRows || !valid_d(d)) return 0;
    Carver c(nullptr, 0);
    GresTargets tg{};
    carve_gres_targets(c, tg, nt, d);
    return c.used;
}

sky_status gres_search(const void* prep, int64_t s, int32_t d, const float* x_soa, int64_t n, int64_t ld,
                       const int64_t* targets, int64_t nt, int32_t g_max, int32_t* g_exit, float* gres,
                       void* ws, size_t ws_bytes, int32_t* dev_status, const sky_gres_opts* opts,
                       void* stream) {
    if (!prep || s < 0 || s > kMaxBuildRows || !valid_d(d) || nt < 0 || nt > kMaxBuildRows || g_max < 2 ||
        g_max > SKY_MAX_G || !dev_status)
        return SKY_ERR_INVALID_ARG;
    if (!targets && nt != s) return SKY_ERR_INVALID_ARG;
    int32_t mapping = 0;
    SKY_TRY(check_opts(opts, &mapping));
    if (nt == 0) return SKY_OK;
    if (targets && (!x_soa || n < 1 || n > kMaxRows || ld < n)) return SKY_ERR_INVALID_ARG;
    if (!ws || ws_bytes < gres_search_bytes(nt, d)) return SKY_ERR_WORKSPACE;
    Carver cp(const_cast<void*>(prep), (size_t)-1);
    GresStore store{};
    carve_gres_store(cp, store, s, d, 1);
    Carver c(ws, ws_bytes);
    GresTargets tg{};
    carve_gres_targets(c, tg, nt, d);
    if (c.overflow) return SKY_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    if (mapping == SKY_GRES_AUTO) mapping = gres_auto_mapping(s, g_max);
    if (s == 0) return SKY_ERR_INVALID_ARG;  // targets need candidates to be tested against
    SKY_TRY(launch_gres_targets(x_soa, n, d, ld, targets, nt, s, store, tg, dev_status, st));
    return launch_gres_search(store, d, (int32_t)s, tg, nt, nullptr, nullptr, nullptr, g_max, mapping, g_exit, gres,
                              opts ? opts->ev_begin : nullptr, opts ? opts->ev_end : nullptr,
                              opts ? opts->dev_tests : nullptr, st);
}

}  // extern "C"
