// Private to the library: the host-side plan of the two-phase skyline and the internal calls
// that the batched path shares with the plain one.
#pragma once

#include "sky_internal.hpp"

struct sky_plan {
    // input
    const float* x = nullptr;
    int64_t n = 0, ld = 0;
    int32_t d = 0;
    int32_t scheme = 0, p = 1, m = 0, slice_dim = 0;
    int32_t* dev_status = nullptr;
    int32_t state = 0;
    // workspace regions
    float* xp = nullptr; int64_t ldp = 0;
    int32_t *rowid = nullptr, *seg = nullptr;
    float* fsum = nullptr;
    int32_t* part_off = nullptr;
    uint8_t* pruned = nullptr;
    double* tan2_dev = nullptr;
    unsigned long long* sel_key = nullptr;  // Sliced: [3 p] boundary keys, active prefixes, maxima
    int32_t* sel_i32 = nullptr;             // Sliced: selection histograms and state
    int64_t* seg_off_dev = nullptr;  // kSchemeSegments: dataset row offsets [p+1]
    int32_t *part_of_row = nullptr, *scan_tmp = nullptr;
    // the build's prefilter (killer rows per partition) and the kept rows
    bool prefilter = false;
    int32_t *pcount = nullptr, *krow = nullptr, *blk = nullptr;
    unsigned long long* kmin = nullptr;
    float* kval = nullptr;
    uint8_t* alive = nullptr;
    uint32_t *k0 = nullptr, *v0 = nullptr, *k1 = nullptr, *v1 = nullptr;
    float* xa = nullptr;  // row-major staging copy for the gathers into curve order
    int32_t reps = 0;     // Representative Filtering: representatives wanted (0 = off)
    int32_t* rep_kept = nullptr;  // [SKY_MAX_REPS] kept flags, then the kept count
    unsigned long long* rep_tests = nullptr;  // row-against-representative tests
    unsigned long long* seg_tests = nullptr;  // [p] local-phase tests per partition
    int32_t* radix_tmp = nullptr;
    sky::EngineBuffers eng{};
    uint8_t *local_flag = nullptr, *final_flag = nullptr, *member_tmp = nullptr;
    int32_t *local_list = nullptr, *final_list = nullptr, *pos_tmp = nullptr, *count_tmp = nullptr;
    int64_t* dinfo = nullptr;  // [kDinfo] device-side counters of sky_info (D_* below)
    int64_t merge_cap = 0;     // sky_idx capacity of the last sky_merge
    hipStream_t last_stream = nullptr;  // stream of the last call that queued work
    // host side
    void* const* ev_begin = nullptr;
    void* const* ev_end = nullptr;
    int32_t ev_cap = 0;
    int32_t ev_used = 0;
    sky_info info{};
};

namespace sky {

// device-side counters of a plan (int64 words of sky_plan::dinfo)
enum {
    D_PRUNED_CELLS = 0, D_PRUNED_ROWS, D_MAX_PART, D_ROUNDS_LOCAL, D_ROUNDS_MERGE, D_LOCAL_COUNT,
    D_SKY_COUNT, D_TESTS_LOCAL, D_TESTS_MERGE, D_TESTS_LOCAL_MAX, D_TESTS_FILTER, kDinfo = 16
};
// count_tmp words: the first round's list length, the union's, the skyline's, the positions
// of the partition-contiguous copy (rows the build kept)
enum { CT_LIST = 0, CT_UNION = 1, CT_SKY = 2, CT_ROWS = 3 };

constexpr int32_t kMaxRows = 0x7FFFFFFF;
constexpr int32_t kMaxBuildRows = 0x3FF00000;  // keeps every engine byte offset within 32 bits

// Workspace bytes of a plan (0 if the sizes are invalid).
size_t plan_bytes(int64_t n, int32_t d, int32_t scheme, int32_t p, int32_t m);
// Carve a plan from ws and (launch) queue its partition step. scheme may be kSchemeSegments,
// with seg_off_host = the p + 1 dataset row offsets (copied to the device before returning).
// reps: Representative Filtering's row count (0 = off); prefilter: drop the rows the killer
// rows of their partition dominate (only without representatives).
sky_status plan_build(const float* x, int64_t n, int32_t d, int64_t ld, int32_t scheme, int32_t p,
                      int32_t m, int32_t slice_dim, const int64_t* seg_off_host, int32_t reps, bool prefilter,
                      void* ws, size_t ws_bytes, int32_t* dev_status, hipStream_t st, sky_plan** out,
                      bool launch);
// Queue the partition step of a plan (re-reads its relation).
sky_status plan_partition(sky_plan* P, hipStream_t st);
// Sec. 3 phase 1 (the local skylines) and phase 2 (the union's skyline, its positions list
// and the ascending rows), never synchronising; no state checks.
sky_status plan_local_phase(sky_plan* P, hipStream_t st);
sky_status plan_final_phase(sky_plan* P, int64_t* sky_idx, int64_t cap, int64_t* dev_count, uint8_t* member,
                            hipStream_t st);

// gres options: the mapping (AUTO when opts is null); rejects unknown values and a lone event
sky_status check_opts(const sky_gres_opts* opts, int32_t* mapping);
// gres_compute's workspace and body; with_keys: also the packed key table of the tile search
// (taken when g_max and d allow it), which gres_compute always asks for
size_t gres_ws_bytes(int64_t s, int32_t d, int32_t g_max, bool with_keys);
sky_status gres_compute_ws(const float* x_soa, int64_t n, int32_t d, int64_t ld, const int64_t* sky_idx,
                           int64_t s, int32_t g_max, int32_t* g_exit, float* gres, void* ws, size_t ws_bytes,
                           bool with_keys, int32_t* dev_status, const sky_gres_opts* opts, hipStream_t st);

}  // namespace sky
