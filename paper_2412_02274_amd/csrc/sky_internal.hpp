// Internal declarations of libsky (not part of the C ABI).
//
// Device-side conventions
//  * Values handled by the kernels are "canonical": finite, in [0, 1), with -0.0 turned into
//    +0.0. For such values the IEEE order equals the order of the 32-bit patterns, so the
//    dominance tests (Def. 1) compare uint32 patterns: exact and independent of the
//    floating-point denormal mode.
//  * Projected keys (Def. 2) are floor(v * g) with one FP32 multiply rounded to nearest even.
//  * Wavefronts are 64 lanes (CDNA4); workgroups are 256 threads unless stated otherwise.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "sky.h"

namespace sky {

constexpr int kWave = 64;
constexpr int kBlock = 256;

// ----------------------------------------------------------------------------------------
// device helpers
// ----------------------------------------------------------------------------------------
__device__ __forceinline__ bool in_domain(float v) { return v >= 0.0f && v < 1.0f; }

// -0.0 -> +0.0 (both compare equal to 0); other values unchanged.
__device__ __forceinline__ float canon(float v) { return v == 0.0f ? 0.0f : v; }

__device__ __forceinline__ uint32_t fbits(float v) { return __float_as_uint(v); }

// Projected key at level g: one IEEE FP32 multiply (round to nearest even), then floor.
__device__ __forceinline__ int32_t qkey(float v, float g) {
    return (int32_t)floorf(__fmul_rn(v, g));
}

// First error wins.
__device__ __forceinline__ void raise_status(int32_t* st, int32_t code) {
    if (st) atomicCAS(st, 0, code);
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Lanes of the wave whose 'key' (low 'bits' bits) equals this lane's key, among the active
// lanes in 'active'.
__device__ __forceinline__ uint64_t match_any(uint32_t key, int bits, uint64_t active) {
    uint64_t m = active;
    for (int b = 0; b < bits; ++b) {
        uint64_t bal = __ballot((key >> b) & 1u);
        m &= ((key >> b) & 1u) ? bal : ~bal;
    }
    return m;
}

// ----------------------------------------------------------------------------------------
// host helpers
// ----------------------------------------------------------------------------------------
#define SKY_HIP(call)                                                      \
    do {                                                                   \
        hipError_t e_ = (call);                                            \
        if (e_ != hipSuccess) return SKY_ERR_HIP;                          \
    } while (0)

#define SKY_TRY(call)                                                      \
    do {                                                                   \
        sky_status s_ = (call);                                            \
        if (s_ != SKY_OK) return s_;                                       \
    } while (0)

// Bump allocator over caller workspace. With base == nullptr it only measures.
struct Carver {
    char* base;
    size_t cap;
    size_t used = 0;
    bool overflow = false;
    Carver(void* b, size_t c) : base(static_cast<char*>(b)), cap(c) {}
    template <class T>
    T* take(size_t count) {
        size_t off = (used + 255) & ~size_t(255);
        size_t bytes = count * sizeof(T);
        used = off + ((bytes + 255) & ~size_t(255));
        if (base && used > cap) overflow = true;
        return base ? reinterpret_cast<T*>(base + off) : nullptr;
    }
};

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

// ----------------------------------------------------------------------------------------
// launchers implemented in the .hip files
// ----------------------------------------------------------------------------------------

// sky_ingest.hip
sky_status launch_ingest(const float* x_rows, int64_t n, int32_t d, float* x_soa, int64_t ld,
                         int32_t* dev_status, hipStream_t st);

// sky_scan.hip: exclusive scan of n int32 values (n < 2^31); tmp needs scan_tmp_elems(n).
int64_t scan_tmp_elems(int64_t n);
sky_status launch_exclusive_scan(const int32_t* in, int32_t* out, int64_t n, int32_t* tmp,
                                 hipStream_t st);

// sky_radix.hip: stable LSD radix sort of (uint32 key, uint32 value) pairs, 8-bit digits,
// over the low 'key_bits' bits. Results end in (k0, v0) (the buffers are ping-ponged).
int64_t radix_tmp_elems(int64_t n);
sky_status launch_radix_sort(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, int64_t n,
                             int key_bits, int32_t* tmp, hipStream_t st);

// sky_partition.hip
struct PartitionArgs {
    const float* x; int64_t n; int32_t d; int64_t ld;
    int32_t scheme; int32_t p; int32_t m; int32_t slice_dim;
    const double* tan2;   // Angular thresholds tan^2(k*pi/(2m)), k = 0..m (device)
    float* xp; int64_t ldp;    // partition-contiguous canonical SoA copy
    int32_t* rowid;            // partitioned position -> original row
    int32_t* seg;              // partitioned position -> partition
    float* fsum;               // partitioned position -> FP32 attribute sum (SFS score)
    int32_t* part_off;         // [p+1]
    uint8_t* pruned;           // [p] Grid: pruned by grid dominance
    int32_t* part_of_row;      // [n] scratch
    int32_t* hist;             // [p * ntiles] scratch
    int32_t* scan_tmp;         // scan scratch
    uint32_t *k0, *v0, *k1, *v1; int32_t* radix_tmp; // Sliced sort scratch
    int32_t* dev_status;
};
int64_t partition_hist_elems(int64_t n, int32_t p);
sky_status launch_partition(const PartitionArgs& a, hipStream_t st);

// sky_skyline.hip: segmented skyline engine (see the file header)
struct EngineBuffers {
    int32_t* w0; int32_t* w1;      // work lists (capacity n)
    int32_t* head;                 // head items, segment-grouped (capacity n)
    int32_t* rest;                 // rest items, segment-grouped (capacity n)
    int32_t* fsky;                 // head skyline items, segment-grouped (capacity n)
    int32_t* out_list;             // confirmed skyline items (capacity n)
    uint32_t* seg_min; uint32_t* seg_max;   // [nseg]
    int32_t* hist;                 // [nseg * kBins]
    int32_t* seg_info;             // [nseg * 12] per-segment counters / offsets
    uint8_t* dom;                  // [n] dominated flags
    int32_t* tile_off;             // [2 * (nseg + 1)] tile offsets for head / rest
    int32_t* counters;             // [16] global counters
    unsigned long long* tests;     // [2] dominance-test counters
    int32_t* scan_tmp;
};
constexpr int kBins = 1024;
struct EngineProblem {
    const float* xp; int64_t ldp; int32_t d; int32_t n_pos;  // rows live at positions [0, n_pos)
    const float* fsum;             // score per position
    const int32_t* seg_of_pos;     // segment of a position (nullptr = single segment)
    int32_t nseg;
    const int32_t* items; int32_t n_items;  // initial work list (positions)
    uint8_t* flag_out;             // [n_pos] set to 1 for skyline items (must be zeroed)
    void* const* ev_begin;         // optional timing events around the test launches
    void* const* ev_end;
    int32_t ev_cap;
    int32_t* ev_used;              // host counter, advanced per recorded pair
};
struct EngineResult { int32_t count; int32_t rounds; int64_t tests; };
sky_status run_engine(const EngineProblem& pb, const EngineBuffers& b, int32_t* out_list,
                      EngineResult* res, hipStream_t st);
// helpers used by the API layer
sky_status launch_iota_filtered(const uint8_t* skip_seg, const int32_t* seg_of_pos, int32_t n,
                                int32_t* out, int32_t* count, hipStream_t st);
sky_status launch_fill_u8(uint8_t* p, int64_t n, uint8_t v, hipStream_t st);
// dst[rowid[q]] = src[q] for q < n (int32 and/or uint8 arrays)
sky_status launch_scatter_rows(const int32_t* src_i32, const uint8_t* src_u8, const int32_t* rowid,
                               int64_t n, int32_t* dst_i32, uint8_t* dst_u8, hipStream_t st);
sky_status launch_compact_flags(const uint8_t* flags, int32_t n, int32_t* out, int32_t* count,
                                hipStream_t st);
sky_status launch_final_output(const int32_t* list, int32_t count, const int32_t* rowid,
                               int64_t n, uint8_t* member_tmp, uint8_t* member_out,
                               int64_t* sky_idx, int64_t cap, int64_t* dev_count,
                               int32_t* pos_tmp, int32_t* scan_tmp, int32_t* dev_status,
                               hipStream_t st);

// sky_gres.hip
struct GresWork {
    float* cand;          // [d * s_pad] canonical candidates in spatial order
    float* lo;            // [d * t_pad] per-tile lower corner
    uint32_t *k0, *v0, *k1, *v1; int32_t* radix_tmp;
    int32_t* ge_sorted;   // [s]
    int64_t s_pad, t_pad;
};
int64_t gres_pad(int64_t s);
sky_status launch_gres(const float* x, int64_t n, int32_t d, int64_t ld, const int64_t* sky_idx,
                       int64_t s, int32_t g_max, int32_t mapping, int32_t* g_exit, float* gres,
                       const GresWork& w, int32_t* dev_status, void* ev_begin, void* ev_end,
                       hipStream_t st);

}  // namespace sky
