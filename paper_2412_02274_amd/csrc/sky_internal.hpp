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

// Exclusive prefix over a workgroup of NT threads of one int32 per thread; *total = the sum.
// ws: NT / kWave int32 of LDS. Every thread of the workgroup must call it.
template <int NT>
__device__ __forceinline__ int32_t block_exscan_t(int32_t v, int32_t* ws, int32_t* total) {
    const int lane = (int)lane_id(), wave = threadIdx.x / kWave;
    int32_t x = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const int32_t t = __shfl_up(x, off, kWave);
        if (lane >= off) x += t;
    }
    if (lane == kWave - 1) ws[wave] = x;
    __syncthreads();
    int32_t pre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NT / kWave; ++w) {
        const int32_t s = ws[w];
        pre += w < wave ? s : 0;
        tot += s;
    }
    __syncthreads();  // ws may be reused at once
    *total = tot;
    return pre + x - v;
}
__device__ __forceinline__ int32_t block_exscan(int32_t v, int32_t* ws, int32_t* total) {
    return block_exscan_t<kBlock>(v, ws, total);
}

// Hilbert-curve key of a point of canonical values in [0, 1): `bits` bits per attribute,
// bits * d <= 32. Coordinates are the top bits of the values (v * 2^bits, exact), mapped to
// the curve with J. Skilling's transposition algorithm ("Programming the Hilbert curve",
// AIP Conf. Proc. 707, 2004) and the transposed form is bit-interleaved into one integer.
// Points that are close on the curve are close in space, which keeps the boxes of tiles of
// consecutive points small.
__device__ __forceinline__ uint32_t hilbert_key(const float* v, int d, int bits) {
    uint32_t X[SKY_MAX_D];
    const float scale = (float)(1u << bits);
    const uint32_t cap = (1u << bits) - 1u;
    for (int k = 0; k < d; ++k) {
        const float t = v[k];
        uint32_t c = (t >= 0.0f && t < 1.0f) ? (uint32_t)(t * scale) : 0u;
        X[k] = c > cap ? cap : c;
    }
    const uint32_t M = 1u << (bits - 1);
    for (uint32_t Q = M; Q > 1; Q >>= 1) {  // inverse undo
        const uint32_t P = Q - 1;
        for (int i = 0; i < d; ++i) {
            if (X[i] & Q) {
                X[0] ^= P;
            } else {
                const uint32_t t = (X[0] ^ X[i]) & P;
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    for (int i = 1; i < d; ++i) X[i] ^= X[i - 1];  // Gray encode
    uint32_t t = 0;
    for (uint32_t Q = M; Q > 1; Q >>= 1)
        if (X[d - 1] & Q) t ^= Q - 1;
    for (int i = 0; i < d; ++i) X[i] ^= t;
    uint32_t code = 0;
    for (int b = bits - 1; b >= 0; --b)
        for (int i = 0; i < d; ++i) code = (code << 1) | ((X[i] >> b) & 1u);
    return code;
}

// bits per attribute of the curve keys: at most 24 bits in all (three 8-bit radix passes);
// 2^24 cells are far finer than the 64-row tiles the order serves
__host__ __device__ __forceinline__ int curve_bits(int d) {
    int b = 24 / d;
    return b > 16 ? 16 : (b < 1 ? 1 : b);
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

// sky_gbar.hip: ell and g_bar of Alg. 1's level range (Sec. 3.2), device outputs
struct GbarBuffers { uint32_t *k0, *v0, *k1, *v1; int32_t* radix_tmp; unsigned long long* minbits; };
void carve_gbar(Carver& c, GbarBuffers& b, int64_t n);
sky_status launch_gbar(const float* x, int64_t n, int32_t d, int64_t ld, const GbarBuffers& b,
                       double* ell, int64_t* g_bar, int32_t* dev_status, hipStream_t st);

// sky_ingest.hip
sky_status launch_project(const float* x, int64_t n, int32_t d, int64_t ld, const int64_t* rows,
                          int64_t s, int32_t g, float* out, int64_t ld_out, int32_t* dev_status,
                          hipStream_t st);
sky_status launch_ingest(const float* x_rows, int64_t n, int32_t d, float* x_soa, int64_t ld,
                         int32_t* dev_status, hipStream_t st);
sky_status launch_literal_level(const uint8_t* member, int64_t s, int32_t g, int32_t* g_exit, int32_t* nil_left,
                                hipStream_t st);

// sky_scan.hip: exclusive scan of n int32 values (n < 2^31); tmp needs scan_tmp_elems(n).
int64_t scan_tmp_elems(int64_t n);
sky_status launch_exclusive_scan(const int32_t* in, int32_t* out, int64_t n, int32_t* tmp,
                                 hipStream_t st);

// sky_radix.hip: stable LSD radix sort of (uint32 key, uint32 value) pairs, 8-bit digits,
// over the low 'key_bits' bits. Results end in (k0, v0) (the buffers are ping-ponged), or, when
// out_k and out_v are given, wherever the last pass left them (no final copy). With n_dev the
// pairs are the first min(*n_dev, n) (a count on the device; n bounds it and sizes the grids).
int64_t radix_tmp_elems(int64_t n);
sky_status launch_radix_sort(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, int64_t n,
                             int key_bits, int32_t* tmp, hipStream_t st,
                             const uint32_t** out_k = nullptr, const uint32_t** out_v = nullptr,
                             const int32_t* n_dev = nullptr);

// sky_partition.hip
// Internal partition scheme of the batched path: partition j = the rows [seg_off[j],
// seg_off[j+1]) of one dataset (datasets are contiguous row ranges of one SoA buffer).
constexpr int32_t kSchemeSegments = 64;

struct PartitionArgs {
    const float* x; int64_t n; int32_t d; int64_t ld;
    int32_t scheme; int32_t p; int32_t m; int32_t slice_dim;
    const int64_t* seg_off;    // kSchemeSegments: [p+1] row offsets of the datasets (device)
    double* tan2;              // Angular thresholds tan^2(k*pi/(2m)), k = 0..m (device, written here)
    unsigned long long* sel_key;  // Sliced: [3 p] scratch: boundary keys, active prefixes, and the
                                  // largest key of each prefix's rows
    int32_t* sel_i32;          // Sliced: [slice_select_elems(p)] scratch
    bool prefilter;            // drop the rows their partition's killer rows dominate (else keep all)
    float* xp; int64_t ldp;    // partition-contiguous canonical SoA copy of the kept rows
    int32_t* rowid;            // position -> original row
    int32_t* seg;              // position -> partition
    float* fsum;               // position -> FP32 attribute sum (SFS score)
    int32_t* n_live;           // device: positions in the copy (rows kept)
    int32_t* part_off;         // [p+1] partition offsets over all rows (partition sizes)
    uint8_t* pruned;           // [p] Grid: pruned by grid dominance
    int32_t* part_of_row;      // [n] partition of every row (p > 1)
    int32_t* pcount;           // [p] scratch: rows per partition
    unsigned long long* kmin;  // [p * SKY_KILLERS] scratch: per-slot minima of (score, row)
    int32_t* krow;             // [p * SKY_KILLERS] scratch: killer rows (-1: none)
    float* kval;               // [p * SKY_KILLERS][row stride] scratch: killer values
    uint8_t* alive;            // [n] scratch: rows kept
    int32_t* blk;              // [partition_blocks(n)] scratch: rows kept per workgroup
    int32_t* scan_tmp;         // scan scratch (scan_tmp_elems(partition_blocks(n)))
    uint32_t *k0, *v0, *k1, *v1; int32_t* radix_tmp;  // sort scratch (n)
    float* xa;                 // [n][partition_row_stride(d)] row-major canonical staging copy
    unsigned long long* seg_tests;  // [p] out: the prefilter's tests per partition
    unsigned long long* tests;      // out: the prefilter's tests in all
    uint32_t* smin; uint32_t* smax; // [p] out: per partition, the smallest and largest score
                                    // (bit pattern) of its positions
    int32_t* iota_out;              // optional [n] out: 0, 1, ... for every position of the copy
    int64_t* stats_out;             // [3] out: pruned non-empty cells, rows inside them, rows of the
                                    // largest partition
    int32_t* dev_status;
};
inline int32_t partition_row_stride(int32_t d) { return d <= 4 ? 4 : (d <= 8 ? 8 : 16); }
// int32 scratch of the Sliced boundary selection: the first digit's histogram (2^14 bins), one
// 256-bin histogram per boundary, and per-boundary state
inline int64_t slice_select_elems(int32_t p) { return 16384 + 256 * (int64_t)p + 4 * (int64_t)p + 64; }
// workgroups of the per-row passes of launch_partition (4096 rows each)
int64_t partition_blocks(int64_t n);
sky_status launch_partition(const PartitionArgs& a, hipStream_t st);


// sky_reps.hip: Representative Filtering (Sec. 3.1)
struct RepArgs {
    const float* fsum; const int32_t* rowid; int32_t n; int32_t d;  // the plan's score per position
    const float* xp; int64_t ldp;       // partition-contiguous copy
    const float* xa; int32_t rs;        // row-major staging copy (stride rs)
    int32_t k;                          // representatives wanted
    uint32_t *k0, *v0, *k1, *v1; int32_t* radix_tmp;  // sort scratch (n)
    int32_t* kept;                      // [SKY_MAX_REPS] out: 1 if kept
    int32_t* nkept;                     // out: kept count (device)
    unsigned long long* tests;          // out: row-against-representative tests (device)
    const int32_t* seg_of_pos;          // segment of a position (nullptr = one segment)
    unsigned long long* seg_tests;      // optional [nseg]: the same tests added per segment
    const uint8_t* skip_seg;            // optional [nseg]: segments whose rows are not tested
    uint8_t* keep;                      // [n] out: 1 for positions no kept representative dominates
};
sky_status launch_representatives(const RepArgs& a, hipStream_t st);

// Persistent launches: workgroups draw work from kWorkCounters counters kCounterStride int32
// apart (one 128-byte line each), so that no single address takes every atomic (measured: one
// counter adds 0.23 ms to the 1M x 6 skyline step; 64 counters beat 32 by 0.5-0.7% there and on
// the 4096-relation batch, 128 gained nothing more; on the gres search 8 were slower than 32).
constexpr int kWorkCounters = 64;
constexpr int kCounterStride = 32;
// Workgroups of `kernel` (block threads, dyn_lds bytes of dynamic LDS) that the current device
// holds at once, from the runtime's occupancy calculation.
sky_status resident_workgroups(const void* kernel, int32_t block, size_t dyn_lds, int32_t* out);
// fn = the instantiation of a kernel template over the attribute count d (0: any d)
#define SKY_KERNEL_PTR_D(d, KERNEL, fn)                                   \
    switch (d) {                                                          \
        case 1: fn = reinterpret_cast<const void*>(&KERNEL<1>); break;    \
        case 2: fn = reinterpret_cast<const void*>(&KERNEL<2>); break;    \
        case 3: fn = reinterpret_cast<const void*>(&KERNEL<3>); break;    \
        case 4: fn = reinterpret_cast<const void*>(&KERNEL<4>); break;    \
        case 5: fn = reinterpret_cast<const void*>(&KERNEL<5>); break;    \
        case 6: fn = reinterpret_cast<const void*>(&KERNEL<6>); break;    \
        case 7: fn = reinterpret_cast<const void*>(&KERNEL<7>); break;    \
        case 8: fn = reinterpret_cast<const void*>(&KERNEL<8>); break;    \
        default: fn = reinterpret_cast<const void*>(&KERNEL<0>); break;   \
    }

// sky_skyline.hip: segmented skyline engine (see the file header)
struct EngineBuffers {
    int32_t* w0;                   // rest groups of every second round (capacity n)
    int32_t* w1;                   // the first round's list (filled by the caller, capacity n)
    int32_t* head;                 // head groups, 64-aligned per segment (capacity hcap)
    int32_t* rest;                 // rest groups of the other rounds (capacity n)
    int32_t* rhb;                  // [n] at the first rest item of each 64-item group: the
                                   // segment's head rows before it in position order
    uint32_t* hval;                // [d][hcap] head candidate bit patterns
    uint32_t* hlo;                 // [d][tcap] per-tile lower corners
    uint32_t* hhi;                 // [d][tcap] per-tile upper corners
    int64_t hcap, tcap;
    uint32_t* seg_min; uint32_t* seg_max;   // [range_elems(nseg)]
    int32_t* hist;                 // [2][nseg * kBins] (by round parity)
    int32_t* seg_info;             // [2][nseg * 8] per-segment counters / offsets (by round parity)
    uint8_t* dom;                  // [n] dominated flags
    int32_t* tile_off;             // [2 * (nseg + 1)] item-tile offsets for head / rest
    int32_t* counters;             // [3 * 16]: the run's counters, then two per-round sets
    unsigned long long* tests;     // [3] dominance-test counters (head, rest, spare)
    int32_t* work;                 // [kWorkCounters * kCounterStride] work counters of the test launch
    int32_t* scan;                 // [engine_scan_elems(n)] per-block counts of the split
    int32_t* scan_tmp;             // scan scratch for n values
};
int64_t engine_head_capacity(int64_t n, int32_t nseg);
// Score ranges of one segment are first gathered in kRangeSlots slots kRangeStride words apart
// (slot 0 at index 0), so that thousands of workgroups do not queue on one address; the
// skyline run's first kernel folds them into index 0. Several segments: one word each.
constexpr int kRangeSlots = 64;
constexpr int kRangeStride = 32;
constexpr int64_t range_elems(int64_t nseg) { return nseg > 1 ? nseg : (int64_t)kRangeSlots * kRangeStride; }
int64_t engine_scan_elems(int64_t n);
constexpr int kBins = 1024;
struct EngineProblem {
    const float* xp; int64_t ldp; int32_t d; int32_t n_pos;  // rows live at positions [0, n_pos)
    const float* fsum;             // score per position
    const int32_t* seg_of_pos;     // segment of a position (nullptr = single segment)
    int32_t nseg;
    unsigned long long* seg_tests; // optional [nseg]: tests added per segment
    bool zero_seg_tests;           // the run zeroes seg_tests first (else the caller has)
    bool ranges_ready;             // the caller has set b.seg_min / b.seg_max: for every segment, a
                                   // range of score bit patterns holding every item's score
    bool range_slots;              // with ranges_ready and one segment: the range is still spread
                                   // over the kRangeSlots slots
    const int32_t* items;          // initial work list (positions); not one of the engine's buffers
    int32_t n_items;               // its length, when n_items_dev is null
    const int32_t* n_items_dev;    // its length on the device (or null)
    int64_t ub_items;              // with n_items_dev: an upper bound on that length
    uint8_t* flag_out;             // [n_pos] zeroed by the run; 1 for every row that entered a head
    int64_t* out_rounds;           // optional device words written at the end of the run: rounds
    int64_t* out_tests;            //   with live items, dominance tests evaluated, and the largest
    int64_t* out_tests_max;        //   count of one segment (the total without seg_tests)
    const unsigned long long* extra_tests;  // optional device word added to out_tests (tests the
                                            // caller evaluated before the run, already in seg_tests)
    void* const* ev_begin;         // optional timing events around the test launches
    void* const* ev_end;
    int32_t ev_cap;
    int32_t* ev_used;              // host counter, advanced per recorded pair
};
// A run queues a fixed launch sequence (no host synchronisation). Afterwards the skyline of
// every segment is the set of positions with flag_out = 1 and b.dom = 0.
sky_status run_engine(const EngineProblem& pb, const EngineBuffers& b, hipStream_t st);
// helpers used by the API layer
// (scan_tmp: scan_tmp_elems(n) int32 of scratch, for these and launch_final_output)
sky_status launch_iota_filtered(const uint8_t* skip_seg, const int32_t* seg_of_pos, int32_t n,
                                int32_t* out, int32_t* count, int32_t* scan_tmp, hipStream_t st,
                                const uint8_t* keep = nullptr);
sky_status launch_fill_u8(uint8_t* p, int64_t n, uint8_t v, hipStream_t st);
// dst[rowid[q]] = src[q] && !(drop && drop[q]) for q < n (q < min(n, *count) with count, a
// device word)
sky_status launch_scatter_rows_live(const uint8_t* src, const uint8_t* drop, const int32_t* rowid, int64_t n,
                                    const int32_t* count, uint8_t* dst, hipStream_t st);
// positions i < n with flags[i] != 0 and (drop null or drop[i] == 0), in order, into out; their
// number into *count32 and *count64 (either may be null); with bake, flags[i] is rewritten to
// the selection. With bound (a device word), only positions i < min(n, *bound) are read and
// rewritten (the caller guarantees that no later position is selected).
sky_status launch_compact_flags(uint8_t* flags, const uint8_t* drop, bool bake, int32_t n, int32_t* out,
                                int32_t* count32, int64_t* count64, int32_t* scan_tmp, hipStream_t st,
                                const int32_t* bound = nullptr);
// ascending rows of the positions list[0, *count) (count on the device, at most n):
// sky_idx[0, min(count, cap)), *dev_count = count (SKY_ERR_CAPACITY above cap), member_out[row]
// (optional), and pos_tmp[row] = the row's index in sky_idx for every skyline row
sky_status launch_final_output(const int32_t* list, const int32_t* count, const int32_t* rowid, int64_t n,
                               uint8_t* member_tmp, uint8_t* member_out, int64_t* sky_idx,
                               int64_t cap, int64_t* dev_count, int32_t* pos_tmp, int32_t* scan_tmp,
                               int32_t* dev_status, hipStream_t st);

// sky_gres.hip
// Prepared candidate store: segments 64-aligned in Hilbert order, padding value 2.0.
struct GresStore {
    float* cand; int64_t ccap;     // [d][ccap]
    float* lo; float* hi; int64_t tcap;  // [d][tcap] per-tile boxes (global tile index)
    uint32_t* ckey;                // [ccap] curve keys (sorted within a segment)
    int32_t* perm;                 // [ccap] caller index of each slot (-1 for padding)
    int32_t* seg_coff;             // [nseg] first slot of each segment (multiple of 64)
    int32_t* seg_cnt;              // [nseg] candidates of each segment
    int32_t nseg;
};
struct GresPrepTmp { uint32_t *k0, *v0, *k1, *v1; int32_t* radix_tmp; };
struct GresTargets {
    float* tval; int64_t tvcap;    // [d][tvcap] target values
    int32_t* thint;                // [tvcap] starting tile of each target (local to its segment)
    int32_t* tout;                 // [tvcap] output index of each target (-1: none)
    int32_t* ge;                   // [tvcap] result per target
    int32_t* gstart;               // [tvcap] highest level worth searching per target
    int32_t* work;                 // work counters of the search (zeroed before each launch)
    int32_t* params;               // [16] the search's shape when its target count is on the device
};
void carve_gres_store(Carver& c, GresStore& st, int64_t s, int32_t d, int32_t nseg);
// Keys of every candidate slot at every level g in [2, levels + 1], packed into one 64-bit word
// per (level, slot): attribute k's key in a field of `width` bits at bit k * width, the field's
// top bit clear (a guard bit for the dominance test's subtraction), width = key_width(d, g_max)
// of the search. Usable when the fields hold every key (g_max <= kKeyTableMaxG,
// d * width <= 64) and g_max - 1 <= levels.
constexpr int32_t kKeyTableMaxG = 64;
struct GresKeys {
    uint64_t* key = nullptr;       // [levels][kslots] candidates (the last 64 slots of a row: padding)
    uint4* tile = nullptr;         // [levels][ktiles] tile boxes: lower corner (x, y), upper (z, w)
    uint64_t* chunk = nullptr;     // [levels][ktiles] lower corner of the 64 tiles from a chunk's first
    int32_t* ok = nullptr;         // set on the device: the store's slots in use fit the tables
    int64_t kslots = 0, ktiles = 0;
    int32_t levels = 0;
    const int32_t* used = nullptr; // slots in use (device; null: the first segment's tiles)
};
// field width for g_max (0: the keys of d attributes do not fit one word)
int32_t key_width(int32_t d, int32_t g_max);
// tables for the store's own capacity, g_max - 1 levels (none when key_width is 0)
void carve_gres_keys(Carver& c, GresKeys& k, const GresStore& store, int32_t d, int32_t g_max);
// tables for `slots` candidate slots (padding tile included), `levels` levels
void carve_gres_keys_slots(Carver& c, GresKeys& k, int64_t slots, int32_t levels);
void carve_gres_prep_tmp(Carver& c, GresPrepTmp& t, int64_t s);
void carve_gres_targets(Carver& c, GresTargets& t, int64_t nt, int32_t d);
sky_status launch_gres_prepare(const float* x, int64_t n, int32_t d, int64_t ld, const int64_t* rows,
                               int64_t s, const GresStore& store, const GresPrepTmp& tmp,
                               int32_t* dev_status, hipStream_t st);
// Store from a plan's partition-contiguous copy xp: the candidates are the rows at positions
// pos[0, s) (ascending, hence curve order), s = min(*s_dev, cap) read on the device (more than
// cap raises SKY_ERR_CAPACITY); perm[slot] = idx_of_row[rowid[pos]]. The store is carved for cap.
// With tg given, every candidate is also written as a target (values, own tile as the hint,
// caller index) with no exit yet (tg.ge = 1), so that the search can skip its own fill (ge_ready).
sky_status launch_gres_prepare_positions(const float* xp, int64_t ldp, int32_t d, const int32_t* pos,
                                         int64_t cap, const int32_t* s_dev, const int32_t* rowid,
                                         const int32_t* idx_of_row, const GresStore& store,
                                         int32_t* dev_status, hipStream_t st, const GresTargets* tg = nullptr);
sky_status launch_gres_targets(const float* x, int64_t n, int32_t d, int64_t ld, const int64_t* rows,
                               int64_t nt, int64_t s, const GresStore& store, const GresTargets& tg,
                               int32_t* dev_status, hipStream_t st);
// Batched relations (segments of one plan): sky_off[j] / cand_off[j] = the first index of
// relation j's rows in the ascending skyline list sky_idx[0, min(*count_dev, cap)) (row_off =
// the relations' row offsets); the candidate store (relation j in curve order from a 64-aligned
// slot, read from the plan's copy at the skyline's positions pos, relation-major) with its tile
// boxes; used[0] = slots in use, used[1] = the largest relation's skyline.
sky_status launch_batch_store(const float* xp, int64_t ldp, int32_t d, const int32_t* pos,
                              const int32_t* rowid, const int32_t* idx_of_row, const int64_t* sky_idx,
                              const int32_t* count_dev, int64_t cap, const int64_t* row_off, int32_t nseg,
                              int64_t* sky_off, int32_t* cand_off, int32_t* used, const GresStore& store,
                              hipStream_t st);
// The gres of every skyline tuple of every relation: targets (tseg[q] = relation of target q),
// with lpt the longest-first order tord (order / rank_off: nseg and nseg + 1 int32 of scratch),
// then one persistent search over all of them; counts and shape read on the device.
sky_status launch_batch_search(const GresStore& store, int32_t d, int64_t cap, const int32_t* cand_off,
                               int32_t nseg, const int32_t* used, bool near_first, bool lpt, int32_t* order,
                               int32_t* rank_off, int32_t* tord, int32_t* tseg, const GresTargets& tg,
                               int32_t g_max, int32_t mapping, int32_t* g_exit, float* gres, void* ev_begin,
                               void* ev_end, unsigned long long* dev_tests, hipStream_t st,
                               const GresKeys* keys = nullptr);
// measured (both mappings with per-target start levels): lanes over 64 levels pay off when
// many levels lie below the start levels (g_max >= 2^17) or on small skylines with
// g_max > 1000; otherwise the banded tile walk is faster
__host__ __device__ inline int32_t gres_auto_mapping(int64_t s, int32_t g_max) {
    if (s > 8192) return SKY_GRES_TILES;
    return (g_max >= (1 << 17) || (g_max > 1000 && s <= 1024)) ? SKY_GRES_LEVELS : SKY_GRES_TILES;
}
// One segment of max_cnt candidates, nt targets. nt_dev: the target count is min(*nt_dev, nt)
// on the device, nt being an upper bound; the mapping (AUTO included) and the work split are then
// decided on the device. tseg (a batch): every target q of segment tseg[q] (in the order tord,
// when given) as persistent work, with tg.params already holding the count and shape. keys
// (tables of at least g_max - 1 levels; for a batch with keys->used set): the tile search runs
// on packed keys, the tables built here, when key_width(d, g_max) allows them and the store's
// slots in use fit them (decided on the device; the values are searched otherwise).
sky_status launch_gres_search(const GresStore& store, int32_t d, int32_t max_cnt,
                              const GresTargets& tg, int64_t nt, const int32_t* nt_dev, const int32_t* tseg,
                              const int32_t* tord, int32_t g_max, int32_t mapping, int32_t* g_exit,
                              float* gres, void* ev_begin, void* ev_end,
                              unsigned long long* dev_tests, hipStream_t st,
                              const GresKeys* keys = nullptr, bool ge_ready = false);

}  // namespace sky
