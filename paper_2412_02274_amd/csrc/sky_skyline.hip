// Segmented skyline engine: the skyline (Def. 1) of every segment of a set of rows, all
// segments at once. Used for the local skylines of the partitions (Sec. 3, phase 1; one
// segment per partition) and for the final skyline of their union (phase 2; one segment).
//
// Rounds of "head skyline, then filter" in the spirit of SFS (the scan order of a monotone
// score; Sec. 2 scoring functions, Sec. 4 SFS):
//   1. per segment, the FP32 attribute sum f of the live rows is binned between the
//      segment's min and max; the head is the set of rows in the lowest bins holding at
//      least H_r rows (all the live rows once there are at most A_r of them, which ends the
//      segment in one all-pairs round instead of several small ones). f is monotone: a row
//      dominating another has f <= the other's f (FP32 additions are monotone), so every
//      dominator of a head row is itself in the head.
//   2. head skyline: every head row is tested against the other head rows of its segment.
//      The survivors are exactly the segment's skyline rows inside the head (their
//      dominators would be in the head), so they are final.
//   3. filter: every other live row is tested against the head rows of its segment (a row
//      dominated by a head row is dominated by a head skyline row, by transitivity, so
//      testing against all head rows is exact); the survivors form the next live set. Every
//      head row leaves the live set, so the rounds terminate.
// Rows are compared through their canonical FP32 bit patterns (exact for [0, 1) data).
//
// Scheduling without the host. The host never reads a count back: every kernel reads its
// item count on the device, grids are sized by upper bounds known before the run, and the
// number of rounds is fixed in advance. Round r uses H_r = 8192 * 4^(r-1) and
// A_r = 65536 * 16^(r-1); the host stops at the first round whose bound on the live rows is at
// most A_r, and that round takes every live row into the head, so the run always ends there
// (two rounds up to about 10^6 rows, three up to 1.6 * 10^7).
// Rounds after the data ran out find no live item and do nothing. A run is therefore a fixed
// launch sequence that a HIP graph can capture.
// The result is a pair of byte arrays: flag_out[pos] = 1 for every row that entered a head,
// dom[pos] = 1 for every row found dominated; the skyline rows are those with flag_out = 1 and
// dom = 0.
//
// Spatial pruning. Positions index a partition-contiguous copy whose rows are in Hilbert-curve
// order inside each partition, and every list of the engine stays in position order
// (stable scan-based compactions). So each segment's head group is a spatially coherent
// sequence; it is stored 64-aligned (values and positions) and cut into tiles of 64 with the
// componentwise minimum `lo` and maximum `hi` of each tile. A tile can hold a dominator of t
// only if lo <= t in every attribute; if moreover hi <= t everywhere and hi < t somewhere,
// every row of the (non-empty) tile dominates t. So an item is tested against the candidates
// of a tile only when the box allows a dominator there and does not already decide (exact: no
// dominator is ever skipped, none is ever invented).
//
// The test kernel is register-tiled like an n-body step: a wavefront holds 64 items (one per
// lane) and walks the head tiles of their segment. Every 64 tiles it keeps only those whose
// lower corner is <= the componentwise maximum of its live items (no other tile can pass any
// of them); each kept tile's box is tested against all items at once, and the tile's 64
// candidates are loaded once and tested against every item that passed the box. The passing
// items are compacted in LDS and broadcast one by one against the 64 candidate lanes, so each
// of the k steps keeps every lane busy. One candidate load serves all the items. A workgroup caches the tile boxes of its
// current segment in LDS when they fit (a barrier only when the segment changes).
// Bound: VALU compares (candidate values are a few hundred KB per segment and stay in cache).
#include "sky_internal.hpp"

namespace sky {

namespace {

constexpr int kHead = 4096;      // head rows per segment in the first round (target)
constexpr int kAllHead = 65536;  // first round: a segment with at most this many live rows takes them all
constexpr int kMaxRounds = 16;   // schedule cap (the last round takes every live row)
constexpr int kTargetWaves = 8192;  // waves per test launch the item split aims at
constexpr int kTile = 64;     // candidates per tile box
constexpr int kProbe = 8;     // best-score candidates of a tile tried first against all items
constexpr uint32_t kPad = 0x7FFFFFFFu;  // padding candidates: above every real value, also as int32
constexpr int kBoxLds = 4096;           // uint32 tile-box values cached in LDS per workgroup
constexpr uint32_t kMaxGrid = 8192;     // workgroups of the grid-stride kernels
constexpr uint32_t kTestGridLater = 2048;  // most workgroups of a test launch after the first round
constexpr uint32_t kGridLater = 1024;      // most workgroups of a row pass after the first round

// seg_info layout per segment (int32 x kInfo)
enum { SI_LIVE = 0, SI_BSTAR, SI_HEADN, SI_HEADOFF, SI_RESTN, SI_RESTOFF, SI_LISTOFF, SI_HEADPRE, kInfo = 8 };
// per-round counters (two sets, alternating with the round's parity)
enum { C_SPARE = 0, C_HTILES, C_RTILES, C_MAXH, C_HTOT, C_RTOT, C_TPUH, C_TPUR, kCounters = 16 };
// counters of the whole run (the set before the two round sets)
enum { G_ROUNDS = 0 };

// head target (grows 4x per round) and all-head limit (16x per round) of round r (from 1)
__host__ __device__ inline int64_t round_head(int32_t r) {
    const int64_t v = (int64_t)kHead << (2 * (r - 1));
    return v < 0x7FFFFFFF ? v : 0x7FFFFFFF;
}
__host__ __device__ inline int64_t round_all(int32_t r) {
    if (r > 5) return 0x7FFFFFFF;
    const int64_t v = (int64_t)kAllHead << (4 * (r - 1));
    return v < 0x7FFFFFFF ? v : 0x7FFFFFFF;
}

template <int D>
__device__ __forceinline__ int dget(int d) { return D > 0 ? D : d; }

// base[idx] with a 32-bit byte offset (a wave-uniform base plus a per-lane offset); callers
// keep idx below 2^30 (rows are capped accordingly).
__device__ __forceinline__ uint32_t ld32(const uint32_t* base, uint32_t idx) {
    return *reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(base) + (idx << 2));
}

__device__ __forceinline__ int32_t seg_of(const int32_t* seg_of_pos, int32_t pos) {
    return seg_of_pos ? seg_of_pos[pos] : 0;
}

// Bitwise OR of v over the 64 lanes (every lane receives it).
__device__ __forceinline__ uint32_t wave_or_u32(uint32_t v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v |= (uint32_t)__shfl_xor((int32_t)v, off);
    return v;
}

// Maximum of v over the 64 lanes (every lane receives it).
__device__ __forceinline__ int32_t wave_max_i32(int32_t v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const int32_t o = __shfl_xor(v, off);
        v = o > v ? o : v;
    }
    return v;
}

// Start of a run: output flags cleared, the round records and histograms of both parities
// cleared, every segment's score range empty (fold: the one segment's range slots folded into
// its range instead), counters zeroed (and the per-segment test counters, when given).
__global__ void __launch_bounds__(kBlock) engine_init_kernel(
    int32_t n_pos, uint8_t* __restrict__ flag_out, int32_t nseg, int32_t* __restrict__ hist2,
    int32_t* __restrict__ info2, uint32_t* __restrict__ smin, uint32_t* __restrict__ smax,
    int32_t fold, int32_t* __restrict__ counters, unsigned long long* __restrict__ tests,
    unsigned long long* __restrict__ seg_tests) {
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t gs = (int64_t)gridDim.x * kBlock;
    const int64_t n16 = n_pos / 16;  // flag_out is 256-byte aligned
    for (int64_t i = g; i < n16; i += gs) reinterpret_cast<uint4*>(flag_out)[i] = make_uint4(0u, 0u, 0u, 0u);
    for (int64_t i = n16 * 16 + g; i < n_pos; i += gs) flag_out[i] = 0;
    for (int64_t i = g; i < 2 * (int64_t)nseg * kBins; i += gs) hist2[i] = 0;
    for (int64_t i = g; i < 2 * (int64_t)nseg * kInfo; i += gs) info2[i] = 0;
    for (int64_t i = g; i < nseg; i += gs) {
        if (smin && !fold) {  // (null: the caller has set the score ranges)
            smin[i] = 0xFFFFFFFFu;
            smax[i] = 0u;
        }
        if (seg_tests) seg_tests[i] = 0ull;
    }
    if (fold && g < kWave) {  // one wave: the slots' minimum and maximum into index 0
        const int lane = (int)g;
        uint32_t a0 = lane < kRangeSlots ? smin[lane * kRangeStride] : 0xFFFFFFFFu;
        uint32_t a1 = lane < kRangeSlots ? smax[lane * kRangeStride] : 0u;
        for (int off = kWave / 2; off > 0; off >>= 1) {
            const uint32_t x = __shfl_xor(a0, off, kWave), y = __shfl_xor(a1, off, kWave);
            a0 = x < a0 ? x : a0;
            a1 = y > a1 ? y : a1;
        }
        if (lane == 0) {
            smin[0] = a0;
            smax[0] = a1;
        }
    }
    if (g < 3 * kCounters) counters[g] = 0;
    if (g < 3) tests[g] = 0ull;
}

// Multi-segment passes over a round's list. The list is in position order and segments are
// runs of positions, so a wavefront's kSegPer * 64 consecutive items (lane l takes items
// l, l + 64, ...) fall into one or a few segments: each lane folds its items into runs of one
// segment, a lane flushes a run only when its segment changes, and the lanes' last runs are
// combined per segment across the wavefront, so the global atomics are a few per wavefront
// instead of one per item (they all land on a few lines per segment).
constexpr int kSegPer = 16;
__host__ __device__ constexpr int64_t seg_pass_blocks(int64_t n) {
    return (n + (int64_t)kBlock * kSegPer - 1) / ((int64_t)kBlock * kSegPer);
}
// Items per lane of a run-folding pass over n items (n read on the device): at most kSegPer,
// fewer when the grid (sized for an upper bound) has more lanes than needed, so that a short
// list still spreads over every wave instead of leaving a few waves a long chain of loads.
__device__ __forceinline__ int seg_per_lane(int64_t n) {
    const int64_t lanes = (int64_t)gridDim.x * kBlock;
    const int64_t pl = (n + lanes - 1) / lanes;
    return pl < 1 ? 1 : (pl > kSegPer ? kSegPer : (int)pl);
}

// Score range (min and max of f) of every segment over the first round's list.
__global__ void __launch_bounds__(kBlock) minmax_kernel(const int32_t* __restrict__ items,
                                                         int32_t n_host, const int32_t* __restrict__ n_dev,
                                                         const float* __restrict__ fsum,
                                                         const int32_t* __restrict__ seg_of_pos,
                                                         uint32_t* __restrict__ smin,
                                                         uint32_t* __restrict__ smax) {
    const int32_t n = n_dev ? *n_dev : n_host;
    const int lane = (int)lane_id();
    const int pl = seg_per_lane(n);
    const int64_t wbase = ((int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave) * (kWave * pl);
    int32_t cs = -1;  // segment of the lane's current run
    uint32_t cmin = 0xFFFFFFFFu, cmax = 0u;
    for (int j = 0; j < pl; ++j) {
        const int64_t i = wbase + (int64_t)j * kWave + lane;
        if (i >= n) break;
        const int32_t pos = items[i];
        const int32_t sg = seg_of(seg_of_pos, pos);
        const uint32_t fb = fbits(fsum[pos]);  // f >= 0: bit order == value order
        if (sg != cs) {
            if (cs >= 0) {
                atomicMin(&smin[cs], cmin);
                atomicMax(&smax[cs], cmax);
            }
            cs = sg;
            cmin = fb;
            cmax = fb;
        } else {
            cmin = fb < cmin ? fb : cmin;
            cmax = fb > cmax ? fb : cmax;
        }
    }
    const bool valid = cs >= 0;
    uint64_t act = __ballot(valid);
    while (act) {
        const int leader = __ffsll((unsigned long long)act) - 1;
        const int32_t sl = __shfl(cs, leader, kWave);
        const bool mine = valid && cs == sl;
        const uint64_t peers = __ballot(mine);
        uint32_t vmin = mine ? cmin : 0xFFFFFFFFu, vmax = mine ? cmax : 0u;
        for (int off = kWave / 2; off > 0; off >>= 1) {
            const uint32_t a = __shfl_xor(vmin, off, kWave), b = __shfl_xor(vmax, off, kWave);
            vmin = a < vmin ? a : vmin;
            vmax = b > vmax ? b : vmax;
        }
        if (lane == leader) {
            atomicMin(&smin[sl], vmin);
            atomicMax(&smax[sl], vmax);
        }
        act &= ~peers;
    }
}

// Single-segment variant: grid-stride with block reductions.
__global__ void __launch_bounds__(kBlock) minmax1_kernel(const int32_t* __restrict__ items,
                                                          int32_t n_host, const int32_t* __restrict__ n_dev,
                                                          const float* __restrict__ fsum,
                                                          uint32_t* __restrict__ smin,
                                                          uint32_t* __restrict__ smax) {
    const int32_t n = n_dev ? *n_dev : n_host;
    __shared__ uint32_t rmin[kBlock / kWave], rmax[kBlock / kWave];
    uint32_t vmin = 0xFFFFFFFFu, vmax = 0u;
    for (int32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        uint32_t fb = fbits(fsum[items[i]]);
        vmin = fb < vmin ? fb : vmin;
        vmax = fb > vmax ? fb : vmax;
    }
    for (int off = kWave / 2; off > 0; off >>= 1) {
        uint32_t a = __shfl_xor(vmin, off, kWave), b = __shfl_xor(vmax, off, kWave);
        vmin = a < vmin ? a : vmin;
        vmax = b > vmax ? b : vmax;
    }
    const int wave = threadIdx.x / kWave;
    if (lane_id() == 0) { rmin[wave] = vmin; rmax[wave] = vmax; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / kWave; ++w) {
            vmin = rmin[w] < vmin ? rmin[w] : vmin;
            vmax = rmax[w] > vmax ? rmax[w] : vmax;
        }
        if (vmin <= vmax) {
            atomicMin(&smin[0], vmin);
            atomicMax(&smax[0], vmax);
        }
    }
}

__device__ __forceinline__ int32_t bin_of(float f, float lo, float scale) {
    // monotone non-decreasing in f
    float t = __fmul_rn(__fsub_rn(f, lo), scale);
    int32_t b = (int32_t)t;
    return b < 0 ? 0 : (b > kBins - 1 ? kBins - 1 : b);
}

__device__ __forceinline__ float seg_scale(uint32_t lo, uint32_t hi) {
    float span = __fsub_rn(__uint_as_float(hi), __uint_as_float(lo));
    return span > 0.0f ? (float)kBins / span : 0.0f;
}

__device__ __forceinline__ int32_t item_bin(const float* fsum, const uint32_t* smin,
                                            const uint32_t* smax, int32_t s, int32_t pos) {
    return bin_of(fsum[pos], __uint_as_float(smin[s]), seg_scale(smin[s], smax[s]));
}

// head threshold of segment s, by one wavefront: the lowest bins holding at least `want` rows
// (all the live rows when there are at most `all_below` of them)
__device__ void thresh_segment(int32_t s, const int32_t* __restrict__ hist, int32_t* __restrict__ info,
                               int32_t want_head, int32_t all_below) {
    const int lane = (int)lane_id();
    const int32_t* h = hist + (int64_t)s * kBins;
    const int32_t live = info[s * kInfo + SI_LIVE];
    // few rows left: all of them form the head, and the segment finishes in this round
    const int32_t want = live <= all_below ? live : want_head;
    int32_t hv[kBins / kWave];  // the whole histogram in flight at once (one round trip)
#pragma unroll
    for (int it = 0; it < kBins / kWave; ++it) hv[it] = h[it * kWave + lane];
    int32_t run = 0, bstar = kBins - 1, headn = live;
#pragma unroll
    for (int it = 0; it < kBins / kWave; ++it) {
        int32_t inc = hv[it];
        for (int off = 1; off < kWave; off <<= 1) {
            int32_t o = __shfl_up(inc, off, kWave);
            if (lane >= off) inc += o;
        }
        uint64_t hit = __ballot(run + inc >= want);
        if (hit) {
            int l = __ffsll((unsigned long long)hit) - 1;
            bstar = it * kWave + l;
            headn = run + __shfl(inc, l, kWave);
            break;
        }
        run += __shfl(inc, kWave - 1, kWave);
    }
    if (lane == 0) {
        info[s * kInfo + SI_BSTAR] = bstar;
        info[s * kInfo + SI_HEADN] = headn;
        info[s * kInfo + SI_RESTN] = live - headn;
    }
}

// the head thresholds of many segments at once, one wave each
__global__ void __launch_bounds__(kBlock) thresh_kernel(int32_t nseg, const int32_t* __restrict__ hist,
                                                         int32_t* __restrict__ info, int32_t want_head,
                                                         int32_t all_below) {
    const int32_t s = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    if (s < nseg) thresh_segment(s, hist, info, want_head, all_below);
}

// Per segment: list offset (scan of live counts), 64-aligned head offset (scan of head counts
// rounded up to 64), rest offset, and the item-tile offsets of both groups; round totals and
// the test launch's work split. Run by one whole workgroup, sequential over blocks of 256
// segments.
__device__ void round_layout(int32_t nseg, int32_t* __restrict__ info, int32_t* __restrict__ tile_off,
                             int32_t* __restrict__ counters) {
    // tiles per unit of the test launch, from the exact counts: split the head tiles of an item
    // group over several units when there are too few groups to fill the chip (kTargetWaves)
    __shared__ int64_t red[3][kBlock / kWave];
    {
        int64_t gh = 0, gr = 0, mt = 0;
        for (int32_t s = threadIdx.x; s < nseg; s += kBlock) {
            const int32_t hn = info[s * kInfo + SI_HEADN], rn = info[s * kInfo + SI_RESTN];
            gh += (hn + kBlock - 1) / kBlock;
            gr += (rn + kBlock - 1) / kBlock;
            const int64_t nt = (hn + kTile - 1) / kTile;
            mt = nt > mt ? nt : mt;
        }
        for (int off = kWave / 2; off > 0; off >>= 1) {
            gh += __shfl_xor(gh, off, kWave);
            gr += __shfl_xor(gr, off, kWave);
            const int64_t o = __shfl_xor(mt, off, kWave);
            mt = o > mt ? o : mt;
        }
        if (lane_id() == 0) {
            red[0][threadIdx.x / kWave] = gh;
            red[1][threadIdx.x / kWave] = gr;
            red[2][threadIdx.x / kWave] = mt;
        }
    }
    __syncthreads();
    int64_t gh = 0, gr = 0, mt = 1;
    for (int w = 0; w < kBlock / kWave; ++w) {
        gh += red[0][w];
        gr += red[1][w];
        mt = red[2][w] > mt ? red[2][w] : mt;
    }
    // rest groups aim at a quarter of the units: their items mostly fall to the first tiles
    // they meet, so tile ranges tested side by side repeat tests more than they gain in
    // parallelism (measured on 10M x 4 rows, one partition: 3% off the step)
    constexpr int64_t kWantUnits = kTargetWaves / (kBlock / kWave);
    auto tpu_of = [&](int64_t groups, int64_t want) -> int32_t {
        const int64_t t = (groups * mt + want - 1) / want;
        return (int32_t)(t < 1 ? 1 : (t > mt ? mt : t));
    };
    const int32_t tpu_h = tpu_of(gh, kWantUnits), tpu_r = tpu_of(gr, kWantUnits / 4);
    constexpr int Q = 6;
    __shared__ int32_t carry[Q];
    __shared__ int32_t wsum[Q][kBlock / kWave];
    __shared__ int32_t wmax[kBlock / kWave];
    __shared__ int32_t maxh;
    if (threadIdx.x == 0) {
        for (int q = 0; q < Q; ++q) carry[q] = 0;
        maxh = 0;
    }
    __syncthreads();
    const int lane = (int)lane_id();
    const int wave = threadIdx.x / kWave;
    for (int base = 0; base < nseg; base += kBlock) {
        int32_t s = base + threadIdx.x;
        int32_t v[Q] = {0, 0, 0, 0, 0, 0};
        int32_t hn = 0;
        if (s < nseg) {
            hn = info[s * kInfo + SI_HEADN];
            int32_t rn = info[s * kInfo + SI_RESTN];
            v[0] = (hn + kTile - 1) / kTile * kTile;    // aligned head slots
            v[1] = rn;                                   // rest items
            const int32_t ntile = (hn + kTile - 1) / kTile;
            v[2] = (hn + kBlock - 1) / kBlock * ((ntile + tpu_h - 1) / tpu_h);  // head units
            v[3] = (rn + kBlock - 1) / kBlock * ((ntile + tpu_r - 1) / tpu_r);  // rest units
            v[4] = info[s * kInfo + SI_LIVE];            // live items
            v[5] = hn;                                   // head items (unaligned)
        }
        int32_t inc[Q];
        for (int q = 0; q < Q; ++q) {
            inc[q] = v[q];
            for (int off = 1; off < kWave; off <<= 1) {
                int32_t o = __shfl_up(inc[q], off, kWave);
                if (lane >= off) inc[q] += o;
            }
            if (lane == kWave - 1) wsum[q][wave] = inc[q];
        }
        int32_t mh = hn;
        for (int off = kWave / 2; off > 0; off >>= 1) {
            int32_t o = __shfl_xor(mh, off, kWave);
            mh = o > mh ? o : mh;
        }
        if (lane == 0) wmax[wave] = mh;
        __syncthreads();
        int32_t excl[Q];
        for (int q = 0; q < Q; ++q) {
            int32_t before = carry[q];
            for (int w = 0; w < wave; ++w) before += wsum[q][w];
            excl[q] = before + inc[q] - v[q];
        }
        if (s < nseg) {
            info[s * kInfo + SI_HEADOFF] = excl[0];
            info[s * kInfo + SI_RESTOFF] = excl[1];
            info[s * kInfo + SI_LISTOFF] = excl[4];
            info[s * kInfo + SI_HEADPRE] = excl[5];
            tile_off[s] = excl[2];
            tile_off[(nseg + 1) + s] = excl[3];
        }
        __syncthreads();
        if (threadIdx.x == kBlock - 1)
            for (int q = 0; q < Q; ++q) carry[q] = excl[q] + v[q];
        if (threadIdx.x == 0)
            for (int w = 0; w < kBlock / kWave; ++w) maxh = wmax[w] > maxh ? wmax[w] : maxh;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        tile_off[nseg] = carry[2];
        tile_off[(nseg + 1) + nseg] = carry[3];
        counters[C_HTILES] = carry[2];
        counters[C_RTILES] = carry[3];
        counters[C_MAXH] = maxh;
        counters[C_HTOT] = carry[0];
        counters[C_RTOT] = carry[1];
        counters[C_TPUH] = tpu_h;
        counters[C_TPUR] = tpu_r;
    }
}

struct StatsArgs {
    const int32_t* items; int32_t n_host; const int32_t* n_dev;  // the round's list
    const uint8_t* dead;         // rounds after the first: items with dead[pos] != 0 are gone
    const float* fsum; const int32_t* seg_of_pos; int32_t nseg;
    const uint32_t* smin; const uint32_t* smax;
    int32_t* hist; int32_t* info;           // this round's (its parity)
    int32_t* hist_next; int32_t* info_next; // the next round's, cleared here
};

// First kernel of a round: clears the next round's records and histograms (the round that last
// used that parity has finished) and adds the round's live items to their segment's live count
// and score histogram. One segment: grid-stride with an LDS histogram. Several: every workgroup
// takes a contiguous range of kBlock * kSegPer-item chunks (segments are runs of consecutive
// items), histograms the segment of each chunk's first item in LDS (flushed when it changes)
// and folds live counts into per-lane runs of one segment.
template <bool MULTI>
__global__ void __launch_bounds__(kBlock) stats_kernel(StatsArgs a) {
    __shared__ int32_t lh[kBins];
    __shared__ int32_t lcnt;
    const int32_t n = a.n_dev ? *a.n_dev : a.n_host;
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t gs = (int64_t)gridDim.x * kBlock;
    for (int64_t i = g; i < (int64_t)a.nseg * kBins; i += gs) a.hist_next[i] = 0;
    for (int64_t i = g; i < (int64_t)a.nseg * kInfo; i += gs) a.info_next[i] = 0;
    for (int b = threadIdx.x; b < kBins; b += kBlock) lh[b] = 0;
    if (threadIdx.x == 0) lcnt = 0;
    __syncthreads();
    const int lane = (int)lane_id();
    if (!MULTI) {
        const float lo = __uint_as_float(a.smin[0]);
        const float scale = seg_scale(a.smin[0], a.smax[0]);
        int32_t c = 0;
        for (int64_t i = g; i < n; i += gs) {
            const int32_t pos = a.items[i];
            if (a.dead && a.dead[pos]) continue;
            atomicAdd(&lh[bin_of(a.fsum[pos], lo, scale)], 1);
            ++c;
        }
        for (int off = kWave / 2; off > 0; off >>= 1) c += __shfl_xor(c, off, kWave);
        if (lane == 0 && c) atomicAdd(&lcnt, c);
        __syncthreads();
        for (int b = threadIdx.x; b < kBins; b += kBlock)
            if (lh[b]) atomicAdd(&a.hist[b], lh[b]);
        if (threadIdx.x == 0 && lcnt) atomicAdd(&a.info[SI_LIVE], lcnt);
        return;
    }
    const int pl = seg_per_lane(n);
    const int64_t kChunk = (int64_t)kBlock * pl;
    const int64_t nchunk = (n + kChunk - 1) / kChunk;
    const int64_t per = (nchunk + gridDim.x - 1) / gridDim.x;
    const int64_t c_end = ((int64_t)blockIdx.x + 1) * per < nchunk ? ((int64_t)blockIdx.x + 1) * per : nchunk;
    int32_t hs = -1;  // segment whose histogram is in lh (block-uniform)
    for (int64_t cidx = (int64_t)blockIdx.x * per; cidx < c_end; ++cidx) {
        const int64_t bbase = cidx * kChunk;
        const int32_t s0 = seg_of(a.seg_of_pos, a.items[bbase]);  // block-uniform
        if (s0 != hs) {
            __syncthreads();
            if (hs >= 0)
                for (int b = threadIdx.x; b < kBins; b += kBlock)
                    if (lh[b]) {
                        atomicAdd(&a.hist[(int64_t)hs * kBins + b], lh[b]);
                        lh[b] = 0;
                    }
            hs = s0;
            __syncthreads();
        }
        const float lo0 = __uint_as_float(a.smin[s0]);
        const float sc0 = seg_scale(a.smin[s0], a.smax[s0]);
        const int64_t wbase = bbase + (int64_t)(threadIdx.x / kWave) * (kWave * pl);
        int32_t cs = -1, ccnt = 0;  // the lane's current run of live items of one segment
        for (int j = 0; j < pl; ++j) {
            const int64_t i = wbase + (int64_t)j * kWave + lane;
            if (i >= n) break;
            const int32_t pos = a.items[i];
            if (a.dead && a.dead[pos]) continue;
            const int32_t sg = seg_of(a.seg_of_pos, pos);
            if (sg == s0) atomicAdd(&lh[bin_of(a.fsum[pos], lo0, sc0)], 1);
            else atomicAdd(&a.hist[(int64_t)sg * kBins + item_bin(a.fsum, a.smin, a.smax, sg, pos)], 1);
            if (sg != cs) {
                if (cs >= 0) atomicAdd(&a.info[cs * kInfo + SI_LIVE], ccnt);
                cs = sg;
                ccnt = 1;
            } else {
                ++ccnt;
            }
        }
        const bool valid = cs >= 0;
        uint64_t act = __ballot(valid);
        while (act) {
            const int leader = __ffsll((unsigned long long)act) - 1;
            const int32_t sl = __shfl(cs, leader, kWave);
            const bool mine = valid && cs == sl;
            const uint64_t peers = __ballot(mine);
            int32_t v = mine ? ccnt : 0;
            for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
            if (lane == leader) atomicAdd(&a.info[sl * kInfo + SI_LIVE], v);
            act &= ~peers;
        }
    }
    __syncthreads();
    if (hs >= 0)
        for (int b = threadIdx.x; b < kBins; b += kBlock)
            if (lh[b]) atomicAdd(&a.hist[(int64_t)hs * kBins + b], lh[b]);
}

// The round's layout, one workgroup: every segment's head (thresh_segment), the offsets of its
// groups and the test launch's split (round_layout); the test launch's work counters cleared;
// the round counted when it has live items.
__global__ void __launch_bounds__(kBlock) layout_kernel(int32_t nseg, const int32_t* __restrict__ hist,
                                                         int32_t* __restrict__ info, int32_t* __restrict__ tile_off,
                                                         int32_t* __restrict__ counters, int32_t* __restrict__ work,
                                                         int32_t* __restrict__ gcounters, int32_t head_want,
                                                         int32_t all_below, int32_t thresh_here) {
    if (thresh_here) {  // few segments: their thresholds first, one wave each
        const int wave = threadIdx.x / kWave;
        for (int32_t s = wave; s < nseg; s += kBlock / kWave) thresh_segment(s, hist, info, head_want, all_below);
        __syncthreads();
    }
    round_layout(nseg, info, tile_off, counters);
    if (work)
        for (int i = threadIdx.x; i < kWorkCounters * kCounterStride; i += kBlock) work[i] = 0;
    if (threadIdx.x == 0 && counters[C_HTOT] > 0) ++gcounters[G_ROUNDS];
}

// ---- stable split of a round's list into head and rest groups ------------------------------
// Chunks of kCItems consecutive list entries; every workgroup takes a contiguous range of
// chunks. Kernel 1 counts the head entries and the live entries of every workgroup's range,
// kernel 2 gets its range's prefixes by summing the counts of the workgroups before it (no
// waiting on other workgroups), ranks entries inside each chunk with wave ballots over 64-entry
// sub-chunks in order, and scatters. The result is in list order (stable).
constexpr int kCItems = 1024;
constexpr int kCChunks = kCItems / kWave;  // 16 sub-chunks of 64 entries
constexpr int64_t kSplitGrid = 1024;       // most workgroups of a split launch

// sum of cnt[0, b) by the whole block (every thread gets it)
__device__ __forceinline__ int32_t block_prefix(const int32_t* __restrict__ cnt, int32_t b) {
    __shared__ int32_t part[kBlock / kWave];
    int32_t v = 0;
    for (int32_t j = threadIdx.x; j < b; j += kBlock) v += cnt[j];
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    if (lane_id() == 0) part[threadIdx.x / kWave] = v;
    __syncthreads();
    int32_t t = 0;
    for (int w = 0; w < kBlock / kWave; ++w) t += part[w];
    __syncthreads();
    return t;
}

// in-order exclusive prefix of the kCChunks sub-chunk counts of a chunk (sub-chunk c is handled
// by wave c % 4); *total gets their sum
__device__ __forceinline__ void chunk_prefix(int32_t* chunk_cnt, int32_t* total) {
    __syncthreads();
    if (threadIdx.x < kWave) {
        const int lane = (int)lane_id();
        int32_t v = lane < kCChunks ? chunk_cnt[lane] : 0;
        int32_t inc = v;
        for (int off = 1; off < kWave; off <<= 1) {
            const int32_t o = __shfl_up(inc, off, kWave);
            if (lane >= off) inc += o;
        }
        if (lane < kCChunks) chunk_cnt[lane] = inc - v;
        if (lane == kCChunks - 1) *total = inc;
    }
    __syncthreads();
}

__device__ __forceinline__ bool is_head(int32_t pos, const float* fsum, const int32_t* seg_of_pos,
                                        const uint32_t* smin, const uint32_t* smax, const int32_t* info,
                                        int32_t& s) {
    s = seg_of(seg_of_pos, pos);
    return item_bin(fsum, smin, smax, s, pos) <= info[s * kInfo + SI_BSTAR];
}

struct SplitArgs {
    const int32_t* items; int32_t n_host; const int32_t* n_dev; const uint8_t* dead;
    const float* fsum; const int32_t* seg_of_pos; const uint32_t* smin; const uint32_t* smax;
    const int32_t* info;
    int32_t* bcnt;              // [2][gridDim.x]: head entries, then live entries, per workgroup
    int32_t* head; int32_t* rest; int32_t* rhb;
    uint8_t* dom_clear;         // first round: dom of every list item cleared (else null)
    uint8_t* flag_out;          // set to 1 for every head item
};

// the workgroup's chunk range [c0, c1)
__device__ __forceinline__ void split_range(int32_t n, int64_t* c0, int64_t* c1) {
    const int64_t nchunk = ((int64_t)n + kCItems - 1) / kCItems;
    const int64_t per = (nchunk + gridDim.x - 1) / gridDim.x;
    *c0 = (int64_t)blockIdx.x * per;
    *c1 = *c0 + per < nchunk ? *c0 + per : nchunk;
}

__global__ void __launch_bounds__(kBlock) split_count_kernel(SplitArgs a) {
    const int32_t n = a.n_dev ? *a.n_dev : a.n_host;
    __shared__ int32_t part[2][kBlock / kWave];
    const int wave = threadIdx.x / kWave;
    const int lane = (int)lane_id();
    int64_t c0, c1;
    split_range(n, &c0, &c1);
    int32_t nh = 0, nl = 0;
    const int64_t end = c1 * kCItems < n ? c1 * kCItems : n;
    for (int64_t i = c0 * kCItems + threadIdx.x; i < end; i += kBlock) {
        const int32_t pos = a.items[i];
        const bool live = !a.dead || a.dead[pos] == 0;
        int32_t sg;
        const bool h = live && is_head(pos, a.fsum, a.seg_of_pos, a.smin, a.smax, a.info, sg);
        nh += h;
        nl += live;
    }
    for (int off = kWave / 2; off > 0; off >>= 1) {
        nh += __shfl_xor(nh, off, kWave);
        nl += __shfl_xor(nl, off, kWave);
    }
    if (lane == 0) {
        part[0][wave] = nh;
        part[1][wave] = nl;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t th = 0, tl = 0;
        for (int w = 0; w < kBlock / kWave; ++w) {
            th += part[0][w];
            tl += part[1][w];
        }
        a.bcnt[blockIdx.x] = th;
        a.bcnt[gridDim.x + blockIdx.x] = tl;
    }
}

// live head entries -> their segment's head group (and flag_out), the other live entries -> its
// rest group, both in list order
__global__ void __launch_bounds__(kBlock) split_scatter_kernel(SplitArgs a) {
    const int32_t n = a.n_dev ? *a.n_dev : a.n_host;
    __shared__ int32_t chunk_h[kCChunks], chunk_l[kCChunks];
    __shared__ int32_t tot_h, tot_l;
    const int wave = threadIdx.x / kWave;
    const int lane = (int)lane_id();
    int64_t c0, c1;
    split_range(n, &c0, &c1);
    int32_t pre_h = block_prefix(a.bcnt, blockIdx.x);
    int32_t pre_l = block_prefix(a.bcnt + gridDim.x, blockIdx.x);
    constexpr int kPer = kCChunks / (kBlock / kWave);
    const uint64_t lt = __lanemask_lt();
    for (int64_t cidx = c0; cidx < c1; ++cidx) {
        int32_t mpos[kPer], mseg[kPer];
        uint64_t mh[kPer], ml[kPer];
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int ch = wave + q * (kBlock / kWave);
            const int64_t i = cidx * kCItems + ch * kWave + lane;
            int32_t pos = -1, sg = 0;
            bool live = false, h = false;
            if (i < n) {
                pos = a.items[i];
                live = !a.dead || a.dead[pos] == 0;
                h = live && is_head(pos, a.fsum, a.seg_of_pos, a.smin, a.smax, a.info, sg);
            }
            mpos[q] = live ? pos : -1;
            mseg[q] = sg;
            mh[q] = __builtin_amdgcn_ballot_w64(h);
            ml[q] = __builtin_amdgcn_ballot_w64(live);
            if (lane == 0) {
                chunk_h[ch] = __popcll(mh[q]);
                chunk_l[ch] = __popcll(ml[q]);
            }
        }
        chunk_prefix(chunk_h, &tot_h);
        chunk_prefix(chunk_l, &tot_l);
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int ch = wave + q * (kBlock / kWave);
            if (mpos[q] < 0) continue;
            const bool h = (mh[q] >> lane) & 1ull;
            const int32_t* si = a.info + mseg[q] * kInfo;
            // head / live items before this one in the whole list, minus those of earlier segments
            const int32_t hr = pre_h + chunk_h[ch] + __popcll(mh[q] & lt) - si[SI_HEADPRE];
            const int32_t lr = pre_l + chunk_l[ch] + __popcll(ml[q] & lt) - si[SI_LISTOFF];
            if (h) {
                a.head[si[SI_HEADOFF] + hr] = mpos[q];
                a.flag_out[mpos[q]] = 1;
            } else {
                const int32_t ri = lr - hr;  // rest index in the segment
                a.rest[si[SI_RESTOFF] + ri] = mpos[q];
                // where the test kernel's wave of items [ri, ri + 64) starts in the head tiles
                if ((ri & (kWave - 1)) == 0) a.rhb[si[SI_RESTOFF] + ri] = hr;
            }
            if (a.dom_clear) a.dom_clear[mpos[q]] = 0;
        }
        pre_h += tot_h;
        pre_l += tot_l;
        __syncthreads();  // chunk_h / chunk_l / totals are rewritten by the next chunk
    }
}

// largest s with info[s].field <= v (the field ascending in s)
__device__ __forceinline__ int32_t find_segment(const int32_t* info, int32_t nseg, int field,
                                                int32_t v) {
    int32_t lo = 0, hi = nseg - 1;
    while (lo < hi) {
        int32_t mid = (lo + hi + 1) >> 1;
        if (info[mid * kInfo + field] <= v) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// One wave per 64-slot tile of the aligned head buffer: candidate values (pads = kPad, pad
// positions = -1) and the tile box: componentwise minimum lo and maximum hi of its rows. Inside
// the tile the rows are put in ascending score order (ties by slot), pads last: a row with a
// smaller attribute sum dominates more of the space around the tile, so the test kernel's
// early-exit probe meets the likeliest dominators first. The box does not depend on the order.
template <int D>
__global__ void __launch_bounds__(kBlock) head_values_kernel(
    const float* __restrict__ xp, int64_t ldp, int32_t d_rt, const float* __restrict__ fsum,
    int32_t nseg, const int32_t* __restrict__ info, const int32_t* __restrict__ counters,
    int32_t* __restrict__ head, uint32_t* __restrict__ hval, int64_t hcap,
    uint32_t* __restrict__ hlo, uint32_t* __restrict__ hhi, int64_t tcap) {
    constexpr int DM = D > 0 ? D : SKY_MAX_D;
    const int d = dget<D>(d_rt);
    const int lane = (int)lane_id();
    const int32_t htot = counters[C_HTOT];
    for (int32_t tile = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; tile * kTile < htot;
         tile += gridDim.x * (kBlock / kWave)) {
        const int32_t j0 = tile * kTile;
        const int32_t j = j0 + lane;
        const int32_t s = find_segment(info, nseg, SI_HEADOFF, j0);
        const bool valid = j < info[s * kInfo + SI_HEADOFF] + info[s * kInfo + SI_HEADN];
        const int32_t pos0 = valid ? head[j] : -1;
        // bitonic sort of (score bits, slot) over the 64 lanes; scores are >= 0, so their bit
        // patterns order like the values, and pads (all ones) go last
        uint64_t key = ((uint64_t)(valid ? fbits(fsum[pos0]) : 0xFFFFFFFFu) << 32) | (uint32_t)lane;
#pragma unroll
        for (int size = 2; size <= kWave; size <<= 1)
#pragma unroll
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                const uint32_t ohi = __shfl_xor((uint32_t)(key >> 32), stride, kWave);
                const uint32_t olo = __shfl_xor((uint32_t)key, stride, kWave);
                const uint64_t o = ((uint64_t)ohi << 32) | olo;
                const bool asc = (lane & size) == 0;
                const bool low = (lane & stride) == 0;
                key = (low == asc) ? (o < key ? o : key) : (o > key ? o : key);
            }
        const int src = (int)(key & (kWave - 1));
        const int32_t pos = __shfl(pos0, src, kWave);
        head[j] = pos;  // -1 for the pads, which now fill the tile's last slots
#pragma unroll
        for (int k = 0; k < DM; ++k)
            if (k < d) {
                uint32_t v = __shfl(valid ? fbits(xp[(int64_t)k * ldp + pos0]) : kPad, src, kWave);
                hval[(int64_t)k * hcap + j] = v;
                uint32_t h = pos >= 0 ? v : 0u;
                for (int off = kWave / 2; off > 0; off >>= 1) {
                    uint32_t o = __shfl_xor(v, off, kWave), q = __shfl_xor(h, off, kWave);
                    v = o < v ? o : v;
                    h = q > h ? q : h;
                }
                if (lane == 0) {
                    hlo[(int64_t)k * tcap + tile] = v;
                    hhi[(int64_t)k * tcap + tile] = h;
                }
            }
    }
}

// Locate the segment of an item tile: largest s with tile_off[s] <= t.
__device__ __forceinline__ int32_t tile_segment(const int32_t* tile_off, int32_t nseg, int32_t t) {
    int32_t lo = 0, hi = nseg - 1;
    while (lo < hi) {
        int32_t mid = (lo + hi + 1) >> 1;
        if (tile_off[mid] <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Dominance tests of items against the head group of their segment, register-tiled.
// A work unit is (segment, a group of 256 items -- 64 per wave, one per lane --, a range of
// the segment's head tiles). For every tile of the range a wave
//   1. tests the tile's box against all its live items at once (lane = item): a tile can hold a
//      dominator of t only if lo <= t everywhere, and if hi <= t everywhere with hi < t
//      somewhere every row of the (non-empty) tile dominates t;
//   2. loads the tile's 64 candidates once (lane = candidate, ascending score order);
//   3. while many items passed the box, broadcasts the candidates one at a time against all
//      of them (lane = item), so items that fall to the tile's first rows leave early;
//   4. tests the items still undecided against all candidates: each item's values are
//      broadcast from LDS against the candidate lanes.
// s dominates t iff max_k(s_k - t_k) <= 0 and min_k(s_k - t_k) < 0 on the bit patterns as
// signed integers (canonical values of [0, 1) are below 2^30, so the differences are exact;
// lanes past the tile's real rows take 0x7FFFFFFF, whose differences are positive).
// One candidate load serves 64 items, so the loop is compute-bound. When a group's tiles are
// split over several units, waves share deaths through dom[] every few tiles.
// mode 0: items = the head group itself; mode 1: items = the rest group. A dominated item
// gets dom[pos] = 1.
template <int D>
__global__ void __launch_bounds__(kBlock) test_kernel(
    const float* __restrict__ xp, int64_t ldp, int32_t d_rt, int32_t nseg,
    const int32_t* __restrict__ unit_off_all, const int32_t* __restrict__ info,
    const int32_t* __restrict__ head, const int32_t* __restrict__ rest,
    const int32_t* __restrict__ rhb, const uint32_t* __restrict__ hval, int64_t hcap,
    const uint32_t* __restrict__ hlo,
    const uint32_t* __restrict__ hhi, int64_t tcap, const int32_t* __restrict__ round_counters,
    uint8_t* __restrict__ dom, unsigned long long* __restrict__ tests,
    unsigned long long* __restrict__ seg_tests, int32_t* __restrict__ work) {
    constexpr int DM = D > 0 ? D : SKY_MAX_D;
    __shared__ uint32_t box[kBoxLds];  // [2][k][ntile] tile boxes (lo, hi) of the current segment
    __shared__ int32_t itemc[kBlock / kWave][kWave][DM];  // each wave's passing items, compacted
    const int d = dget<D>(d_rt);
    const int lane = (int)lane_id();
    // (left as a vector value: marking it uniform made the partitioned launches slower)
    const int wave = threadIdx.x / kWave;
    const int32_t tpu_h = round_counters[C_TPUH], tpu_r = round_counters[C_TPUR];
    const int32_t nunits_h = unit_off_all[nseg];
    const int32_t nunits = nunits_h + unit_off_all[(nseg + 1) + nseg];
    int32_t cached = -1;  // segment whose boxes are in LDS (uniform per workgroup)
    unsigned long long ntests_h = 0, ntests_r = 0;
    // the wave's tests of the segment it worked on last, added to seg_tests when it moves on
    int32_t acc_seg = -1;
    unsigned long long acc = 0;
    // one wave's share of unit ug: its items part * 64 .. part * 64 + 63 of the unit's group
    auto unit = [&](const int32_t ug, const int32_t part) {
        // head units first (few items, latency-bound), then rest units
        const int mode = ug < nunits_h ? 0 : 1;
        const int32_t u = mode == 0 ? ug : ug - nunits_h;
        const int32_t* uoff = unit_off_all + (mode == 0 ? 0 : (nseg + 1));
        const int32_t tpu = mode == 0 ? tpu_h : tpu_r;
        const int32_t* items_all = mode == 0 ? head : rest;
        unsigned long long ntests = 0;
        const int32_t s = tile_segment(uoff, nseg, u);
        const int32_t* si = info + s * kInfo;
        const int32_t hoff = si[SI_HEADOFF];
        const int32_t hn = si[SI_HEADN];
        const int32_t ntile = (hn + kTile - 1) / kTile;
        const int32_t t0 = hoff / kTile;
        const int32_t nb = ntile * d;
        const bool in_lds = 2 * nb <= kBoxLds;
        if (!work && in_lds && s != cached) {  // (with work, the one segment's boxes are loaded)
            __syncthreads();  // every wave is done with the previous boxes
            for (int32_t e = threadIdx.x; e < nb; e += kBlock) {
                const int32_t k = e / ntile, tl = e - k * ntile;
                box[e] = hlo[(int64_t)k * tcap + t0 + tl];
                box[nb + e] = hhi[(int64_t)k * tcap + t0 + tl];
            }
            __syncthreads();
            cached = s;
        }
        const int32_t nr = (ntile + tpu - 1) / tpu;  // tile ranges per item group
        const int32_t lu = u - uoff[s];
        const int32_t grp = lu / nr;
        const int32_t c0 = (lu - grp * nr) * tpu;
        const int32_t span = ntile - c0 < tpu ? ntile - c0 : tpu;
        const int32_t ioff = mode == 0 ? hoff : si[SI_RESTOFF];
        const int32_t icnt = mode == 0 ? hn : si[SI_RESTN];
        const int32_t ibase = grp * kBlock + part * kWave;
        const bool have = ibase + lane < icnt;
        const uint32_t myidx = (uint32_t)(ioff + ibase + (have ? lane : 0));
        const int32_t mypos = have ? items_all[myidx] : 0;
        int32_t tv[DM];
#pragma unroll
        for (int k = 0; k < DM; ++k)
            if (k < d) {
                tv[k] = !have ? 0
                              : (int32_t)(mode == 0 ? ld32(hval + k * hcap, myidx)
                                                    : ld32(reinterpret_cast<const uint32_t*>(xp) + k * ldp,
                                                           (uint32_t)mypos));
            }
        const uint64_t born = __builtin_amdgcn_ballot_w64(have && dom[mypos] == 0);
        uint64_t live = born, written = 0;
        // start at the head tile nearest the wave's items on the curve (the likeliest place of
        // their dominators) and go forward: a head group's own tile, or for rest items the tile
        // of the head rows that precede the wave's first item; a unit whose tile range does not
        // hold that tile starts at the beginning of its range
        int32_t own = 0;
        if (mode == 0) own = ibase / kTile;
        else if (ibase < icnt) own = rhb[ioff + ibase] / kTile;
        own = own < ntile ? own : ntile - 1;
        const int32_t start = (own >= c0 && own < c0 + span) ? own - c0 : 0;
        int32_t done_steps = 0;
        bool probe = true;  // uniform: whether the unit still probes its tiles' best rows first
        // the unit's tiles in visiting order c(step) = c0 + (start + step) mod span, 64 at a time
        for (int32_t b0 = 0; b0 < span && live; b0 += kWave) {
            // a tile can pass a live item only if its lower corner is <= the componentwise
            // maximum of the live items: one test per tile, lanes over the next 64 tiles
            const bool lv = (live >> lane) & 1ull;
            int32_t mxk[DM];
#pragma unroll
            for (int k = 0; k < DM; ++k)
                if (k < d) mxk[k] = wave_max_i32(lv ? tv[k] : INT32_MIN);
            const int32_t sl = b0 + lane;
            bool maybe = sl < span;
            if (maybe) {
                int32_t cl = start + sl;
                cl = (cl < span ? cl : cl - span) + c0;
#pragma unroll
                for (int k = 0; k < DM; ++k)
                    if (k < d)
                        maybe &= (int32_t)(in_lds ? box[k * ntile + cl] : hlo[(int64_t)k * tcap + t0 + cl]) <= mxk[k];
            }
            uint64_t tmask = __builtin_amdgcn_ballot_w64(maybe);
            while (tmask && live) {
                const int32_t step = b0 + (__ffsll((unsigned long long)tmask) - 1);
                tmask &= tmask - 1;
                int32_t c = start + step;
                c = c < span ? c : c - span;
                c += c0;
                // 1. box of tile c against every live item (lane = item)
                bool pass = (live >> lane) & 1ull, hle = true, hlt = false;
#pragma unroll
                for (int k = 0; k < DM; ++k)
                    if (k < d) {
                        const int32_t lo = (int32_t)(in_lds ? box[k * ntile + c] : hlo[(int64_t)k * tcap + t0 + c]);
                        const int32_t hi = (int32_t)(in_lds ? box[nb + k * ntile + c] : hhi[(int64_t)k * tcap + t0 + c]);
                        pass &= lo <= tv[k];
                        hle &= hi <= tv[k];
                        hlt |= hi < tv[k];
                    }
                live &= ~__builtin_amdgcn_ballot_w64(pass && hle && hlt);
                uint64_t todo = __builtin_amdgcn_ballot_w64(pass) & live;
                if (todo) {
                    // 2. the tile's candidates (lane = candidate, in registers), in ascending
                    // score order
                    const uint32_t slot = (uint32_t)((t0 + c) * kTile + lane);
                    const int32_t creal = hn - c * kTile < kTile ? hn - c * kTile : kTile;
                    // slots past the tile's real rows act as padding (their values are stale)
                    const bool cin = lane < creal;
                    int32_t cv[DM];
#pragma unroll
                    for (int k = 0; k < DM; ++k)
                        if (k < d) cv[k] = cin ? (int32_t)ld32(hval + k * hcap, slot) : (int32_t)kPad;
                    // 3. probe (lane = item): the tile's kProbe best-score rows, read from the
                    // candidate lanes, against every passing item at once. On data where most
                    // rows fall to the first candidates they meet, this replaces a full tile
                    // of tests per item; a unit stops probing after a probe that decided
                    // fewer than a quarter of its items.
                    int32_t q = 0;
                    if (probe && 2 * __popcll(todo) >= creal) {
                        q = creal < kProbe ? creal : kProbe;
                        bool hit = false;
#pragma unroll
                        for (int32_t j = 0; j < kProbe; ++j)
                            if (j < q) {
                                int32_t mx = INT32_MIN, mn = INT32_MAX;
#pragma unroll
                                for (int k = 0; k < DM; ++k)
                                    if (k < d) {
                                        const int32_t e = __builtin_amdgcn_readlane(cv[k], j) - tv[k];
                                        mx = e > mx ? e : mx;
                                        mn = e < mn ? e : mn;
                                    }
                                hit |= ((mx - 1) & mn) < 0;
                            }
                        const int32_t left = __popcll(todo);
                        ntests += (unsigned long long)left * (unsigned long long)q;
                        const uint64_t killed = __builtin_amdgcn_ballot_w64(((todo >> lane) & 1ull) && hit);
                        todo &= ~killed;
                        live &= ~killed;
                        probe = 4 * __popcll(killed) >= left;
                    }
                    if (todo) {
                        // 4. every candidate against every item still undecided: the items are
                        // compacted in rank order in LDS and broadcast one by one, so every step
                        // keeps all 64 lanes busy (padding never dominates; the q candidates the
                        // probe already tried are tried again, which changes nothing and is not
                        // counted: the count stays one test per pair)
                        const int32_t kk = __popcll(todo);
                        ntests += (unsigned long long)kk * (unsigned long long)(creal - q);
                        const uint32_t rank = __builtin_amdgcn_mbcnt_hi(
                            (uint32_t)(todo >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)todo, 0u));
                        const bool mine = (todo >> lane) & 1ull;
                        if (mine) {
#pragma unroll
                            for (int k = 0; k < DM; ++k)
                                if (k < d) itemc[wave][rank][k] = tv[k];
                        }
                        __builtin_amdgcn_wave_barrier();
                        // each lane marks, by rank, the items its candidate dominates (no
                        // cross-lane step inside the loop); one OR over the lanes gives the dead
                        uint32_t mlo = 0, mhi = 0;
                        const int32_t k1 = kk < 32 ? kk : 32;
#pragma unroll 4
                        for (int32_t r = 0; r < k1; ++r) {
                            int32_t mx = INT32_MIN, mn = INT32_MAX;
#pragma unroll
                            for (int k = 0; k < DM; ++k)
                                if (k < d) {
                                    const int32_t e = cv[k] - itemc[wave][r][k];
                                    mx = e > mx ? e : mx;
                                    mn = e < mn ? e : mn;
                                }
                            // mx <= 0 and mn < 0  <=>  the sign bit of (mx - 1) & mn is set
                            mlo |= ((uint32_t)((mx - 1) & mn) >> 31) << r;
                        }
#pragma unroll 4
                        for (int32_t r = 32; r < kk; ++r) {
                            int32_t mx = INT32_MIN, mn = INT32_MAX;
#pragma unroll
                            for (int k = 0; k < DM; ++k)
                                if (k < d) {
                                    const int32_t e = cv[k] - itemc[wave][r][k];
                                    mx = e > mx ? e : mx;
                                    mn = e < mn ? e : mn;
                                }
                            mhi |= ((uint32_t)((mx - 1) & mn) >> 31) << (r - 32);
                        }
                        mlo = wave_or_u32(mlo);
                        if (kk > 32) mhi = wave_or_u32(mhi);
                        const uint64_t dead = ((uint64_t)mhi << 32) | mlo;
                        __builtin_amdgcn_wave_barrier();  // itemc is rewritten by the next tile
                        live &= ~__builtin_amdgcn_ballot_w64(mine && ((dead >> (rank & 63u)) & 1ull));
                    }
                }
                if (nr > 1 && (++done_steps & 7) == 0) {
                    // share deaths with the units testing the same items on other tiles
                    const uint64_t newly = born & ~live & ~written;
                    if ((newly >> lane) & 1ull) dom[mypos] = 1;
                    written |= newly;
                    live &= ~__builtin_amdgcn_ballot_w64(have && dom[mypos] != 0);
                }
            }
        }
        if ((((born & ~live & ~written) >> lane) & 1ull) != 0) dom[mypos] = 1;
        if (mode == 0) ntests_h += ntests; else ntests_r += ntests;
        if (seg_tests) {
            if (s != acc_seg) {
                if (lane == 0 && acc) atomicAdd(&seg_tests[acc_seg], acc);
                acc_seg = s;
                acc = 0;
            }
            acc += ntests;
        }
    };
    if (work) {
        // one segment, persistent workgroups: its tile boxes are loaded once, then every wave
        // takes (unit, part) pairs from the striped counters until its counter passes the total
        // (no barrier after the load, so waves that run out of work simply end)
        const int32_t* si = info;
        const int32_t ntile = (si[SI_HEADN] + kTile - 1) / kTile;
        const int32_t t0 = si[SI_HEADOFF] / kTile;
        const int32_t nb = ntile * d;
        if (2 * nb <= kBoxLds) {
            for (int32_t e = threadIdx.x; e < nb; e += kBlock) {
                const int32_t k = e / ntile, tl = e - k * ntile;
                box[e] = hlo[(int64_t)k * tcap + t0 + tl];
                box[nb + e] = hhi[(int64_t)k * tcap + t0 + tl];
            }
        }
        __syncthreads();
        cached = 0;
        const int32_t total = nunits * (kBlock / kWave);
        const int32_t nctr = gridDim.x >= (uint32_t)kWorkCounters ? kWorkCounters : 1;
        const int32_t x = (int32_t)(blockIdx.x % (uint32_t)nctr);
        for (;;) {
            int32_t k = 0;
            if (lane == 0) k = atomicAdd(work + kCounterStride * x, 1);
            k = __builtin_amdgcn_readfirstlane(k);
            const int32_t item = x + nctr * k;
            if (item >= total) break;
            unit(item / (kBlock / kWave), item % (kBlock / kWave));
        }
    } else {
        // a contiguous range of units per workgroup (one unit each when the grid covers them):
        // the units of a segment are consecutive, so its tile boxes stay in LDS
        const int32_t per = (nunits + (int32_t)gridDim.x - 1) / (int32_t)gridDim.x;
        const int32_t u1 = ((int32_t)blockIdx.x + 1) * per < nunits ? ((int32_t)blockIdx.x + 1) * per : nunits;
        for (int32_t ug = (int32_t)blockIdx.x * per; ug < u1; ++ug) unit(ug, wave);
    }
    // one atomic per workgroup and counter: the waves' counts summed through LDS (thousands of
    // waves adding to one address at the end of a launch would queue behind each other)
    __shared__ unsigned long long wred[kBlock / kWave][2];
    if (lane == 0) {
        wred[wave][0] = ntests_h;
        wred[wave][1] = ntests_r;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        unsigned long long t = 0;
        for (int w = 0; w < kBlock / kWave; ++w) t += wred[w][threadIdx.x];
        if (t) atomicAdd(&tests[threadIdx.x], t);
    }
    if (seg_tests && lane == 0 && acc) atomicAdd(&seg_tests[acc_seg], acc);
}

// End of a run: the dominance tests it evaluated (head and rest groups), the largest count of
// one segment (the sum when no per-segment counters are kept) and the rounds that had live
// items, as int64 words for the caller (each output may be null).
__global__ void __launch_bounds__(kBlock) engine_finish_kernel(const unsigned long long* __restrict__ tests,
                                                                const unsigned long long* __restrict__ seg_tests,
                                                                const unsigned long long* __restrict__ extra,
                                                                int32_t nseg, const int32_t* __restrict__ gcounters,
                                                                int64_t* __restrict__ out_rounds,
                                                                int64_t* __restrict__ out_tests,
                                                                int64_t* __restrict__ out_max) {
    __shared__ unsigned long long part[kBlock / kWave];
    unsigned long long m = 0;
    if (seg_tests)
        for (int32_t i = threadIdx.x; i < nseg; i += kBlock) m = seg_tests[i] > m ? seg_tests[i] : m;
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(m, off);
        m = o > m ? o : m;
    }
    if (lane_id() == 0) part[threadIdx.x / kWave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / kWave; ++w) m = part[w] > m ? part[w] : m;
        const unsigned long long total = tests[0] + tests[1] + (extra ? *extra : 0ull);
        if (out_rounds) *out_rounds = gcounters[G_ROUNDS];
        if (out_tests) *out_tests = (int64_t)total;
        if (out_max) *out_max = (int64_t)(seg_tests ? m : total);
    }
}

__global__ void __launch_bounds__(kBlock) scatter_rows_u8_kernel(const uint8_t* __restrict__ src,
                                                                  const uint8_t* __restrict__ drop,
                                                                  const int32_t* __restrict__ rowid,
                                                                  int64_t n, const int32_t* __restrict__ count,
                                                                  uint8_t* __restrict__ dst) {
    int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t m = count ? (*count < n ? (int64_t)*count : n) : n;
    if (q < m) dst[rowid[q]] = (drop && drop[q]) ? 0 : src[q];
}
__global__ void fill_u8_kernel(uint8_t* __restrict__ p, int64_t n, uint8_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// every position in order
__global__ void __launch_bounds__(kBlock) iota_kernel(int32_t n, int32_t* __restrict__ out,
                                                       int32_t* __restrict__ count) {
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) out[i] = i;
    if (i == 0) *count = n;
}

// p[0, n) = 0 (p 16-byte aligned; grid-stride, 16 bytes per store)
__global__ void __launch_bounds__(kBlock) zero_bytes_kernel(uint8_t* __restrict__ p, int64_t n) {
    const int64_t n16 = n / 16;
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x, gs = (int64_t)gridDim.x * kBlock;
    for (int64_t i = g; i < n16; i += gs) reinterpret_cast<uint4*>(p)[i] = make_uint4(0u, 0u, 0u, 0u);
    for (int64_t i = n16 * 16 + g; i < n; i += gs) p[i] = 0;
}

// member[rowid[list[i]]] = 1 for i < *count (grid-stride)
__global__ void __launch_bounds__(kBlock) mark_rows_kernel(const int32_t* __restrict__ list,
                                                            const int32_t* __restrict__ count,
                                                            const int32_t* __restrict__ rowid,
                                                            uint8_t* __restrict__ member) {
    const int32_t c = *count;
    for (int32_t i = blockIdx.x * kBlock + threadIdx.x; i < c; i += gridDim.x * kBlock) member[rowid[list[i]]] = 1;
}

// ---- stable selection in three launches: per-block counts, their scan, then each block
// re-derives its positions' predicate bits and writes the selected ones at its offset ---------
constexpr int kSelPer = 16;                  // consecutive positions per thread
constexpr int kSelChunk = kBlock * kSelPer;  // positions per block

// position i is selected iff flags[i] != 0 (no flags: every position), keep[i] != 0 (if given),
// drop[i] == 0 (if given) and its segment is not skipped (if skip_seg is given)
struct SelPred {
    const uint8_t* flags;
    const uint8_t* keep;
    const uint8_t* drop;
    const uint8_t* skip_seg;
    const int32_t* seg;
};

// bit j = (byte j of the 16 at ptr != 0); ptr 16-byte aligned
__device__ __forceinline__ uint32_t nonzero16(const uint8_t* ptr) {
    const uint4 q = *reinterpret_cast<const uint4*>(ptr);
    const uint32_t w[4] = {q.x, q.y, q.z, q.w};
    uint32_t m = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) m |= (((w[j >> 2] >> (8 * (j & 3))) & 0xFFu) != 0u ? 1u : 0u) << j;
    return m;
}

__device__ __forceinline__ bool aligned16(const void* ptr) { return ((uintptr_t)ptr & 15u) == 0; }

__device__ __forceinline__ uint32_t sel_bits(const SelPred& p, int64_t base, int64_t n) {
    if (base + kSelPer <= n && !p.skip_seg && (!p.flags || aligned16(p.flags)) && (!p.keep || aligned16(p.keep)) &&
        (!p.drop || aligned16(p.drop))) {
        // whole runs of 16 positions: one 16-byte load per byte array
        uint32_t m = 0xFFFFu;
        if (p.flags) m &= nonzero16(p.flags + base);
        if (p.keep) m &= nonzero16(p.keep + base);
        if (p.drop) m &= ~nonzero16(p.drop + base) & 0xFFFFu;
        return m;
    }
    uint32_t m = 0;
#pragma unroll
    for (int j = 0; j < kSelPer; ++j) {
        const int64_t i = base + j;
        if (i < n) {
            bool v = p.flags ? p.flags[i] != 0 : true;
            if (p.keep) v = v && p.keep[i] != 0;
            if (p.drop) v = v && p.drop[i] == 0;
            if (p.skip_seg) v = v && !p.skip_seg[p.seg[i]];
            m |= (v ? 1u : 0u) << j;
        }
    }
    return m;
}

// block-wide exclusive scan of one value per thread; *total gets the block's sum
__device__ __forceinline__ int32_t sel_block_scan(int32_t v, int32_t* total) {
    __shared__ int32_t wsum[kBlock / kWave];
    const int lane = (int)lane_id();
    const int wave = threadIdx.x / kWave;
    int32_t inc = v;
    for (int off = 1; off < kWave; off <<= 1) {
        const int32_t o = __shfl_up(inc, off, kWave);
        if (lane >= off) inc += o;
    }
    if (lane == kWave - 1) wsum[wave] = inc;
    __syncthreads();
    int32_t before = 0, t = 0;
    for (int w = 0; w < kBlock / kWave; ++w) {
        before += w < wave ? wsum[w] : 0;
        t += wsum[w];
    }
    *total = t;
    return before + inc - v;
}

// the positions a selection covers: [0, n), or [0, min(n, *bound)) with a device bound
__device__ __forceinline__ int64_t sel_extent(int64_t n, const int32_t* bound) {
    if (!bound) return n;
    const int64_t b = *bound;
    return b < 0 ? 0 : (b < n ? b : n);
}

__global__ void __launch_bounds__(kBlock) sel_count_kernel(SelPred p, int64_t n, const int32_t* __restrict__ bound,
                                                           int32_t* __restrict__ blk) {
    n = sel_extent(n, bound);
    if ((int64_t)blockIdx.x * kSelChunk >= n) {  // past the bound (uniform per workgroup)
        if (threadIdx.x == 0) blk[blockIdx.x] = 0;
        return;
    }
    const int64_t base = (int64_t)blockIdx.x * kSelChunk + (int64_t)threadIdx.x * kSelPer;
    int32_t total = 0;
    sel_block_scan(__popc(sel_bits(p, base, n)), &total);
    if (threadIdx.x == 0) blk[blockIdx.x] = total;
}

// out32[k] = the k-th selected position (int32 output), or out64[k] for k < cap (int64 output);
// all_idx[i] (if given) = number of selected positions before i, for every selected i; flags_copy (if
// given) = the selection as bytes (it may be the flags array itself: each thread rewrites only
// the positions it has read); the last block stores the total in *count32 / *count64 and raises
// SKY_ERR_CAPACITY when it exceeds cap (int64 output)
__global__ void __launch_bounds__(kBlock) sel_write_kernel(SelPred p, int64_t n, const int32_t* __restrict__ bound,
                                                            const int32_t* __restrict__ blk_off,
                                                            int32_t* __restrict__ out32,
                                                            int64_t* __restrict__ out64, int64_t cap,
                                                            int32_t* __restrict__ all_idx,
                                                            uint8_t* flags_copy,
                                                            int32_t* __restrict__ count32,
                                                            int64_t* __restrict__ count64,
                                                            int32_t* dev_status) {
    n = sel_extent(n, bound);
    const bool past = (int64_t)blockIdx.x * kSelChunk >= n;  // uniform per workgroup
    if (past && blockIdx.x != gridDim.x - 1) return;
    const int64_t base = (int64_t)blockIdx.x * kSelChunk + (int64_t)threadIdx.x * kSelPer;
    const uint32_t m = past ? 0u : sel_bits(p, base, n);
    int32_t total = 0;
    int32_t k = blk_off[blockIdx.x] + sel_block_scan(__popc(m), &total);
    if (flags_copy && base + kSelPer <= n && aligned16(flags_copy)) {
        uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int j = 0; j < kSelPer; ++j) w[j >> 2] |= ((m >> j) & 1u) << (8 * (j & 3));
        *reinterpret_cast<uint4*>(flags_copy + base) = make_uint4(w[0], w[1], w[2], w[3]);
        flags_copy = nullptr;  // written
    }
    if (m || flags_copy) {
#pragma unroll
        for (int j = 0; j < kSelPer; ++j) {
            const int64_t i = base + j;
            if (i >= n) break;
            const bool v = (m >> j) & 1u;
            if (all_idx && v) all_idx[i] = k;
            if (flags_copy) flags_copy[i] = v ? 1 : 0;
            if (v) {
                if (out32) out32[k] = (int32_t)i;
                if (out64 && k < cap) out64[k] = i;
                ++k;
            }
        }
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        const int64_t c = (int64_t)blk_off[blockIdx.x] + total;
        if (count32) *count32 = (int32_t)c;
        if (count64) {
            *count64 = c;
            if (c > cap) raise_status(dev_status, SKY_ERR_CAPACITY);
        }
    }
}

}  // namespace

#define SKY_DISPATCH_D(d, KERNEL, ...)                                            \
    switch (d) {                                                                  \
        case 1: hipLaunchKernelGGL(KERNEL<1>, __VA_ARGS__); break;                \
        case 2: hipLaunchKernelGGL(KERNEL<2>, __VA_ARGS__); break;                \
        case 3: hipLaunchKernelGGL(KERNEL<3>, __VA_ARGS__); break;                \
        case 4: hipLaunchKernelGGL(KERNEL<4>, __VA_ARGS__); break;                \
        case 5: hipLaunchKernelGGL(KERNEL<5>, __VA_ARGS__); break;                \
        case 6: hipLaunchKernelGGL(KERNEL<6>, __VA_ARGS__); break;                \
        case 7: hipLaunchKernelGGL(KERNEL<7>, __VA_ARGS__); break;                \
        case 8: hipLaunchKernelGGL(KERNEL<8>, __VA_ARGS__); break;                \
        default: hipLaunchKernelGGL(KERNEL<0>, __VA_ARGS__); break;               \
    }

int64_t engine_head_capacity(int64_t n, int32_t nseg) { return n + (int64_t)kTile * nseg + kTile; }

int64_t engine_scan_elems(int64_t n) { return 2 * (ceil_div(n > 0 ? n : 1, kCItems) + 1); }

// The rounds of a run over at most `ub` live items: round r is the last one when its bound is
// at most A_r (every segment then takes all of its live rows into the head). With one segment
// every round takes at least H_r rows out of the live set, which lowers the next bound; with
// several, a segment may hold every live row, so the bound stays.
int32_t engine_rounds(int64_t ub, int32_t nseg, int64_t* ub_of_round) {
    for (int32_t r = 1;; ++r) {
        ub_of_round[r - 1] = ub;
        if (ub <= round_all(r) || r == kMaxRounds) return r;
        if (nseg == 1) ub = ub > round_head(r) ? ub - round_head(r) : 0;
    }
}

sky_status run_engine(const EngineProblem& pb, const EngineBuffers& b, hipStream_t st) {
    const int32_t nseg = pb.nseg;
    int32_t* const gctr = b.counters;
    auto ctr = [&](int32_t r) { return b.counters + kCounters * (1 + (r & 1)); };
    auto hist_of = [&](int32_t r) { return b.hist + (int64_t)(r & 1) * nseg * kBins; };
    auto info_of = [&](int32_t r) { return b.seg_info + (int64_t)(r & 1) * nseg * kInfo; };
    auto grid = [](int64_t want) -> uint32_t {
        return (uint32_t)(want < 1 ? 1 : (want > kMaxGrid ? kMaxGrid : want));
    };
    {
        const bool fold = pb.ranges_ready && pb.range_slots && nseg == 1;
        int64_t work = pb.n_pos / 16;
        if (2 * (int64_t)nseg * kBins > work) work = 2 * (int64_t)nseg * kBins;
        hipLaunchKernelGGL(engine_init_kernel, dim3(grid(ceil_div(work, kBlock))), dim3(kBlock), 0, st,
                           pb.n_pos, pb.flag_out, nseg, b.hist, b.seg_info,
                           pb.ranges_ready && !fold ? nullptr : b.seg_min,
                           pb.ranges_ready && !fold ? nullptr : b.seg_max, fold ? 1 : 0, b.counters, b.tests,
                           pb.zero_seg_tests ? pb.seg_tests : nullptr);
        SKY_HIP(hipGetLastError());
    }
    // optional timing hooks around the dominance-test launches
    auto ev_rec = [&](bool begin) -> hipError_t {
        if (!pb.ev_begin || !pb.ev_end || !pb.ev_used || *pb.ev_used >= pb.ev_cap) return hipSuccess;
        hipEvent_t e = (hipEvent_t)(begin ? pb.ev_begin[*pb.ev_used] : pb.ev_end[*pb.ev_used]);
        hipError_t r = hipEventRecord(e, st);
        if (!begin) ++*pb.ev_used;
        return r;
    };
    const int64_t ub0 = pb.n_items_dev ? pb.ub_items : pb.n_items;
    if (ub0 > 0) {
        int64_t ubs[kMaxRounds];
        const int32_t R = engine_rounds(ub0, nseg, ubs);
        // round r writes its rest groups into rest_buf[r & 1] and reads the previous round's
        // (the caller's list in the first round)
        int32_t* rest_buf[2] = {b.rest, b.w0};
        for (int32_t r = 1; r <= R; ++r) {
            const int64_t ub = ubs[r - 1];
            // rounds after the first often turn out empty (the host bound cannot see that):
            // their grid-stride launches use fewer workgroups, which costs little when they are
            // not
            auto later = [&](uint32_t g) -> uint32_t { return r > 1 && g > kGridLater ? kGridLater : g; };
            const int32_t* items = r == 1 ? pb.items : rest_buf[(r - 1) & 1];
            const int32_t n_host = r == 1 ? pb.n_items : 0;
            const int32_t* n_dev = r == 1 ? pb.n_items_dev : ctr(r - 1) + C_RTOT;
            const uint8_t* dead = r == 1 ? nullptr : b.dom;
            const uint32_t iblocks = (uint32_t)ceil_div(ub, kBlock);
            if (r == 1 && !pb.ranges_ready) {
                if (nseg == 1)
                    hipLaunchKernelGGL(minmax1_kernel, dim3(iblocks < 256 ? iblocks : 256), dim3(kBlock), 0, st,
                                       items, n_host, n_dev, pb.fsum, b.seg_min, b.seg_max);
                else
                    hipLaunchKernelGGL(minmax_kernel, dim3((uint32_t)seg_pass_blocks(ub)), dim3(kBlock), 0, st,
                                       items, n_host, n_dev, pb.fsum, pb.seg_of_pos, b.seg_min, b.seg_max);
                SKY_HIP(hipGetLastError());
            }
            // the test launch: one segment runs persistent workgroups fed from work counters when
            // more workgroups are wanted than the device holds at once
            const int64_t want_wg = kTargetWaves / (kBlock / kWave);
            const int64_t groups_ub = ceil_div(ub, kBlock) + 2 * (int64_t)nseg;
            uint32_t tgrid = grid(groups_ub + 2 * want_wg);
            if (r > 1 && tgrid > kTestGridLater) tgrid = kTestGridLater;
            int32_t* work = nullptr;
            if (nseg == 1) {
                const void* fn = nullptr;
                SKY_KERNEL_PTR_D(pb.d, test_kernel, fn);
                int32_t resident = 0;
                SKY_TRY(resident_workgroups(fn, kBlock, 0, &resident));
                if ((int64_t)tgrid > resident) {
                    tgrid = (uint32_t)resident;
                    work = b.work;
                }
            }
            StatsArgs sa{};
            sa.items = items; sa.n_host = n_host; sa.n_dev = n_dev; sa.dead = dead;
            sa.fsum = pb.fsum; sa.seg_of_pos = pb.seg_of_pos; sa.nseg = nseg;
            sa.smin = b.seg_min; sa.smax = b.seg_max;
            sa.hist = hist_of(r); sa.info = info_of(r);
            sa.hist_next = hist_of(r + 1); sa.info_next = info_of(r + 1);
            if (nseg == 1)
                hipLaunchKernelGGL(stats_kernel<false>, dim3(iblocks < 256 ? iblocks : 256), dim3(kBlock), 0, st, sa);
            else
                hipLaunchKernelGGL(stats_kernel<true>, dim3(later(grid(seg_pass_blocks(ub)))), dim3(kBlock), 0, st, sa);
            SKY_HIP(hipGetLastError());
            const int32_t want_head = (int32_t)round_head(r);
            const int32_t all_below = r == R ? (int32_t)0x7FFFFFFF : (int32_t)round_all(r);
            const bool thresh_here = nseg <= kBlock / kWave;
            if (!thresh_here)
                hipLaunchKernelGGL(thresh_kernel, dim3((uint32_t)ceil_div(nseg, kBlock / kWave)), dim3(kBlock), 0, st,
                                   nseg, (const int32_t*)hist_of(r), info_of(r), want_head, all_below);
            hipLaunchKernelGGL(layout_kernel, dim3(1), dim3(kBlock), 0, st, nseg, (const int32_t*)hist_of(r),
                               info_of(r), b.tile_off, ctr(r), work, gctr, want_head, all_below,
                               (int32_t)thresh_here);
            SKY_HIP(hipGetLastError());
            SplitArgs xa{};
            xa.items = items; xa.n_host = n_host; xa.n_dev = n_dev; xa.dead = dead;
            xa.fsum = pb.fsum; xa.seg_of_pos = pb.seg_of_pos; xa.smin = b.seg_min; xa.smax = b.seg_max;
            xa.info = info_of(r); xa.bcnt = b.scan;
            xa.head = b.head; xa.rest = rest_buf[r & 1]; xa.rhb = b.rhb;
            xa.dom_clear = r == 1 ? b.dom : nullptr;
            xa.flag_out = pb.flag_out;
            const int64_t cb = ceil_div(ub, kCItems);
            const uint32_t cblocks = (uint32_t)(cb > kSplitGrid ? kSplitGrid : cb);
            hipLaunchKernelGGL(split_count_kernel, dim3(cblocks), dim3(kBlock), 0, st, xa);
            hipLaunchKernelGGL(split_scatter_kernel, dim3(cblocks), dim3(kBlock), 0, st, xa);
            SKY_HIP(hipGetLastError());
            const int64_t slot_bound = ub + (int64_t)kTile * nseg;
            SKY_DISPATCH_D(pb.d, head_values_kernel, dim3(later(grid(ceil_div(slot_bound, kTile * (kBlock / kWave))))),
                           dim3(kBlock), 0, st, pb.xp, pb.ldp, pb.d, pb.fsum, nseg, (const int32_t*)info_of(r),
                           (const int32_t*)ctr(r), b.head, b.hval, b.hcap, b.hlo, b.hhi, b.tcap);
            SKY_HIP(hipGetLastError());
            // one launch: the head skyline (every head row against the head rows of its segment)
            // and the filter of the rest against the same head rows -- independent tests
            SKY_HIP(ev_rec(true));
            SKY_DISPATCH_D(pb.d, test_kernel, dim3(tgrid),
                           dim3(kBlock), 0, st, pb.xp, pb.ldp, pb.d, nseg, (const int32_t*)b.tile_off,
                           (const int32_t*)info_of(r), (const int32_t*)b.head, (const int32_t*)rest_buf[r & 1],
                           (const int32_t*)b.rhb, (const uint32_t*)b.hval, b.hcap, (const uint32_t*)b.hlo,
                           (const uint32_t*)b.hhi, b.tcap, (const int32_t*)ctr(r), b.dom, b.tests,
                           pb.seg_tests, work);
            SKY_HIP(hipGetLastError());
            SKY_HIP(ev_rec(false));
        }
    }
    hipLaunchKernelGGL(engine_finish_kernel, dim3(1), dim3(kBlock), 0, st, (const unsigned long long*)b.tests,
                       (const unsigned long long*)pb.seg_tests, pb.extra_tests, nseg, (const int32_t*)gctr, pb.out_rounds,
                       pb.out_tests, pb.out_tests_max);
    SKY_HIP(hipGetLastError());
    return SKY_OK;
}

// Stable selection of the positions [0, n) that satisfy p (see sel_write_kernel for the
// outputs). tmp: scan_tmp_elems(n) int32 of scratch.
static sky_status launch_select(const SelPred& p, int64_t n, int32_t* out32, int64_t* out64, int64_t cap,
                                int32_t* all_idx, uint8_t* flags_copy, int32_t* count32, int64_t* count64,
                                int32_t* dev_status, int32_t* tmp, hipStream_t st, const int32_t* bound = nullptr) {
    const int64_t nblk = ceil_div(n > 0 ? n : 1, kSelChunk);
    int32_t* blk = tmp;  // block counts, then their exclusive scan (the layout of scan_tmp_elems)
    hipLaunchKernelGGL(sel_count_kernel, dim3((uint32_t)nblk), dim3(kBlock), 0, st, p, n, bound, blk);
    SKY_HIP(hipGetLastError());
    SKY_TRY(launch_exclusive_scan(blk, blk, nblk, tmp + round_up(nblk, 64), st));
    hipLaunchKernelGGL(sel_write_kernel, dim3((uint32_t)nblk), dim3(kBlock), 0, st, p, n, bound,
                       (const int32_t*)blk, out32, out64, cap, all_idx, flags_copy, count32, count64,
                       dev_status);
    SKY_HIP(hipGetLastError());
    return SKY_OK;
}

// Positions [0, n) in order, without those whose segment is skipped (stable).
sky_status launch_iota_filtered(const uint8_t* skip_seg, const int32_t* seg_of_pos, int32_t n,
                                int32_t* out, int32_t* count, int32_t* scan_tmp, hipStream_t st,
                                const uint8_t* keep) {
    const uint32_t nb = (uint32_t)ceil_div(n > 0 ? n : 1, kBlock);
    if (!skip_seg && !keep) {  // nothing skipped: the list is every position
        hipLaunchKernelGGL(iota_kernel, dim3(nb), dim3(kBlock), 0, st, n, out, count);
        SKY_HIP(hipGetLastError());
        return SKY_OK;
    }
    const SelPred p{nullptr, keep, nullptr, skip_seg, skip_seg ? seg_of_pos : nullptr};
    return launch_select(p, n, out, nullptr, 0, nullptr, nullptr, count, nullptr, nullptr, scan_tmp, st);
}

// Positions i with flags[i] != 0 and (drop null or drop[i] == 0), in order (stable); with
// bake, flags[i] is rewritten to the selection.
sky_status launch_compact_flags(uint8_t* flags, const uint8_t* drop, bool bake, int32_t n, int32_t* out,
                                int32_t* count32, int64_t* count64, int32_t* scan_tmp, hipStream_t st,
                                const int32_t* bound) {
    const SelPred p{flags, nullptr, drop, nullptr, nullptr};
    return launch_select(p, n, out, nullptr, (int64_t)n, nullptr, bake ? flags : nullptr, count32, count64,
                         nullptr, scan_tmp, st, bound);
}

sky_status launch_scatter_rows_live(const uint8_t* src, const uint8_t* drop, const int32_t* rowid, int64_t n,
                                    const int32_t* count, uint8_t* dst, hipStream_t st) {
    if (n <= 0) return SKY_OK;
    hipLaunchKernelGGL(scatter_rows_u8_kernel, dim3((uint32_t)ceil_div(n, kBlock)), dim3(kBlock), 0, st, src,
                       drop, rowid, n, count, dst);
    SKY_HIP(hipGetLastError());
    return SKY_OK;
}

sky_status launch_fill_u8(uint8_t* p, int64_t n, uint8_t v, hipStream_t st) {
    if (n > 0)
        hipLaunchKernelGGL(fill_u8_kernel, dim3((uint32_t)ceil_div(n, 256)), dim3(256), 0, st, p, n, v);
    SKY_HIP(hipGetLastError());
    return SKY_OK;
}

// The final skyline's rows in ascending order: member_tmp cleared, set at the rows of the
// positions list[0, *count) (count on the device, at most n), then a selection over the rows.
sky_status launch_final_output(const int32_t* list, const int32_t* count, const int32_t* rowid, int64_t n,
                               uint8_t* member_tmp, uint8_t* member_out, int64_t* sky_idx,
                               int64_t cap, int64_t* dev_count, int32_t* pos_tmp, int32_t* scan_tmp,
                               int32_t* dev_status, hipStream_t st) {
    const int64_t n16 = ceil_div(n, 16);
    hipLaunchKernelGGL(zero_bytes_kernel, dim3((uint32_t)(ceil_div(n16, kBlock) > 2048 ? 2048 : ceil_div(n16, kBlock))),
                       dim3(kBlock), 0, st, member_tmp, n);
    const int64_t mb = ceil_div(n, kBlock);
    hipLaunchKernelGGL(mark_rows_kernel, dim3((uint32_t)(mb > 1024 ? 1024 : mb)), dim3(kBlock), 0, st, list, count,
                       rowid, member_tmp);
    SKY_HIP(hipGetLastError());
    // ascending rows: pos_tmp[row] = the row's index in sky_idx (kept for the gres store)
    const SelPred p{member_tmp, nullptr, nullptr, nullptr, nullptr};
    return launch_select(p, n, nullptr, sky_idx, cap, pos_tmp, member_out, nullptr, dev_count, dev_status,
                         scan_tmp, st);
}

}  // namespace sky
