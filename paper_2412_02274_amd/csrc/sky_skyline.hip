// Segmented skyline engine: the skyline (Def. 1) of every segment of a set of rows, all
// segments at once. Used for the local skylines of the partitions (Sec. 3, phase 1; one
// segment per partition) and for the final skyline of their union (phase 2; one segment).
//
// Rounds of "head skyline, then filter" in the spirit of SFS (the scan order of a monotone
// score; Sec. 2 scoring functions, Sec. 4 SFS):
//   1. per segment, the FP32 attribute sum f of the live rows is binned between the
//      segment's min and max; the head is the set of rows in the lowest bins holding at
//      least kHead rows. f is monotone: a row dominating another has f <= the other's f
//      (FP32 additions are monotone), so every dominator of a head row is itself in the head.
//   2. head skyline: every head row is tested against every other head row of its segment
//      (all pairs, early exit). The survivors are exactly the segment's skyline rows inside
//      the head (their dominators would be in the head), so they are final.
//   3. filter: every other live row is tested against the head skyline of its segment; the
//      survivors form the next round's live set. A row dominated by some row of the head is
//      dominated by a head skyline row (transitivity), so no skyline row is ever dropped, and
//      every row of the head leaves the live set, so the rounds terminate.
// Rows are compared through their canonical FP32 bit patterns (exact for [0, 1) data).
//
// Layout: positions index a partition-contiguous SoA copy xp[k*ldp + pos]; lists hold
// positions. Head/rest lists are grouped by segment (offsets from a scan over segments);
// the test kernels run one workgroup per tile of <= 256 items of one segment, stage 256
// candidate rows at a time in LDS, and stop as soon as every item of the tile is dominated.
// Bound: VALU compares (skyline-heavy data) or the filter's HBM reads (uniform data).
#include "sky_internal.hpp"

namespace sky {

namespace {

constexpr int kHead = 8192;   // head rows per segment and round (target)
constexpr int kItems = kBlock; // items per test tile
constexpr int kLdsBytes = 40 * 1024;  // LDS for the staged candidate chunk
constexpr int kMinBlocks = 2048; // test grids are split along candidates up to this many blocks

// seg_info layout per segment (int32 x kInfo)
enum { SI_LIVE = 0, SI_BSTAR, SI_HEADN, SI_HEADOFF, SI_RESTN, SI_RESTOFF, SI_HCUR, SI_RCUR,
       SI_FCUR, kInfo = 12 };
// global counters
enum { C_NEXT = 0, C_OUT, C_HTILES, C_RTILES, C_MAXH, C_HTOT, C_RTOT, kCounters = 16 };

template <int D>
__device__ __forceinline__ int dget(int d) { return D > 0 ? D : d; }

__device__ __forceinline__ int32_t seg_of(const int32_t* seg_of_pos, int32_t pos) {
    return seg_of_pos ? seg_of_pos[pos] : 0;
}

// Wave-aggregated "slot = atomicAdd(&ctr[key*stride], 1)": one atomic per distinct key in the
// wave; every active lane gets a unique slot.
__device__ __forceinline__ int32_t wave_slot(int32_t* ctr, int32_t stride, int32_t key, bool active) {
    const int lane = (int)lane_id();
    const uint64_t lt = __lanemask_lt();
    uint64_t act = __ballot(active);
    int32_t slot = 0;
    while (act) {
        const int leader = __ffsll((unsigned long long)act) - 1;
        const int32_t kl = __shfl(key, leader, kWave);
        const bool mine = active && key == kl;
        const uint64_t peers = __ballot(mine);
        int32_t base = 0;
        if (lane == leader) base = atomicAdd(&ctr[(int64_t)kl * stride], (int32_t)__popcll(peers));
        base = __shfl(base, leader, kWave);
        if (mine) slot = base + (int32_t)__popcll(peers & lt);
        act &= ~peers;
    }
    return slot;
}

__global__ void init_segments_kernel(int32_t nseg, uint32_t* __restrict__ smin,
                                     uint32_t* __restrict__ smax, int32_t* __restrict__ hist,
                                     int32_t* __restrict__ info, int32_t* __restrict__ counters) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < (int64_t)nseg * kBins) hist[i] = 0;
    if (i < nseg) {
        smin[i] = 0xFFFFFFFFu;
        smax[i] = 0u;
        for (int j = 0; j < kInfo; ++j) info[i * kInfo + j] = 0;
    }
    if (i == 0) counters[C_NEXT] = 0;
}

__global__ void __launch_bounds__(kBlock) minmax_kernel(const int32_t* __restrict__ items, int32_t n,
                                                         const float* __restrict__ fsum,
                                                         const int32_t* __restrict__ seg_of_pos,
                                                         uint32_t* __restrict__ smin,
                                                         uint32_t* __restrict__ smax,
                                                         int32_t* __restrict__ info) {
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    const bool valid = i < n;
    int32_t s = 0;
    uint32_t fb = 0;
    if (valid) {
        int32_t pos = items[i];
        s = seg_of(seg_of_pos, pos);
        fb = fbits(fsum[pos]);  // f >= 0: bit order == value order
    }
    const int lane = (int)lane_id();
    uint64_t act = __ballot(valid);
    while (act) {
        const int leader = __ffsll((unsigned long long)act) - 1;
        const int32_t sl = __shfl(s, leader, kWave);
        const bool mine = valid && s == sl;
        const uint64_t peers = __ballot(mine);
        uint32_t vmin = mine ? fb : 0xFFFFFFFFu, vmax = mine ? fb : 0u;
        for (int off = kWave / 2; off > 0; off >>= 1) {
            uint32_t a = __shfl_xor(vmin, off, kWave), b = __shfl_xor(vmax, off, kWave);
            vmin = a < vmin ? a : vmin;
            vmax = b > vmax ? b : vmax;
        }
        if (lane == leader) {
            atomicMin(&smin[sl], vmin);
            atomicMax(&smax[sl], vmax);
            atomicAdd(&info[sl * kInfo + SI_LIVE], (int32_t)__popcll(peers));
        }
        act &= ~peers;
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

__global__ void __launch_bounds__(kBlock) hist_kernel(const int32_t* __restrict__ items, int32_t n,
                                                       const float* __restrict__ fsum,
                                                       const int32_t* __restrict__ seg_of_pos,
                                                       const uint32_t* __restrict__ smin,
                                                       const uint32_t* __restrict__ smax,
                                                       int32_t* __restrict__ hist) {
    int32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int32_t pos = items[i];
    int32_t s = seg_of(seg_of_pos, pos);
    int32_t b = bin_of(fsum[pos], __uint_as_float(smin[s]), seg_scale(smin[s], smax[s]));
    atomicAdd(&hist[(int64_t)s * kBins + b], 1);
}

// One wave per segment: smallest bin b* whose cumulative count reaches kHead.
__global__ void __launch_bounds__(kWave) thresh_kernel(int32_t nseg, const int32_t* __restrict__ hist,
                                                        int32_t* __restrict__ info) {
    int32_t s = blockIdx.x;
    if (s >= nseg) return;
    const int lane = (int)lane_id();
    const int32_t* h = hist + (int64_t)s * kBins;
    int32_t live = info[s * kInfo + SI_LIVE];
    int32_t run = 0, bstar = kBins - 1, headn = live;
    bool done = false;
    for (int base = 0; base < kBins && !done; base += kWave) {
        int32_t v = h[base + lane];
        int32_t inc = v;
        for (int off = 1; off < kWave; off <<= 1) {
            int32_t o = __shfl_up(inc, off, kWave);
            if (lane >= off) inc += o;
        }
        uint64_t hit = __ballot(run + inc >= kHead);
        if (hit) {
            int l = __ffsll((unsigned long long)hit) - 1;
            bstar = base + l;
            headn = run + __shfl(inc, l, kWave);
            done = true;
        }
        run += __shfl(inc, kWave - 1, kWave);
    }
    if (lane == 0) {
        info[s * kInfo + SI_BSTAR] = bstar;
        info[s * kInfo + SI_HEADN] = headn;
        info[s * kInfo + SI_RESTN] = live - headn;
    }
}

// Offsets of every segment's head / rest group, their tile offsets, and round totals
// (single workgroup, sequential over blocks of 256 segments).
__global__ void __launch_bounds__(kBlock) seg_offsets_kernel(int32_t nseg, int32_t* __restrict__ info,
                                                              int32_t* __restrict__ tile_off,
                                                              int32_t* __restrict__ counters) {
    __shared__ int32_t carry[4];
    __shared__ int32_t wsum[4][kBlock / kWave];
    __shared__ int32_t wmax[kBlock / kWave];
    __shared__ int32_t maxh;
    if (threadIdx.x == 0) { carry[0] = carry[1] = carry[2] = carry[3] = 0; maxh = 0; }
    __syncthreads();
    const int lane = (int)lane_id();
    const int wave = threadIdx.x / kWave;
    for (int base = 0; base < nseg; base += kBlock) {
        int32_t s = base + threadIdx.x;
        int32_t hn = 0, rn = 0, ht = 0, rt = 0;
        if (s < nseg) {
            hn = info[s * kInfo + SI_HEADN];
            rn = info[s * kInfo + SI_RESTN];
            ht = (hn + kItems - 1) / kItems;
            rt = (rn + kItems - 1) / kItems;
        }
        int32_t v[4] = {hn, rn, ht, rt}, inc[4];
        for (int q = 0; q < 4; ++q) {
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
        int32_t excl[4];
        for (int q = 0; q < 4; ++q) {
            int32_t before = carry[q];
            for (int w = 0; w < wave; ++w) before += wsum[q][w];
            excl[q] = before + inc[q] - v[q];
        }
        if (s < nseg) {
            info[s * kInfo + SI_HEADOFF] = excl[0];
            info[s * kInfo + SI_RESTOFF] = excl[1];
            tile_off[s] = excl[2];
            tile_off[(nseg + 1) + s] = excl[3];
            info[s * kInfo + SI_HCUR] = 0;
            info[s * kInfo + SI_RCUR] = 0;
            info[s * kInfo + SI_FCUR] = 0;
        }
        __syncthreads();
        if (threadIdx.x == kBlock - 1)
            for (int q = 0; q < 4; ++q) carry[q] = excl[q] + v[q];
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
    }
}

__global__ void __launch_bounds__(kBlock) split_kernel(const int32_t* __restrict__ items, int32_t n,
                                                        const float* __restrict__ fsum,
                                                        const int32_t* __restrict__ seg_of_pos,
                                                        const uint32_t* __restrict__ smin,
                                                        const uint32_t* __restrict__ smax,
                                                        int32_t* __restrict__ info,
                                                        int32_t* __restrict__ head,
                                                        int32_t* __restrict__ rest,
                                                        uint8_t* __restrict__ dom) {
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    const bool valid = i < n;
    int32_t pos = 0, s = 0;
    bool is_head = false;
    if (valid) {
        pos = items[i];
        s = seg_of(seg_of_pos, pos);
        int32_t b = bin_of(fsum[pos], __uint_as_float(smin[s]), seg_scale(smin[s], smax[s]));
        is_head = b <= info[s * kInfo + SI_BSTAR];
        dom[pos] = 0;
    }
    const int32_t hs = wave_slot(info + SI_HCUR, kInfo, s, valid && is_head);
    const int32_t rs = wave_slot(info + SI_RCUR, kInfo, s, valid && !is_head);
    if (valid) {
        if (is_head) head[info[s * kInfo + SI_HEADOFF] + hs] = pos;
        else rest[info[s * kInfo + SI_RESTOFF] + rs] = pos;
    }
}

// Locate the segment of a tile: largest s with tile_off[s] <= t (tile_off[0..nseg] ascending).
__device__ __forceinline__ int32_t tile_segment(const int32_t* tile_off, int32_t nseg, int32_t t) {
    int32_t lo = 0, hi = nseg - 1;
    while (lo < hi) {
        int32_t mid = (lo + hi + 1) >> 1;
        if (tile_off[mid] <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Items of one segment tile (blockIdx.x, 256 items, 64 per wave) against a range of that
// segment's candidates (blockIdx.y selects the range when the grid is split along
// candidates). mode 0: items and candidates = the head group; mode 1: items = the rest group,
// candidates = the head-skyline group (count in SI_FCUR).
// The candidate range is staged in LDS chunk by chunk (structure of arrays, lane-consecutive).
// Each wave takes its items one at a time; the 64 lanes test 64 candidates at once and a
// ballot ends the item at its first dominator, so lanes never idle behind other items.
// A dominated item gets dom[pos] = 1 (idempotent; items already flagged are skipped).
template <int D>
__global__ void __launch_bounds__(kBlock) test_kernel(
    int mode, const float* __restrict__ xp, int64_t ldp, int32_t d_rt, int32_t nseg,
    const int32_t* __restrict__ tile_off, const int32_t* __restrict__ info,
    const int32_t* __restrict__ items_all, const int32_t* __restrict__ cand_all, int32_t span,
    int32_t chunk, uint8_t* __restrict__ dom, unsigned long long* __restrict__ tests) {
    extern __shared__ uint32_t cvs[];  // [d][chunk]
    constexpr int DM = D > 0 ? D : SKY_MAX_D;
    const int d = dget<D>(d_rt);
    const int lane = (int)lane_id();
    const int wave = threadIdx.x / kWave;
    const int32_t* toff = tile_off + (mode == 0 ? 0 : (nseg + 1));
    const int32_t t = blockIdx.x;
    if (t >= toff[nseg]) return;  // uniform per workgroup
    const int32_t s = tile_segment(toff, nseg, t);
    const int32_t* si = info + s * kInfo;
    const int32_t ioff = mode == 0 ? si[SI_HEADOFF] : si[SI_RESTOFF];
    const int32_t icnt = mode == 0 ? si[SI_HEADN] : si[SI_RESTN];
    const int32_t coff = si[SI_HEADOFF];
    const int32_t ccnt = mode == 0 ? si[SI_HEADN] : si[SI_FCUR];
    const int32_t r0 = (int32_t)blockIdx.y * span;
    if (r0 >= ccnt) return;  // uniform
    const int32_t r1 = (ccnt - r0) < span ? ccnt : r0 + span;
    const int32_t ibase = (t - toff[s]) * kItems + wave * kWave;
    const int32_t nmine = icnt - ibase < kWave ? (icnt - ibase > 0 ? icnt - ibase : 0) : kWave;
    // this wave's items: position held by lane i (uniform reads below via shuffles)
    const int32_t mypos = lane < nmine ? items_all[ioff + ibase + lane] : 0;
    uint64_t done = __ballot(lane < nmine ? dom[mypos] != 0 : true);  // bit i: item i finished
    unsigned long long ntests = 0;
    for (int32_t c0 = r0; c0 < r1; c0 += chunk) {
        const int32_t nc = (r1 - c0) < chunk ? (r1 - c0) : chunk;
        // barrier: the previous chunk is fully consumed; stop when every item is finished
        if (__syncthreads_or(done != ~0ull) == 0) break;
        for (int32_t j = threadIdx.x; j < nc; j += kBlock) {
            const int32_t cp = cand_all[coff + c0 + j];
#pragma unroll
            for (int k = 0; k < DM; ++k)
                if (k < d) cvs[k * chunk + j] = fbits(xp[(int64_t)k * ldp + cp]);
        }
        __syncthreads();
        uint64_t todo = ~done;
        while (todo) {
            const int i = __ffsll((unsigned long long)todo) - 1;
            todo &= todo - 1;
            const int32_t pos = __shfl(mypos, i, kWave);
            uint32_t tv[DM];
#pragma unroll
            for (int k = 0; k < DM; ++k)
                if (k < d) tv[k] = fbits(xp[(int64_t)k * ldp + pos]);
            int32_t j0 = 0;
            bool found = false;
            for (; j0 < nc; j0 += kWave) {
                const int32_t j = j0 + lane;
                bool le = j < nc, lt = false;
#pragma unroll
                for (int k = 0; k < DM; ++k)
                    if (k < d) {
                        const uint32_t c = le ? cvs[k * chunk + j] : 0u;
                        le &= c <= tv[k];
                        lt |= c < tv[k];
                    }
                if (__ballot(le && lt)) { found = true; break; }
            }
            ntests += (unsigned long long)((j0 + kWave) < nc ? (j0 + kWave) : nc);
            if (found) {
                done |= 1ull << i;
                if (lane == 0) dom[pos] = 1;
            }
        }
    }
    // per-wave tally (lane 0 holds the wave's count)
    if (lane == 0 && ntests) atomicAdd(&tests[mode], ntests);
}

// Head survivors -> head-skyline group of their segment, output flags and output list.
__global__ void __launch_bounds__(kBlock) compact_head_kernel(
    const int32_t* __restrict__ head, const int32_t* __restrict__ counters,
    const int32_t* __restrict__ seg_of_pos, const uint8_t* __restrict__ dom,
    int32_t* __restrict__ info, int32_t* __restrict__ fsky, uint8_t* __restrict__ flag_out,
    int32_t* __restrict__ out_list, int32_t* __restrict__ out_counter) {
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    const bool valid = i < counters[C_HTOT];
    int32_t pos = 0, s = 0;
    bool keep = false;
    if (valid) {
        pos = head[i];
        s = seg_of(seg_of_pos, pos);
        keep = dom[pos] == 0;
    }
    const int32_t fs = wave_slot(info + SI_FCUR, kInfo, s, keep);
    const int32_t os = wave_slot(out_counter, 0, 0, keep);
    if (keep) {
        fsky[info[s * kInfo + SI_HEADOFF] + fs] = pos;
        flag_out[pos] = 1;
        out_list[os] = pos;
    }
}

// Rest survivors -> next work list.
__global__ void __launch_bounds__(kBlock) compact_rest_kernel(const int32_t* __restrict__ rest,
                                                               int32_t* __restrict__ counters,
                                                               const uint8_t* __restrict__ dom,
                                                               int32_t* __restrict__ next) {
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    const bool valid = i < counters[C_RTOT];
    int32_t pos = 0;
    bool keep = false;
    if (valid) {
        pos = rest[i];
        keep = dom[pos] == 0;
    }
    const int32_t slot = wave_slot(counters + C_NEXT, 0, 0, keep);
    if (keep) next[slot] = pos;
}

__global__ void zero_i32_kernel(int32_t* __restrict__ p, int32_t n) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ void zero_u64_kernel(unsigned long long* __restrict__ p, int32_t n) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// positions [0, n) whose segment is not skipped
__global__ void __launch_bounds__(kBlock) iota_filtered_kernel(const uint8_t* __restrict__ skip,
                                                                const int32_t* __restrict__ seg,
                                                                int32_t n, int32_t* __restrict__ out,
                                                                int32_t* __restrict__ count) {
    int32_t i = blockIdx.x * kBlock + threadIdx.x;
    bool keep = i < n && !(skip && skip[seg[i]]);
    uint64_t m = __ballot(keep);
    int32_t base = 0;
    if (lane_id() == 0 && m) base = atomicAdd(count, (int32_t)__popcll(m));
    base = __shfl(base, 0, kWave);
    if (keep) out[base + (int32_t)__popcll(m & __lanemask_lt())] = i;
}

__global__ void __launch_bounds__(kBlock) compact_flags_kernel(const uint8_t* __restrict__ flags,
                                                                int32_t n, int32_t* __restrict__ out,
                                                                int32_t* __restrict__ count) {
    int32_t i = blockIdx.x * kBlock + threadIdx.x;
    bool keep = i < n && flags[i];
    uint64_t m = __ballot(keep);
    int32_t base = 0;
    if (lane_id() == 0 && m) base = atomicAdd(count, (int32_t)__popcll(m));
    base = __shfl(base, 0, kWave);
    if (keep) out[base + (int32_t)__popcll(m & __lanemask_lt())] = i;
}

// ---- final output: ascending original row ids ------------------------------------------------
__global__ void __launch_bounds__(kBlock) mark_rows_kernel(const int32_t* __restrict__ list,
                                                            int32_t count,
                                                            const int32_t* __restrict__ rowid,
                                                            uint8_t* __restrict__ member) {
    int32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < count) member[rowid[list[i]]] = 1;
}

__global__ void __launch_bounds__(kBlock) u8_to_i32_kernel(const uint8_t* __restrict__ m, int64_t n,
                                                            int32_t* __restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) out[i] = m[i];
}

__global__ void __launch_bounds__(kBlock) write_idx_kernel(const uint8_t* __restrict__ m, int64_t n,
                                                            const int32_t* __restrict__ pos,
                                                            int64_t* __restrict__ sky_idx,
                                                            int64_t cap,
                                                            uint8_t* __restrict__ member_out) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    uint8_t v = m[i];
    if (member_out) member_out[i] = v;
    if (v) {
        int64_t p = pos[i];
        if (p < cap) sky_idx[p] = i;
    }
}

__global__ void finish_count_kernel(const int32_t* __restrict__ pos, const uint8_t* __restrict__ m,
                                    int64_t n, int64_t cap, int64_t* __restrict__ dev_count,
                                    int32_t* dev_status) {
    int64_t c = (int64_t)pos[n - 1] + (int64_t)m[n - 1];
    *dev_count = c;
    if (c > cap) raise_status(dev_status, SKY_ERR_CAPACITY);
}

__global__ void __launch_bounds__(kBlock) scatter_rows_i32_kernel(const int32_t* __restrict__ src,
                                                                   const int32_t* __restrict__ rowid,
                                                                   int64_t n, int32_t* __restrict__ dst) {
    int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q < n) dst[rowid[q]] = src[q];
}

__global__ void __launch_bounds__(kBlock) scatter_rows_u8_kernel(const uint8_t* __restrict__ src,
                                                                  const int32_t* __restrict__ rowid,
                                                                  int64_t n, uint8_t* __restrict__ dst) {
    int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q < n) dst[rowid[q]] = src[q];
}

__global__ void fill_u8_kernel(uint8_t* __restrict__ p, int64_t n, uint8_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
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

sky_status run_engine(const EngineProblem& pb, const EngineBuffers& b, int32_t* out_list,
                      EngineResult* res, hipStream_t st) {
    res->count = 0;
    res->rounds = 0;
    res->tests = 0;
    const int32_t nseg = pb.nseg;
    int32_t live = pb.n_items;
    const int32_t* cur = pb.items;
    int32_t* next = b.w0;
    int32_t* other = b.w1;
    hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(64), 0, st, b.counters, (int32_t)kCounters);
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, st, b.tests, 2);
    SKY_HIP(hipGetLastError());
    // LDS chunk of candidates (d x chunk uint32) and the split of the candidate range across
    // workgroups (grid.y) so that tiles x splits reaches kMinBlocks
    const int32_t chunk = (int32_t)((kLdsBytes / (4 * pb.d)) / kWave * kWave);
    const size_t lds = (size_t)pb.d * (size_t)chunk * sizeof(uint32_t);
    auto split = [&](int64_t tiles, int64_t maxc, int32_t* span) -> uint32_t {
        if (tiles <= 0 || maxc <= 0) { *span = chunk; return 1; }
        int64_t y = ceil_div(kMinBlocks, tiles);
        int64_t ymax = ceil_div(maxc, kWave * 8);  // at least 512 candidates per split
        if (y > ymax) y = ymax;
        if (y < 1) y = 1;
        int64_t sp = round_up(ceil_div(maxc, y), kWave);
        *span = (int32_t)sp;
        return (uint32_t)ceil_div(maxc, sp);
    };
    // optional timing hooks around the dominance-test launches
    auto ev_rec = [&](bool begin) -> hipError_t {
        if (!pb.ev_begin || !pb.ev_end || !pb.ev_used || *pb.ev_used >= pb.ev_cap) return hipSuccess;
        hipEvent_t e = (hipEvent_t)(begin ? pb.ev_begin[*pb.ev_used] : pb.ev_end[*pb.ev_used]);
        hipError_t r = hipEventRecord(e, st);
        if (!begin) ++*pb.ev_used;
        return r;
    };
    int guard = 0;
    while (live > 0) {
        if (++guard > 1000000) return SKY_ERR_HIP;
        res->rounds++;
        const uint32_t iblocks = (uint32_t)ceil_div(live, kBlock);
        const int64_t hn = (int64_t)nseg * kBins;
        hipLaunchKernelGGL(init_segments_kernel, dim3((uint32_t)ceil_div(hn > nseg ? hn : nseg, 256)),
                           dim3(256), 0, st, nseg, b.seg_min, b.seg_max, b.hist, b.seg_info,
                           b.counters);
        hipLaunchKernelGGL(minmax_kernel, dim3(iblocks), dim3(kBlock), 0, st, cur, live, pb.fsum,
                           pb.seg_of_pos, b.seg_min, b.seg_max, b.seg_info);
        hipLaunchKernelGGL(hist_kernel, dim3(iblocks), dim3(kBlock), 0, st, cur, live, pb.fsum,
                           pb.seg_of_pos, (const uint32_t*)b.seg_min, (const uint32_t*)b.seg_max,
                           b.hist);
        hipLaunchKernelGGL(thresh_kernel, dim3((uint32_t)nseg), dim3(kWave), 0, st, nseg,
                           (const int32_t*)b.hist, b.seg_info);
        hipLaunchKernelGGL(seg_offsets_kernel, dim3(1), dim3(kBlock), 0, st, nseg, b.seg_info,
                           b.tile_off, b.counters);
        hipLaunchKernelGGL(split_kernel, dim3(iblocks), dim3(kBlock), 0, st, cur, live, pb.fsum,
                           pb.seg_of_pos, (const uint32_t*)b.seg_min, (const uint32_t*)b.seg_max,
                           b.seg_info, b.head, b.rest, b.dom);
        SKY_HIP(hipGetLastError());
        int32_t cnt[kCounters];
        SKY_HIP(hipMemcpyAsync(cnt, b.counters, sizeof(cnt), hipMemcpyDeviceToHost, st));
        SKY_HIP(hipStreamSynchronize(st));
        const int32_t htiles = cnt[C_HTILES], rtiles = cnt[C_RTILES], maxh = cnt[C_MAXH];
        const int32_t htot = cnt[C_HTOT], rtot = cnt[C_RTOT];
        if (htot <= 0 || htot + rtot != live) return SKY_ERR_HIP;  // internal consistency
        // head skyline: all pairs inside every segment's head
        int32_t span = chunk;
        uint32_t ychunks = split(htiles, maxh, &span);
        SKY_HIP(ev_rec(true));
        SKY_DISPATCH_D(pb.d, test_kernel, dim3((uint32_t)htiles, ychunks), dim3(kBlock), lds, st, 0,
                       pb.xp, pb.ldp, pb.d, nseg, (const int32_t*)b.tile_off,
                       (const int32_t*)b.seg_info, (const int32_t*)b.head, (const int32_t*)b.head,
                       span, chunk, b.dom, b.tests);
        SKY_HIP(ev_rec(false));
        hipLaunchKernelGGL(compact_head_kernel, dim3((uint32_t)ceil_div(htot, kBlock)), dim3(kBlock), 0,
                           st, (const int32_t*)b.head, (const int32_t*)b.counters, pb.seg_of_pos,
                           (const uint8_t*)b.dom, b.seg_info, b.fsky, pb.flag_out, out_list,
                           b.counters + C_OUT);
        SKY_HIP(hipGetLastError());
        if (rtot > 0) {
            // filter the rest against the head skylines
            ychunks = split(rtiles, maxh, &span);
            SKY_HIP(ev_rec(true));
            SKY_DISPATCH_D(pb.d, test_kernel, dim3((uint32_t)rtiles, ychunks), dim3(kBlock), lds, st, 1,
                           pb.xp, pb.ldp, pb.d, nseg, (const int32_t*)b.tile_off,
                           (const int32_t*)b.seg_info, (const int32_t*)b.rest,
                           (const int32_t*)b.fsky, span, chunk, b.dom, b.tests);
            SKY_HIP(ev_rec(false));
            hipLaunchKernelGGL(compact_rest_kernel, dim3((uint32_t)ceil_div(rtot, kBlock)), dim3(kBlock),
                               0, st, (const int32_t*)b.rest, b.counters, (const uint8_t*)b.dom, next);
            SKY_HIP(hipGetLastError());
        }
        int32_t nl = 0;
        if (rtot > 0) {
            SKY_HIP(hipMemcpyAsync(&nl, b.counters + C_NEXT, sizeof(int32_t), hipMemcpyDeviceToHost, st));
            SKY_HIP(hipStreamSynchronize(st));
        }
        // every round removes the head rows from the live set
        if (nl >= live) return SKY_ERR_HIP;
        live = nl;
        cur = next;
        int32_t* t = next; next = other; other = t;
    }
    int32_t outc = 0;
    unsigned long long tests[2] = {0, 0};
    SKY_HIP(hipMemcpyAsync(&outc, b.counters + C_OUT, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    SKY_HIP(hipMemcpyAsync(tests, b.tests, sizeof(tests), hipMemcpyDeviceToHost, st));
    SKY_HIP(hipStreamSynchronize(st));
    res->count = outc;
    res->tests = (int64_t)(tests[0] + tests[1]);
    return SKY_OK;
}

sky_status launch_iota_filtered(const uint8_t* skip_seg, const int32_t* seg_of_pos, int32_t n,
                                int32_t* out, int32_t* count, hipStream_t st) {
    hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(64), 0, st, count, 1);
    if (n > 0)
        hipLaunchKernelGGL(iota_filtered_kernel, dim3((uint32_t)ceil_div(n, kBlock)), dim3(kBlock), 0,
                           st, skip_seg, seg_of_pos, n, out, count);
    SKY_HIP(hipGetLastError());
    return SKY_OK;
}

sky_status launch_compact_flags(const uint8_t* flags, int32_t n, int32_t* out, int32_t* count,
                                hipStream_t st) {
    hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(64), 0, st, count, 1);
    if (n > 0)
        hipLaunchKernelGGL(compact_flags_kernel, dim3((uint32_t)ceil_div(n, kBlock)), dim3(kBlock), 0,
                           st, flags, n, out, count);
    SKY_HIP(hipGetLastError());
    return SKY_OK;
}

sky_status launch_scatter_rows(const int32_t* src_i32, const uint8_t* src_u8, const int32_t* rowid,
                               int64_t n, int32_t* dst_i32, uint8_t* dst_u8, hipStream_t st) {
    if (n <= 0) return SKY_OK;
    const uint32_t nb = (uint32_t)ceil_div(n, kBlock);
    if (dst_i32)
        hipLaunchKernelGGL(scatter_rows_i32_kernel, dim3(nb), dim3(kBlock), 0, st, src_i32, rowid, n,
                           dst_i32);
    if (dst_u8)
        hipLaunchKernelGGL(scatter_rows_u8_kernel, dim3(nb), dim3(kBlock), 0, st, src_u8, rowid, n,
                           dst_u8);
    SKY_HIP(hipGetLastError());
    return SKY_OK;
}

sky_status launch_fill_u8(uint8_t* p, int64_t n, uint8_t v, hipStream_t st) {
    if (n > 0)
        hipLaunchKernelGGL(fill_u8_kernel, dim3((uint32_t)ceil_div(n, 256)), dim3(256), 0, st, p, n, v);
    SKY_HIP(hipGetLastError());
    return SKY_OK;
}

sky_status launch_final_output(const int32_t* list, int32_t count, const int32_t* rowid, int64_t n,
                               uint8_t* member_tmp, uint8_t* member_out, int64_t* sky_idx,
                               int64_t cap, int64_t* dev_count, int32_t* pos_tmp, int32_t* scan_tmp,
                               int32_t* dev_status, hipStream_t st) {
    SKY_TRY(launch_fill_u8(member_tmp, n, 0, st));
    if (count > 0)
        hipLaunchKernelGGL(mark_rows_kernel, dim3((uint32_t)ceil_div(count, kBlock)), dim3(kBlock), 0,
                           st, list, count, rowid, member_tmp);
    const uint32_t nb = (uint32_t)ceil_div(n, kBlock);
    hipLaunchKernelGGL(u8_to_i32_kernel, dim3(nb), dim3(kBlock), 0, st, (const uint8_t*)member_tmp, n,
                       pos_tmp);
    SKY_HIP(hipGetLastError());
    SKY_TRY(launch_exclusive_scan(pos_tmp, pos_tmp, n, scan_tmp, st));
    hipLaunchKernelGGL(write_idx_kernel, dim3(nb), dim3(kBlock), 0, st, (const uint8_t*)member_tmp, n,
                       (const int32_t*)pos_tmp, sky_idx, cap, member_out);
    hipLaunchKernelGGL(finish_count_kernel, dim3(1), dim3(1), 0, st, (const int32_t*)pos_tmp,
                       (const uint8_t*)member_tmp, n, cap, dev_count, dev_status);
    SKY_HIP(hipGetLastError());
    return SKY_OK;
}

}  // namespace sky
