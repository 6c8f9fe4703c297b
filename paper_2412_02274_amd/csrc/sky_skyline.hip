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
constexpr int kCand = 256;    // candidates staged in LDS per step

// seg_info layout per segment (int32 x 8)
enum { SI_LIVE = 0, SI_BSTAR, SI_HEADN, SI_HEADOFF, SI_RESTN, SI_RESTOFF, SI_HCUR, SI_RCUR };
// counters layout
enum { C_NEXT = 0, C_OUT, C_FCUR_BASE };

template <int D>
__device__ __forceinline__ int dget(int d) { return D > 0 ? D : d; }

__device__ __forceinline__ int32_t seg_of(const int32_t* seg_of_pos, int32_t pos) {
    return seg_of_pos ? seg_of_pos[pos] : 0;
}

__global__ void init_segments_kernel(int32_t nseg, uint32_t* __restrict__ smin,
                                     uint32_t* __restrict__ smax, int32_t* __restrict__ hist,
                                     int32_t* __restrict__ info) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < (int64_t)nseg * kBins) hist[i] = 0;
    if (i < nseg) {
        smin[i] = 0xFFFFFFFFu;
        smax[i] = 0u;
        for (int j = 0; j < 8; ++j) info[i * 8 + j] = 0;
    }
}

__global__ void __launch_bounds__(kBlock) minmax_kernel(const int32_t* __restrict__ items, int32_t n,
                                                         const float* __restrict__ fsum,
                                                         const int32_t* __restrict__ seg_of_pos,
                                                         uint32_t* __restrict__ smin,
                                                         uint32_t* __restrict__ smax,
                                                         int32_t* __restrict__ info) {
    int32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int32_t pos = items[i];
    int32_t s = seg_of(seg_of_pos, pos);
    uint32_t fb = fbits(fsum[pos]);  // f >= 0: bit order == value order
    atomicMin(&smin[s], fb);
    atomicMax(&smax[s], fb);
    atomicAdd(&info[s * 8 + SI_LIVE], 1);
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
    int32_t live = info[s * 8 + SI_LIVE];
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
        info[s * 8 + SI_BSTAR] = bstar;
        info[s * 8 + SI_HEADN] = headn;
        info[s * 8 + SI_RESTN] = live - headn;
    }
}

// Offsets of every segment's head / rest group and their tile offsets (single workgroup,
// sequential over blocks of segments).
__global__ void __launch_bounds__(kBlock) seg_offsets_kernel(int32_t nseg, int32_t* __restrict__ info,
                                                              int32_t* __restrict__ tile_off) {
    __shared__ int32_t carry[4];
    if (threadIdx.x == 0) { carry[0] = carry[1] = carry[2] = carry[3] = 0; }
    __syncthreads();
    const int lane = (int)lane_id();
    const int wave = threadIdx.x / kWave;
    __shared__ int32_t wsum[4][4];
    for (int base = 0; base < nseg; base += kBlock) {
        int32_t s = base + threadIdx.x;
        int32_t hn = 0, rn = 0, ht = 0, rt = 0;
        if (s < nseg) {
            hn = info[s * 8 + SI_HEADN];
            rn = info[s * 8 + SI_RESTN];
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
        __syncthreads();
        int32_t excl[4];
        for (int q = 0; q < 4; ++q) {
            int32_t before = carry[q];
            for (int w = 0; w < wave; ++w) before += wsum[q][w];
            excl[q] = before + inc[q] - v[q];
        }
        if (s < nseg) {
            info[s * 8 + SI_HEADOFF] = excl[0];
            info[s * 8 + SI_RESTOFF] = excl[1];
            tile_off[s] = excl[2];
            tile_off[(nseg + 1) + s] = excl[3];
            info[s * 8 + SI_HCUR] = 0;
            info[s * 8 + SI_RCUR] = 0;
        }
        __syncthreads();
        if (threadIdx.x == kBlock - 1)
            for (int q = 0; q < 4; ++q) carry[q] = excl[q] + v[q];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        tile_off[nseg] = carry[2];
        tile_off[(nseg + 1) + nseg] = carry[3];
    }
}

__global__ void __launch_bounds__(kBlock) split_kernel(const int32_t* __restrict__ items, int32_t n,
                                                        const float* __restrict__ fsum,
                                                        const int32_t* __restrict__ seg_of_pos,
                                                        const uint32_t* __restrict__ smin,
                                                        const uint32_t* __restrict__ smax,
                                                        int32_t* __restrict__ info,
                                                        int32_t* __restrict__ head,
                                                        int32_t* __restrict__ rest) {
    int32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int32_t pos = items[i];
    int32_t s = seg_of(seg_of_pos, pos);
    int32_t b = bin_of(fsum[pos], __uint_as_float(smin[s]), seg_scale(smin[s], smax[s]));
    if (b <= info[s * 8 + SI_BSTAR]) {
        int32_t at = atomicAdd(&info[s * 8 + SI_HCUR], 1);
        head[info[s * 8 + SI_HEADOFF] + at] = pos;
    } else {
        int32_t at = atomicAdd(&info[s * 8 + SI_RCUR], 1);
        rest[info[s * 8 + SI_RESTOFF] + at] = pos;
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

// Dominance (Def. 1) of candidate c (values in LDS, column j) over item t (values in regs),
// on canonical bit patterns.
template <int D>
__device__ __forceinline__ bool dominated_by(const uint32_t* tv, const uint32_t (*cv)[kCand], int j,
                                             int d) {
    bool le = true, lt = false;
#pragma unroll
    for (int k = 0; k < (D > 0 ? D : SKY_MAX_D); ++k)
        if (k < d) {
            uint32_t c = cv[k][j];
            le &= c <= tv[k];
            lt |= c < tv[k];
        }
    return le && lt;
}

// mode 0 (head): items = head group of segment s, candidates = the same group; survivors go
//   to fsky (segment group at the head offset, counter SI_HCUR reused) and to out/flag.
// mode 1 (filter): items = rest group of s, candidates = fsky group of s; survivors go to the
//   next work list.
template <int D>
__global__ void __launch_bounds__(kBlock) test_kernel(
    int mode, const float* __restrict__ xp, int64_t ldp, int32_t d_rt, int32_t nseg,
    const int32_t* __restrict__ tile_off, int32_t* __restrict__ info,
    const int32_t* __restrict__ items_all, const int32_t* __restrict__ cand_all,
    const int32_t* __restrict__ fsky_count, int32_t* __restrict__ out_items,
    int32_t* __restrict__ out_counter, uint8_t* __restrict__ flag_out,
    int32_t* __restrict__ out_list, int32_t* __restrict__ out_list_counter,
    unsigned long long* __restrict__ tests) {
    __shared__ uint32_t cv[D > 0 ? D : SKY_MAX_D][kCand];
    __shared__ int32_t cpos[kCand];
    const int d = dget<D>(d_rt);
    const int32_t* toff = tile_off + (mode == 0 ? 0 : (nseg + 1));
    const int32_t t = blockIdx.x;
    if (t >= toff[nseg]) return;  // uniform per workgroup
    const int32_t s = tile_segment(toff, nseg, t);
    const int32_t* si = info + s * 8;
    const int32_t ioff = mode == 0 ? si[SI_HEADOFF] : si[SI_RESTOFF];
    const int32_t icnt = mode == 0 ? si[SI_HEADN] : si[SI_RESTN];
    const int32_t coff = si[SI_HEADOFF];
    const int32_t ccnt = mode == 0 ? si[SI_HEADN] : fsky_count[s];
    const int32_t first = (t - toff[s]) * kItems;
    const int32_t me = first + (int32_t)threadIdx.x;
    const bool valid = me < icnt;
    int32_t pos = valid ? items_all[ioff + me] : -1;
    uint32_t tv[D > 0 ? D : SKY_MAX_D];
#pragma unroll
    for (int k = 0; k < (D > 0 ? D : SKY_MAX_D); ++k)
        if (k < d) tv[k] = valid ? fbits(xp[(int64_t)k * ldp + pos]) : 0u;
    bool alive = valid;
    unsigned long long ntests = 0;
    for (int32_t c0 = 0; c0 < ccnt; c0 += kCand) {
        if (__syncthreads_or(alive) == 0) break;
        const int32_t nc = (ccnt - c0) < kCand ? (ccnt - c0) : kCand;
        if ((int)threadIdx.x < nc) {
            int32_t cp = cand_all[coff + c0 + threadIdx.x];
            cpos[threadIdx.x] = cp;
#pragma unroll
            for (int k = 0; k < (D > 0 ? D : SKY_MAX_D); ++k)
                if (k < d) cv[k][threadIdx.x] = fbits(xp[(int64_t)k * ldp + cp]);
        }
        __syncthreads();
        if (alive) {
            int j = 0;
            for (; j < nc; ++j) {
                if (dominated_by<D>(tv, cv, j, d)) { alive = false; ++j; break; }
            }
            ntests += (unsigned long long)j;
        }
        __syncthreads();
    }
    (void)cpos;
    if (valid && alive) {
        if (mode == 0) {
            int32_t at = atomicAdd(&info[s * 8 + SI_HCUR], 1);
            out_items[coff + at] = pos;  // fsky group of s (same offsets as the head group)
            flag_out[pos] = 1;
            int32_t o = atomicAdd(out_list_counter, 1);
            out_list[o] = pos;
        } else {
            int32_t at = atomicAdd(out_counter, 1);
            out_items[at] = pos;
        }
    }
    // wave-level reduction of the test count
    for (int off = kWave / 2; off > 0; off >>= 1) ntests += __shfl_down(ntests, off, kWave);
    if (lane_id() == 0 && ntests) atomicAdd(&tests[mode], ntests);
}

__global__ void fsky_count_kernel(int32_t nseg, int32_t* __restrict__ info,
                                  int32_t* __restrict__ fcount) {
    int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < nseg) {
        fcount[s] = info[s * 8 + SI_HCUR];
        info[s * 8 + SI_HCUR] = 0;  // reused by the head kernel as the fsky cursor
    }
}

__global__ void copy_count_kernel(const int32_t* __restrict__ fcount, int32_t nseg,
                                  int32_t* __restrict__ info) {
    int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < nseg) info[s * 8 + SI_HCUR] = 0;
    (void)fcount;
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
    // counters: [C_NEXT]=next list size, [C_OUT]=out_list size
    hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(64), 0, st, b.counters, 16);
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, st, b.tests, 2);
    SKY_HIP(hipGetLastError());
    int32_t* fcount = b.seg_info + (int64_t)nseg * 8;  // [nseg] after the info table
    while (live > 0) {
        res->rounds++;
        const uint32_t iblocks = (uint32_t)ceil_div(live, kBlock);
        const int64_t hn = (int64_t)nseg * kBins;
        hipLaunchKernelGGL(init_segments_kernel, dim3((uint32_t)ceil_div(hn > nseg ? hn : nseg, 256)),
                           dim3(256), 0, st, nseg, b.seg_min, b.seg_max, b.hist, b.seg_info);
        hipLaunchKernelGGL(minmax_kernel, dim3(iblocks), dim3(kBlock), 0, st, cur, live, pb.fsum,
                           pb.seg_of_pos, b.seg_min, b.seg_max, b.seg_info);
        hipLaunchKernelGGL(hist_kernel, dim3(iblocks), dim3(kBlock), 0, st, cur, live, pb.fsum,
                           pb.seg_of_pos, (const uint32_t*)b.seg_min, (const uint32_t*)b.seg_max,
                           b.hist);
        hipLaunchKernelGGL(thresh_kernel, dim3((uint32_t)nseg), dim3(kWave), 0, st, nseg,
                           (const int32_t*)b.hist, b.seg_info);
        hipLaunchKernelGGL(seg_offsets_kernel, dim3(1), dim3(kBlock), 0, st, nseg, b.seg_info,
                           b.tile_off);
        hipLaunchKernelGGL(split_kernel, dim3(iblocks), dim3(kBlock), 0, st, cur, live, pb.fsum,
                           pb.seg_of_pos, (const uint32_t*)b.seg_min, (const uint32_t*)b.seg_max,
                           b.seg_info, b.head, b.rest);
        SKY_HIP(hipGetLastError());
        // head skyline: reset the per-segment cursor (reused for fsky), then test all pairs
        hipLaunchKernelGGL(copy_count_kernel, dim3((uint32_t)ceil_div(nseg, 256)), dim3(256), 0, st,
                           (const int32_t*)fcount, nseg, b.seg_info);
        const uint32_t max_tiles = (uint32_t)(ceil_div(live, kItems) + nseg);
        SKY_DISPATCH_D(pb.d, test_kernel, dim3(max_tiles), dim3(kBlock), 0, st, 0, pb.xp, pb.ldp,
                       pb.d, nseg, (const int32_t*)b.tile_off, b.seg_info,
                       (const int32_t*)b.head, (const int32_t*)b.head, (const int32_t*)fcount,
                       b.fsky, b.counters + C_NEXT, pb.flag_out, out_list, b.counters + C_OUT,
                       b.tests);
        SKY_HIP(hipGetLastError());
        hipLaunchKernelGGL(fsky_count_kernel, dim3((uint32_t)ceil_div(nseg, 256)), dim3(256), 0, st,
                           nseg, b.seg_info, fcount);
        // filter the rest against the head skylines
        hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(64), 0, st, b.counters + C_NEXT, 1);
        SKY_DISPATCH_D(pb.d, test_kernel, dim3(max_tiles), dim3(kBlock), 0, st, 1, pb.xp, pb.ldp,
                       pb.d, nseg, (const int32_t*)b.tile_off, b.seg_info,
                       (const int32_t*)b.rest, (const int32_t*)b.fsky, (const int32_t*)fcount,
                       next, b.counters + C_NEXT, pb.flag_out, out_list, b.counters + C_OUT,
                       b.tests);
        SKY_HIP(hipGetLastError());
        int32_t nl = 0;
        SKY_HIP(hipMemcpyAsync(&nl, b.counters + C_NEXT, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        SKY_HIP(hipStreamSynchronize(st));
        // every round removes the head rows from the live set; anything else is an internal
        // error and must not loop
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
