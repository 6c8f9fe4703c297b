// Grid resistance (Def. 2) of the skyline tuples via Alg. 1 in per-tuple form.
//
// For every skyline tuple t the result is g_exit(t) = the largest g in [2, g_max] at which
// the projection of some other skyline tuple s dominates the projection of t (Alg. 1 scans g
// downwards and records the first g at which t leaves the projected skyline), or 1. gres is
// stable (dominated tuples never matter), so the candidates s are the skyline tuples
// themselves. Projections are compared through integer keys K_g(v) = floor(fl32(v * g)).
//
// Exact pruning used by both mappings (no candidate that could dominate is ever skipped):
//  * tile boxes -- candidates are sorted along a Morton curve and cut into tiles of 64; lo
//    is the tile's componentwise minimum. K_g is non-decreasing in v (an FP32 multiply by
//    g > 0 rounded to nearest is monotone, floor too), so K_g(s_k) >= K_g(lo_k) for every s
//    of the tile, and K_g(s) <= K_g(t) componentwise requires K_g(lo) <= K_g(t)
//    componentwise. Tiles failing that test at level g hold no dominator at level g.
//  * level bound -- if s_k > t_k, K_g(s_k) <= K_g(t_k) needs fl(s_k g) - fl(t_k g) < 1, and
//    with FP32 relative rounding error at most u = 2^-24 on values below g this gives
//    g (s_k - t_k - 2u) < 1. So with delta = max_k (s_k - t_k) (or the same from a tile's lo,
//    which bounds every member from below), no level g with g (delta - 2^-23) >= 1 can see s
//    dominate t. Evaluated in double with a 1e-9 margin.
//
// Mappings (both one wavefront per tuple t, which keeps the control flow wave-uniform and
// lets the search stop at the first dominator):
//  * TILES  -- levels in order g_max..2; per level the 64 lanes first test 64 tile boxes at
//    once (ballot), then, tile by tile, the 64 lanes test the tile's 64 candidates (ballot);
//    the first dominator ends the level and the search. Best when S is large and g_max
//    small.
//  * LEVELS -- lanes hold 64 consecutive levels; candidates are read as wave-uniform values
//    and each lane tests its own level; the highest level with a dominator in the block of
//    64 levels ends the search. Best when S is small and g_max large.
// Bound: VALU compare/convert throughput and L2 latency (the candidate set of a dataset is
// at most a few MB and stays in L2).
#include "sky_internal.hpp"

namespace sky {

namespace {

constexpr int kTileC = 64;  // candidates per tile

template <int D>
__device__ __forceinline__ int dget(int d) { return D > 0 ? D : d; }

// Morton code of canonical values in [0, 1): b bits per attribute, attribute 0 most significant
// within every bit level.
__global__ void __launch_bounds__(kBlock) morton_kernel(const float* __restrict__ x, int64_t n,
                                                         int32_t d, int64_t ld,
                                                         const int64_t* __restrict__ sky_idx,
                                                         int32_t s, int bits,
                                                         uint32_t* __restrict__ keys,
                                                         uint32_t* __restrict__ vals,
                                                         int32_t* dev_status) {
    int32_t j = blockIdx.x * kBlock + threadIdx.x;
    bool bad_idx = false, bad_val = false;
    if (j < s) {
        int64_t row = sky_idx[j];
        uint32_t q[SKY_MAX_D];
        if (row < 0 || row >= n) {
            bad_idx = true;
            for (int k = 0; k < d; ++k) q[k] = 0;
        } else {
            const float scale = (float)(1u << bits);
            for (int k = 0; k < d; ++k) {
                float v = x[(int64_t)k * ld + row];
                bad_val |= !in_domain(v);
                v = canon(v);
                float t = v * scale;  // exact: power-of-two scaling
                uint32_t c = in_domain(v) ? (uint32_t)t : 0u;
                uint32_t cap = (1u << bits) - 1u;
                q[k] = c > cap ? cap : c;
            }
        }
        uint32_t code = 0;
        for (int l = bits - 1; l >= 0; --l)
            for (int k = 0; k < d; ++k) code = (code << 1) | ((q[k] >> l) & 1u);
        keys[j] = code;
        vals[j] = (uint32_t)j;
    }
    if (__ballot(bad_idx) && lane_id() == 0) raise_status(dev_status, SKY_ERR_INVALID_ARG);
    if (__ballot(bad_val) && lane_id() == 0) raise_status(dev_status, SKY_ERR_DOMAIN);
}

__global__ void __launch_bounds__(kBlock) gather_sorted_kernel(const float* __restrict__ x, int64_t n,
                                                                int32_t d, int64_t ld,
                                                                const int64_t* __restrict__ sky_idx,
                                                                int32_t s,
                                                                const uint32_t* __restrict__ order,
                                                                float* __restrict__ cand,
                                                                int64_t s_pad) {
    int32_t q = blockIdx.x * kBlock + threadIdx.x;
    if (q >= s) return;
    int64_t row = sky_idx[order[q]];
    bool ok = row >= 0 && row < n;
    for (int k = 0; k < d; ++k) {
        float v = ok ? canon(x[(int64_t)k * ld + row]) : 0.0f;
        cand[(int64_t)k * s_pad + q] = v;
    }
}

// one wave per tile: componentwise minimum of its (up to 64) candidates
__global__ void __launch_bounds__(kBlock) tile_lo_kernel(const float* __restrict__ cand,
                                                          int64_t s_pad, int32_t s, int32_t d,
                                                          int32_t ntile, float* __restrict__ lo,
                                                          int64_t t_pad) {
    int32_t tile = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    if (tile >= ntile) return;
    const int lane = (int)lane_id();
    int32_t j = tile * kTileC + lane;
    for (int k = 0; k < d; ++k) {
        float v = j < s ? cand[(int64_t)k * s_pad + j] : 1.0f;
        for (int off = kWave / 2; off > 0; off >>= 1) v = fminf(v, __shfl_xor(v, off, kWave));
        if (lane == 0) lo[(int64_t)k * t_pad + tile] = v;
    }
}

template <int D>
__global__ void __launch_bounds__(kBlock) gres_tiles_kernel(const float* __restrict__ cand,
                                                             int64_t s_pad, int32_t s, int32_t d_rt,
                                                             const float* __restrict__ lo,
                                                             int64_t t_pad, int32_t ntile,
                                                             int32_t g_max,
                                                             int32_t* __restrict__ ge_sorted) {
    constexpr int DM = D > 0 ? D : SKY_MAX_D;
    const int d = dget<D>(d_rt);
    const int lane = (int)lane_id();
    const int32_t q = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    if (q >= s) return;  // whole wave
    float tv[DM];
#pragma unroll
    for (int k = 0; k < DM; ++k)
        if (k < d) tv[k] = cand[(int64_t)k * s_pad + q];
    const int32_t nchunk = (ntile + kWave - 1) / kWave;
    const int32_t c0 = (q / kTileC) / kWave;  // start near the tuple's own tile
    int32_t result = 1;
    for (int32_t g = g_max; g >= 2; --g) {
        const float fg = (float)g;
        int32_t kt[DM];
#pragma unroll
        for (int k = 0; k < DM; ++k)
            if (k < d) kt[k] = qkey(tv[k], fg);
        bool found = false;
        for (int32_t ci = 0; ci < nchunk && !found; ++ci) {
            int32_t c = c0 + ci;
            if (c >= nchunk) c -= nchunk;
            const int32_t tile = c * kWave + lane;
            bool pass = tile < ntile;
            if (pass) {
#pragma unroll
                for (int k = 0; k < DM; ++k)
                    if (k < d) pass &= qkey(lo[(int64_t)k * t_pad + tile], fg) <= kt[k];
            }
            uint64_t mask = __ballot(pass);
            while (mask) {
                const int tb = __ffsll((unsigned long long)mask) - 1;
                mask &= mask - 1;
                const int32_t j = (c * kWave + tb) * kTileC + lane;
                bool dom = false;
                if (j < s && j != q) {
                    bool le = true, lt = false;
#pragma unroll
                    for (int k = 0; k < DM; ++k)
                        if (k < d) {
                            int32_t ks = qkey(cand[(int64_t)k * s_pad + j], fg);
                            le &= ks <= kt[k];
                            lt |= ks < kt[k];
                        }
                    dom = le && lt;
                }
                if (__ballot(dom)) { found = true; break; }
            }
        }
        if (found) { result = g; break; }
    }
    if (lane == 0) ge_sorted[q] = result;
}

// no level g >= g_low can see a candidate whose (lower-bounding) excess over t is delta
__device__ __forceinline__ bool beyond_levels(double delta, int32_t g_low) {
    const double w = delta - 0x1p-23;
    return w > 0.0 && (double)g_low * w >= 1.0 + 1e-9;
}

template <int D>
__global__ void __launch_bounds__(kBlock) gres_levels_kernel(const float* __restrict__ cand,
                                                              int64_t s_pad, int32_t s, int32_t d_rt,
                                                              const float* __restrict__ lo,
                                                              int64_t t_pad, int32_t ntile,
                                                              int32_t g_max,
                                                              int32_t* __restrict__ ge_sorted) {
    constexpr int DM = D > 0 ? D : SKY_MAX_D;
    const int d = dget<D>(d_rt);
    const int lane = (int)lane_id();
    const int32_t q = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    if (q >= s) return;  // whole wave
    float tv[DM];
#pragma unroll
    for (int k = 0; k < DM; ++k)
        if (k < d) tv[k] = cand[(int64_t)k * s_pad + q];
    int32_t result = 1;
    for (int32_t gh = g_max; gh >= 2; gh -= kWave) {
        const int32_t g = gh - lane;
        const bool lv = g >= 2;
        const int32_t g_low = (gh - (kWave - 1)) > 2 ? (gh - (kWave - 1)) : 2;
        const float fg = (float)(lv ? g : 2);
        int32_t kt[DM];
#pragma unroll
        for (int k = 0; k < DM; ++k)
            if (k < d) kt[k] = qkey(tv[k], fg);
        const uint64_t lvmask = __ballot(lv);
        uint64_t hit = 0;
        for (int32_t tile = 0; tile < ntile; ++tile) {
            const uint64_t need =
                (hit ? ((1ull << (__ffsll((unsigned long long)hit) - 1)) - 1ull) : ~0ull) & lvmask;
            if (!need) break;
            // uniform bound on the whole tile
            double dt = -1.0;
#pragma unroll
            for (int k = 0; k < DM; ++k)
                if (k < d) {
                    double e = (double)lo[(int64_t)k * t_pad + tile] - (double)tv[k];
                    dt = e > dt ? e : dt;
                }
            if (beyond_levels(dt, g_low)) continue;
            bool pass = (need >> lane) & 1ull;
#pragma unroll
            for (int k = 0; k < DM; ++k)
                if (k < d) pass &= qkey(lo[(int64_t)k * t_pad + tile], fg) <= kt[k];
            if (!__ballot(pass)) continue;
            const int32_t base = tile * kTileC;
            const int32_t cnt = (s - base) < kTileC ? (s - base) : kTileC;
            for (int32_t i = 0; i < cnt; ++i) {
                const int32_t j = base + i;
                if (j == q) continue;
                float sv[DM];
                double ds = -1.0;
#pragma unroll
                for (int k = 0; k < DM; ++k)
                    if (k < d) {
                        sv[k] = cand[(int64_t)k * s_pad + j];
                        double e = (double)sv[k] - (double)tv[k];
                        ds = e > ds ? e : ds;
                    }
                if (beyond_levels(ds, g_low)) continue;
                bool le = true, lt = false;
#pragma unroll
                for (int k = 0; k < DM; ++k)
                    if (k < d) {
                        int32_t ks = qkey(sv[k], fg);
                        le &= ks <= kt[k];
                        lt |= ks < kt[k];
                    }
                hit |= __ballot(pass && le && lt);
                if (hit & 1ull) break;
            }
            if (hit & 1ull) break;
        }
        if (hit) {
            result = gh - (__ffsll((unsigned long long)hit) - 1);
            break;
        }
    }
    if (lane == 0) ge_sorted[q] = result;
}

__global__ void __launch_bounds__(kBlock) gres_output_kernel(const int32_t* __restrict__ ge_sorted,
                                                              const uint32_t* __restrict__ order,
                                                              int32_t s, int32_t* __restrict__ g_exit,
                                                              float* __restrict__ gres) {
    int32_t q = blockIdx.x * kBlock + threadIdx.x;
    if (q >= s) return;
    int32_t j = (int32_t)order[q];
    int32_t g = ge_sorted[q];
    if (g_exit) g_exit[j] = g;
    if (gres) gres[j] = __fdiv_rn(1.0f, (float)g);
}

}  // namespace

int64_t gres_pad(int64_t s) { return round_up(s > 0 ? s : 1, kWave * kTileC); }

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

sky_status launch_gres(const float* x, int64_t n, int32_t d, int64_t ld, const int64_t* sky_idx,
                       int64_t s64, int32_t g_max, int32_t mapping, int32_t* g_exit, float* gres,
                       const GresWork& w, int32_t* dev_status, void* ev_begin, void* ev_end,
                       hipStream_t st) {
    if (s64 <= 0) return SKY_OK;
    const int32_t s = (int32_t)s64;
    const int32_t ntile = (int32_t)ceil_div(s, kTileC);
    const uint32_t sblocks = (uint32_t)ceil_div(s, kBlock);
    int bits = 32 / d;
    if (bits > 16) bits = 16;
    if (bits < 1) bits = 1;
    hipLaunchKernelGGL(morton_kernel, dim3(sblocks), dim3(kBlock), 0, st, x, n, d, ld, sky_idx, s,
                       bits, w.k0, w.v0, dev_status);
    SKY_HIP(hipGetLastError());
    SKY_TRY(launch_radix_sort(w.k0, w.v0, w.k1, w.v1, s, bits * d, w.radix_tmp, st));
    hipLaunchKernelGGL(gather_sorted_kernel, dim3(sblocks), dim3(kBlock), 0, st, x, n, d, ld, sky_idx,
                       s, (const uint32_t*)w.v0, w.cand, w.s_pad);
    hipLaunchKernelGGL(tile_lo_kernel, dim3((uint32_t)ceil_div(ntile, kBlock / kWave)), dim3(kBlock),
                       0, st, (const float*)w.cand, w.s_pad, s, d, ntile, w.lo, w.t_pad);
    SKY_HIP(hipGetLastError());
    if (mapping == SKY_GRES_AUTO) mapping = (g_max > 64 && s <= 8192) ? SKY_GRES_LEVELS : SKY_GRES_TILES;
    const uint32_t wblocks = (uint32_t)ceil_div(s, kBlock / kWave);
    if (ev_begin) SKY_HIP(hipEventRecord((hipEvent_t)ev_begin, st));
    if (mapping == SKY_GRES_LEVELS) {
        SKY_DISPATCH_D(d, gres_levels_kernel, dim3(wblocks), dim3(kBlock), 0, st,
                       (const float*)w.cand, w.s_pad, s, d, (const float*)w.lo, w.t_pad, ntile, g_max,
                       w.ge_sorted);
    } else {
        SKY_DISPATCH_D(d, gres_tiles_kernel, dim3(wblocks), dim3(kBlock), 0, st,
                       (const float*)w.cand, w.s_pad, s, d, (const float*)w.lo, w.t_pad, ntile, g_max,
                       w.ge_sorted);
    }
    SKY_HIP(hipGetLastError());
    if (ev_end) SKY_HIP(hipEventRecord((hipEvent_t)ev_end, st));
    hipLaunchKernelGGL(gres_output_kernel, dim3(sblocks), dim3(kBlock), 0, st,
                       (const int32_t*)w.ge_sorted, (const uint32_t*)w.v0, s, g_exit, gres);
    SKY_HIP(hipGetLastError());
    return SKY_OK;
}

}  // namespace sky
