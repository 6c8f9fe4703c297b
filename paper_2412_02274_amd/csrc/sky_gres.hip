// Grid resistance (Def. 2) of the skyline tuples via Alg. 1 in per-tuple form.
//
// For every skyline tuple t the result is g_exit(t) = the largest g in [2, g_max] at which
// the projection of some other skyline tuple s dominates the projection of t (Alg. 1 scans g
// downwards and records the first g at which t leaves the projected skyline), or 1. gres is
// stable (dominated tuples never matter), so the candidates s are the skyline tuples
// themselves. Projections are compared through integer keys K_g(v) = floor(fl32(v * g)).
//
// Exact pruning used by both mappings (no candidate that could dominate is ever skipped):
//  * tile boxes -- candidates are sorted along a Hilbert curve and cut into tiles of 64; lo
//    and hi are the tile's componentwise minimum and maximum. K_g is non-decreasing in v (an
//    FP32 multiply by g > 0 rounded to nearest is monotone, floor too), so
//    K_g(lo) <= K_g(s) <= K_g(hi) for every s of the tile. K_g(s) <= K_g(t) componentwise
//    requires K_g(lo) <= K_g(t): tiles failing that hold no dominator at level g. If
//    K_g(hi) <= K_g(t) everywhere and < somewhere, every s of the tile dominates t at level g
//    (t itself in the tile would force K_g(hi) = K_g(t)), so the level is decided without
//    looking at the candidates.
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
constexpr int kGresBlock = 512;         // threads per workgroup of the TILES mapping
constexpr int kBatch = 4;               // candidate tiles fetched per round trip
constexpr int kGresLdsBytes = 64 * 1024; // tile boxes cached in LDS when they fit

template <int D>
__device__ __forceinline__ int dget(int d) { return D > 0 ? D : d; }

// Hilbert key of every candidate (and checks of the row index and the domain)
__global__ void __launch_bounds__(kBlock) curve_kernel(const float* __restrict__ x, int64_t n,
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
        float v[SKY_MAX_D];
        if (row < 0 || row >= n) {
            bad_idx = true;
            for (int k = 0; k < d; ++k) v[k] = 0.0f;
        } else {
            for (int k = 0; k < d; ++k) {
                float t = x[(int64_t)k * ld + row];
                bad_val |= !in_domain(t);
                v[k] = canon(t);
            }
        }
        keys[j] = hilbert_key(v, d, bits);
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

// one wave per tile: componentwise minimum (lo) and maximum (hi) of its (up to 64) candidates
__global__ void __launch_bounds__(kBlock) tile_box_kernel(const float* __restrict__ cand,
                                                           int64_t s_pad, int32_t s, int32_t d,
                                                           int32_t ntile, float* __restrict__ lo,
                                                           float* __restrict__ hi, int64_t t_pad) {
    int32_t tile = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    if (tile >= ntile) return;
    const int lane = (int)lane_id();
    int32_t j = tile * kTileC + lane;
    for (int k = 0; k < d; ++k) {
        float v = j < s ? cand[(int64_t)k * s_pad + j] : 1.0f;
        float h = j < s ? v : 0.0f;
        for (int off = kWave / 2; off > 0; off >>= 1) {
            v = fminf(v, __shfl_xor(v, off, kWave));
            h = fmaxf(h, __shfl_xor(h, off, kWave));
        }
        if (lane == 0) {
            lo[(int64_t)k * t_pad + tile] = v;
            hi[(int64_t)k * t_pad + tile] = h;
        }
    }
}

// Iterate the set bits of a 64-bit mask starting at bit r (wrapping around).
__device__ __forceinline__ uint64_t rotr64(uint64_t m, int r) {
    return r ? ((m >> r) | (m << (64 - r))) : m;
}

template <int D>
__global__ void __launch_bounds__(kGresBlock) gres_tiles_kernel(const float* __restrict__ cand,
                                                                 int64_t s_pad, int32_t s, int32_t d_rt,
                                                                 const float* __restrict__ lo,
                                                                 const float* __restrict__ hi,
                                                                 int64_t t_pad, int32_t ntile,
                                                                 int32_t g_max, int use_lds,
                                                                 int32_t* __restrict__ ge_sorted) {
    constexpr int DM = D > 0 ? D : SKY_MAX_D;
    extern __shared__ float sbox[];  // [d][ntile] lo, [d][ntile] hi, [d][nchunk] chunk lo, hi
    const int d = dget<D>(d_rt);
    const int lane = (int)lane_id();
    const int wave = threadIdx.x / kWave;
    constexpr int kWaves = kGresBlock / kWave;
    const int32_t nchunk = (ntile + kWave - 1) / kWave;
    float* blo = sbox;
    float* bhi = sbox + (int64_t)d * ntile;
    float* clo = sbox + 2 * (int64_t)d * ntile;
    float* chi = clo + (int64_t)d * nchunk;
    if (use_lds) {
        // tile boxes, then the boxes of chunks of 64 tiles
        for (int32_t e = threadIdx.x; e < d * ntile; e += kGresBlock) {
            const int32_t k = e / ntile, tl = e - k * ntile;
            blo[e] = lo[(int64_t)k * t_pad + tl];
            bhi[e] = hi[(int64_t)k * t_pad + tl];
        }
        __syncthreads();
        for (int32_t e = threadIdx.x; e < d * nchunk; e += kGresBlock) {
            const int32_t k = e / nchunk, c = e - k * nchunk;
            float mn = 1.0f, mx = 0.0f;
            for (int32_t tl = c * kWave; tl < ntile && tl < (c + 1) * kWave; ++tl) {
                mn = fminf(mn, blo[k * ntile + tl]);
                mx = fmaxf(mx, bhi[k * ntile + tl]);
            }
            clo[e] = mn;
            chi[e] = mx;
        }
        __syncthreads();
    }
    for (int32_t q = blockIdx.x * kWaves + wave; q < s; q += gridDim.x * kWaves) {
        float tv[DM];
#pragma unroll
        for (int k = 0; k < DM; ++k)
            if (k < d) tv[k] = cand[(int64_t)k * s_pad + q];
        const int32_t my_tile = q / kTileC;
        const int32_t my_chunk = my_tile / kWave;
        int32_t result = 1;
        for (int32_t g = g_max; g >= 2; --g) {
            const float fg = (float)g;
            int32_t kt[DM];
#pragma unroll
            for (int k = 0; k < DM; ++k)
                if (k < d) kt[k] = qkey(tv[k], fg);
            bool found = false;
            // chunks that may hold a dominator (one ballot over chunk boxes when cached)
            uint64_t cmask;
            if (use_lds) {
                bool cp = lane < nchunk;
#pragma unroll
                for (int k = 0; k < DM; ++k)
                    if (k < d) cp &= cp && qkey(clo[k * nchunk + lane], fg) <= kt[k];
                cmask = rotr64(__ballot(cp), my_chunk);
            } else {
                cmask = nchunk >= 64 ? ~0ull : ((1ull << nchunk) - 1ull);
                cmask = rotr64(cmask, my_chunk % 64);
            }
            for (int32_t cbase = 0; cbase < nchunk && !found; cbase += kWave) {
                uint64_t cm = use_lds ? cmask : (cbase == 0 ? cmask : ~0ull);
                while (cm && !found) {
                    const int cb = __ffsll((unsigned long long)cm) - 1;
                    cm &= cm - 1;
                    // undo the rotation: bit cb of the rotated mask is chunk (cb + start) mod 64
                    const int32_t c = use_lds ? (cb + my_chunk) % kWave
                                              : (cbase == 0 ? (cb + my_chunk % kWave) % kWave : cbase + cb);
                    if (c >= nchunk) continue;
                    const int32_t tile = c * kWave + lane;
                    bool pass = tile < ntile, hle = true, hlt = false;
                    if (pass) {
#pragma unroll
                        for (int k = 0; k < DM; ++k)
                            if (k < d) {
                                const float l = use_lds ? blo[k * ntile + tile] : lo[(int64_t)k * t_pad + tile];
                                const float h = use_lds ? bhi[k * ntile + tile] : hi[(int64_t)k * t_pad + tile];
                                pass &= qkey(l, fg) <= kt[k];
                                const int32_t kh = qkey(h, fg);
                                hle &= kh <= kt[k];
                                hlt |= kh < kt[k];
                            }
                    }
                    // every candidate of a tile whose upper corner's keys dominate t's keys
                    // dominates t (t itself in the tile would force equal keys)
                    if (__ballot(pass && hle && hlt)) { found = true; break; }
                    const int r = c == my_chunk ? my_tile % kWave : 0;
                    uint64_t mask = rotr64(__ballot(pass), r);
                    while (mask) {
                        // up to kBatch passing tiles per round trip: all loads issued together
                        int32_t jb[kBatch];
#pragma unroll
                        for (int b = 0; b < kBatch; ++b) {
                            jb[b] = -1;
                            if (mask) {
                                const int tb = ((__ffsll((unsigned long long)mask) - 1) + r) % kWave;
                                mask &= mask - 1;
                                jb[b] = (c * kWave + tb) * kTileC + lane;
                            }
                        }
                        float sv[kBatch][DM];
#pragma unroll
                        for (int b = 0; b < kBatch; ++b) {
                            const bool ok = jb[b] >= 0 && jb[b] < s && jb[b] != q;
#pragma unroll
                            for (int k = 0; k < DM; ++k)
                                if (k < d) sv[b][k] = ok ? cand[(int64_t)k * s_pad + jb[b]] : 2.0f;
                        }
                        bool dom = false;
#pragma unroll
                        for (int b = 0; b < kBatch; ++b) {
                            bool le = true, lt = false;
#pragma unroll
                            for (int k = 0; k < DM; ++k)
                                if (k < d) {
                                    const int32_t ks = qkey(sv[b][k], fg);
                                    le &= ks <= kt[k];
                                    lt |= ks < kt[k];
                                }
                            dom |= le && lt;
                        }
                        if (__ballot(dom)) { found = true; break; }
                    }
                }
                if (use_lds) break;  // all chunks were covered by the chunk mask
            }
            if (found) { result = g; break; }
        }
        if (lane == 0) ge_sorted[q] = result;
    }
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
                                                              const float* __restrict__ hi,
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
            bool pass = (need >> lane) & 1ull, hle = true, hlt = false;
#pragma unroll
            for (int k = 0; k < DM; ++k)
                if (k < d) {
                    pass &= qkey(lo[(int64_t)k * t_pad + tile], fg) <= kt[k];
                    const int32_t kh = qkey(hi[(int64_t)k * t_pad + tile], fg);
                    hle &= kh <= kt[k];
                    hlt |= kh < kt[k];
                }
            // the whole tile dominates t at this lane's level
            hit |= __ballot(pass && hle && hlt);
            if (hit & 1ull) break;
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
    const int bits = curve_bits(d);
    hipLaunchKernelGGL(curve_kernel, dim3(sblocks), dim3(kBlock), 0, st, x, n, d, ld, sky_idx, s,
                       bits, w.k0, w.v0, dev_status);
    SKY_HIP(hipGetLastError());
    SKY_TRY(launch_radix_sort(w.k0, w.v0, w.k1, w.v1, s, bits * d, w.radix_tmp, st));
    hipLaunchKernelGGL(gather_sorted_kernel, dim3(sblocks), dim3(kBlock), 0, st, x, n, d, ld, sky_idx,
                       s, (const uint32_t*)w.v0, w.cand, w.s_pad);
    hipLaunchKernelGGL(tile_box_kernel, dim3((uint32_t)ceil_div(ntile, kBlock / kWave)), dim3(kBlock),
                       0, st, (const float*)w.cand, w.s_pad, s, d, ntile, w.lo, w.hi, w.t_pad);
    SKY_HIP(hipGetLastError());
    if (mapping == SKY_GRES_AUTO) mapping = (g_max > 64 && s <= 8192) ? SKY_GRES_LEVELS : SKY_GRES_TILES;
    const uint32_t wblocks = (uint32_t)ceil_div(s, kBlock / kWave);
    if (ev_begin) SKY_HIP(hipEventRecord((hipEvent_t)ev_begin, st));
    if (mapping == SKY_GRES_LEVELS) {
        SKY_DISPATCH_D(d, gres_levels_kernel, dim3(wblocks), dim3(kBlock), 0, st,
                       (const float*)w.cand, w.s_pad, s, d, (const float*)w.lo, (const float*)w.hi,
                       w.t_pad, ntile, g_max, w.ge_sorted);
    } else {
        const int32_t nchunk = (int32_t)ceil_div(ntile, kWave);
        const size_t lds = sizeof(float) * 2 * (size_t)d * (size_t)(ntile + nchunk);
        const int use_lds = (lds <= (size_t)kGresLdsBytes && nchunk <= kWave) ? 1 : 0;
        const int64_t want = ceil_div(s, kGresBlock / kWave);
        const uint32_t blocks = (uint32_t)(want < 1024 ? want : 1024);
        SKY_DISPATCH_D(d, gres_tiles_kernel, dim3(blocks), dim3(kGresBlock), use_lds ? lds : 0, st,
                       (const float*)w.cand, w.s_pad, s, d, (const float*)w.lo, (const float*)w.hi,
                       w.t_pad, ntile, g_max, use_lds, w.ge_sorted);
    }
    SKY_HIP(hipGetLastError());
    if (ev_end) SKY_HIP(hipEventRecord((hipEvent_t)ev_end, st));
    hipLaunchKernelGGL(gres_output_kernel, dim3(sblocks), dim3(kBlock), 0, st,
                       (const int32_t*)w.ge_sorted, (const uint32_t*)w.v0, s, g_exit, gres);
    SKY_HIP(hipGetLastError());
    return SKY_OK;
}

}  // namespace sky
