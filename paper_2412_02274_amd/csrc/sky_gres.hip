// Grid resistance (Def. 2) of skyline tuples via Alg. 1 in per-tuple form.
//
// For a tuple t the result is g_exit(t) = the largest g in [2, g_max] at which the projection
// of some candidate s dominates the projection of t (Alg. 1 scans g downwards and records the
// first g at which t leaves the projected skyline), or 1. gres is stable (dominated tuples
// never matter), so the candidates are the skyline tuples. Projections are compared through
// integer keys K_g(v) = floor(fl32(v * g)); in the kernels this is done on the products
// themselves: K_g(v) <= K_g(t) <=> fl(v g) < K_g(t) + 1 and K_g(v) < K_g(t) <=> fl(v g) < K_g(t)
// (K_g(t) and K_g(t) + 1 are small integers, exact in FP32).
//
// Two phases:
//  * prepare -- the candidate set is put in Hilbert-curve order inside each segment (one
//    segment per dataset), stored 64-aligned per segment with padding candidates of value 2.0
//    (their products are >= g, above every key of a value in [0, 1): they never dominate),
//    and cut into tiles of 64 with the componentwise minimum (lo) and maximum (hi) of each.
//  * search -- for each target tuple (all candidates, or any rows of the relation), one
//    wavefront runs the level scan. Exact pruning (no candidate that could dominate is ever
//    skipped, none that cannot is ever counted):
//      - K_g is non-decreasing in v (an FP32 multiply by g > 0 rounded to nearest is monotone,
//        floor too), so K_g(lo) <= K_g(s) <= K_g(hi) for every s of a tile. K_g(s) <= K_g(t)
//        everywhere requires K_g(lo) <= K_g(t): tiles failing that hold no dominator at level
//        g. If K_g(hi) <= K_g(t) everywhere and < somewhere, every s of the tile dominates t
//        (t itself in the tile would force K_g(hi) = K_g(t)), and the level is decided at once.
//      - the same test on the minimum over 64 consecutive tiles (a chunk) skips whole chunks.
//      - LEVELS mapping only: if s_k > t_k, K_g(s_k) <= K_g(t_k) needs fl(s_k g) - fl(t_k g) < 1,
//        and FP32 rounding (relative error <= 2^-24 below g) turns this into
//        g (s_k - t_k - 2^-23) < 1; with delta = max_k (s_k - t_k), or the same from a tile's
//        lo (a lower bound for every member), no level g with g (delta - 2^-23) >= 1 can see
//        s dominate t. Evaluated in double with a 1e-9 margin.
//
// Mappings (both one wavefront per target, wave-uniform control flow, first dominator ends
// the level):
//  * TILES  -- levels g_max..2; per level the 64 lanes test 64 chunk boxes, then 64 tile
//    boxes per chunk (cached in LDS when they fit), then up to 4 passing tiles of 64
//    candidates per memory round trip, starting near the target's own place on the curve.
//    Best when S is large and g_max small.
//  * LEVELS -- lanes hold 64 consecutive levels; candidates are read as wave-uniform values
//    and each lane tests its own level; the highest level with a dominator in the block of
//    64 levels ends the search. Best when S is small and g_max large.
// Bound: VALU compare/multiply throughput and L2 latency (a candidate set is at most a few MB
// and stays in L2).
#include "sky_internal.hpp"

namespace sky {

namespace {

constexpr int kTileC = 64;               // candidates per tile
constexpr int kGresBlock = 512;          // threads per workgroup of the search kernels
constexpr int kWaves = kGresBlock / kWave;
constexpr int kBatch = 4;                // candidate tiles fetched per round trip (measured best)
constexpr int kChunkBatch = 4;           // chunks' tile boxes fetched per round trip (packed keys)
constexpr int kGresLdsBytes = 64 * 1024; // tile boxes cached in LDS when they fit
constexpr float kPadValue = 2.0f;
constexpr int kBandLevels = 6;           // levels per band of the TILES search
constexpr int kMaxBands = 8;
constexpr int kStartLevels = 64;         // above this g_max, searches start at per-target bounds
constexpr int kLevelWaves = 4096;        // LEVELS: waves wanted in flight (targets x bands)
constexpr int kMaxLevelBands = 16;
constexpr int kGresLdsDevBytes = 40 * 1024;  // box LDS of searches whose count is on the device
constexpr int kStrideGrid = 4096;       // workgroups of searches whose count is on the device

template <int D>
__device__ __forceinline__ int dget(int d) { return D > 0 ? D : d; }

// f32 load base[idx] with a 32-bit byte offset from a wave-uniform base
__device__ __forceinline__ float ldf(const float* base, uint32_t idx) {
    return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + (idx << 2));
}

// Iterate the set bits of a 64-bit mask starting at bit r (wrapping around).
__device__ __forceinline__ uint64_t rotr64(uint64_t m, int r) {
    return r ? ((m >> r) | (m << (64 - r))) : m;
}

// ---------------------------------------------------------------------------------- prepare

// Hilbert key of every candidate (and checks of the row index and the domain)
__global__ void __launch_bounds__(kBlock) curve_kernel(const float* __restrict__ x, int64_t n,
                                                        int32_t d, int64_t ld,
                                                        const int64_t* __restrict__ rows,
                                                        int32_t s, int bits,
                                                        uint32_t* __restrict__ keys,
                                                        uint32_t* __restrict__ vals,
                                                        int32_t* dev_status) {
    int32_t j = blockIdx.x * kBlock + threadIdx.x;
    bool bad_idx = false, bad_val = false;
    if (j < s) {
        int64_t row = rows[j];
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

// every slot of the store: candidate values, curve key and caller index (padding: 2.0, ~0, -1)
__global__ void __launch_bounds__(kBlock) store_kernel(const float* __restrict__ x, int64_t n,
                                                        int32_t d, int64_t ld,
                                                        const int64_t* __restrict__ rows, int32_t s,
                                                        const uint32_t* __restrict__ skeys,
                                                        const uint32_t* __restrict__ order,
                                                        float* __restrict__ cand, int64_t ccap,
                                                        uint32_t* __restrict__ ckey,
                                                        int32_t* __restrict__ perm) {
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= ccap) return;
    const bool real = q < s;
    const int32_t j = real ? (int32_t)order[q] : -1;
    const int64_t row = real ? rows[j] : -1;
    const bool ok = real && row >= 0 && row < n;
    for (int k = 0; k < d; ++k)
        cand[(int64_t)k * ccap + q] = ok ? canon(x[(int64_t)k * ld + row]) : (real ? 0.0f : kPadValue);
    ckey[q] = real ? skeys[q] : 0xFFFFFFFFu;
    perm[q] = j;
}

// the store from a plan's partition-contiguous copy: the candidates are the rows at positions
// pos[0, s), already in curve order (the copy is), so no sort is needed; the caller index of a
// slot is idx_of_row[row]. s = min(*s_dev, cap) when s_dev is given. Slots from s to the end of
// its tile, and the store's last tile, get padding (2.0, ~0, -1); slots beyond are never read.
// With tval given, every candidate is also a target: its values, its own tile as the hint, its
// caller index, and no exit yet (ge = 1). With seg_coff given, the store's one segment is
// recorded (s candidates from slot 0; a device count above s_host raises SKY_ERR_CAPACITY).
__global__ void __launch_bounds__(kBlock) store_pos_kernel(const float* __restrict__ xp, int64_t ldp,
                                                            int32_t d, const int32_t* __restrict__ pos,
                                                            int32_t s_host, const int32_t* __restrict__ s_dev,
                                                            const int32_t* __restrict__ rowid,
                                                            const int32_t* __restrict__ idx_of_row,
                                                            float* __restrict__ cand, int64_t ccap,
                                                            uint32_t* __restrict__ ckey,
                                                            int32_t* __restrict__ perm, float* __restrict__ tval,
                                                            int64_t tvcap, int32_t* __restrict__ thint,
                                                            int32_t* __restrict__ tout, int32_t* __restrict__ ge,
                                                            int32_t* __restrict__ seg_coff,
                                                            int32_t* __restrict__ seg_cnt, int32_t* dev_status,
                                                            float* __restrict__ lo, float* __restrict__ hi,
                                                            int64_t tcap) {
    int32_t s = s_host;
    if (s_dev) s = *s_dev < s_host ? *s_dev : s_host;
    if (seg_coff && blockIdx.x == 0 && threadIdx.x == 0) {  // the store's one segment
        if (s_dev && *s_dev > s_host) raise_status(dev_status, SKY_ERR_CAPACITY);
        seg_coff[0] = 0;
        seg_cnt[0] = s;
    }
    // one wave per tile (lane = slot): the tiles holding candidates, then the store's last tile
    // [ccap - 64, ccap); each candidate tile's box (componentwise minimum and maximum of its real
    // candidates) as tile_box_kernel takes it
    const int64_t ntl = ((int64_t)s + kTileC - 1) / kTileC;
    const int lane = (int)lane_id();
    const int64_t nwaves = (int64_t)gridDim.x * (kBlock / kWave);
    for (int64_t t = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; t <= ntl; t += nwaves) {
        const int64_t q = t < ntl ? t * kTileC + lane : ccap - kTileC + lane;
        const bool real = q < s;
        const int32_t p = real ? pos[q] : 0;
        float v[SKY_MAX_D];
        for (int k = 0; k < d; ++k) {
            v[k] = real ? xp[(int64_t)k * ldp + p] : kPadValue;
            cand[(int64_t)k * ccap + q] = v[k];
        }
        ckey[q] = real ? hilbert_key(v, d, curve_bits(d)) : 0xFFFFFFFFu;
        const int32_t pm = real ? idx_of_row[rowid[p]] : -1;
        perm[q] = pm;
        if (tval && real) {
            for (int k = 0; k < d; ++k) tval[(int64_t)k * tvcap + q] = v[k];
            thint[q] = (int32_t)(q / kTileC);
            tout[q] = pm;
            ge[q] = 1;
        }
        if (t < ntl)  // (uniform per wave)
            for (int k = 0; k < d; ++k) {
                float mn = real ? v[k] : 1.0f, mx = real ? v[k] : 0.0f;
                for (int off = kWave / 2; off > 0; off >>= 1) {
                    mn = fminf(mn, __shfl_xor(mn, off, kWave));
                    mx = fmaxf(mx, __shfl_xor(mx, off, kWave));
                }
                if (lane == 0) {
                    lo[(int64_t)k * tcap + t] = mn;
                    hi[(int64_t)k * tcap + t] = mx;
                }
            }
    }
}

// one wave per tile: componentwise minimum (lo) and maximum (hi) of its real candidates (padding
// slots hold kPadValue in every attribute; a tile of padding only gets lo = 1, which no key test
// passes: fl(1 g) = g is above every key of a value in [0, 1))
__global__ void __launch_bounds__(kBlock) tile_box_kernel(const float* __restrict__ cand, int64_t ccap,
                                                           int32_t d, int32_t ntile_host,
                                                           const int32_t* __restrict__ s_dev, int32_t s_cap,
                                                           float* __restrict__ lo,
                                                           float* __restrict__ hi, int64_t tcap) {
    int32_t ntile = ntile_host;
    if (s_dev) ntile = ((*s_dev < s_cap ? *s_dev : s_cap) + kTileC - 1) / kTileC;
    const int lane = (int)lane_id();
    for (int32_t tile = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; tile < ntile;
         tile += gridDim.x * (kBlock / kWave)) {
        const int64_t j = (int64_t)tile * kTileC + lane;
        const bool real = cand[j] < kPadValue;
        for (int k = 0; k < d; ++k) {
            const float c = cand[(int64_t)k * ccap + j];
            float v = real ? c : 1.0f;
            float h = real ? c : 0.0f;
            for (int off = kWave / 2; off > 0; off >>= 1) {
                v = fminf(v, __shfl_xor(v, off, kWave));
                h = fmaxf(h, __shfl_xor(h, off, kWave));
            }
            if (lane == 0) {
                lo[(int64_t)k * tcap + tile] = v;
                hi[(int64_t)k * tcap + tile] = h;
            }
        }
    }
}

// Packed keys at every level g in [2, levels + 1]: attribute k's key floor(fl32(v g)) at bit
// k * w of one 64-bit word. Keys are clamped to the field's largest value 2^(w-1) - 1, which
// only the padding value 2.0 reaches (a value in [0, 1) has keys of at most g <= 2^(w-1) - 2),
// so padding never dominates a target.
template <int D>
__device__ __forceinline__ uint64_t pack_keys(const float* v, int d, float fg, int w, uint32_t kmax) {
    constexpr int DM = D > 0 ? D : SKY_MAX_D;
    uint64_t kv = 0;
#pragma unroll
    for (int k = 0; k < DM; ++k)
        if (k < d) {
            uint32_t q = (uint32_t)floorf(__fmul_rn(v[k], fg));
            q = q < kmax ? q : kmax;
            kv |= (uint64_t)q << (k * w);
        }
    return kv;
}

// The key tables of a store, every level, when its slots in use (used[0], or the first
// segment's tiles when used is null) fit them (*ok, written by workgroup 0; nothing else is
// written otherwise):
//  * blocks [0, cblocks): candidate slots [0, used) from the store, and the padding tile
//    [kslots - 64, kslots) (the clamp value in every field), key[(g - 2) * kslots + slot];
//  * blocks [cblocks, cblocks + tblocks): one thread per tile in use, its packed box corners,
//    tile[(g - 2) * ktiles + tile];
//  * the other blocks: for each chunk of 64 tiles from a segment's first tile, the packed
//    minimum of their lower corners at chunk[(g - 2) * ktiles + first tile] (one wave per chunk
//    of a single segment, one wave per segment of many).
template <int D>
__global__ void __launch_bounds__(kBlock) level_keys_kernel(
    const float* __restrict__ cand, int64_t ccap, const float* __restrict__ lo, const float* __restrict__ hi,
    int64_t tcap, int32_t d_rt, const int32_t* __restrict__ seg_coff, const int32_t* __restrict__ seg_cnt,
    int32_t nseg, const int32_t* __restrict__ used_dev, int32_t levels, int32_t w, int32_t cblocks,
    int32_t tblocks, uint64_t* __restrict__ key, int64_t kslots, uint4* __restrict__ tile,
    uint64_t* __restrict__ chunk, int64_t ktiles, int32_t* __restrict__ ok) {
    constexpr int DM = D > 0 ? D : SKY_MAX_D;
    const int d = dget<D>(d_rt);
    const uint32_t kmax = (1u << (w - 1)) - 1u;
    const int64_t used = used_dev ? (int64_t)used_dev[0] : (int64_t)(seg_cnt[0] + kTileC - 1) / kTileC * kTileC;
    const int64_t ntl = used / kTileC;  // tiles in use
    const bool fits = used + kTileC <= kslots && ntl <= ktiles;
    if (blockIdx.x == 0 && threadIdx.x == 0) *ok = fits ? 1 : 0;
    if (!fits) return;
    const int32_t b = (int32_t)blockIdx.x;
    if (b < cblocks) {
        for (int64_t i = (int64_t)b * kBlock + threadIdx.x; i < used + kTileC; i += (int64_t)cblocks * kBlock) {
            if (i >= used) {  // padding: above every key of a target
                uint64_t pad = 0;
                for (int k = 0; k < d; ++k) pad |= (uint64_t)kmax << (k * w);
                for (int32_t l = 0; l < levels; ++l) key[(int64_t)l * kslots + kslots - kTileC + (i - used)] = pad;
                continue;
            }
            float v[DM];
#pragma unroll
            for (int k = 0; k < DM; ++k)
                if (k < d) v[k] = cand[(int64_t)k * ccap + i];
            for (int32_t l = 0; l < levels; ++l)
                key[(int64_t)l * kslots + i] = pack_keys<D>(v, d, (float)(l + 2), w, kmax);
        }
        return;
    }
    if (b < cblocks + tblocks) {
        for (int64_t t = (int64_t)(b - cblocks) * kBlock + threadIdx.x; t < ntl; t += (int64_t)tblocks * kBlock) {
            float vl[DM], vh[DM];
#pragma unroll
            for (int k = 0; k < DM; ++k)
                if (k < d) {
                    vl[k] = lo[(int64_t)k * tcap + t];
                    vh[k] = hi[(int64_t)k * tcap + t];
                }
            for (int32_t l = 0; l < levels; ++l) {
                const float fg = (float)(l + 2);
                const uint64_t a = pack_keys<D>(vl, d, fg, w, kmax), h = pack_keys<D>(vh, d, fg, w, kmax);
                tile[(int64_t)l * ktiles + t] = make_uint4((uint32_t)a, (uint32_t)(a >> 32), (uint32_t)h,
                                                           (uint32_t)(h >> 32));
            }
        }
        return;
    }
    const int lane = (int)lane_id();
    const int32_t wpb = kBlock / kWave;
    const int32_t nwaves = ((int32_t)gridDim.x - cblocks - tblocks) * wpb;
    const int32_t w0 = (b - cblocks - tblocks) * wpb + (int32_t)(threadIdx.x / kWave);
    // the chunk of tiles [t0 + c0, t0 + c0 + 64) of a segment of nts tiles
    auto do_chunk = [&](int32_t t0, int32_t nts, int32_t c0) {
        const bool real = c0 + lane < nts;
        float vl[DM];
#pragma unroll
        for (int k = 0; k < DM; ++k)
            if (k < d) {
                vl[k] = real ? lo[(int64_t)k * tcap + t0 + c0 + lane] : kPadValue;
                for (int off = kWave / 2; off > 0; off >>= 1) vl[k] = fminf(vl[k], __shfl_xor(vl[k], off, kWave));
            }
        if (lane < levels) chunk[(int64_t)lane * ktiles + t0 + c0] = pack_keys<D>(vl, d, (float)(lane + 2), w, kmax);
    };
    if (nseg == 1) {  // one wave per chunk
        const int32_t nts = (seg_cnt[0] + kTileC - 1) / kTileC;
        for (int32_t c = w0; c * kWave < nts; c += nwaves) do_chunk(seg_coff[0] / kTileC, nts, c * kWave);
        return;
    }
    for (int32_t sg = w0; sg < nseg; sg += nwaves) {  // one wave per segment
        const int32_t t0 = seg_coff[sg] / kTileC;
        const int32_t nts = (seg_cnt[sg] + kTileC - 1) / kTileC;
        for (int32_t c0 = 0; c0 < nts; c0 += kWave) do_chunk(t0, nts, c0);
    }
}

// largest j in [0, cnt) with off[j] <= q (off non-decreasing; empty segments share their offset
// with the next one, so the search lands on the segment that holds q)
__device__ __forceinline__ int32_t find_seg(const int32_t* __restrict__ off, int32_t cnt, int64_t q) {
    int32_t lo = 0, hi = cnt - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (off[mid] <= q) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// segment of every element in the curve order (key of the stable second sort)
__global__ void __launch_bounds__(kBlock) seg_key_kernel(const uint32_t* __restrict__ order, int32_t s,
                                                          const int32_t* __restrict__ cand_off,
                                                          int32_t nseg, uint32_t* __restrict__ keys) {
    const int32_t q = blockIdx.x * kBlock + threadIdx.x;
    if (q < s) keys[q] = (uint32_t)find_seg(cand_off, nseg, (int64_t)order[q]);
}

// every slot of a segmented store: slot q of segment sg holds the (q - coff)-th element of the
// segment in curve order, or padding past the segment's count
__global__ void __launch_bounds__(kBlock) store_seg_kernel(
    const float* __restrict__ x, int64_t n, int32_t d, int64_t ld, const int64_t* __restrict__ rows,
    const uint32_t* __restrict__ order, const int32_t* __restrict__ cand_off,
    const int32_t* __restrict__ seg_coff, const int32_t* __restrict__ seg_cnt, int32_t nseg, int bits,
    float* __restrict__ cand, int64_t ccap, uint32_t* __restrict__ ckey, int32_t* __restrict__ perm) {
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= ccap) return;
    const int32_t sg = find_seg(seg_coff, nseg, q);
    const int64_t r = q - seg_coff[sg];
    const bool real = r >= 0 && r < seg_cnt[sg];
    const int32_t j = real ? (int32_t)order[cand_off[sg] + r] : -1;
    const int64_t row = real ? rows[j] : -1;
    const bool ok = real && row >= 0 && row < n;
    float v[SKY_MAX_D];
    for (int k = 0; k < d; ++k) {
        v[k] = ok ? canon(x[(int64_t)k * ld + row]) : (real ? 0.0f : kPadValue);
        cand[(int64_t)k * ccap + q] = v[k];
    }
    ckey[q] = real ? hilbert_key(v, d, bits) : 0xFFFFFFFFu;
    perm[q] = j;
}

// one segment of s candidates; with s_dev, s = min(*s_dev, s), and a larger count raises
// SKY_ERR_CAPACITY (the store was carved for s)
__global__ void single_segment_kernel(int32_t* __restrict__ seg_coff, int32_t* __restrict__ seg_cnt,
                                      int32_t s, const int32_t* __restrict__ s_dev, int32_t* dev_status) {
    if (threadIdx.x == 0) {
        int32_t c = s;
        if (s_dev) {
            if (*s_dev > s) raise_status(dev_status, SKY_ERR_CAPACITY);
            else c = *s_dev;
        }
        seg_coff[0] = 0;
        seg_cnt[0] = c;
    }
}

// ---------------------------------------------------------------------------------- targets

// targets = every candidate of the store (slot order): values, hint tile, output index
__global__ void __launch_bounds__(kBlock) targets_all_kernel(const float* __restrict__ cand, int64_t ccap,
                                                              int32_t s_host, const int32_t* __restrict__ s_dev,
                                                              int32_t d, const int32_t* __restrict__ perm,
                                                              float* __restrict__ tval, int64_t tvcap,
                                                              int32_t* __restrict__ thint,
                                                              int32_t* __restrict__ tout) {
    int32_t s = s_host;
    if (s_dev) s = *s_dev < s_host ? *s_dev : s_host;
    for (int32_t q = blockIdx.x * kBlock + threadIdx.x; q < s; q += gridDim.x * kBlock) {
        for (int k = 0; k < d; ++k) tval[(int64_t)k * tvcap + q] = cand[(int64_t)k * ccap + q];
        thint[q] = q / kTileC;
        tout[q] = perm[q];
    }
}

// targets = every candidate of a segmented store in element order: element q of segment sg
// sits at slot seg_coff[sg] + (q - cand_off[sg]); tseg[q] = sg. The count is cand_off[nseg].
__global__ void __launch_bounds__(kBlock) targets_seg_kernel(
    const float* __restrict__ cand, int64_t ccap, int32_t d,
    const int32_t* __restrict__ cand_off, const int32_t* __restrict__ seg_coff, int32_t nseg,
    const int32_t* __restrict__ perm, int32_t near_first, float* __restrict__ tval, int64_t tvcap,
    int32_t* __restrict__ thint, int32_t* __restrict__ tout, int32_t* __restrict__ tseg) {
    const int32_t s = cand_off[nseg];
    for (int32_t q = blockIdx.x * kBlock + threadIdx.x; q < s; q += gridDim.x * kBlock) {
        const int32_t sg = find_seg(cand_off, nseg, q);
        const int32_t r = q - cand_off[sg];
        const int64_t slot = (int64_t)seg_coff[sg] + r;
        for (int k = 0; k < d; ++k) tval[(int64_t)k * tvcap + q] = cand[(int64_t)k * ccap + slot];
        thint[q] = near_first ? r / kTileC : 0;
        tout[q] = perm[slot];
        tseg[q] = sg;
    }
}

__global__ void __launch_bounds__(kBlock) fill_i32_kernel(int32_t* __restrict__ p, int32_t n, int32_t v) {
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = v;
}

// ------------------------------------------------------------- search shape on the device
// The targets of a search whose count is on the device: its shape, as the host would pick it
// for that count (params[P_*]).
enum { P_NT = 0, P_MAPPING, P_PER_WG, P_BLOCKS, P_LBANDS };

__host__ __device__ inline void search_shape(int32_t nt, int32_t g_max, int32_t* per_wg, int32_t* blocks,
                                             int32_t* lbands) {
    // ~2 targets per wave when there are plenty (measured best on large skylines: fewer leaves
    // waves idle on the longest searches), fewer otherwise
    int64_t want = ((int64_t)nt + kWaves * 2 - 1) / (kWaves * 2);
    if (want < 256) want = ((int64_t)nt + kWaves - 1) / kWaves;
    int32_t b = (int32_t)(want < 1 ? 1 : want);
    const int32_t pw = nt > 0 ? (nt + b - 1) / b : 1;
    *per_wg = pw;
    *blocks = nt > 0 ? (nt + pw - 1) / pw : 0;
    // LEVELS with few targets: each target's levels split over several waves so the chip fills
    int64_t lb = nt > 0 && nt < kLevelWaves ? ((int64_t)kLevelWaves + nt - 1) / nt : 1;
    const int64_t lmax = ((int64_t)g_max - 1 + kWave - 1) / kWave;  // at least 64 levels per band
    lb = lb > lmax ? lmax : lb;
    lb = lb > kMaxLevelBands ? kMaxLevelBands : (lb < 1 ? 1 : lb);
    *lbands = (int32_t)lb;
}

__global__ void search_setup_kernel(const int32_t* __restrict__ nt_dev, int32_t nt_cap, int32_t g_max,
                                    int32_t mapping, int32_t* __restrict__ params, int32_t* __restrict__ work) {
    if (work)  // the work counters of the persistent search, cleared
        for (int i = threadIdx.x; i < kWorkCounters * kCounterStride; i += blockDim.x) work[i] = 0;
    if (threadIdx.x != 0) return;
    const int32_t nt = *nt_dev < nt_cap ? *nt_dev : nt_cap;
    int32_t per_wg, blocks, lb;
    search_shape(nt, g_max, &per_wg, &blocks, &lb);
    params[P_NT] = nt;
    params[P_MAPPING] = mapping == SKY_GRES_AUTO ? gres_auto_mapping(nt, g_max) : mapping;
    params[P_PER_WG] = per_wg;
    params[P_BLOCKS] = blocks;
    params[P_LBANDS] = lb;
}

// p[0, n) = v, n = params[P_NT] when params is given (grid-stride)
__global__ void __launch_bounds__(kBlock) fill_targets_kernel(int32_t* __restrict__ p, int32_t n,
                                                               const int32_t* __restrict__ params, int32_t v) {
    if (params) n = params[P_NT];
    for (int32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) p[i] = v;
}

// first position of every relation's rows in the ascending skyline list sky_idx[0, *count)
// (lower bound of its first row), as int64 offsets for the caller and int32 element offsets
// for the store
__global__ void __launch_bounds__(kBlock) batch_offsets_kernel(const int64_t* __restrict__ sky_idx,
                                                                const int32_t* __restrict__ count_dev,
                                                                int32_t cap,
                                                                const int64_t* __restrict__ row_off,
                                                                int32_t nseg, int64_t* __restrict__ sky_off,
                                                                int32_t* __restrict__ cand_off) {
    const int32_t j = blockIdx.x * kBlock + threadIdx.x;
    if (j > nseg) return;
    const int32_t count = *count_dev < cap ? *count_dev : cap;
    int32_t lo = 0, hi = count;
    if (j == nseg) {
        lo = count;
    } else {
        const int64_t key = row_off[j];
        while (lo < hi) {
            const int32_t mid = (lo + hi) >> 1;
            if (sky_idx[mid] < key) lo = mid + 1; else hi = mid;
        }
    }
    sky_off[j] = lo;
    cand_off[j] = lo;
}

// ------------------------------------------------------------------ batched store and order
// Layout of a batch's candidate store, one workgroup: relation j holds cnt_j = cand_off[j+1] -
// cand_off[j] candidates from slot seg_coff[j] (64-aligned); used[0] = the slots in use,
// used[1] = the largest cnt_j.
__global__ void __launch_bounds__(1024) batch_layout_kernel(const int32_t* __restrict__ cand_off, int32_t nseg,
                                                             int32_t* __restrict__ seg_coff,
                                                             int32_t* __restrict__ seg_cnt,
                                                             int32_t* __restrict__ used) {
    __shared__ int32_t wsum[1024 / kWave], wmax[1024 / kWave];
    __shared__ int32_t carry, mx_all;
    const int lane = (int)lane_id(), wave = threadIdx.x / kWave;
    if (threadIdx.x == 0) { carry = 0; mx_all = 0; }
    __syncthreads();
    for (int32_t base = 0; base < nseg; base += 1024) {
        const int32_t j = base + threadIdx.x;
        const int32_t c = j < nseg ? cand_off[j + 1] - cand_off[j] : 0;
        const int32_t v = (c + kTileC - 1) / kTileC * kTileC;
        int32_t inc = v, m = c;
        for (int off = 1; off < kWave; off <<= 1) {
            const int32_t o = __shfl_up(inc, off, kWave);
            if (lane >= off) inc += o;
        }
        for (int off = kWave / 2; off > 0; off >>= 1) {
            const int32_t o = __shfl_xor(m, off, kWave);
            m = o > m ? o : m;
        }
        if (lane == kWave - 1) wsum[wave] = inc;
        if (lane == 0) wmax[wave] = m;
        __syncthreads();
        int32_t before = carry;
        for (int w = 0; w < wave; ++w) before += wsum[w];
        if (j < nseg) {
            seg_coff[j] = before + inc - v;
            seg_cnt[j] = c;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 0; w < 1024 / kWave; ++w) {
                carry += wsum[w];
                mx_all = wmax[w] > mx_all ? wmax[w] : mx_all;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        used[0] = carry;
        used[1] = mx_all;
    }
}

// The search's shape for all S = cand_off[nseg] targets of a batch (as search_setup_kernel
// gives it; AUTO judged by the largest relation's count, used[1]).
__global__ void batch_params_kernel(const int32_t* __restrict__ cand_off, int32_t nseg,
                                    const int32_t* __restrict__ used, int32_t g_max, int32_t mapping,
                                    int32_t* __restrict__ params) {
    if (threadIdx.x != 0) return;
    const int32_t nt = cand_off[nseg];
    int32_t per_wg, blocks, lb;
    search_shape(nt, g_max, &per_wg, &blocks, &lb);
    params[P_NT] = nt;
    params[P_MAPPING] = mapping == SKY_GRES_AUTO ? gres_auto_mapping(used[1], g_max) : mapping;
    params[P_PER_WG] = per_wg;
    params[P_BLOCKS] = blocks;
    params[P_LBANDS] = lb;
}

// Longest-first order of the relations: rank_of = the number of relations with more candidates
// (equal counts in relation order); order[rank] = relation. Every workgroup holds all counts.
__global__ void __launch_bounds__(kBlock) batch_rank_kernel(const int32_t* __restrict__ seg_cnt, int32_t nseg,
                                                             int32_t* __restrict__ order) {
    __shared__ int32_t c[SKY_MAX_CELLS];
    for (int32_t i = threadIdx.x; i < nseg; i += kBlock) c[i] = seg_cnt[i];
    __syncthreads();
    const int32_t j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= nseg) return;
    const int32_t cj = c[j];
    int32_t rank = 0;
    for (int32_t i = 0; i < nseg; ++i) rank += (c[i] > cj) || (c[i] == cj && i < j);
    order[rank] = j;
}

// rank_off[i] = targets of the relations ranked before i (one workgroup)
__global__ void __launch_bounds__(1024) batch_rank_scan_kernel(const int32_t* __restrict__ seg_cnt,
                                                                const int32_t* __restrict__ order, int32_t nseg,
                                                                int32_t* __restrict__ rank_off) {
    __shared__ int32_t wsum[1024 / kWave];
    __shared__ int32_t carry;
    const int lane = (int)lane_id(), wave = threadIdx.x / kWave;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int32_t base = 0; base < nseg; base += 1024) {
        const int32_t i = base + threadIdx.x;
        const int32_t v = i < nseg ? seg_cnt[order[i]] : 0;
        int32_t inc = v;
        for (int off = 1; off < kWave; off <<= 1) {
            const int32_t o = __shfl_up(inc, off, kWave);
            if (lane >= off) inc += o;
        }
        if (lane == kWave - 1) wsum[wave] = inc;
        __syncthreads();
        int32_t before = carry;
        for (int w = 0; w < wave; ++w) before += wsum[w];
        if (i < nseg) rank_off[i] = before + inc - v;
        __syncthreads();
        if (threadIdx.x == 0)
            for (int w = 0; w < 1024 / kWave; ++w) carry += wsum[w];
        __syncthreads();
    }
    if (threadIdx.x == 0) rank_off[nseg] = carry;
}

// tord: the targets in longest-first relation order, one workgroup per relation rank
__global__ void __launch_bounds__(kBlock) batch_tord_kernel(const int32_t* __restrict__ order,
                                                             const int32_t* __restrict__ rank_off,
                                                             const int32_t* __restrict__ cand_off,
                                                             int32_t nseg, int32_t* __restrict__ tord) {
    for (int32_t i = blockIdx.x; i < nseg; i += gridDim.x) {
        const int32_t j = order[i];
        const int32_t a = rank_off[i], c = rank_off[i + 1] - a, e = cand_off[j];
        for (int32_t r = threadIdx.x; r < c; r += kBlock) tord[a + r] = e + r;
    }
}

// The slots of a batch's store from the plan's partition-contiguous copy: slot r of relation j
// holds element cand_off[j] + r of the skyline's positions list (relation-major, curve order
// inside each relation, as the copy is); slots past a relation's count, and the store's last
// tile, hold padding. perm = the row's index in the ascending skyline list (idx_of_row).
__global__ void __launch_bounds__(kBlock) store_seg_pos_kernel(
    const float* __restrict__ xp, int64_t ldp, int32_t d, const int32_t* __restrict__ pos,
    const int32_t* __restrict__ cand_off, const int32_t* __restrict__ seg_coff,
    const int32_t* __restrict__ seg_cnt, int32_t nseg, const int32_t* __restrict__ used,
    const int32_t* __restrict__ rowid, const int32_t* __restrict__ idx_of_row, float* __restrict__ cand,
    int64_t ccap, uint32_t* __restrict__ ckey, int32_t* __restrict__ perm) {
    const int64_t u = used[0];
    const int64_t lim = u + kTileC;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < lim; i += (int64_t)gridDim.x * kBlock) {
        const int64_t q = i < u ? i : ccap - kTileC + (i - u);
        bool real = false;
        int32_t p = 0;
        if (i < u) {
            const int32_t sg = find_seg(seg_coff, nseg, q);
            const int64_t r = q - seg_coff[sg];
            real = r < seg_cnt[sg];
            if (real) p = pos[cand_off[sg] + r];
        }
        float v[SKY_MAX_D];
        for (int k = 0; k < d; ++k) {
            v[k] = real ? xp[(int64_t)k * ldp + p] : kPadValue;
            cand[(int64_t)k * ccap + q] = v[k];
        }
        ckey[q] = real ? hilbert_key(v, d, curve_bits(d)) : 0xFFFFFFFFu;
        perm[q] = real ? idx_of_row[rowid[p]] : -1;
    }
}

// targets = given rows of the relation: values, hint tile (where the row's curve key falls
// among the sorted candidate keys), output index = position in the target list
__global__ void __launch_bounds__(kBlock) targets_rows_kernel(const float* __restrict__ x, int64_t n,
                                                               int32_t d, int64_t ld,
                                                               const int64_t* __restrict__ rows,
                                                               int32_t nt, int bits,
                                                               const uint32_t* __restrict__ ckey,
                                                               int32_t s,
                                                               float* __restrict__ tval, int64_t tvcap,
                                                               int32_t* __restrict__ thint,
                                                               int32_t* __restrict__ tout,
                                                               int32_t* dev_status) {
    const int32_t q = blockIdx.x * kBlock + threadIdx.x;
    bool bad_idx = false, bad_val = false;
    if (q < nt) {
        const int64_t row = rows[q];
        float v[SKY_MAX_D];
        if (row < 0 || row >= n) {
            bad_idx = true;
            for (int k = 0; k < d; ++k) v[k] = kPadValue;  // never dominated (keys >= g)
        } else {
            for (int k = 0; k < d; ++k) {
                float t = x[(int64_t)k * ld + row];
                bad_val |= !in_domain(t);
                v[k] = canon(t);
            }
        }
        for (int k = 0; k < d; ++k) tval[(int64_t)k * tvcap + q] = v[k];
        const uint32_t key = bad_idx ? 0u : hilbert_key(v, d, bits);
        int32_t lo = 0, hi = s;  // first slot with key >= the target's key
        while (lo < hi) {
            const int32_t mid = (lo + hi) >> 1;
            if (ckey[mid] < key) lo = mid + 1; else hi = mid;
        }
        const int32_t slot = lo < s ? lo : (s > 0 ? s - 1 : 0);
        thint[q] = slot / kTileC;
        tout[q] = q;
    }
    if (__ballot(bad_idx) && lane_id() == 0) raise_status(dev_status, SKY_ERR_INVALID_ARG);
    if (__ballot(bad_val) && lane_id() == 0) raise_status(dev_status, SKY_ERR_DOMAIN);
}

// ----------------------------------------------------------------------------------- search

// Work of one workgroup of a one-segment search: targets [blk * per_wg, ...) of segment 0.
struct WgWork { int32_t seg, t0, t1; };

__device__ __forceinline__ WgWork wg_work(int32_t per_wg, int32_t nt, int32_t blk) {
    WgWork w;
    w.seg = 0;
    w.t0 = blk * per_wg;
    w.t1 = w.t0 + per_wg < nt ? w.t0 + per_wg : nt;
    return w;
}

// The candidate tests of a workgroup of the search kernels, added to *dev_tests with one atomic
// (every wave's count summed through LDS: thousands of waves adding to one address at the end
// of a launch would queue behind each other). Every wave of the workgroup calls it.
__device__ __forceinline__ void add_block_tests(unsigned long long* dev_tests, unsigned long long ntests) {
    __shared__ unsigned long long wred[kWaves];
    if (!dev_tests) return;
    if (lane_id() == 0) wred[threadIdx.x / kWave] = ntests;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < kWaves; ++w) t += wred[w];
        if (t) atomicAdd(dev_tests, t);
    }
}

template <int D>
// 8 waves per SIMD: the search waits on cache round trips, so more waves in flight pay.
// Three ways to hand out the work, (target, band) pairs in band-major order (every target's
// highest band first):
//  * work == nullptr (one segment, few targets): workgroup b searches band b / nblk of the
//    contiguous range of targets b % nblk * per_wg ..., each wave taking the range's next
//    target from a counter in LDS when it is free;
//  * work != nullptr, tseg == nullptr (one segment): the grid is what the device holds at once,
//    and every wave takes the next pair from the counters until none is left, so a workgroup's
//    tile boxes are loaded once and no wave waits for a slow one to free its slot;
//  * tseg != nullptr (many segments, one per relation of a batch): the same persistent pairs
//    over every target of every relation, tseg[q] naming the target's relation and tord (when
//    given) the order of the targets (the heaviest relations first); a wave reads the tile boxes
//    of its target's relation from L2.
__global__ void __launch_bounds__(kGresBlock) __attribute__((amdgpu_waves_per_eu(8))) gres_tiles_kernel(
    const float* __restrict__ cand, int64_t ccap, const float* __restrict__ lo,
    const float* __restrict__ hi, int64_t tcap, const int32_t* __restrict__ seg_coff,
    const int32_t* __restrict__ seg_cnt, int32_t d_rt, const float* __restrict__ tval,
    int64_t tvcap, int32_t nt, const int32_t* __restrict__ thint, int32_t per_wg, int32_t g_max,
    int32_t lds_floats, int32_t* __restrict__ ge_out, unsigned long long* __restrict__ dev_tests,
    int32_t nblk, int32_t band_len, const int32_t* __restrict__ gstart, int32_t nbands,
    int32_t* __restrict__ work, const int32_t* __restrict__ params, const int32_t* __restrict__ tseg,
    const int32_t* __restrict__ tord, const uint64_t* __restrict__ lkey, const uint4* __restrict__ tkey,
    const uint64_t* __restrict__ ckey, int32_t kw, const int32_t* __restrict__ kok, int64_t kslots,
    int64_t ktiles) {
    constexpr int DM = D > 0 ? D : SKY_MAX_D;
    extern __shared__ float sbox[];  // [d][ntile] lo, [d][ntile] hi, [d][nchunk] chunk lo
    if (params) {  // target count and mapping decided on the device
        if (params[P_MAPPING] != SKY_GRES_TILES) return;
        nt = params[P_NT];
    }
    unsigned long long ntests = 0;   // candidate tests (target against candidate at one level)
    const int d = dget<D>(d_rt);
    const int lane = (int)lane_id();
    const uint32_t padslot = (uint32_t)(ccap - kTileC);
    // packed keys, when the store's slots fit the tables: the guard bit of every field
    const bool use_keys = lkey && *kok;
    uint64_t guard = 0;
    if (use_keys)
        for (int k = 0; k < d; ++k) guard |= 1ull << (k * kw + kw - 1);
    // a segment's place in the store (and whether its boxes fit in LDS)
    struct Seg { uint32_t coff; int32_t ntile, nchunk; uint32_t t0; bool use_lds; };
    auto seg_at = [&](int32_t sg, bool lds_ok) -> Seg {
        Seg v;
        v.coff = (uint32_t)seg_coff[sg];
        const int32_t cnt = seg_cnt[sg];
        v.ntile = (cnt + kTileC - 1) / kTileC;
        v.nchunk = (v.ntile + kWave - 1) / kWave;
        v.t0 = v.coff / kTileC;  // first tile of the segment
        v.use_lds = lds_ok && v.nchunk <= kWave && d * (2 * v.ntile + v.nchunk) <= lds_floats;
        return v;
    };
    int32_t band0 = 0;
    WgWork w{0, 0, nt};
    if (!work) {
        band0 = blockIdx.x / nblk;
        w = wg_work(per_wg, nt, blockIdx.x - band0 * nblk);
        if (w.t0 >= w.t1) return;  // uniform
    }
    // one segment: its boxes in LDS when they fit
    const Seg sv0 = seg_at(0, tseg == nullptr && !use_keys);
    float* blo = sbox;
    float* bhi = sbox + d * sv0.ntile;
    float* clo = sbox + 2 * d * sv0.ntile;
    if (sv0.use_lds) {
        const int32_t ntile = sv0.ntile, nchunk = sv0.nchunk;
        for (int32_t e = threadIdx.x; e < d * ntile; e += kGresBlock) {
            const int32_t k = e / ntile, tl = e - k * ntile;
            blo[e] = lo[(int64_t)k * tcap + sv0.t0 + tl];
            bhi[e] = hi[(int64_t)k * tcap + sv0.t0 + tl];
        }
        __syncthreads();
        for (int32_t e = threadIdx.x; e < d * nchunk; e += kGresBlock) {
            const int32_t k = e / nchunk, c = e - k * nchunk;
            float mn = 1.0f;
            for (int32_t tl = c * kWave; tl < ntile && tl < (c + 1) * kWave; ++tl)
                mn = fminf(mn, blo[k * ntile + tl]);
            clo[e] = mn;
        }
        __syncthreads();
    }
    // the level scan of target q over the levels of band `band`, in segment sv
    auto search = [&](const int32_t q, const int32_t band, const Seg& sv) {
        const uint32_t coff = sv.coff;
        const int32_t ntile = sv.ntile, nchunk = sv.nchunk;
        const uint32_t t0 = sv.t0;
        const bool use_lds = sv.use_lds;
        float tv[DM];
#pragma unroll
        for (int k = 0; k < DM; ++k)
            if (k < d) tv[k] = ldf(tval + k * tvcap, (uint32_t)q);
        int32_t my_tile = thint[q];
        my_tile = my_tile < 0 ? 0 : (my_tile >= ntile ? ntile - 1 : my_tile);
        const int32_t my_chunk = my_tile / kWave;
        int32_t result = 1;
        // a higher band may already have found the exit of q at or above this band's levels
        int32_t seen = __hip_atomic_load(&ge_out[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // the bands split [2, g_max], or [2, start level] when the target has one (no exit lies
        // above it, gres_start_kernel), into nbands ranges, highest first
        int32_t gtop = g_max, blen = band_len;
        if (gstart) {
            gtop = gstart[q] < g_max ? gstart[q] : g_max;
            blen = gtop > 2 ? (gtop - 2 + nbands) / nbands : 1;
        }
        const int32_t g_hi = gtop - band * blen;
        const int32_t g_lo = g_hi - blen + 1 > 2 ? g_hi - blen + 1 : 2;
        for (int32_t g = g_hi; g >= g_lo && ntile > 0; --g) {
            if (seen >= g) break;
            const int32_t seen_next =
                __hip_atomic_load(&ge_out[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const float fg = (float)g;
            // key(v) <= key(t) <=> fl(v g) < key(t) + 1;  key(v) < key(t) <=> fl(v g) < key(t)
            float tle[DM], tlt[DM];
#pragma unroll
            for (int k = 0; k < DM; ++k)
                if (k < d) {
                    const float kt = floorf(__fmul_rn(tv[k], fg));
                    tlt[k] = kt;
                    tle[k] = kt + 1.0f;
                }
            bool found = false;
            // chunks [cbase, cbase + 64), the first group from the target's own chunk on: bit cb
            // of the mask is chunk cbase + (cb + rot) mod 64
            for (int32_t cbase = 0; cbase < nchunk && !found; cbase += kWave) {
                const int rot = cbase == 0 ? my_chunk % kWave : 0;
                uint64_t cm;
                if (use_lds) {  // (one group: nchunk <= 64)
                    const bool inr = lane < nchunk;
                    const int32_t ci = inr ? lane : 0;
                    bool cp = inr;
#pragma unroll
                    for (int k = 0; k < DM; ++k)
                        if (k < d) cp &= __fmul_rn(clo[k * nchunk + ci], fg) < tle[k];
                    cm = __ballot(cp);
                } else {
                    cm = nchunk - cbase >= kWave ? ~0ull : ((1ull << (nchunk - cbase)) - 1ull);
                }
                cm = rotr64(cm, rot);
                while (cm && !found) {
                    const int cb = __ffsll((unsigned long long)cm) - 1;
                    cm &= cm - 1;
                    const int32_t c = cbase + (cb + rot) % kWave;
                    if (c >= nchunk) continue;
                    const int32_t tile = c * kWave + lane;
                    const bool inr = tile < ntile;
                    const uint32_t ti = inr ? (uint32_t)tile : 0u;
                    bool pass = inr, hle = true, hlt = false;
#pragma unroll
                    for (int k = 0; k < DM; ++k)
                        if (k < d) {
                            const float l = use_lds ? blo[k * ntile + ti] : ldf(lo + k * tcap, t0 + ti);
                            const float h = use_lds ? bhi[k * ntile + ti] : ldf(hi + k * tcap, t0 + ti);
                            pass &= __fmul_rn(l, fg) < tle[k];
                            const float ph = __fmul_rn(h, fg);
                            hle &= ph < tle[k];
                            hlt |= ph < tlt[k];
                        }
                    // every candidate of a tile whose upper corner's keys dominate t's keys
                    // dominates t
                    if (__ballot(pass && hle && hlt)) { found = true; break; }
                    const int r = c == my_chunk ? my_tile % kWave : 0;
                    uint64_t mask = rotr64(__ballot(pass), r);
                    while (mask) {
                        // up to kBatch passing tiles per round trip, branch-free loads
                        uint32_t jb[kBatch];
#pragma unroll
                        for (int b = 0; b < kBatch; ++b) {
                            jb[b] = padslot + (uint32_t)lane;
                            if (mask) {
                                const int tb = ((__ffsll((unsigned long long)mask) - 1) + r) % kWave;
                                mask &= mask - 1;
                                jb[b] = coff + (uint32_t)((c * kWave + tb) * kTileC + lane);
                                ntests += kTileC;
                            }
                        }
                        float sv[kBatch][DM];
#pragma unroll
                        for (int b = 0; b < kBatch; ++b)
#pragma unroll
                            for (int k = 0; k < DM; ++k)
                                if (k < d) sv[b][k] = ldf(cand + k * ccap, jb[b]);
                        bool dom = false;
#pragma unroll
                        for (int b = 0; b < kBatch; ++b) {
                            // padding candidates hold 2.0: never below t's keys
                            bool le = true, lt = false;
#pragma unroll
                            for (int k = 0; k < DM; ++k)
                                if (k < d) {
                                    const float p = __fmul_rn(sv[b][k], fg);
                                    le &= p < tle[k];
                                    lt |= p < tlt[k];
                                }
                            dom |= le && lt;
                        }
                        if (__ballot(dom)) { found = true; break; }
                    }
                }
            }
            if (found) { result = g; break; }
            seen = seen_next;
        }
        // ge_out starts at 1 (no exit); each band raises it to its highest exit level
        if (lane == 0 && result > 1) atomicMax(&ge_out[q], result);
    };
    // The same scan on the packed key tables (boxes from L2), arranged for few dependent round
    // trips per level: the chunk keys, the target's own chunk's tile boxes and its own tile's
    // candidates are loaded together, the other passing chunks' tile boxes kChunkBatch at a
    // time, candidates kBatch tiles at a time.
    const uint32_t kpad = (uint32_t)(kslots - kTileC);  // the key table's padding tile
    auto search_keys = [&](const int32_t q, const int32_t band, const Seg& sv) {
        const uint32_t coff = sv.coff;
        const int32_t ntile = sv.ntile, nchunk = sv.nchunk;
        const uint32_t t0 = sv.t0;
        float tv[DM];
#pragma unroll
        for (int k = 0; k < DM; ++k)
            if (k < d) tv[k] = ldf(tval + k * tvcap, (uint32_t)q);
        int32_t my_tile = thint[q];
        my_tile = my_tile < 0 ? 0 : (my_tile >= ntile ? ntile - 1 : my_tile);
        const int32_t my_chunk = my_tile / kWave;
        const int r_own = my_tile % kWave;
        int32_t result = 1;
        int32_t seen = __hip_atomic_load(&ge_out[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int32_t gtop = g_max, blen = band_len;
        if (gstart) {
            gtop = gstart[q] < g_max ? gstart[q] : g_max;
            blen = gtop > 2 ? (gtop - 2 + nbands) / nbands : 1;
        }
        const int32_t g_hi = gtop - band * blen;
        const int32_t g_lo = g_hi - blen + 1 > 2 ? g_hi - blen + 1 : 2;
        for (int32_t g = g_hi; g >= g_lo && ntile > 0; --g) {
            if (seen >= g) break;
            const int32_t seen_next =
                __hip_atomic_load(&ge_out[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const float fg = (float)g;
            uint64_t tk = 0;  // t's packed keys
#pragma unroll
            for (int k = 0; k < DM; ++k)
                if (k < d) tk |= (uint64_t)(uint32_t)floorf(__fmul_rn(tv[k], fg)) << (k * kw);
            // (t | guard) - s: no field borrows (t's field plus the guard bit exceeds s's field),
            // and a field keeps its guard bit exactly when s's key <= t's key
            const uint64_t tg = tk | guard;
            auto keys_le = [&](uint64_t kv) { return ((tg - kv) & guard) == guard; };
            const uint64_t* krow = lkey + (int64_t)(g - 2) * kslots;
            const uint4* trow = tkey + (int64_t)(g - 2) * ktiles + t0;
            const uint64_t* crow = ckey + (int64_t)(g - 2) * ktiles + t0;  // chunk c at crow[64 c]
            // candidates of kBatch passing tiles of chunk c per round trip (mask rotated by r)
            auto test_tiles = [&](uint64_t mask, int32_t c, int r) -> bool {
                while (mask) {
                    uint32_t jb[kBatch];
#pragma unroll
                    for (int b = 0; b < kBatch; ++b) {
                        jb[b] = kpad + (uint32_t)lane;
                        if (mask) {
                            const int tb = ((__ffsll((unsigned long long)mask) - 1) + r) % kWave;
                            mask &= mask - 1;
                            jb[b] = coff + (uint32_t)((c * kWave + tb) * kTileC + lane);
                            ntests += kTileC;
                        }
                    }
                    uint64_t kv[kBatch];
#pragma unroll
                    for (int b = 0; b < kBatch; ++b) kv[b] = krow[jb[b]];
                    bool dom = false;
#pragma unroll
                    for (int b = 0; b < kBatch; ++b) dom |= keys_le(kv[b]) && kv[b] != tk;
                    if (__ballot(dom)) return true;
                }
                return false;
            };
            // pass: the tile's lower corner's keys are all <= t's (some candidate may dominate);
            // tdom: so are its upper corner's, one of them below t's (every candidate dominates)
            auto tile_pass = [&](const uint4& b, bool inr, bool* tdom) {
                const uint64_t kl = ((uint64_t)b.y << 32) | b.x, kh = ((uint64_t)b.w << 32) | b.z;
                *tdom = inr && keys_le(kh) && kh != tk;
                return inr && keys_le(kl);
            };
            // one round trip: the first 64 chunks' keys, the own chunk's boxes, the own tile
            const bool c_in = lane < nchunk;
            const uint64_t ck = crow[c_in ? lane * kWave : 0];
            const int32_t own_t = my_chunk * kWave + lane;
            const bool own_in = own_t < ntile;
            const uint4 ob = trow[own_in ? own_t : 0];
            const uint64_t okv = krow[coff + (uint32_t)my_tile * kTileC + lane];
            ntests += kTileC;
            bool found = __ballot(keys_le(okv) && okv != tk) != 0;
            if (!found) {
                bool tdom;
                const bool pass = tile_pass(ob, own_in, &tdom);
                found = __ballot(tdom) != 0 || test_tiles(rotr64(__ballot(pass), r_own) & ~1ull, my_chunk, r_own);
            }
            // the other chunks whose lower corner passes, from the one after the own chunk on
            for (int32_t cbase = 0; cbase < nchunk && !found; cbase += kWave) {
                uint64_t cm;
                if (cbase == 0) {
                    cm = __ballot(c_in && keys_le(ck));
                } else {
                    const int32_t ci = cbase + lane;
                    cm = __ballot(ci < nchunk && keys_le(crow[ci < nchunk ? ci * kWave : 0]));
                }
                if (my_chunk >= cbase && my_chunk < cbase + kWave) cm &= ~(1ull << (my_chunk - cbase));
                const int rot = my_chunk >= cbase && my_chunk < cbase + kWave ? my_chunk - cbase : 0;
                cm = rotr64(cm, rot);
                while (cm && !found) {
                    // up to kChunkBatch chunks' tile boxes per round trip
                    int32_t cs[kChunkBatch];
                    uint4 bx[kChunkBatch];
#pragma unroll
                    for (int j = 0; j < kChunkBatch; ++j) {
                        cs[j] = -1;
                        if (cm) {
                            cs[j] = cbase + ((__ffsll((unsigned long long)cm) - 1) + rot) % kWave;
                            cm &= cm - 1;
                        }
                        const int32_t t = (cs[j] < 0 ? 0 : cs[j]) * kWave + lane;
                        bx[j] = trow[t < ntile ? t : 0];
                    }
#pragma unroll
                    for (int j = 0; j < kChunkBatch; ++j) {
                        if (found || cs[j] < 0) continue;
                        bool tdom;
                        const bool pass = tile_pass(bx[j], cs[j] * kWave + lane < ntile, &tdom);
                        found = __ballot(tdom) != 0 || test_tiles(__ballot(pass), cs[j], 0);
                    }
                }
            }
            if (found) { result = g; break; }
            seen = seen_next;
        }
        if (lane == 0 && result > 1) atomicMax(&ge_out[q], result);
    };
    if (work) {
        const int64_t total = (int64_t)nt * nbands;
        // kWorkCounters counters, 128 bytes apart, so that no single address takes every
        // atomic: workgroup b draws from counter b % nctr, which hands out the pairs
        // x, x + nctr, x + 2 nctr, ... (every pair belongs to exactly one counter, and every
        // counter has workgroups when the grid holds at least nctr of them)
        const int32_t nctr = gridDim.x >= (uint32_t)kWorkCounters ? kWorkCounters : 1;
        const int32_t x = (int32_t)(blockIdx.x % (uint32_t)nctr);
        for (;;) {
            int32_t k = 0;
            if (lane == 0) k = atomicAdd(work + kCounterStride * x, 1);
            k = __builtin_amdgcn_readfirstlane(k);
            const int64_t item = x + (int64_t)nctr * k;
            if (item >= total) break;  // every wave ends here once its counter passes the total
            const int32_t b = (int32_t)(item / nt);
            const int32_t r = (int32_t)(item - (int64_t)b * nt);
            if (tseg) {
                const int32_t q = tord ? tord[r] : r;
                if (use_keys) search_keys(q, b, seg_at(tseg[q], false));
                else search(q, b, seg_at(tseg[q], false));
            } else if (use_keys) {
                search_keys(r, b, sv0);
            } else {
                search(r, b, sv0);
            }
        }
    } else {
        // the workgroup's range, one target at a time to whichever wave is free
        __shared__ int32_t next_q;
        if (threadIdx.x == 0) next_q = w.t0;
        __syncthreads();
        for (;;) {
            int32_t q = 0;
            if (lane == 0) q = atomicAdd(&next_q, 1);
            q = __builtin_amdgcn_readfirstlane(q);
            if (q >= w.t1) break;
            if (use_keys) search_keys(q, band0, sv0);
            else search(q, band0, sv0);
        }
    }
    add_block_tests(dev_tests, ntests);
}

// no level g >= g_low can see a candidate whose (lower-bounding) excess over t is delta
__device__ __forceinline__ bool beyond_levels(double delta, int32_t g_low) {
    const double wv = delta - 0x1p-23;
    return wv > 0.0 && (double)g_low * wv >= 1.0 + 1e-9;
}

// A level bound B for a candidate whose excess over t is delta: beyond_levels(delta, g) holds
// for every g > B (with one level to spare against the rounding of the quotient); g_max when
// the excess excludes no level.
__device__ __forceinline__ int32_t collapse_bound(double delta, int32_t g_max) {
    const double wv = delta - 0x1p-23;
    if (!(wv > 0.0)) return g_max;
    const double r = (1.0 + 1e-9) / wv;
    return r >= (double)g_max ? g_max : (int32_t)r + 1;
}

// Highest level worth searching for each target. A candidate s can dominate the projection of
// t at level g only if s is below t in some attribute (keys are monotone, so s >= t everywhere
// gives keys >= t's keys), and only while every attribute where s is above t can still collapse
// onto t's key (collapse_bound). The start level of t is the largest bound over the candidates
// that qualify (1 when none does), so no level above it holds an exit. A tile's lower corner
// bounds all of its candidates at once: a tile with no attribute below t is skipped, and so is
// one whose bound does not exceed the start level found so far.
template <int D>
__global__ void __launch_bounds__(kGresBlock) gres_start_kernel(
    const float* __restrict__ cand, int64_t ccap, const float* __restrict__ lo, int64_t tcap,
    const int32_t* __restrict__ seg_coff, const int32_t* __restrict__ seg_cnt, int32_t d_rt,
    const float* __restrict__ tval, int64_t tvcap, int32_t nt, const int32_t* __restrict__ tseg,
    int32_t per_wg, int32_t g_max, int32_t* __restrict__ gstart, const int32_t* __restrict__ params) {
    constexpr int DM = D > 0 ? D : SKY_MAX_D;
    const int d = dget<D>(d_rt);
    const int lane = (int)lane_id();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform
    int32_t nblk = (int32_t)gridDim.x;
    if (params) {  // the target count and the split are on the device: grid-stride over the blocks
        nt = params[P_NT];
        per_wg = params[P_PER_WG];
        nblk = params[P_BLOCKS];
    }
    for (int32_t vb = blockIdx.x; vb < nblk; vb += gridDim.x) {
    const WgWork w = wg_work(per_wg, nt, vb);
    for (int32_t q = w.t0 + wave; q < w.t1; q += kWaves) {
        const int32_t sg = tseg ? tseg[q] : 0;  // the target's segment (a relation of a batch)
        const int64_t coff = seg_coff[sg];
        const int32_t cnt = seg_cnt[sg];
        const int32_t ntile = (cnt + kTileC - 1) / kTileC;
        const int64_t t0 = coff / kTileC;
        float tv[DM];
#pragma unroll
        for (int k = 0; k < DM; ++k)
            if (k < d) tv[k] = tval[(int64_t)k * tvcap + q];
        int32_t best = 1;  // wave-uniform
        for (int32_t tb = 0; tb < ntile && best < g_max; tb += kWave) {
            // lanes over tiles
            const int32_t tile = tb + lane;
            int32_t tbound = 1;
            if (tile < ntile) {
                bool below = false;
                double dt = -1.0;
#pragma unroll
                for (int k = 0; k < DM; ++k)
                    if (k < d) {
                        const float l = lo[(int64_t)k * tcap + t0 + tile];
                        below |= l < tv[k];
                        const double e = (double)l - (double)tv[k];
                        dt = e > dt ? e : dt;
                    }
                if (below) tbound = collapse_bound(dt, g_max);
            }
            uint64_t todo = __ballot(tbound > best);
            while (todo && best < g_max) {
                const int i = __ffsll((unsigned long long)todo) - 1;
                todo &= todo - 1;
                if (__shfl(tbound, i) <= best) continue;
                // lanes over the tile's candidates (padding slots hold 2.0: never below t)
                const int64_t j = coff + (int64_t)(tb + i) * kTileC + lane;
                bool below = false;
                double ds = -1.0;
#pragma unroll
                for (int k = 0; k < DM; ++k)
                    if (k < d) {
                        const float v = cand[(int64_t)k * ccap + j];
                        below |= v < tv[k];
                        const double e = (double)v - (double)tv[k];
                        ds = e > ds ? e : ds;
                    }
                int32_t b = below ? collapse_bound(ds, g_max) : 1;
                for (int off = kWave / 2; off > 0; off >>= 1) {
                    const int32_t o = __shfl_xor(b, off);
                    b = o > b ? o : b;
                }
                best = b > best ? b : best;
            }
        }
        if (lane == 0) gstart[q] = best;
    }
    }
}

template <int D>
// Lanes over 64 consecutive levels, candidates wave-uniform. Work: the levels of each target
// split into nbands bands, blocks band-major over contiguous target ranges (per_wg), or, with
// tseg (the relations of a batch), persistent waves taking (target, band) pairs from the work
// counters like the tile search.
__global__ void __launch_bounds__(kGresBlock) gres_levels_kernel(
    const float* __restrict__ cand, int64_t ccap, const float* __restrict__ lo,
    const float* __restrict__ hi, int64_t tcap, const int32_t* __restrict__ seg_coff,
    const int32_t* __restrict__ seg_cnt, int32_t d_rt, const float* __restrict__ tval,
    int64_t tvcap, int32_t nt, int32_t per_wg, int32_t g_max,
    int32_t* __restrict__ ge_out, unsigned long long* __restrict__ dev_tests,
    const int32_t* __restrict__ gstart, int32_t nblk, const int32_t* __restrict__ params,
    int32_t* __restrict__ work, const int32_t* __restrict__ tseg, const int32_t* __restrict__ tord) {
    constexpr int DM = D > 0 ? D : SKY_MAX_D;
    unsigned long long ntests = 0;  // candidate tests (target against candidate at one level)
    const int d = dget<D>(d_rt);
    const int lane = (int)lane_id();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform
    int32_t nbands = (int32_t)(gridDim.x / (uint32_t)nblk);
    if (params) {  // target count, mapping and split decided on the device: grid-stride
        if (params[P_MAPPING] != SKY_GRES_LEVELS) return;
        nt = params[P_NT];
        per_wg = params[P_PER_WG];
        nblk = params[P_BLOCKS];
        nbands = params[P_LBANDS];
    }
    // the level scan of target q over the levels of band `band`, in segment sg
    auto search = [&](const int32_t q, const int32_t band, const int32_t sg) {
        const int64_t coff = seg_coff[sg];
        const int32_t cnt = seg_cnt[sg];
        const int32_t ntile = (cnt + kTileC - 1) / kTileC;
        const int64_t t0 = coff / kTileC;
        float tv[DM];
#pragma unroll
        for (int k = 0; k < DM; ++k)
            if (k < d) tv[k] = tval[(int64_t)k * tvcap + q];
        int32_t result = 1;
        // the bands split [2, g_max], or [2, start level] when the target has one (no exit lies
        // above it, gres_start_kernel), into nbands ranges, highest first
        const int32_t gtop = gstart ? (gstart[q] < g_max ? gstart[q] : g_max) : g_max;
        const int32_t blen = gtop > 2 ? (gtop - 2 + nbands) / nbands : 1;
        const int32_t g_hi = gtop - band * blen;
        const int32_t g_lo = g_hi - blen + 1 > 2 ? g_hi - blen + 1 : 2;
        for (int32_t gh = g_hi; gh >= g_lo; gh -= kWave) {
            // a higher band has already found an exit at or above every level left here
            if (nbands > 1 &&
                __hip_atomic_load(&ge_out[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= gh)
                break;
            const int32_t g = gh - lane;
            const bool lv = g >= g_lo;
            const int32_t g_low = (gh - (kWave - 1)) > g_lo ? (gh - (kWave - 1)) : g_lo;
            const float fg = (float)(lv ? g : 2);
            float tle[DM], tlt[DM];
#pragma unroll
            for (int k = 0; k < DM; ++k)
                if (k < d) {
                    const float kt = floorf(__fmul_rn(tv[k], fg));
                    tlt[k] = kt;
                    tle[k] = kt + 1.0f;
                }
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
                        double e = (double)lo[(int64_t)k * tcap + t0 + tile] - (double)tv[k];
                        dt = e > dt ? e : dt;
                    }
                if (beyond_levels(dt, g_low)) continue;
                bool pass = (need >> lane) & 1ull, hle = true, hlt = false;
#pragma unroll
                for (int k = 0; k < DM; ++k)
                    if (k < d) {
                        pass &= __fmul_rn(lo[(int64_t)k * tcap + t0 + tile], fg) < tle[k];
                        const float ph = __fmul_rn(hi[(int64_t)k * tcap + t0 + tile], fg);
                        hle &= ph < tle[k];
                        hlt |= ph < tlt[k];
                    }
                // the whole tile dominates t at this lane's level
                hit |= __ballot(pass && hle && hlt);
                if (hit & 1ull) break;
                const uint64_t pmask = __ballot(pass);
                if (!pmask) continue;
                const int32_t base = tile * kTileC;
                const int32_t cnt_t = (cnt - base) < kTileC ? (cnt - base) : kTileC;
                ntests += (unsigned long long)cnt_t * (unsigned long long)__popcll(pmask);
                for (int32_t i = 0; i < cnt_t; ++i) {
                    const int64_t j = coff + base + i;
                    float sv[DM];
                    double ds = -1.0;
#pragma unroll
                    for (int k = 0; k < DM; ++k)
                        if (k < d) {
                            sv[k] = cand[(int64_t)k * ccap + j];
                            double e = (double)sv[k] - (double)tv[k];
                            ds = e > ds ? e : ds;
                        }
                    if (beyond_levels(ds, g_low)) continue;
                    bool le = true, lt = false;
#pragma unroll
                    for (int k = 0; k < DM; ++k)
                        if (k < d) {
                            const float p = __fmul_rn(sv[k], fg);
                            le &= p < tle[k];
                            lt |= p < tlt[k];
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
        // ge_out starts at 1 (no exit); each band raises it to its highest exit level
        if (lane == 0 && result > 1) atomicMax(&ge_out[q], result);
    };
    if (tseg) {
        const int64_t total = (int64_t)nt * nbands;
        const int32_t nctr = gridDim.x >= (uint32_t)kWorkCounters ? kWorkCounters : 1;
        const int32_t x = (int32_t)(blockIdx.x % (uint32_t)nctr);
        for (;;) {
            int32_t k = 0;
            if (lane == 0) k = atomicAdd(work + kCounterStride * x, 1);
            k = __builtin_amdgcn_readfirstlane(k);
            const int64_t item = x + (int64_t)nctr * k;
            if (item >= total) break;
            const int32_t b = (int32_t)(item / nt);
            const int32_t r = (int32_t)(item - (int64_t)b * nt);
            const int32_t q = tord ? tord[r] : r;
            search(q, b, tseg[q]);
        }
    } else {
        // blocks are band-major: every target's highest band first
        for (int32_t vb = blockIdx.x; vb < nblk * nbands; vb += gridDim.x) {
            const int32_t band = vb / nblk;
            const WgWork w = wg_work(per_wg, nt, vb - band * nblk);
            for (int32_t q = w.t0 + wave; q < w.t1; q += kWaves) search(q, band, 0);
        }
    }
    add_block_tests(dev_tests, ntests);
}

__global__ void __launch_bounds__(kBlock) gres_output_kernel(const int32_t* __restrict__ ge_t,
                                                              const int32_t* __restrict__ tout,
                                                              int32_t nt, const int32_t* __restrict__ params,
                                                              int32_t out_cap, int32_t* __restrict__ g_exit,
                                                              float* __restrict__ gres) {
    if (params) nt = params[P_NT];
    for (int32_t q = blockIdx.x * kBlock + threadIdx.x; q < nt; q += gridDim.x * kBlock) {
        const int32_t j = tout[q];
        if (j < 0 || j >= out_cap) continue;  // (beyond the outputs only after a capacity error)
        const int32_t g = ge_t[q];
        if (g_exit) g_exit[j] = g;
        if (gres) gres[j] = __fdiv_rn(1.0f, (float)g);
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

void carve_gres_store(Carver& c, GresStore& st, int64_t s, int32_t d, int32_t nseg) {
    // every segment 64-aligned, plus one padding tile at the end
    st.ccap = round_up(s > 0 ? s : 1, kTileC) + (int64_t)kTileC * (nseg + 1);
    st.tcap = round_up(ceil_div(st.ccap, kTileC), 64);
    st.cand = c.take<float>((size_t)(d * st.ccap));
    st.lo = c.take<float>((size_t)(d * st.tcap));
    st.hi = c.take<float>((size_t)(d * st.tcap));
    st.ckey = c.take<uint32_t>((size_t)st.ccap);
    st.perm = c.take<int32_t>((size_t)st.ccap);
    st.seg_coff = c.take<int32_t>((size_t)nseg);
    st.seg_cnt = c.take<int32_t>((size_t)nseg);
    st.nseg = nseg;
}

void carve_gres_prep_tmp(Carver& c, GresPrepTmp& t, int64_t s) {
    const int64_t sp = round_up(s > 0 ? s : 1, 64);
    t.k0 = c.take<uint32_t>((size_t)sp);
    t.v0 = c.take<uint32_t>((size_t)sp);
    t.k1 = c.take<uint32_t>((size_t)sp);
    t.v1 = c.take<uint32_t>((size_t)sp);
    t.radix_tmp = c.take<int32_t>((size_t)radix_tmp_elems(s > 0 ? s : 1));
}

void carve_gres_targets(Carver& c, GresTargets& t, int64_t nt, int32_t d) {
    t.tvcap = round_up(nt > 0 ? nt : 1, 64);
    t.tval = c.take<float>((size_t)(d * t.tvcap));
    t.thint = c.take<int32_t>((size_t)t.tvcap);
    t.tout = c.take<int32_t>((size_t)t.tvcap);
    t.ge = c.take<int32_t>((size_t)t.tvcap);
    t.gstart = c.take<int32_t>((size_t)t.tvcap);
    t.work = c.take<int32_t>((size_t)kWorkCounters * kCounterStride);
    t.params = c.take<int32_t>(16);
}

int32_t key_width(int32_t d, int32_t g_max) {
    if (g_max < 2 || g_max > kKeyTableMaxG) return 0;
    // keys 0..g_max and the clamp value 2^(w-1) - 1 above them: w - 1 = bit length of g_max + 1
    int32_t b = 0;
    while ((1 << b) <= g_max + 1) ++b;
    const int32_t w = b + 1;
    return d * w <= 64 ? w : 0;
}

void carve_gres_keys_slots(Carver& c, GresKeys& k, int64_t slots, int32_t levels) {
    k.kslots = round_up(slots > kTileC ? slots : kTileC + 1, kTileC);
    k.ktiles = round_up(ceil_div(k.kslots, kTileC), kWave);
    k.levels = levels;
    k.key = c.take<uint64_t>((size_t)(levels * k.kslots));
    k.tile = c.take<uint4>((size_t)(levels * k.ktiles));
    k.chunk = c.take<uint64_t>((size_t)(levels * k.ktiles));
    k.ok = c.take<int32_t>(64);
}

void carve_gres_keys(Carver& c, GresKeys& k, const GresStore& store, int32_t d, int32_t g_max) {
    if (key_width(d, g_max)) carve_gres_keys_slots(c, k, store.ccap, g_max - 1);
}

sky_status launch_gres_prepare(const float* x, int64_t n, int32_t d, int64_t ld, const int64_t* rows,
                               int64_t s64, const GresStore& store, const GresPrepTmp& tmp,
                               int32_t* dev_status, hipStream_t st) {
    const int32_t s = (int32_t)s64;
    const int bits = curve_bits(d);
    hipLaunchKernelGGL(single_segment_kernel, dim3(1), dim3(64), 0, st, store.seg_coff, store.seg_cnt, s,
                       (const int32_t*)nullptr, dev_status);
    if (s > 0) {
        hipLaunchKernelGGL(curve_kernel, dim3((uint32_t)ceil_div(s, kBlock)), dim3(kBlock), 0, st, x, n,
                           d, ld, rows, s, bits, tmp.k0, tmp.v0, dev_status);
        SKY_HIP(hipGetLastError());
        SKY_TRY(launch_radix_sort(tmp.k0, tmp.v0, tmp.k1, tmp.v1, s, bits * d, tmp.radix_tmp, st));
    }
    hipLaunchKernelGGL(store_kernel, dim3((uint32_t)ceil_div(store.ccap, kBlock)), dim3(kBlock), 0, st,
                       x, n, d, ld, rows, s, (const uint32_t*)tmp.k0, (const uint32_t*)tmp.v0,
                       store.cand, store.ccap, store.ckey, store.perm);
    const int32_t ntile = (int32_t)ceil_div(s, kTileC);
    if (ntile > 0)
        hipLaunchKernelGGL(tile_box_kernel, dim3((uint32_t)ceil_div(ntile, kBlock / kWave)), dim3(kBlock), 0,
                           st, (const float*)store.cand, store.ccap, d, ntile, (const int32_t*)nullptr, 0,
                           store.lo, store.hi, store.tcap);
    SKY_HIP(hipGetLastError());
    return SKY_OK;
}

sky_status launch_gres_prepare_positions(const float* xp, int64_t ldp, int32_t d, const int32_t* pos,
                                         int64_t cap64, const int32_t* s_dev, const int32_t* rowid,
                                         const int32_t* idx_of_row, const GresStore& store,
                                         int32_t* dev_status, hipStream_t st, const GresTargets* tg) {
    const int32_t cap = (int32_t)cap64;
    auto grid = [](int64_t want, int64_t most) -> uint32_t {
        return (uint32_t)(want < 1 ? 1 : (want > most ? most : want));
    };
    // the store, its tile boxes, and (tg) the targets: one wave per tile
    const int64_t ntile = ceil_div(cap, kTileC);
    hipLaunchKernelGGL(store_pos_kernel, dim3(grid(ceil_div(ntile + 1, kBlock / kWave), 2048)),
                       dim3(kBlock), 0, st, xp, ldp, d, pos, cap, s_dev, rowid, idx_of_row, store.cand, store.ccap,
                       store.ckey, store.perm, tg ? tg->tval : nullptr, tg ? tg->tvcap : 0,
                       tg ? tg->thint : nullptr, tg ? tg->tout : nullptr, tg ? tg->ge : nullptr, store.seg_coff,
                       store.seg_cnt, dev_status, store.lo, store.hi, store.tcap);
    SKY_HIP(hipGetLastError());
    return SKY_OK;
}

sky_status launch_gres_targets(const float* x, int64_t n, int32_t d, int64_t ld,
                               const int64_t* rows /* null: all candidates */, int64_t nt64,
                               int64_t s64, const GresStore& store, const GresTargets& tg,
                               int32_t* dev_status, hipStream_t st) {
    const int32_t nt = (int32_t)nt64;
    if (nt <= 0) return SKY_OK;
    if (!rows) {
        hipLaunchKernelGGL(targets_all_kernel, dim3((uint32_t)ceil_div(nt, kBlock)), dim3(kBlock), 0, st,
                           (const float*)store.cand, store.ccap, nt, (const int32_t*)nullptr, d,
                           (const int32_t*)store.perm, tg.tval, tg.tvcap, tg.thint, tg.tout);
    } else {
        hipLaunchKernelGGL(targets_rows_kernel, dim3((uint32_t)ceil_div(nt, kBlock)), dim3(kBlock), 0, st,
                           x, n, d, ld, rows, nt, curve_bits(d), (const uint32_t*)store.ckey,
                           (int32_t)s64, tg.tval, tg.tvcap, tg.thint, tg.tout, dev_status);
    }
    SKY_HIP(hipGetLastError());
    return SKY_OK;
}

sky_status launch_batch_store(const float* xp, int64_t ldp, int32_t d, const int32_t* pos,
                              const int32_t* rowid, const int32_t* idx_of_row, const int64_t* sky_idx,
                              const int32_t* count_dev, int64_t cap, const int64_t* row_off, int32_t nseg,
                              int64_t* sky_off, int32_t* cand_off, int32_t* used, const GresStore& store,
                              hipStream_t st) {
    hipLaunchKernelGGL(batch_offsets_kernel, dim3((uint32_t)ceil_div(nseg + 1, kBlock)), dim3(kBlock), 0, st,
                       sky_idx, count_dev, (int32_t)cap, row_off, nseg, sky_off, cand_off);
    hipLaunchKernelGGL(batch_layout_kernel, dim3(1), dim3(1024), 0, st, (const int32_t*)cand_off, nseg,
                       store.seg_coff, store.seg_cnt, used);
    const int64_t slots = round_up(cap > 0 ? cap : 1, kTileC) + (int64_t)kTileC * (nseg + 1);
    const int64_t sb = ceil_div(slots, kBlock);
    hipLaunchKernelGGL(store_seg_pos_kernel, dim3((uint32_t)(sb > 2048 ? 2048 : sb)), dim3(kBlock), 0, st, xp, ldp,
                       d, pos, (const int32_t*)cand_off, (const int32_t*)store.seg_coff,
                       (const int32_t*)store.seg_cnt, nseg, (const int32_t*)used, rowid, idx_of_row, store.cand,
                       store.ccap, store.ckey, store.perm);
    const int64_t ntile = ceil_div(slots, kTileC);
    const int64_t tb = ceil_div(ntile, kBlock / kWave);
    hipLaunchKernelGGL(tile_box_kernel, dim3((uint32_t)(tb > 2048 ? 2048 : tb)), dim3(kBlock), 0, st,
                       (const float*)store.cand, store.ccap, d, (int32_t)ntile, (const int32_t*)used,
                       (int32_t)(ntile * kTileC), store.lo, store.hi, store.tcap);
    SKY_HIP(hipGetLastError());
    return SKY_OK;
}

sky_status launch_batch_search(const GresStore& store, int32_t d, int64_t cap, const int32_t* cand_off,
                               int32_t nseg, const int32_t* used, bool near_first, bool lpt, int32_t* order,
                               int32_t* rank_off, int32_t* tord, int32_t* tseg, const GresTargets& tg,
                               int32_t g_max, int32_t mapping, int32_t* g_exit, float* gres, void* ev_begin,
                               void* ev_end, unsigned long long* dev_tests, hipStream_t st, const GresKeys* keys) {
    if (cap <= 0) return SKY_OK;
    if (lpt) {  // the targets of the relations with the most candidates first
        hipLaunchKernelGGL(batch_rank_kernel, dim3((uint32_t)ceil_div(nseg, kBlock)), dim3(kBlock), 0, st,
                           (const int32_t*)store.seg_cnt, nseg, order);
        hipLaunchKernelGGL(batch_rank_scan_kernel, dim3(1), dim3(1024), 0, st, (const int32_t*)store.seg_cnt,
                           (const int32_t*)order, nseg, rank_off);
        hipLaunchKernelGGL(batch_tord_kernel, dim3((uint32_t)(nseg < 4096 ? nseg : 4096)), dim3(kBlock), 0, st,
                           (const int32_t*)order, (const int32_t*)rank_off, cand_off, nseg, tord);
        SKY_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(batch_params_kernel, dim3(1), dim3(64), 0, st, cand_off, nseg, used, g_max, mapping,
                       tg.params);
    const int64_t qb = ceil_div(cap, kBlock);
    hipLaunchKernelGGL(targets_seg_kernel, dim3((uint32_t)(qb > 2048 ? 2048 : qb)), dim3(kBlock), 0, st,
                       (const float*)store.cand, store.ccap, d, cand_off, (const int32_t*)store.seg_coff, nseg,
                       (const int32_t*)store.perm, near_first ? 1 : 0, tg.tval, tg.tvcap, tg.thint, tg.tout, tseg);
    SKY_HIP(hipGetLastError());
    return launch_gres_search(store, d, 0, tg, cap, nullptr, tseg, lpt ? tord : nullptr, g_max, mapping, g_exit,
                              gres, ev_begin, ev_end, dev_tests, st, keys);
}

sky_status resident_workgroups(const void* kernel, int32_t block, size_t dyn_lds, int32_t* out) {
    int dev = 0, cus = 0, per_cu = 0;
    SKY_HIP(hipGetDevice(&dev));
    SKY_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    SKY_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, dyn_lds));
    *out = (cus > 0 ? cus : 1) * (per_cu > 0 ? per_cu : 1);
    return SKY_OK;
}

sky_status launch_gres_search(const GresStore& store, int32_t d, int32_t max_cnt,
                              const GresTargets& tg, int64_t nt64, const int32_t* nt_dev, const int32_t* tseg,
                              const int32_t* tord, int32_t g_max, int32_t mapping, int32_t* g_exit,
                              float* gres, void* ev_begin, void* ev_end,
                              unsigned long long* dev_tests, hipStream_t st, const GresKeys* keys,
                              bool ge_ready) {
    const int32_t nt = (int32_t)nt64;  // with a count on the device: an upper bound of it
    if (nt <= 0) return SKY_OK;
    const bool batch = tseg != nullptr;
    const bool on_dev = nt_dev || batch;
    // packed key tables, when given for this g_max (whether the store's slots fit them is
    // decided on the device: the search falls back to the values otherwise)
    const uint64_t* lkey = nullptr;
    int32_t kw = 0;
    const uint4* tkey = nullptr;
    const uint64_t* ckey = nullptr;
    const int32_t* kok = nullptr;
    if (mapping != SKY_GRES_LEVELS && keys && keys->key && key_width(d, g_max) && g_max - 1 <= keys->levels &&
        (!batch || keys->used)) {
        kw = key_width(d, g_max);
        const int64_t kb = ceil_div(keys->kslots, kBlock);
        const int32_t cblocks = (int32_t)(kb > 2048 ? 2048 : kb);
        const int64_t tb = ceil_div(keys->ktiles, kBlock);
        const int32_t tblocks = (int32_t)(tb < 1 ? 1 : (tb > 1024 ? 1024 : tb));
        const int32_t nseg = batch ? store.nseg : 1;
        const int64_t sb = ceil_div(batch ? nseg : keys->ktiles / kWave, kBlock / kWave);
        const int32_t sblocks = (int32_t)(sb > 256 ? 256 : sb);
        SKY_DISPATCH_D(d, level_keys_kernel, dim3((uint32_t)(cblocks + tblocks + sblocks)), dim3(kBlock), 0, st,
                       (const float*)store.cand, store.ccap, (const float*)store.lo, (const float*)store.hi,
                       store.tcap, d, (const int32_t*)store.seg_coff, (const int32_t*)store.seg_cnt, nseg,
                       batch ? keys->used : nullptr, g_max - 1, kw, cblocks, tblocks, keys->key, keys->kslots,
                       keys->tile, keys->chunk, keys->ktiles, keys->ok);
        SKY_HIP(hipGetLastError());
        lkey = keys->key;
        tkey = keys->tile;
        ckey = keys->chunk;
        kok = keys->ok;
    }
    // LDS for the tile boxes of the one segment, when they fit; with the count on the device,
    // a fixed 40 KB (the kernel checks the real size), which costs no occupancy at 8 waves per
    // SIMD; a batch reads every relation's boxes from L2
    const int32_t ntile = (int32_t)ceil_div(max_cnt, kTileC);
    const int32_t nchunk = (int32_t)ceil_div(ntile, kWave);
    int64_t floats = (int64_t)d * (2 * ntile + nchunk);
    if (floats * 4 > kGresLdsBytes || nchunk > kWave) floats = 0;
    if (nt_dev) floats = kGresLdsDevBytes / 4;
    if (batch) floats = 0;
    const size_t lds = (size_t)floats * sizeof(float);
    int32_t per_wg = 0, lbands = 1, blocks = 0;
    search_shape(nt, g_max, &per_wg, &blocks, &lbands);
    int32_t* params = on_dev ? tg.params : nullptr;
    if (nt_dev) {  // the shape from the device count; it also clears the work counters of the
                   // persistent tile search (a batch's own setup has filled params)
        hipLaunchKernelGGL(search_setup_kernel, dim3(1), dim3(256), 0, st, nt_dev, nt, g_max, mapping, params,
                           mapping != SKY_GRES_LEVELS ? tg.work : nullptr);
        SKY_HIP(hipGetLastError());
    }
    // TILES: the levels are split into bands searched by separate workgroups (band-major
    // order), so a tuple that scans many levels is not one long sequential chain
    int32_t nbands = (int32_t)ceil_div(g_max - 1, kBandLevels);
    nbands = nbands < 1 ? 1 : (nbands > kMaxBands ? kMaxBands : nbands);
    const int32_t band_len = (int32_t)ceil_div(g_max - 1, nbands);
    const bool run_tiles = on_dev ? mapping != SKY_GRES_LEVELS : mapping != SKY_GRES_LEVELS;
    // (AUTO picks LEVELS only above g_max 1000, gres_auto_mapping)
    const bool run_levels = on_dev ? mapping == SKY_GRES_LEVELS || (mapping == SKY_GRES_AUTO && g_max > 1000)
                                   : mapping == SKY_GRES_LEVELS;
    // grids of the kernels that stride over the blocks a device-side count asks for
    const uint32_t stride_grid = (uint32_t)(blocks < kStrideGrid ? (blocks < 1 ? 1 : blocks) : kStrideGrid);
    // many levels: each target's highest level worth searching, from the candidates' bounds
    const int32_t* gstart = nullptr;
    if (g_max > kStartLevels) {
        SKY_DISPATCH_D(d, gres_start_kernel, dim3(on_dev ? stride_grid : (uint32_t)blocks), dim3(kGresBlock), 0,
                       st, (const float*)store.cand, store.ccap, (const float*)store.lo, store.tcap,
                       (const int32_t*)store.seg_coff, (const int32_t*)store.seg_cnt, d,
                       (const float*)tg.tval, tg.tvcap, nt, tseg, per_wg, g_max, tg.gstart,
                       (const int32_t*)params);
        SKY_HIP(hipGetLastError());
        gstart = tg.gstart;
    }
    // no exit (1) until a band finds one
    if (!ge_ready) {
        const int64_t fb = ceil_div(nt, kBlock);
        hipLaunchKernelGGL(fill_targets_kernel, dim3((uint32_t)(fb > 1024 ? 1024 : fb)), dim3(kBlock), 0, st, tg.ge,
                           nt, (const int32_t*)params, 1);
        SKY_HIP(hipGetLastError());
    }
    // persistent launches (one segment with many targets, a count on the device, a batch): as
    // many workgroups as the device holds at once, fed from the work counters
    uint32_t grid = (uint32_t)blocks * (uint32_t)nbands;
    int32_t* work = nullptr;
    uint32_t resident_tiles = 0;
    if (run_tiles) {
        const void* fn = nullptr;
        SKY_KERNEL_PTR_D(d, gres_tiles_kernel, fn);
        int32_t resident = 0;
        SKY_TRY(resident_workgroups(fn, kGresBlock, lds, &resident));
        resident_tiles = (uint32_t)resident;
        if ((int64_t)grid > resident || on_dev) {
            grid = resident_tiles;
            work = tg.work;
        }
    }
    uint32_t lgrid = (uint32_t)blocks * (uint32_t)lbands;
    if (run_levels && on_dev) {
        if (batch) {
            const void* fn = nullptr;
            SKY_KERNEL_PTR_D(d, gres_levels_kernel, fn);
            int32_t resident = 0;
            SKY_TRY(resident_workgroups(fn, kGresBlock, 0, &resident));
            lgrid = (uint32_t)resident;
            work = tg.work;
        } else {
            lgrid = stride_grid * (uint32_t)kMaxLevelBands > (uint32_t)kStrideGrid
                        ? (uint32_t)kStrideGrid : stride_grid * (uint32_t)kMaxLevelBands;
        }
    }
    if (work && !(nt_dev && mapping != SKY_GRES_LEVELS)) {  // (else cleared by the setup)
        hipLaunchKernelGGL(fill_i32_kernel, dim3(kWorkCounters * kCounterStride / kBlock), dim3(kBlock), 0,
                           st, work, kWorkCounters * kCounterStride, 0);
        SKY_HIP(hipGetLastError());
    }
    if (ev_begin) SKY_HIP(hipEventRecord((hipEvent_t)ev_begin, st));
    if (run_levels) {
        SKY_DISPATCH_D(d, gres_levels_kernel, dim3(lgrid), dim3(kGresBlock), 0, st,
                       (const float*)store.cand, store.ccap, (const float*)store.lo,
                       (const float*)store.hi, store.tcap, (const int32_t*)store.seg_coff,
                       (const int32_t*)store.seg_cnt, d, (const float*)tg.tval, tg.tvcap, nt,
                       per_wg, g_max, tg.ge, dev_tests, gstart, (int32_t)blocks, (const int32_t*)params,
                       work, tseg, tord);
        SKY_HIP(hipGetLastError());
    }
    if (run_tiles) {
        SKY_DISPATCH_D(d, gres_tiles_kernel, dim3(grid), dim3(kGresBlock), lds, st,
                       (const float*)store.cand, store.ccap, (const float*)store.lo,
                       (const float*)store.hi, store.tcap, (const int32_t*)store.seg_coff,
                       (const int32_t*)store.seg_cnt, d, (const float*)tg.tval, tg.tvcap, nt,
                       (const int32_t*)tg.thint, per_wg, g_max, (int32_t)floats, tg.ge,
                       dev_tests, (int32_t)blocks, band_len, gstart, nbands, work, (const int32_t*)params,
                       tseg, tord, lkey, tkey, ckey, kw, kok, lkey ? keys->kslots : 0,
                       lkey ? keys->ktiles : 0);
        SKY_HIP(hipGetLastError());
    }
    if (ev_end) SKY_HIP(hipEventRecord((hipEvent_t)ev_end, st));
    const int64_t ob = ceil_div(nt, kBlock);
    hipLaunchKernelGGL(gres_output_kernel, dim3((uint32_t)(ob > 1024 ? 1024 : ob)), dim3(kBlock), 0, st,
                       (const int32_t*)tg.ge, (const int32_t*)tg.tout, nt, (const int32_t*)params, nt, g_exit,
                       gres);
    SKY_HIP(hipGetLastError());
    return SKY_OK;
}

}  // namespace sky
