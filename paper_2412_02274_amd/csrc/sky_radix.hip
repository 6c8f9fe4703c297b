// Stable LSD radix sort of (uint32 key, uint32 value) pairs, 8-bit digits.
//
// One pass = histogram (per wave tile of 1024 items, 256 digit counters in LDS), exclusive
// scan of the digit-major histogram table, and a stable scatter: each wave walks its tile in
// order, 64 items at a time, and ranks equal digits inside the wave with ballots (no
// atomics), so equal keys keep their input order. Used for the Sliced partitioning order
// (key = FP32 pattern of the slicing attribute, value = row) and for the spatial order of
// the gres candidates.
#include "sky_internal.hpp"

namespace sky {

namespace {

constexpr int kTile = 1024;                     // items per wave tile
constexpr int kWavesPerBlock = kBlock / kWave;  // 4
constexpr int kChunks = kTile / kWave;          // 16

__global__ void __launch_bounds__(kBlock) radix_hist_kernel(const uint32_t* __restrict__ keys,
                                                             int64_t n, int shift,
                                                             int32_t* __restrict__ hist,
                                                             int64_t ntiles) {
    __shared__ int32_t cnt[kWavesPerBlock][256];
    const int wave = threadIdx.x / kWave;
    const int lane = (int)lane_id();
    const int64_t tile = (int64_t)blockIdx.x * kWavesPerBlock + wave;
    for (int i = lane; i < 256; i += kWave) cnt[wave][i] = 0;
    __syncthreads();
    if (tile < ntiles) {
        for (int c = 0; c < kChunks; ++c) {
            int64_t idx = tile * kTile + c * kWave + lane;
            if (idx < n) atomicAdd(&cnt[wave][(keys[idx] >> shift) & 0xFFu], 1);
        }
    }
    __syncthreads();
    if (tile < ntiles)
        for (int i = lane; i < 256; i += kWave) hist[(int64_t)i * ntiles + tile] = cnt[wave][i];
}

__global__ void __launch_bounds__(kBlock) radix_scatter_kernel(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint32_t* __restrict__ kout,
    uint32_t* __restrict__ vout, int64_t n, int shift, const int32_t* __restrict__ offs,
    int64_t ntiles) {
    __shared__ int32_t base[kWavesPerBlock][256];
    const int wave = threadIdx.x / kWave;
    const int lane = (int)lane_id();
    const int64_t tile = (int64_t)blockIdx.x * kWavesPerBlock + wave;
    if (tile >= ntiles) return;  // no block-wide barrier below
    for (int i = lane; i < 256; i += kWave) base[wave][i] = offs[(int64_t)i * ntiles + tile];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    const uint64_t lt = __lanemask_lt();
    for (int c = 0; c < kChunks; ++c) {
        int64_t idx = tile * kTile + c * kWave + lane;
        bool valid = idx < n;
        uint32_t k = valid ? kin[idx] : 0u;
        uint32_t v = valid ? vin[idx] : 0u;
        uint32_t dig = (k >> shift) & 0xFFu;
        uint64_t act = __ballot(valid);
        if (act == 0) break;
        uint64_t peers = match_any(dig, 8, act);
        int32_t b = valid ? base[wave][dig] : 0;
        __builtin_amdgcn_wave_barrier();
        if (valid) {
            int32_t pos = b + (int32_t)__popcll(peers & lt);
            kout[pos] = k;
            vout[pos] = v;
            if ((peers & lt) == 0) base[wave][dig] = b + (int32_t)__popcll(peers);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
    }
}

__global__ void copy_pairs_kernel(const uint32_t* __restrict__ ks, const uint32_t* __restrict__ vs,
                                  uint32_t* __restrict__ kd, uint32_t* __restrict__ vd, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) { kd[i] = ks[i]; vd[i] = vs[i]; }
}

}  // namespace

int64_t radix_tmp_elems(int64_t n) {
    int64_t ntiles = ceil_div(n > 0 ? n : 1, kTile);
    int64_t h = 256 * ntiles;
    return round_up(h, 64) + scan_tmp_elems(h);
}

sky_status launch_radix_sort(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, int64_t n,
                             int key_bits, int32_t* tmp, hipStream_t st, const uint32_t** out_k,
                             const uint32_t** out_v) {
    if (out_k) *out_k = k0;
    if (out_v) *out_v = v0;
    if (n <= 1) return SKY_OK;
    const int64_t ntiles = ceil_div(n, kTile);
    const int64_t blocks = ceil_div(ntiles, kWavesPerBlock);
    int32_t* hist = tmp;
    int32_t* stmp = tmp + round_up(256 * ntiles, 64);
    int passes = (key_bits + 7) / 8;
    uint32_t *ka = k0, *va = v0, *kb = k1, *vb = v1;
    for (int p = 0; p < passes; ++p) {
        int shift = 8 * p;
        hipLaunchKernelGGL(radix_hist_kernel, dim3((uint32_t)blocks), dim3(kBlock), 0, st, ka, n,
                           shift, hist, ntiles);
        SKY_HIP(hipGetLastError());
        SKY_TRY(launch_exclusive_scan(hist, hist, 256 * ntiles, stmp, st));
        hipLaunchKernelGGL(radix_scatter_kernel, dim3((uint32_t)blocks), dim3(kBlock), 0, st, ka,
                           va, kb, vb, n, shift, (const int32_t*)hist, ntiles);
        SKY_HIP(hipGetLastError());
        uint32_t* t;
        t = ka; ka = kb; kb = t;
        t = va; va = vb; vb = t;
    }
    if (out_k && out_v) {  // the caller reads the result where the last pass left it
        *out_k = ka;
        *out_v = va;
        return SKY_OK;
    }
    if (ka != k0) {
        hipLaunchKernelGGL(copy_pairs_kernel, dim3((uint32_t)ceil_div(n, kBlock)), dim3(kBlock), 0,
                           st, ka, va, k0, v0, n);
        SKY_HIP(hipGetLastError());
    }
    return SKY_OK;
}

}  // namespace sky
