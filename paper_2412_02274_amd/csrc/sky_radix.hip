// Stable LSD radix sort of (uint32 key, uint32 value) pairs, 8-bit digits.
//
// One pass over tiles of 1024 or 4096 pairs (by the count) is three launches:
//   1. per-tile digit counts (wave-private LDS histograms), stored digit-major;
//   2. one workgroup per digit scans that digit's row of tile counts (exclusive, in place)
//      and records the digit's total;
//   3. every tile ranks its pairs by digit (each wave walks its quarter in order, 64 at a
//      time, ranking equal digits with ballots; waves are combined in wave order), sorts them
//      by digit in LDS, and writes each digit's run at that digit's global offset: consecutive
//      lanes write consecutive addresses, so the writes coalesce.
// Equal keys keep their input order. The item count may come from the device (a count an
// earlier kernel produced): the count and scatter grids are capped at 1024 workgroups that
// loop over the tiles below the count, so no pass waits on the host and a count far below the
// host's bound costs few empty workgroups.
#include "sky_internal.hpp"

namespace sky {

namespace {

constexpr int kRT = 4096;                            // pairs per tile (large counts)
constexpr int kRTSmall = 1024;                       // pairs per tile (counts up to kRBig)
constexpr int64_t kRBig = int64_t(1) << 21;
constexpr int kRWaves = kBlock / kWave;              // 4
constexpr int kRChunks = kRT / kRWaves / kWave;      // at most 16 chunks of 64 per wave
constexpr int kRPer = kRT / kBlock;                  // at most 16 pairs per thread in the count pass
constexpr int64_t kRGridCap = 1024;                  // most workgroups of a count or scatter launch

// Pairs per tile for a pass over n pairs (n known on the device): small tiles for small counts
// (more tiles in flight, each ranking a quarter as many chunks in sequence), large tiles for
// large counts (longer digit runs, so better coalesced writes). Every kernel of a pass derives
// the same value from the same count.
__device__ __forceinline__ int tile_pairs(int64_t n) { return n > kRBig ? kRT : kRTSmall; }

__device__ __forceinline__ int64_t item_count(const int32_t* n_dev, int64_t n_host) {
    if (!n_dev) return n_host;
    const int64_t c = *n_dev;
    return c < 0 ? 0 : (c < n_host ? c : n_host);
}

__global__ void __launch_bounds__(kBlock) rs_count_kernel(const uint32_t* __restrict__ keys,
                                                          const int32_t* __restrict__ n_dev, int64_t n_host,
                                                          int shift, int32_t* __restrict__ hist,
                                                          int64_t stride) {
    __shared__ int32_t cnt[kRWaves][256];
    const int64_t n = item_count(n_dev, n_host);
    const int T = tile_pairs(n);
    const int wave = threadIdx.x / kWave;
    // tiles blockIdx.x, + gridDim.x, ...: the grid is capped, so a count far below the bound
    // costs few empty workgroups
    for (int64_t tile = blockIdx.x; tile * T < n; tile += gridDim.x) {
        const int64_t t0 = tile * T;
        for (int i = (int)lane_id(); i < 256; i += kWave) cnt[wave][i] = 0;
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kRPer; ++i) {
            const int64_t idx = t0 + (int64_t)i * kBlock + threadIdx.x;
            if (i * kBlock < T && idx < n) atomicAdd(&cnt[wave][(keys[idx] >> shift) & 0xFFu], 1);
        }
        __syncthreads();
        const int dg = threadIdx.x;  // 256 threads, one digit each
        hist[(int64_t)dg * stride + tile] = cnt[0][dg] + cnt[1][dg] + cnt[2][dg] + cnt[3][dg];
        __syncthreads();  // cnt is cleared for the next tile
    }
}

// One workgroup per digit: exclusive scan of its tile counts in place, and its total.
__global__ void __launch_bounds__(kBlock) rs_scan_kernel(int32_t* __restrict__ hist, int64_t stride,
                                                         const int32_t* __restrict__ n_dev, int64_t n_host,
                                                         int32_t* __restrict__ totals) {
    __shared__ int32_t ws[kRWaves];
    const int64_t n = item_count(n_dev, n_host);
    const int T = tile_pairs(n);
    const int64_t nt = (n + T - 1) / T;
    int32_t* row = hist + (int64_t)blockIdx.x * stride;
    const int64_t per = (nt + kBlock - 1) / kBlock;
    const int64_t b0 = (int64_t)threadIdx.x * per;
    const int64_t b1 = b0 + per < nt ? b0 + per : nt;
    int32_t s = 0;
    for (int64_t i = b0; i < b1; ++i) s += row[i];
    int32_t total = 0;
    int32_t run = block_exscan(s, ws, &total);
    for (int64_t i = b0; i < b1; ++i) {
        const int32_t v = row[i];
        row[i] = run;
        run += v;
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kBlock) rs_scatter_kernel(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint32_t* __restrict__ kout,
    uint32_t* __restrict__ vout, const int32_t* __restrict__ n_dev, int64_t n_host, int shift,
    const int32_t* __restrict__ hist, int64_t stride, const int32_t* __restrict__ totals) {
    __shared__ uint32_t sk[kRT];
    __shared__ uint32_t sv[kRT];
    __shared__ int32_t wc[kRWaves][256];  // per-wave digit counts, then the waves' prefixes
    __shared__ int32_t dstart[256];       // first slot of each digit in the tile's sorted order
    __shared__ int32_t gbase[256];        // global position of that slot
    __shared__ int32_t ws[kRWaves];
    const int64_t n = item_count(n_dev, n_host);
    const int T = tile_pairs(n);
    const int nch = T / (kRWaves * kWave);  // chunks of 64 per wave: 4 or 16
    const int wave = threadIdx.x / kWave;
    const int lane = (int)lane_id();
    // tiles blockIdx.x, + gridDim.x, ... (the grid is capped, as for the counts)
    for (int64_t tile = blockIdx.x; tile * T < n; tile += gridDim.x) {
        const int64_t t0 = tile * T;
        __syncthreads();  // the previous tile's LDS is free
        for (int i = lane; i < 256; i += kWave) wc[wave][i] = 0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        // 1. the wave's share of the tile in order, ranked inside the wave by digit
        const int64_t w0 = t0 + (int64_t)wave * nch * kWave;
        uint32_t k[kRChunks], v[kRChunks];
        int32_t r[kRChunks];
#pragma unroll
        for (int c = 0; c < kRChunks; ++c) {
            const int64_t idx = w0 + c * kWave + lane;
            const bool in = c < nch && idx < n;
            k[c] = in ? kin[idx] : 0u;
            v[c] = in ? vin[idx] : 0u;
        }
        const uint64_t lt = __lanemask_lt();
#pragma unroll
        for (int c = 0; c < kRChunks; ++c) {
            r[c] = 0;
            if (c < nch) {  // (uniform)
                const bool valid = w0 + c * kWave + lane < n;
                const uint64_t act = __ballot(valid);
                const uint32_t dg = (k[c] >> shift) & 0xFFu;
                const uint64_t peers = match_any(dg, 8, act);
                const int32_t b = valid ? wc[wave][dg] : 0;
                __builtin_amdgcn_wave_barrier();
                r[c] = b + (int32_t)__popcll(peers & lt);
                if (valid && (peers & lt) == 0) wc[wave][dg] = b + (int32_t)__popcll(peers);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                __builtin_amdgcn_wave_barrier();
            }
        }
        __syncthreads();
        // 2. per digit (thread = digit): wave prefixes, the tile's digit starts, global bases
        {
            const int dg = threadIdx.x;
            const int32_t c0 = wc[0][dg], c1 = wc[1][dg], c2 = wc[2][dg], c3 = wc[3][dg];
            int32_t unused = 0;
            const int32_t st = block_exscan(c0 + c1 + c2 + c3, ws, &unused);
            const int32_t gpre = block_exscan(totals[dg], ws, &unused);
            wc[0][dg] = 0;
            wc[1][dg] = c0;
            wc[2][dg] = c0 + c1;
            wc[3][dg] = c0 + c1 + c2;
            dstart[dg] = st;
            gbase[dg] = gpre + hist[(int64_t)dg * stride + tile];
        }
        __syncthreads();
        // 3. the tile sorted by digit in LDS
#pragma unroll
        for (int c = 0; c < kRChunks; ++c) {
            if (c < nch && w0 + c * kWave + lane < n) {
                const uint32_t dg = (k[c] >> shift) & 0xFFu;
                const int32_t lp = dstart[dg] + wc[wave][dg] + r[c];
                sk[lp] = k[c];
                sv[lp] = v[c];
            }
        }
        __syncthreads();
        // 4. every digit's run written at its global offset
        const int32_t cnt = n - t0 < T ? (int32_t)(n - t0) : T;
        for (int32_t j = threadIdx.x; j < cnt; j += kBlock) {
            const uint32_t kk = sk[j];
            const uint32_t dg = (kk >> shift) & 0xFFu;
            const int64_t o = (int64_t)gbase[dg] + (j - dstart[dg]);
            kout[o] = kk;
            vout[o] = sv[j];
        }
    }
}

__global__ void copy_pairs_kernel(const uint32_t* __restrict__ ks, const uint32_t* __restrict__ vs,
                                  uint32_t* __restrict__ kd, uint32_t* __restrict__ vd,
                                  const int32_t* __restrict__ n_dev, int64_t n_host) {
    const int64_t n = item_count(n_dev, n_host);
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) { kd[i] = ks[i]; vd[i] = vs[i]; }
}

// hist columns: enough for the small tiles of any count up to n
int64_t tile_stride(int64_t n) { return round_up(ceil_div(n > 0 ? n : 1, kRTSmall), 64); }

}  // namespace

int64_t radix_tmp_elems(int64_t n) { return 256 * tile_stride(n) + 256; }

sky_status launch_radix_sort(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, int64_t n,
                             int key_bits, int32_t* tmp, hipStream_t st, const uint32_t** out_k,
                             const uint32_t** out_v, const int32_t* n_dev) {
    if (out_k) *out_k = k0;
    if (out_v) *out_v = v0;
    if (n <= 1 && !n_dev) return SKY_OK;
    if (n <= 0) return SKY_OK;
    const int64_t stride = tile_stride(n);
    const int64_t ntiles = ceil_div(n, n > kRBig ? kRT : kRTSmall);  // at most what the device count needs
    const uint32_t tiles = (uint32_t)(ntiles < kRGridCap ? ntiles : kRGridCap);
    int32_t* hist = tmp;
    int32_t* totals = tmp + 256 * stride;
    const int passes = (key_bits + 7) / 8;
    uint32_t *ka = k0, *va = v0, *kb = k1, *vb = v1;
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        hipLaunchKernelGGL(rs_count_kernel, dim3(tiles), dim3(kBlock), 0, st, ka, n_dev, n, shift, hist, stride);
        hipLaunchKernelGGL(rs_scan_kernel, dim3(256), dim3(kBlock), 0, st, hist, stride, n_dev, n, totals);
        hipLaunchKernelGGL(rs_scatter_kernel, dim3(tiles), dim3(kBlock), 0, st, ka, va, kb, vb, n_dev, n, shift,
                           (const int32_t*)hist, stride, (const int32_t*)totals);
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
        hipLaunchKernelGGL(copy_pairs_kernel, dim3((uint32_t)ceil_div(n, kBlock)), dim3(kBlock), 0, st, ka, va,
                           k0, v0, n_dev, n);
        SKY_HIP(hipGetLastError());
    }
    return SKY_OK;
}

}  // namespace sky
