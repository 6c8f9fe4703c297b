// Exclusive prefix sum of int32 values (totals must fit in int32), used for partition and
// histogram offsets. Three phases per level: block sums, scan of the block sums (recursive),
// block-local scan plus the block's offset. Each block covers kChunk consecutive values,
// staged through LDS so that global reads and writes are coalesced. in == out is allowed.
#include "sky_internal.hpp"

namespace sky {

namespace {

constexpr int kPer = 16;
constexpr int kChunk = kBlock * kPer;  // 4096 values per block

// Exclusive scan of one value per thread across the workgroup; returns the block total.
__device__ int32_t block_exclusive_scan(int32_t v, int32_t* excl) {
    __shared__ int32_t wsum[kBlock / kWave];
    const int lane = (int)lane_id();
    const int wave = threadIdx.x / kWave;
    int32_t inc = v;
    for (int off = 1; off < kWave; off <<= 1) {
        int32_t o = __shfl_up(inc, off, kWave);
        if (lane >= off) inc += o;
    }
    if (lane == kWave - 1) wsum[wave] = inc;
    __syncthreads();
    int32_t before = 0, total = 0;
    for (int w = 0; w < kBlock / kWave; ++w) {
        if (w < wave) before += wsum[w];
        total += wsum[w];
    }
    *excl = before + inc - v;
    __syncthreads();
    return total;
}

__global__ void __launch_bounds__(kBlock) block_sums_kernel(const int32_t* __restrict__ in,
                                                             int64_t n, int32_t* __restrict__ sums) {
    const int64_t base = (int64_t)blockIdx.x * kChunk;
    int32_t acc = 0;
    for (int i = threadIdx.x; i < kChunk; i += kBlock) {
        int64_t g = base + i;
        if (g < n) acc += in[g];
    }
    int32_t excl;
    int32_t total = block_exclusive_scan(acc, &excl);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kBlock) block_scan_kernel(const int32_t* in, int64_t n,
                                                             const int32_t* __restrict__ offs,
                                                             int32_t* out) {
    __shared__ int32_t buf[kChunk];
    const int64_t base = (int64_t)blockIdx.x * kChunk;
    for (int i = threadIdx.x; i < kChunk; i += kBlock) {
        int64_t g = base + i;
        buf[i] = g < n ? in[g] : 0;
    }
    __syncthreads();
    int32_t local[kPer];
    int32_t acc = 0;
    for (int j = 0; j < kPer; ++j) {
        local[j] = buf[threadIdx.x * kPer + j];
        acc += local[j];
    }
    int32_t excl;
    block_exclusive_scan(acc, &excl);
    int32_t run = excl + (offs ? offs[blockIdx.x] : 0);
    for (int j = 0; j < kPer; ++j) {
        buf[threadIdx.x * kPer + j] = run;
        run += local[j];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kChunk; i += kBlock) {
        int64_t g = base + i;
        if (g < n) out[g] = buf[i];
    }
}

}  // namespace

int64_t scan_tmp_elems(int64_t n) {
    int64_t total = 0;
    int64_t m = n;
    while (m > kChunk) {
        m = ceil_div(m, kChunk);
        total += round_up(m, 64);
    }
    return total + 64;
}

sky_status launch_exclusive_scan(const int32_t* in, int32_t* out, int64_t n, int32_t* tmp,
                                 hipStream_t st) {
    if (n <= 0) return SKY_OK;
    int64_t blocks = ceil_div(n, kChunk);
    if (blocks == 1) {
        hipLaunchKernelGGL(block_scan_kernel, dim3(1), dim3(kBlock), 0, st, in, n,
                           (const int32_t*)nullptr, out);
        SKY_HIP(hipGetLastError());
        return SKY_OK;
    }
    int32_t* sums = tmp;
    int32_t* rest = tmp + round_up(blocks, 64);
    hipLaunchKernelGGL(block_sums_kernel, dim3((uint32_t)blocks), dim3(kBlock), 0, st, in, n, sums);
    SKY_HIP(hipGetLastError());
    SKY_TRY(launch_exclusive_scan(sums, sums, blocks, rest, st));
    hipLaunchKernelGGL(block_scan_kernel, dim3((uint32_t)blocks), dim3(kBlock), 0, st, in, n,
                       (const int32_t*)sums, out);
    SKY_HIP(hipGetLastError());
    return SKY_OK;
}

}  // namespace sky
