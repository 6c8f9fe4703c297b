// Measurement aids, not part of the path: probes of the two rates the kernels' rooflines are
// priced against, measured on the device itself.
//  * VALU: 32-bit integer add / xor / max / min (the dominance test's instruction mix) in four
//    independent chains per lane, so that every lane issues one full-rate VALU op per cycle of
//    its SIMD when the chip is saturated. Each loop iteration is 24 ops per lane.
//  * HBM: a streaming 16-byte copy (every byte read once and written once).
#include "sky_internal.hpp"

namespace sky {

namespace {

constexpr int kProbeChains = 4;
constexpr int kProbeOpsPerChain = 6;  // add, max, xor, xor, min, add

__global__ void __launch_bounds__(kBlock) valu_probe_kernel(int64_t iters, uint32_t salt,
                                                             uint32_t* __restrict__ sink) {
    uint32_t a[kProbeChains], b[kProbeChains];
#pragma unroll
    for (int c = 0; c < kProbeChains; ++c) {
        a[c] = (uint32_t)threadIdx.x * 2654435761u + salt + (uint32_t)c;
        b[c] = (uint32_t)blockIdx.x * 40503u ^ (salt + 17u * (uint32_t)c);
    }
    for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < kProbeChains; ++c) {
            // loop-carried and data-dependent, so nothing folds across iterations
            const int32_t x = (int32_t)(a[c] + 0x9E3779B9u);
            a[c] = (uint32_t)max(x, (int32_t)b[c]) ^ 0x85EBCA6Bu;
            const int32_t y = (int32_t)(b[c] ^ 0xC2B2AE35u);
            b[c] = (uint32_t)min(y, (int32_t)a[c]) + 0x27D4EB2Fu;
        }
    }
    uint32_t r = 0;
#pragma unroll
    for (int c = 0; c < kProbeChains; ++c) r ^= a[c] ^ b[c];
    // one word per workgroup keeps the chains live
    r = __shfl_xor(r, 1, kWave) ^ r;
    if (threadIdx.x == 0) sink[blockIdx.x] = r;
}

__global__ void __launch_bounds__(kBlock) copy_probe_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                             int64_t n16) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n16; i += (int64_t)gridDim.x * kBlock)
        dst[i] = src[i];
}

}  // namespace

}  // namespace sky

using namespace sky;

extern "C" {

sky_status sky_probe_valu(int64_t iters, int32_t grid, uint32_t* sink, void* ev_begin, void* ev_end,
                          void* stream, int64_t* lane_ops) {
    if (iters < 1 || grid < 1 || !sink || !lane_ops || (!ev_begin) != (!ev_end)) return SKY_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    if (ev_begin) SKY_HIP(hipEventRecord((hipEvent_t)ev_begin, st));
    hipLaunchKernelGGL(valu_probe_kernel, dim3((uint32_t)grid), dim3(kBlock), 0, st, iters, 0x5EEDu, sink);
    SKY_HIP(hipGetLastError());
    if (ev_end) SKY_HIP(hipEventRecord((hipEvent_t)ev_end, st));
    *lane_ops = (int64_t)grid * kBlock * iters * kProbeChains * kProbeOpsPerChain;
    return SKY_OK;
}

sky_status sky_probe_copy(const void* src, void* dst, int64_t bytes, void* ev_begin, void* ev_end, void* stream) {
    if (!src || !dst || bytes < 16 || (bytes & 15) || ((uintptr_t)src & 15) || ((uintptr_t)dst & 15) ||
        (!ev_begin) != (!ev_end))
        return SKY_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    const int64_t n16 = bytes / 16;
    const int64_t want = ceil_div(n16, kBlock);
    if (ev_begin) SKY_HIP(hipEventRecord((hipEvent_t)ev_begin, st));
    hipLaunchKernelGGL(copy_probe_kernel, dim3((uint32_t)(want < 16384 ? want : 16384)), dim3(kBlock), 0, st,
                       reinterpret_cast<const uint4*>(src), reinterpret_cast<uint4*>(dst), n16);
    SKY_HIP(hipGetLastError());
    if (ev_end) SKY_HIP(hipEventRecord((hipEvent_t)ev_end, st));
    return SKY_OK;
}

}  // extern "C"
