// Input step: row-major FP32 relation -> validated, canonical structure-of-arrays copy.
// The domain is the one the paper assumes for its data (values in [0, 1), Sec. 3.1 / Sec. 4).
//
// Bound: HBM (4d bytes read + 4d bytes written per row). Each workgroup stages a tile of
// 256 rows through LDS so that both the row-major reads and the SoA writes are coalesced.
#include "sky_internal.hpp"

namespace sky {

namespace {

constexpr int kRows = 256;  // rows per workgroup tile

__global__ void __launch_bounds__(kBlock) ingest_kernel(const float* __restrict__ x_rows,
                                                         int64_t n, int32_t d,
                                                         float* __restrict__ x_soa, int64_t ld,
                                                         int32_t* dev_status) {
    __shared__ float tile[SKY_MAX_D * (kRows + 1)];
    const int64_t row0 = (int64_t)blockIdx.x * kRows;
    const int rows = (int)((n - row0) < kRows ? (n - row0) : kRows);
    const int elems = rows * d;
    bool bad = false;
    // coalesced read of the contiguous block of rows*d floats
    const float* src = x_rows + row0 * d;
    for (int e = threadIdx.x; e < elems; e += kBlock) {
        float v = src[e];
        bad |= !in_domain(v);
        int r = e / d;
        int k = e - r * d;
        tile[k * (kRows + 1) + r] = canon(v);
    }
    __syncthreads();
    // coalesced SoA writes
    for (int k = 0; k < d; ++k)
        for (int r = threadIdx.x; r < rows; r += kBlock)
            x_soa[(int64_t)k * ld + row0 + r] = tile[k * (kRows + 1) + r];
    if (__ballot(bad) != 0 && lane_id() == 0) raise_status(dev_status, SKY_ERR_DOMAIN);
}

}  // namespace

sky_status launch_ingest(const float* x_rows, int64_t n, int32_t d, float* x_soa, int64_t ld,
                         int32_t* dev_status, hipStream_t st) {
    if (n == 0) return SKY_OK;
    int64_t blocks = ceil_div(n, kRows);
    hipLaunchKernelGGL(ingest_kernel, dim3((uint32_t)blocks), dim3(kBlock), 0, st, x_rows, n, d,
                       x_soa, ld, dev_status);
    SKY_HIP(hipGetLastError());
    return SKY_OK;
}

}  // namespace sky
