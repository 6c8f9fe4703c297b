// Input step: row-major FP32 relation -> validated, canonical structure-of-arrays copy.
// The domain is the one the paper assumes for its data (values in [0, 1), Sec. 3.1 / Sec. 4).
//
// Bound: HBM (4d bytes read + 4d bytes written per row). Each workgroup stages a tile of
// 256 rows through LDS so that both the row-major reads and the SoA writes are coalesced.
#include "sky_internal.hpp"

namespace sky {

namespace {

constexpr int kRows = 256;  // rows per workgroup tile

// D > 0: d known at compile time (the row/attribute split of an element index is then a
// division by a constant); D = 0: any d.
template <int D>
__global__ void __launch_bounds__(kBlock) ingest_kernel(const float* __restrict__ x_rows,
                                                         int64_t n, int32_t d_rt,
                                                         float* __restrict__ x_soa, int64_t ld,
                                                         int32_t* dev_status) {
    __shared__ float tile[SKY_MAX_D * (kRows + 1)];
    const int d = D > 0 ? D : d_rt;
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

// Grid projection (Def. 2) of the rows rows[0, s) at level g, as a relation of its own:
// out[k*ld_out + j] = floor(fl32(x[k][rows[j]] * g)) * 2^-b with 2^b >= g. The scale keeps the
// values in [0, 1) and exact in FP32 (keys < 2^24), and orders them like floor(t g) / g.
__global__ void __launch_bounds__(kBlock) project_kernel(const float* __restrict__ x, int64_t n, int32_t d,
                                                          int64_t ld, const int64_t* __restrict__ rows,
                                                          int64_t s, int32_t g, float scale,
                                                          float* __restrict__ out, int64_t ld_out,
                                                          int32_t* dev_status) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    bool bad_idx = false, bad_val = false;
    if (j < s) {
        const int64_t row = rows[j];
        bad_idx = row < 0 || row >= n;
        const float fg = (float)g;
        for (int k = 0; k < d; ++k) {
            const float v = bad_idx ? 0.0f : x[(int64_t)k * ld + row];
            bad_val |= !in_domain(v);
            out[(int64_t)k * ld_out + j] = __fmul_rn((float)qkey(canon(v), fg), scale);
        }
    }
    if (__ballot(bad_idx) && lane_id() == 0) raise_status(dev_status, SKY_ERR_INVALID_ARG);
    if (__ballot(bad_val) && lane_id() == 0) raise_status(dev_status, SKY_ERR_DOMAIN);
}

}  // namespace

// One level of Alg. 1 as written: a tuple whose projection is not in the skyline of the
// projected candidates at level g, and that has no level yet (0), exits at g; *nil_left (if
// given) gets the number of tuples still without a level added to it. Level 1 ends the scan:
// every tuple without a level gets 1 (it never left the skyline).
__global__ void __launch_bounds__(kBlock) literal_level_kernel(const uint8_t* __restrict__ member, int64_t s,
                                                                int32_t g, int32_t* __restrict__ g_exit,
                                                                int32_t* __restrict__ nil_left) {
    int32_t left = 0;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < s; j += (int64_t)gridDim.x * kBlock) {
        if (g_exit[j] != 0) continue;
        if (g == 1 || !member[j]) g_exit[j] = g;
        else ++left;
    }
    if (nil_left) {
        for (int off = kWave / 2; off > 0; off >>= 1) left += __shfl_xor(left, off, kWave);
        if (lane_id() == 0 && left) atomicAdd(nil_left, left);
    }
}

sky_status launch_literal_level(const uint8_t* member, int64_t s, int32_t g, int32_t* g_exit, int32_t* nil_left,
                                hipStream_t st) {
    if (s <= 0) return SKY_OK;
    const int64_t b = ceil_div(s, kBlock);
    hipLaunchKernelGGL(literal_level_kernel, dim3((uint32_t)(b > 1024 ? 1024 : b)), dim3(kBlock), 0, st, member, s,
                       g, g_exit, nil_left);
    SKY_HIP(hipGetLastError());
    return SKY_OK;
}

sky_status launch_project(const float* x, int64_t n, int32_t d, int64_t ld, const int64_t* rows,
                          int64_t s, int32_t g, float* out, int64_t ld_out, int32_t* dev_status,
                          hipStream_t st) {
    if (s <= 0) return SKY_OK;
    int b = 0;
    while ((int64_t(1) << b) < g) ++b;
    const float scale = ldexpf(1.0f, -b);
    hipLaunchKernelGGL(project_kernel, dim3((uint32_t)ceil_div(s, kBlock)), dim3(kBlock), 0, st, x, n, d,
                       ld, rows, s, g, scale, out, ld_out, dev_status);
    SKY_HIP(hipGetLastError());
    return SKY_OK;
}

sky_status launch_ingest(const float* x_rows, int64_t n, int32_t d, float* x_soa, int64_t ld,
                         int32_t* dev_status, hipStream_t st) {
    if (n == 0) return SKY_OK;
    int64_t blocks = ceil_div(n, kRows);
    switch (d) {
#define SKY_INGEST_D(DD) \
        case DD: hipLaunchKernelGGL(ingest_kernel<DD>, dim3((uint32_t)blocks), dim3(kBlock), 0, st, x_rows, n, d, \
                                    x_soa, ld, dev_status); break;
        SKY_INGEST_D(1) SKY_INGEST_D(2) SKY_INGEST_D(3) SKY_INGEST_D(4)
        SKY_INGEST_D(5) SKY_INGEST_D(6) SKY_INGEST_D(7) SKY_INGEST_D(8)
#undef SKY_INGEST_D
        default:
            hipLaunchKernelGGL(ingest_kernel<0>, dim3((uint32_t)blocks), dim3(kBlock), 0, st, x_rows, n, d, x_soa,
                               ld, dev_status);
    }
    SKY_HIP(hipGetLastError());
    return SKY_OK;
}

}  // namespace sky
