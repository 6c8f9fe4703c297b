// Upper end of Alg. 1's level range (Sec. 3.2): ell, the smallest non-zero difference between
// two values of one attribute over all pairs of rows, and g_bar = floor(1 / ell).
//
// Per attribute, the canonical values' 32-bit patterns are radix-sorted (non-negative floats
// order like their patterns, and canonical values are below 2^30 as patterns, so 4 digit
// passes). In sorted order the smallest non-zero difference is between neighbours. Each
// neighbour gap is taken in FP64 and min-reduced into one 64-bit word: the pattern of a
// positive double orders like the double, so an unsigned atomic minimum is the minimum.
// Bound: HBM (the sort's passes over 8-byte pairs, then one read of the sorted keys).
#include "sky_internal.hpp"

namespace sky {

namespace {

constexpr unsigned long long kInfBits = 0x7FF0000000000000ull;  // +inf as a double pattern
constexpr int kGapGrid = 1024;                                 // blocks of the gap pass

__global__ void __launch_bounds__(kBlock) gbar_init_kernel(unsigned long long* minbits) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *minbits = kInfBits;
}

__global__ void __launch_bounds__(kBlock) gbar_keys_kernel(const float* __restrict__ x, int64_t n,
                                                            uint32_t* __restrict__ keys,
                                                            uint32_t* __restrict__ vals,
                                                            int32_t* dev_status) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    bool bad = false;
    if (i < n) {
        const float v = x[i];
        bad = !in_domain(v);
        keys[i] = bad ? 0u : fbits(canon(v));
        vals[i] = (uint32_t)i;
    }
    if (__ballot(bad) && lane_id() == 0) raise_status(dev_status, SKY_ERR_DOMAIN);
}

// The value of a canonical FP32 pattern as a double, built from its fields (exact, and
// independent of how the FP32 denormal mode treats subnormal inputs).
__device__ __forceinline__ double pattern_value(uint32_t b) {
    const uint32_t e = b >> 23, m = b & 0x7FFFFFu;
    const int32_t ex = e == 0 ? -149 : (int32_t)e - 150;  // value = mant * 2^ex
    const uint32_t mant = e == 0 ? m : (m | 0x800000u);
    const double scale = __longlong_as_double((long long)((uint64_t)(ex + 1023) << 52));
    return (double)mant * scale;
}

__global__ void __launch_bounds__(kBlock) gbar_gap_kernel(const uint32_t* __restrict__ keys,
                                                           int64_t n,
                                                           unsigned long long* minbits) {
    __shared__ unsigned long long part[kBlock / kWave];
    unsigned long long m = kInfBits;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x + 1; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const uint32_t a = keys[i - 1], b = keys[i];
        if (a != b) {
            const double e = __dsub_rn(pattern_value(b), pattern_value(a));  // > 0: b > a
            const unsigned long long eb = (unsigned long long)__double_as_longlong(e);
            m = eb < m ? eb : m;
        }
    }
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(m, off);
        m = o < m ? o : m;
    }
    if (lane_id() == 0) part[threadIdx.x / kWave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / kWave; ++w) m = part[w] < m ? part[w] : m;
        if (m < kInfBits) atomicMin(minbits, m);
    }
}

__global__ void gbar_final_kernel(const unsigned long long* __restrict__ minbits,
                                  double* __restrict__ ell, int64_t* __restrict__ g_bar) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const unsigned long long b = *minbits;
    const double e = __longlong_as_double((long long)b);
    if (ell) *ell = e;
    int64_t g = 1;  // no ell: every level is alike, nothing to search above 1
    if (b < kInfBits) {
        const double r = floor(__ddiv_rn(1.0, e));
        g = r >= 0x1p62 ? ((int64_t)1 << 62) : (int64_t)r;
    }
    if (g_bar) *g_bar = g;
}

}  // namespace

void carve_gbar(Carver& c, GbarBuffers& b, int64_t n) {
    const int64_t m = n > 0 ? n : 1;
    b.k0 = c.take<uint32_t>((size_t)m);
    b.v0 = c.take<uint32_t>((size_t)m);
    b.k1 = c.take<uint32_t>((size_t)m);
    b.v1 = c.take<uint32_t>((size_t)m);
    b.radix_tmp = c.take<int32_t>((size_t)radix_tmp_elems(m));
    b.minbits = c.take<unsigned long long>(1);
}

sky_status launch_gbar(const float* x, int64_t n, int32_t d, int64_t ld, const GbarBuffers& b,
                       double* ell, int64_t* g_bar, int32_t* dev_status, hipStream_t st) {
    hipLaunchKernelGGL(gbar_init_kernel, dim3(1), dim3(kWave), 0, st, b.minbits);
    SKY_HIP(hipGetLastError());
    if (n >= 2) {
        const int64_t gap_blocks = ceil_div(n, kBlock);
        for (int32_t k = 0; k < d; ++k) {
            hipLaunchKernelGGL(gbar_keys_kernel, dim3((uint32_t)ceil_div(n, kBlock)), dim3(kBlock), 0, st,
                               x + (int64_t)k * ld, n, b.k0, b.v0, dev_status);
            SKY_HIP(hipGetLastError());
            SKY_TRY(launch_radix_sort(b.k0, b.v0, b.k1, b.v1, n, 30, b.radix_tmp, st));
            hipLaunchKernelGGL(gbar_gap_kernel,
                               dim3((uint32_t)(gap_blocks < kGapGrid ? gap_blocks : kGapGrid)),
                               dim3(kBlock), 0, st, (const uint32_t*)b.k0, n, b.minbits);
            SKY_HIP(hipGetLastError());
        }
    }
    hipLaunchKernelGGL(gbar_final_kernel, dim3(1), dim3(kWave), 0, st,
                       (const unsigned long long*)b.minbits, ell, g_bar);
    SKY_HIP(hipGetLastError());
    return SKY_OK;
}

}  // namespace sky
