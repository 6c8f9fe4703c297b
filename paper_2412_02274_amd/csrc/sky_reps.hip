// Representative Filtering (Sec. 3.1): a few strong rows shared by every partition, so that the
// rows they dominate leave the local skylines early.
//
// The representatives are the k rows with the smallest FP32 attribute sum (the plan's score,
// summed in attribute order), equal sums in row order: a stable radix sort of (score pattern,
// row) pairs in row order (non-negative floats order like their patterns). Those dominated by
// another representative add no pruning power and are dropped (an all-pairs test over at most
// SKY_MAX_REPS rows, staged through LDS). Every position is then tested against the kept
// representatives; the survivors form the local phase's initial item list.
// Bound: the sort (HBM); the tests are n x kept compares.
#include "sky_internal.hpp"

namespace sky {

namespace {

constexpr int kRepChunk = 256;  // representatives staged in LDS at a time

__global__ void zero_counters_kernel(int32_t* __restrict__ nkept, unsigned long long* __restrict__ tests) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *nkept = 0;
        *tests = 0;
    }
}

__global__ void __launch_bounds__(kBlock) rep_keys_kernel(const float* __restrict__ fsum,
                                                          const int32_t* __restrict__ rowid, int32_t n,
                                                          uint32_t* __restrict__ keys,
                                                          uint32_t* __restrict__ vals) {
    const int32_t p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= n) return;
    const int32_t row = rowid[p];
    keys[row] = fbits(fsum[p]);  // f >= 0
    vals[row] = (uint32_t)row;
}

// The values of row `row` from the row-major staging copy (stride rs floats).
__device__ __forceinline__ void rep_row(const float* __restrict__ xa, int32_t rs, int32_t d, int32_t row,
                                        float* v) {
    for (int k = 0; k < d; ++k) v[k] = xa[(int64_t)row * rs + k];
}

__device__ __forceinline__ bool dominates_f(const float* s, const float* t, int d) {
    bool le = true, lt = false;
    for (int k = 0; k < d; ++k) {
        le &= s[k] <= t[k];
        lt |= s[k] < t[k];
    }
    return le && lt;
}

// kept[j] = 1 when no other representative dominates representative j (rows[0, k))
__global__ void __launch_bounds__(kBlock) rep_skyline_kernel(const float* __restrict__ xa, int32_t rs,
                                                             int32_t d, const uint32_t* __restrict__ rows,
                                                             int32_t k, int32_t* __restrict__ kept,
                                                             int32_t* __restrict__ nkept) {
    __shared__ float cv[kRepChunk * SKY_MAX_D];
    const int32_t j = blockIdx.x * kBlock + threadIdx.x;
    float t[SKY_MAX_D];
    if (j < k) rep_row(xa, rs, d, (int32_t)rows[j], t);
    bool dom = false;
    for (int32_t c0 = 0; c0 < k; c0 += kRepChunk) {
        const int32_t cn = k - c0 < kRepChunk ? k - c0 : kRepChunk;
        __syncthreads();
        for (int32_t e = threadIdx.x; e < cn * d; e += kBlock) {
            const int32_t q = e / d, a = e - q * d;
            cv[q * d + a] = xa[(int64_t)rows[c0 + q] * rs + a];
        }
        __syncthreads();
        if (j < k && !dom)
            for (int32_t q = 0; q < cn && !dom; ++q)
                if (c0 + q != j) dom = dominates_f(cv + q * d, t, d);
    }
    if (j < k) {
        kept[j] = dom ? 0 : 1;
        if (!dom) atomicAdd(nkept, 1);
    }
}

// keep[p] = 1 for positions no kept representative dominates (0 for the others); tests holds
// the row-against-representative tests made (each row stops at its first dominator), and
// seg_tests (when given) the same tests per segment of the rows. Rows of skipped segments
// (pruned Grid cells, which the local phase disregards) are not tested.
__global__ void __launch_bounds__(kBlock) rep_filter_kernel(const float* __restrict__ xp, int64_t ldp,
                                                            int32_t d, int32_t n,
                                                            const float* __restrict__ xa, int32_t rs,
                                                            const uint32_t* __restrict__ rows,
                                                            const int32_t* __restrict__ kept, int32_t k,
                                                            uint8_t* __restrict__ keep,
                                                            unsigned long long* __restrict__ tests,
                                                            const int32_t* __restrict__ seg_of_pos,
                                                            unsigned long long* __restrict__ seg_tests,
                                                            const uint8_t* __restrict__ skip_seg) {
    __shared__ float cv[kRepChunk * SKY_MAX_D];
    __shared__ int32_t cok[kRepChunk];
    const int32_t p = blockIdx.x * kBlock + threadIdx.x;
    const int32_t sg = (seg_of_pos && p < n) ? seg_of_pos[p] : 0;
    const bool act = p < n && !(skip_seg && skip_seg[sg]);
    float t[SKY_MAX_D];
    if (act)
        for (int a = 0; a < d; ++a) t[a] = xp[(int64_t)a * ldp + p];
    bool dom = false;
    unsigned long long nt = 0;
    for (int32_t c0 = 0; c0 < k; c0 += kRepChunk) {
        const int32_t cn = k - c0 < kRepChunk ? k - c0 : kRepChunk;
        __syncthreads();
        for (int32_t e = threadIdx.x; e < cn * d; e += kBlock) {
            const int32_t q = e / d, a = e - q * d;
            cv[q * d + a] = xa[(int64_t)rows[c0 + q] * rs + a];
        }
        for (int32_t q = threadIdx.x; q < cn; q += kBlock) cok[q] = kept[c0 + q];
        __syncthreads();
        if (act && !dom)
            for (int32_t q = 0; q < cn && !dom; ++q)
                if (cok[q]) {
                    ++nt;
                    dom = dominates_f(cv + q * d, t, d);
                }
    }
    if (p < n) keep[p] = dom ? 0 : 1;
    // per segment: one add per wave when its rows share a segment (segments are runs of
    // positions, so nearly every wave does), else one per lane
    const int32_t s0 = __shfl(sg, 0);
    const bool mixed = __builtin_amdgcn_ballot_w64(p < n && sg != s0) != 0;
    if (seg_tests && mixed && nt) atomicAdd(&seg_tests[sg], nt);
    for (int off = kWave / 2; off > 0; off >>= 1) nt += __shfl_xor(nt, off);
    if (lane_id() == 0 && nt) {
        atomicAdd(tests, nt);
        if (seg_tests && !mixed) atomicAdd(&seg_tests[s0], nt);
    }
}

}  // namespace

sky_status launch_representatives(const RepArgs& a, hipStream_t st) {
    const uint32_t nb = (uint32_t)ceil_div(a.n, kBlock);
    hipLaunchKernelGGL(rep_keys_kernel, dim3(nb), dim3(kBlock), 0, st, a.fsum, a.rowid, a.n, a.k0, a.v0);
    SKY_HIP(hipGetLastError());
    const uint32_t* sorted_rows = nullptr;
    const uint32_t* sorted_keys = nullptr;
    SKY_TRY(launch_radix_sort(a.k0, a.v0, a.k1, a.v1, a.n, 32, a.radix_tmp, st, &sorted_keys, &sorted_rows));
    const int32_t k = a.k < a.n ? a.k : a.n;
    hipLaunchKernelGGL(zero_counters_kernel, dim3(1), dim3(kWave), 0, st, a.nkept, a.tests);
    hipLaunchKernelGGL(rep_skyline_kernel, dim3((uint32_t)ceil_div(k, kBlock)), dim3(kBlock), 0, st, a.xa,
                       a.rs, a.d, sorted_rows, k, a.kept, a.nkept);
    hipLaunchKernelGGL(rep_filter_kernel, dim3(nb), dim3(kBlock), 0, st, a.xp, a.ldp, a.d, a.n, a.xa, a.rs,
                       sorted_rows, (const int32_t*)a.kept, k, a.keep, a.tests,
                       a.seg_of_pos, a.seg_tests, a.skip_seg);
    SKY_HIP(hipGetLastError());
    return SKY_OK;
}

}  // namespace sky
