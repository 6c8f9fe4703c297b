// Partition assignment and the partition-contiguous copy (Sec. 3.1).
//
//  Grid     partition of t = sum_k floor(t_k * m) * m^k (first attribute fastest), the
//           coordinate taken with one FP32 multiply and clamped to m-1; cells that a
//           non-empty cell grid-dominates (Def. 3: strictly smaller coordinate in every
//           dimension) are flagged as pruned.
//  Angular  Eq. (1): partition = sum_a floor(2 phi_a m / pi) * m^a over the d-1 hyper-
//           spherical angles phi_a = atan2(sqrt(sum_{j>a} t_j^2), t_a) in [0, pi/2]. The
//           bucket is evaluated without trigonometry: floor(2 phi m / pi) counts the k >= 1
//           with phi >= k pi/(2m), i.e. (tan is increasing on [0, pi/2)) with
//           sum_{j>a} t_j^2 >= t_a^2 tan^2(k pi/(2m)); found by binary search over a table of
//           tan^2 values, in double precision; clamped to m-1; a zero sub-vector has angle 0.
//  Sliced   rows ordered by (t[dim], row index); the i-th (0-based) goes to floor(i p / n).
//  None     one partition.
//
// Every path validates the domain (SKY_ERR_DOMAIN) and writes a canonical SoA copy in partition
// order, with the rows of each partition along a Hilbert curve (a stable radix sort of the
// Hilbert keys followed by a stable counting sort by partition), the original row of every
// position, its partition, and the FP32 attribute sum used as the monotone score that orders
// the skyline filter (Sec. 2, scoring function). The spatial order inside partitions keeps
// the tile boxes of the dominance tests tight.
//
// Grid/Angular use a counting sort: per wave-tile histograms of the partition ids, one
// exclusive scan of the partition-major table, then a stable scatter where each wave ranks
// equal ids among its 64 lanes with ballots. Bound: HBM.
#include "sky_internal.hpp"

namespace sky {

namespace {

// Row stride (floats) of the row-major staging copy: the smallest of 4, 8, 16 that holds d.
template <int D>
constexpr int row_stride() { return D == 0 ? 16 : (D <= 4 ? 4 : (D <= 8 ? 8 : 16)); }

// The canonical values of row i from the staging copy.
template <int D>
__device__ __forceinline__ void load_row(const float* __restrict__ xa, int64_t i, float* v) {
    constexpr int RS = row_stride<D>();
    const float4* row = reinterpret_cast<const float4*>(xa + i * RS);
#pragma unroll
    for (int c = 0; c < RS / 4; ++c) {
        const float4 q = row[c];
        v[4 * c] = q.x; v[4 * c + 1] = q.y; v[4 * c + 2] = q.z; v[4 * c + 3] = q.w;
    }
}

constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int64_t kHistCap = int64_t(1) << 22;  // max entries of the histogram table

int bits_for(int32_t p) {
    int b = 0;
    while ((int64_t(1) << b) < p) ++b;
    return b;
}

template <int D>
__device__ __forceinline__ int dget(int d) { return D > 0 ? D : d; }

// ---- per-row partition id (Grid / Angular) + validation --------------------------------------
template <int D>
__global__ void __launch_bounds__(kBlock) part_id_kernel(const float* __restrict__ x, int64_t n,
                                                          int32_t d_rt, int64_t ld, int32_t scheme,
                                                          int32_t m, const double* __restrict__ tan2,
                                                          int32_t* __restrict__ part,
                                                          int32_t* dev_status) {
    const int d = dget<D>(d_rt);
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    bool bad = false;
    if (i < n) {
        float v[SKY_MAX_D];
#pragma unroll
        for (int k = 0; k < (D > 0 ? D : SKY_MAX_D); ++k)
            if (k < d) {
                float t = x[(int64_t)k * ld + i];
                bad |= !in_domain(t);
                v[k] = canon(t);
            }
        int32_t id = 0;
        if (scheme == SKY_GRID) {
            const float fm = (float)m;
            int32_t w = 1;
#pragma unroll
            for (int k = 0; k < (D > 0 ? D : SKY_MAX_D); ++k)
                if (k < d) {
                    int32_t c = qkey(v[k], fm);
                    c = c < 0 ? 0 : (c > m - 1 ? m - 1 : c);
                    id += c * w;
                    w *= m;
                }
        } else {  // SKY_ANGULAR
            // weights m^a for a = 0..d-2; suffix sums of squares from the last attribute down
            int32_t w[SKY_MAX_D];
            w[0] = 1;
            for (int a = 1; a < d - 1; ++a) w[a] = w[a - 1] * m;
            double r2 = 0.0;
            for (int a = d - 2; a >= 0; --a) {
                double nx = (double)v[a + 1];
                r2 += nx * nx;
                double xa = (double)v[a];
                double xa2 = xa * xa;
                int32_t b = 0;
                if (r2 > 0.0) {
                    // largest k in [0, m-1] with r2 >= xa2 * tan2[k] (tan2[0] = 0 always holds)
                    int lo = 0, hi = m - 1;
                    while (lo < hi) {
                        int mid = (lo + hi + 1) >> 1;
                        if (r2 >= xa2 * tan2[mid]) lo = mid; else hi = mid - 1;
                    }
                    b = lo;
                }
                id += b * w[a];
            }
        }
        part[i] = id;
    }
    if (__ballot(bad) != 0 && lane_id() == 0) raise_status(dev_status, SKY_ERR_DOMAIN);
}

// ---- per-row partition id (batched datasets): the dataset holding the row ---------------------
// largest j in [0, p) with seg_off[j] <= i; empty datasets share their offset with the next one,
// so the search lands on the non-empty dataset that holds row i
__global__ void __launch_bounds__(kBlock) seg_part_kernel(const int64_t* __restrict__ seg_off,
                                                           int32_t p, int64_t n,
                                                           int32_t* __restrict__ part) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int32_t lo = 0, hi = p - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (seg_off[mid] <= i) lo = mid; else hi = mid - 1;
    }
    part[i] = lo;
}

// ---- wave-tile histogram of partition ids ----------------------------------------------------
__global__ void __launch_bounds__(kBlock) part_hist_kernel(const int32_t* __restrict__ part,
                                                            const uint32_t* __restrict__ order,
                                                            int64_t n, int32_t p, int chunks,
                                                            int32_t* __restrict__ hist,
                                                            int64_t ntiles) {
    extern __shared__ int32_t cnt[];  // [kWavesPerBlock][p]
    const int wave = threadIdx.x / kWave;
    const int lane = (int)lane_id();
    const int64_t tile = (int64_t)blockIdx.x * kWavesPerBlock + wave;
    int32_t* my = cnt + (int64_t)wave * p;
    for (int i = lane; i < p; i += kWave) my[i] = 0;
    __syncthreads();
    if (tile < ntiles) {
        const int64_t base = tile * (int64_t)chunks * kWave;
        for (int c = 0; c < chunks; ++c) {
            int64_t idx = base + (int64_t)c * kWave + lane;
            if (idx < n) atomicAdd(&my[part[order ? (int64_t)order[idx] : idx]], 1);
        }
    }
    __syncthreads();
    if (tile < ntiles)
        for (int i = lane; i < p; i += kWave) hist[(int64_t)i * ntiles + tile] = my[i];
}

// ---- stable scatter into partition-contiguous order ---------------------------------------------
template <int D>
__global__ void __launch_bounds__(kBlock) part_scatter_kernel(
    const float* __restrict__ xa, int64_t n, int32_t d_rt,
    const int32_t* __restrict__ part, const uint32_t* __restrict__ order, int32_t p, int pbits,
    int chunks, const int32_t* __restrict__ offs, int64_t ntiles, float* __restrict__ xp, int64_t ldp,
    int32_t* __restrict__ rowid, int32_t* __restrict__ seg, float* __restrict__ fsum) {
    extern __shared__ int32_t base[];  // [kWavesPerBlock][p]
    const int d = dget<D>(d_rt);
    const int wave = threadIdx.x / kWave;
    const int lane = (int)lane_id();
    const int64_t tile = (int64_t)blockIdx.x * kWavesPerBlock + wave;
    if (tile >= ntiles) return;  // only wave-level synchronisation below
    int32_t* my = base + (int64_t)wave * p;
    for (int i = lane; i < p; i += kWave) my[i] = offs[(int64_t)i * ntiles + tile];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    const uint64_t lt = __lanemask_lt();
    const int64_t tbase = tile * (int64_t)chunks * kWave;
    for (int c = 0; c < chunks; ++c) {
        const int64_t q = tbase + (int64_t)c * kWave + lane;
        bool valid = q < n;
        uint64_t act = __ballot(valid);
        if (act == 0) break;
        const int64_t i = valid ? (order ? (int64_t)order[q] : q) : 0;
        int32_t id = valid ? part[i] : 0;
        uint64_t peers = match_any((uint32_t)id, pbits, act);
        int32_t b = valid ? my[id] : 0;
        __builtin_amdgcn_wave_barrier();
        if (valid) {
            int32_t pos = b + (int32_t)__popcll(peers & lt);
            float v[row_stride<D>()];
            load_row<D>(xa, i, v);
            float f = 0.0f;
#pragma unroll
            for (int k = 0; k < (D > 0 ? D : SKY_MAX_D); ++k)
                if (k < d) {
                    xp[(int64_t)k * ldp + pos] = v[k];
                    f = __fadd_rn(f, v[k]);
                }
            rowid[pos] = (int32_t)i;
            seg[pos] = id;
            fsum[pos] = f;
            if ((peers & lt) == 0) my[id] = b + (int32_t)__popcll(peers);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
    }
}

__global__ void part_offsets_kernel(const int32_t* __restrict__ offs, int64_t ntiles, int32_t p,
                                    int64_t n, int32_t* __restrict__ part_off) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < p) part_off[j] = offs[(int64_t)j * ntiles];
    if (j == p) part_off[p] = (int32_t)n;
}

// ---- Grid cell pruning (Def. 3) ---------------------------------------------------------------
// A[c] = "some non-empty cell lies in the closed lower orthant of c" via prefix-OR along every
// axis; cell h is pruned iff all its coordinates are >= 1 and A[h - (1,...,1)].
__global__ void __launch_bounds__(1024) grid_prune_kernel(const int32_t* __restrict__ part_off,
                                                           int32_t m, int32_t d, int32_t cells,
                                                           uint8_t* __restrict__ pruned) {
    __shared__ uint8_t A[SKY_MAX_CELLS];
    for (int c = threadIdx.x; c < cells; c += blockDim.x)
        A[c] = part_off[c + 1] > part_off[c] ? 1 : 0;
    __syncthreads();
    int32_t stride = 1;
    for (int k = 0; k < d; ++k) {
        // lines along axis k: cells with coordinate k == 0
        for (int c = threadIdx.x; c < cells; c += blockDim.x) {
            if ((c / stride) % m != 0) continue;
            uint8_t acc = 0;
            for (int j = 0; j < m; ++j) {
                int q = c + j * stride;
                acc |= A[q];
                A[q] = acc;
            }
        }
        __syncthreads();
        stride *= m;
    }
    int32_t diag = 0;
    {
        int32_t w = 1;
        for (int k = 0; k < d; ++k) { diag += w; w *= m; }
    }
    for (int h = threadIdx.x; h < cells; h += blockDim.x) {
        bool all_pos = true;
        int32_t q = h;
        for (int k = 0; k < d; ++k) {
            if (q % m == 0) all_pos = false;
            q /= m;
        }
        pruned[h] = (all_pos && A[h - diag]) ? 1 : 0;
    }
}

// ---- Hilbert key of every row (canonical values), with validation ----------------------------
// Used to order the rows of each partition along a space-filling curve, so that consecutive
// rows are close in space (tight tile boxes for the dominance tests).
// Curve key of every row, and the row's canonical values copied row-major (stride
// row_stride<D>(), zero padded): the gathers into curve order then read one contiguous row
// per item instead of d scattered values.
template <int D>
__global__ void __launch_bounds__(kBlock) curve_rows_kernel(const float* __restrict__ x, int64_t n,
                                                             int32_t d_rt, int64_t ld, int bits,
                                                             uint32_t* __restrict__ keys,
                                                             uint32_t* __restrict__ vals,
                                                             float* __restrict__ xa,
                                                             int32_t* dev_status) {
    constexpr int RS = row_stride<D>();
    const int d = dget<D>(d_rt);
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    bool bad = false;
    if (i < n) {
        float v[RS];
#pragma unroll
        for (int k = 0; k < RS; ++k) {
            float t = k < d ? x[(int64_t)k * ld + i] : 0.0f;
            bad |= !in_domain(t);
            v[k] = canon(t);
        }
        keys[i] = hilbert_key(v, d, bits);
        vals[i] = (uint32_t)i;
        float4* row = reinterpret_cast<float4*>(xa + i * RS);
#pragma unroll
        for (int c = 0; c < RS / 4; ++c) row[c] = make_float4(v[4 * c], v[4 * c + 1], v[4 * c + 2], v[4 * c + 3]);
    }
    if (__ballot(bad) != 0 && lane_id() == 0) raise_status(dev_status, SKY_ERR_DOMAIN);
}


// Sliced: the row at rank q of the (value, row) order goes to partition floor(q p / n)
__global__ void __launch_bounds__(kBlock) slice_parts_kernel(const uint32_t* __restrict__ order,
                                                              int64_t n, int32_t p,
                                                              int32_t* __restrict__ part) {
    int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q < n) part[order[q]] = (int32_t)((q * (int64_t)p) / n);
}

// ---- Sliced: sort keys, gather ----------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) slice_keys_kernel(const float* __restrict__ x, int64_t n,
                                                             int32_t d, int64_t ld, int32_t dim,
                                                             uint32_t* __restrict__ keys,
                                                             uint32_t* __restrict__ vals,
                                                             int32_t* dev_status) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    bool bad = false;
    if (i < n) {
        for (int k = 0; k < d; ++k) bad |= !in_domain(x[(int64_t)k * ld + i]);
        // canonical non-negative FP32 values: the bit pattern orders like the value
        keys[i] = fbits(canon(x[(int64_t)dim * ld + i]));
        vals[i] = (uint32_t)i;
    }
    if (__ballot(bad) != 0 && lane_id() == 0) raise_status(dev_status, SKY_ERR_DOMAIN);
}

template <int D>
__global__ void __launch_bounds__(kBlock) slice_gather_kernel(
    const float* __restrict__ xa, int64_t n, int32_t d_rt, int32_t p,
    const uint32_t* __restrict__ order, float* __restrict__ xp, int64_t ldp,
    int32_t* __restrict__ rowid, int32_t* __restrict__ seg, float* __restrict__ fsum) {
    const int d = dget<D>(d_rt);
    int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= n) return;
    int64_t i = order[q];
    float v[row_stride<D>()];
    load_row<D>(xa, i, v);
    float f = 0.0f;
#pragma unroll
    for (int k = 0; k < (D > 0 ? D : SKY_MAX_D); ++k)
        if (k < d) {
            xp[(int64_t)k * ldp + q] = v[k];
            f = __fadd_rn(f, v[k]);
        }
    rowid[q] = (int32_t)i;
    seg[q] = (int32_t)((q * (int64_t)p) / n);
    fsum[q] = f;
}

__global__ void slice_offsets_kernel(int64_t n, int32_t p, int32_t* __restrict__ part_off,
                                     uint8_t* __restrict__ pruned) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    // first rank q with floor(q p / n) >= j is ceil(j n / p)
    if (j <= p) part_off[j] = (int32_t)(((int64_t)j * n + p - 1) / p);
    if (j < p) pruned[j] = 0;
}

__global__ void fill_u8_kernel(uint8_t* __restrict__ p, int64_t n, uint8_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

// items per histogram tile for p partitions over n rows
static int part_chunks(int64_t n, int32_t p) {
    int64_t min_items = ceil_div((int64_t)p * n, kHistCap);
    int64_t chunks = ceil_div(min_items, kWave);
    if (chunks < 16) chunks = 16;
    return (int)chunks;
}

int64_t partition_hist_elems(int64_t n, int32_t p) {
    if (n <= 0 || p <= 0) return 64;
    const int chunks = part_chunks(n, p);
    const int64_t ntiles = ceil_div(n, (int64_t)chunks * kWave);
    return round_up((int64_t)p * ntiles, 64);
}

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

// Angular bucket thresholds (Eq. (1)): tan2[k] = tan^2(k pi / (2m)) in FP64, tan2[0] = 0. A
// row's bucket along an angle is the number of k in [1, m-1] whose threshold its ratio reaches.
__global__ void angular_table_kernel(int32_t m, double* __restrict__ tan2) {
    for (int32_t k = threadIdx.x; k <= m; k += blockDim.x) {
        const double t = tan((double)k * 3.14159265358979323846 / (2.0 * (double)m));
        tan2[k] = k == 0 ? 0.0 : t * t;
    }
}

// Partition statistics as int64 words: out[0] = Grid cells pruned by grid dominance that hold
// rows, out[1] = the rows inside them, out[2] = rows of the largest partition (one workgroup).
__global__ void __launch_bounds__(kBlock) partition_stats_kernel(const int32_t* __restrict__ part_off,
                                                                  const uint8_t* __restrict__ pruned,
                                                                  int32_t p, int64_t* __restrict__ out) {
    __shared__ int64_t red[3][kBlock / kWave];
    int64_t pc = 0, pr = 0, mx = 0;
    for (int32_t j = threadIdx.x; j < p; j += kBlock) {
        const int64_t sz = (int64_t)part_off[j + 1] - part_off[j];
        mx = sz > mx ? sz : mx;
        if (pruned[j] && sz > 0) {
            ++pc;
            pr += sz;
        }
    }
    for (int off = kWave / 2; off > 0; off >>= 1) {
        pc += __shfl_xor(pc, off, kWave);
        pr += __shfl_xor(pr, off, kWave);
        const int64_t o = __shfl_xor(mx, off, kWave);
        mx = o > mx ? o : mx;
    }
    if (lane_id() == 0) {
        red[0][threadIdx.x / kWave] = pc;
        red[1][threadIdx.x / kWave] = pr;
        red[2][threadIdx.x / kWave] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / kWave; ++w) {
            pc += red[0][w];
            pr += red[1][w];
            mx = red[2][w] > mx ? red[2][w] : mx;
        }
        out[0] = pc;
        out[1] = pr;
        out[2] = mx;
    }
}

sky_status launch_partition_stats(const int32_t* part_off, const uint8_t* pruned, int32_t p, int64_t* out,
                                  hipStream_t st) {
    hipLaunchKernelGGL(partition_stats_kernel, dim3(1), dim3(kBlock), 0, st, part_off, pruned, p, out);
    SKY_HIP(hipGetLastError());
    return SKY_OK;
}

sky_status launch_partition(const PartitionArgs& a, hipStream_t st) {
    const int64_t n = a.n;
    const uint32_t rblocks = (uint32_t)ceil_div(n, kBlock);
    // 1. partition of every row (Grid / Angular directly, Sliced from the rank order)
    if (a.scheme == SKY_ANGULAR) {
        hipLaunchKernelGGL(angular_table_kernel, dim3(1), dim3(256), 0, st, a.m, a.tan2);
        SKY_HIP(hipGetLastError());
    }
    if (a.scheme == SKY_GRID || a.scheme == SKY_ANGULAR) {
        SKY_DISPATCH_D(a.d, part_id_kernel, dim3(rblocks), dim3(kBlock), 0, st, a.x, n, a.d, a.ld,
                       a.scheme, a.m, a.tan2, a.part_of_row, a.dev_status);
        SKY_HIP(hipGetLastError());
    } else if (a.scheme == SKY_SLICED) {
        hipLaunchKernelGGL(slice_keys_kernel, dim3(rblocks), dim3(kBlock), 0, st, a.x, n, a.d, a.ld,
                           a.slice_dim, a.k0, a.v0, a.dev_status);
        SKY_HIP(hipGetLastError());
        SKY_TRY(launch_radix_sort(a.k0, a.v0, a.k1, a.v1, n, 32, a.radix_tmp, st));
        hipLaunchKernelGGL(slice_parts_kernel, dim3(rblocks), dim3(kBlock), 0, st,
                           (const uint32_t*)a.v0, n, a.p, a.part_of_row);
        SKY_HIP(hipGetLastError());
    } else if (a.scheme == kSchemeSegments) {
        hipLaunchKernelGGL(seg_part_kernel, dim3(rblocks), dim3(kBlock), 0, st, a.seg_off, a.p, n,
                           a.part_of_row);
        SKY_HIP(hipGetLastError());
    }
    // 2. every row in Hilbert order (stable): the order rows take inside their partition
    const int bits = curve_bits(a.d);
    SKY_DISPATCH_D(a.d, curve_rows_kernel, dim3(rblocks), dim3(kBlock), 0, st, a.x, n, a.d, a.ld, bits,
                   a.k0, a.v0, a.xa, a.dev_status);
    SKY_HIP(hipGetLastError());
    const uint32_t* sorted_keys = nullptr;
    const uint32_t* order = nullptr;
    SKY_TRY(launch_radix_sort(a.k0, a.v0, a.k1, a.v1, n, bits * a.d, a.radix_tmp, st, &sorted_keys, &order));
    if (a.p == 1) {
        SKY_DISPATCH_D(a.d, slice_gather_kernel, dim3(rblocks), dim3(kBlock), 0, st,
                       (const float*)a.xa, n, a.d, 1, order, a.xp, a.ldp, a.rowid, a.seg, a.fsum);
        SKY_HIP(hipGetLastError());
        hipLaunchKernelGGL(slice_offsets_kernel, dim3(1), dim3(64), 0, st, n, 1, a.part_off, a.pruned);
        SKY_HIP(hipGetLastError());
        return SKY_OK;
    }
    // 3. stable counting sort by partition over the curve order
    const int chunks = part_chunks(n, a.p);
    const int64_t ntiles = ceil_div(n, (int64_t)chunks * kWave);
    if ((int64_t)a.p * ntiles > a.hist_cap) return SKY_ERR_WORKSPACE;  // never with the API's sizes
    const uint32_t tblocks = (uint32_t)ceil_div(ntiles, kWavesPerBlock);
    const size_t lds = sizeof(int32_t) * (size_t)kWavesPerBlock * (size_t)a.p;
    hipLaunchKernelGGL(part_hist_kernel, dim3(tblocks), dim3(kBlock), lds, st,
                       (const int32_t*)a.part_of_row, order, n, a.p, chunks, a.hist, ntiles);
    SKY_HIP(hipGetLastError());
    SKY_TRY(launch_exclusive_scan(a.hist, a.hist, (int64_t)a.p * ntiles, a.scan_tmp, st));
    const int pbits = bits_for(a.p);
    SKY_DISPATCH_D(a.d, part_scatter_kernel, dim3(tblocks), dim3(kBlock), lds, st,
                   (const float*)a.xa, n, a.d, (const int32_t*)a.part_of_row, order, a.p, pbits, chunks,
                   (const int32_t*)a.hist, ntiles, a.xp, a.ldp, a.rowid, a.seg, a.fsum);
    SKY_HIP(hipGetLastError());
    hipLaunchKernelGGL(part_offsets_kernel, dim3((uint32_t)ceil_div(a.p + 1, 256)), dim3(256), 0,
                       st, (const int32_t*)a.hist, ntiles, a.p, n, a.part_off);
    SKY_HIP(hipGetLastError());
    if (a.scheme == SKY_GRID) {
        hipLaunchKernelGGL(grid_prune_kernel, dim3(1), dim3(1024), 0, st,
                           (const int32_t*)a.part_off, a.m, a.d, a.p, a.pruned);
    } else {
        hipLaunchKernelGGL(fill_u8_kernel, dim3((uint32_t)ceil_div(a.p, 256)), dim3(256), 0, st,
                           a.pruned, (int64_t)a.p, (uint8_t)0);
    }
    SKY_HIP(hipGetLastError());
    return SKY_OK;
}

}  // namespace sky
