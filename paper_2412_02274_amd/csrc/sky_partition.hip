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
// The steps, for every scheme:
//  1. classify (one pass over the relation): validate the domain (SKY_ERR_DOMAIN), take the
//     canonical values, the partition and the FP32 attribute sum (the monotone score of the
//     skyline filter, Sec. 2), count the rows of every partition, and keep, per partition, the
//     row of smallest score of each workgroup's 4096 consecutive rows, folded into
//     SKY_KILLERS slots (slot = workgroup mod SKY_KILLERS, minimum per slot).
//  2. partition offsets, then Grid pruning (Def. 3) from the partition sizes.
//  3. prefilter: every row of an unpruned partition is tested against that partition's slot
//     rows (the "killers"; a row is not tested against itself). A row one of them dominates
//     belongs to no skyline of its partition (Def. 1 inside the partition), so it is dropped
//     before any sorting. On uniform data a few rows of smallest score dominate almost every
//     row of their partition (10M x 4 in 81 cells: about 3% of the rows remain); on
//     anticorrelated data the prefilter keeps most rows and costs one streaming pass. With
//     Representative Filtering, or when the caller turns it off, every row is kept (the
//     representatives are drawn from all rows, pruned cells included). The kept rows'
//     canonical values go to a row-major staging copy (at their row index).
//  4. the kept rows, in row order, with sort keys (partition, Hilbert key of the values);
//  5. a stable radix sort of those keys over the kept rows only (their count stays on the
//     device);
//  6. the partition-contiguous canonical SoA copy of the kept rows in key order: inside every
//     partition the rows follow a Hilbert curve, which keeps the tile boxes of the dominance
//     tests tight; with the original row, the partition and the score of every position.
// Bound: HBM (steps 1 and 3 stream the relation; the sort and the copy touch the kept rows).
#include "sky_internal.hpp"

namespace sky {

namespace {

// Row stride (floats) of the row-major staging copy: the smallest of 4, 8, 16 that holds d.
template <int D>
constexpr int row_stride() { return D == 0 ? 16 : (D <= 4 ? 4 : (D <= 8 ? 8 : 16)); }

// The first row_stride<D>() floats at p (16-byte aligned).
template <int D>
__device__ __forceinline__ void load_row(const float* __restrict__ p, float* v) {
    constexpr int RS = row_stride<D>();
    const float4* row = reinterpret_cast<const float4*>(p);
#pragma unroll
    for (int c = 0; c < RS / 4; ++c) {
        const float4 q = row[c];
        v[4 * c] = q.x; v[4 * c + 1] = q.y; v[4 * c + 2] = q.z; v[4 * c + 3] = q.w;
    }
}

// The classify/filter/compact passes: workgroups of 1024 threads, 4 rows per thread. Wide
// workgroups keep many waves per CU on a 1M-row relation while the per-workgroup flushes of
// partition counters into global memory stay at one per 4096 rows (with one partition they all
// meet on the same few addresses).
constexpr int kPT = 1024;
constexpr int kPPer = 4;
constexpr int kPRows = kPT * kPPer;
constexpr int kKill = SKY_KILLERS;

int bits_for(int32_t p) {
    int b = 0;
    while ((int64_t(1) << b) < p) ++b;
    return b;
}

template <int D>
__device__ __forceinline__ int dget(int d) { return D > 0 ? D : d; }

// ---- the partition of a row from its canonical values (Grid / Angular) ------------------------
template <int D>
__device__ __forceinline__ int32_t cell_of(const float* v, int d, int32_t scheme, int32_t m,
                                           const double* __restrict__ tan2) {
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
        return id;
    }
    // SKY_ANGULAR: weights m^a for a = 0..d-2; suffix sums of squares from the last attribute
    int32_t w[SKY_MAX_D];
    w[0] = 1;
    for (int a = 1; a < d - 1; ++a) w[a] = w[a - 1] * m;
    double r2 = 0.0;
    for (int a = d - 2; a >= 0; --a) {
        const double nx = (double)v[a + 1];
        r2 += nx * nx;
        const double xa = (double)v[a];
        const double xa2 = xa * xa;
        int32_t b = 0;
        if (r2 > 0.0) {
            // largest k in [0, m-1] with r2 >= xa2 * tan2[k] (tan2[0] = 0 always holds)
            int lo = 0, hi = m - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (r2 >= xa2 * tan2[mid]) lo = mid; else hi = mid - 1;
            }
            b = lo;
        }
        id += b * w[a];
    }
    return id;
}

// The dataset holding row i (batched path): largest j in [0, p) with seg_off[j] <= i; empty
// datasets share their offset with the next one, so the search lands on the non-empty one.
__device__ __forceinline__ int32_t dataset_of(const int64_t* __restrict__ seg_off, int32_t p, int64_t i) {
    int32_t lo = 0, hi = p - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (seg_off[mid] <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ---- 0. per-build counters -----------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) partition_init_kernel(int32_t p, int32_t* __restrict__ pcount,
                                                                unsigned long long* __restrict__ kmin,
                                                                unsigned long long* __restrict__ seg_tests,
                                                                unsigned long long* __restrict__ tests,
                                                                uint32_t* __restrict__ smin,
                                                                uint32_t* __restrict__ smax,
                                                                uint8_t* __restrict__ pruned) {
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g < p) {
        pcount[g] = 0;
        seg_tests[g] = 0ull;
        pruned[g] = 0;  // (Grid rewrites them after the counts)
    }
    if (g < (p > 1 ? p : kRangeSlots)) {  // one partition: its range slots
        const int64_t at = p > 1 ? g : g * kRangeStride;
        smin[at] = 0xFFFFFFFFu;
        smax[at] = 0u;
    }
    if (g < (int64_t)p * kKill) kmin[g] = ~0ull;
    if (g == 0) *tests = 0ull;
}

// ---- 1. classify -----------------------------------------------------------------------------------
// A row's key in the (value, row) order of the slicing attribute: the canonical value's bits
// above the row index (rows < 2^30)
__device__ __forceinline__ unsigned long long slice_key(float v, int64_t row) {
    return ((unsigned long long)fbits(v) << 30) | (unsigned long long)row;
}

struct ClassifyArgs {
    const float* x; int64_t n; int32_t d; int64_t ld;
    int32_t scheme; int32_t p; int32_t m; int32_t slice_dim;
    const double* tan2;             // Angular thresholds
    const int64_t* seg_off;         // batched datasets
    const unsigned long long* bkey; // Sliced: [p - 1] boundary keys (slice_key order)
    int32_t* part_of_row;           // written (every scheme but None), null (None)
    int32_t* pcount;                // [p] rows per partition (+=)
    unsigned long long* kmin;       // [p][kKill] minima of (score bits << 32 | row)
    int32_t* dev_status;
};

template <int D>
__global__ void __launch_bounds__(kPT) classify_kernel(ClassifyArgs a) {
    constexpr int DM = D > 0 ? D : SKY_MAX_D;
    extern __shared__ unsigned long long lmin[];  // [p], Sliced: [p - 1] boundary keys, then int32 counts [p]
    unsigned long long* lbk = lmin + a.p;
    const bool sliced = a.scheme == SKY_SLICED;
    int32_t* lcnt = reinterpret_cast<int32_t*>(lmin + a.p + (sliced ? a.p - 1 : 0));
    const int d = dget<D>(a.d);
    for (int32_t j = threadIdx.x; j < a.p; j += kPT) {
        lmin[j] = ~0ull;
        lcnt[j] = 0;
        if (sliced && j < a.p - 1) lbk[j] = a.bkey[j];
    }
    __syncthreads();
    bool bad = false;
    const int64_t b0 = (int64_t)blockIdx.x * kPRows;
    for (int it = 0; it < kPPer; ++it) {
        const int64_t i = b0 + (int64_t)it * kPT + threadIdx.x;
        const bool valid = i < a.n;
        int32_t part = -1;
        unsigned long long key = ~0ull;
        if (valid) {
            float v[DM];
            float f = 0.0f, vs = 0.0f;
#pragma unroll
            for (int k = 0; k < DM; ++k)
                if (k < d) {
                    const float t = a.x[(int64_t)k * a.ld + i];
                    bad |= !in_domain(t);
                    v[k] = canon(t);
                    f = __fadd_rn(f, v[k]);
                    if (k == a.slice_dim) vs = v[k];
                }
            if (a.scheme == SKY_NONE) part = 0;
            else if (sliced) {  // the boundaries at or below the row's key (binary search)
                const unsigned long long kr = slice_key(vs, i);
                int32_t lo = 0, hi = a.p - 1;
                while (lo < hi) {
                    const int32_t mid = (lo + hi) >> 1;
                    if (lbk[mid] <= kr) lo = mid + 1; else hi = mid;
                }
                part = lo;
            }
            else if (a.scheme == kSchemeSegments) part = dataset_of(a.seg_off, a.p, i);
            else part = cell_of<D>(v, d, a.scheme, a.m, a.tan2);
            if (a.part_of_row) a.part_of_row[i] = part;
            key = ((unsigned long long)fbits(f) << 32) | (uint32_t)i;
        }
        // count and minimum per partition in LDS; a wave whose rows share one partition (one
        // relation, or one dataset of a batch) folds them into one update
        const uint64_t act = __ballot(valid);
        const int32_t p0 = __builtin_amdgcn_readfirstlane(part);
        if ((act & 1ull) && __ballot(valid && part != p0) == 0) {
            unsigned long long mk = key;
#pragma unroll
            for (int off = kWave / 2; off > 0; off >>= 1) {
                const unsigned long long o = __shfl_xor(mk, off, kWave);
                mk = o < mk ? o : mk;
            }
            if (lane_id() == 0) {
                atomicMin(&lmin[p0], mk);
                atomicAdd(&lcnt[p0], (int32_t)__popcll(act));
            }
        } else if (valid) {
            // (the minimum only falls: most rows lose to it without an atomic)
            if (key < lmin[part]) atomicMin(&lmin[part], key);
            atomicAdd(&lcnt[part], 1);
        }
    }
    __syncthreads();
    const int32_t slot = (int32_t)(blockIdx.x % (uint32_t)kKill);
    for (int32_t j = threadIdx.x; j < a.p; j += kPT) {
        const int32_t c = lcnt[j];
        if (c) {
            atomicAdd(&a.pcount[j], c);
            atomicMin(&a.kmin[(int64_t)j * kKill + slot], lmin[j]);
        }
    }
    if (__ballot(bad) != 0 && lane_id() == 0) raise_status(a.dev_status, SKY_ERR_DOMAIN);
}

// Partition statistics (out[0..3) = pruned non-empty cells, rows inside them, rows of the
// largest partition) by the whole workgroup (at most 1024 threads), once part_off (and pruned,
// when given) are written: every thread calls it.
__device__ void partition_stats_block(const int32_t* __restrict__ part_off, const uint8_t* __restrict__ pruned,
                                      int32_t p, int64_t* __restrict__ out) {
    __shared__ int64_t red[3][1024 / kWave];
    __syncthreads();  // part_off / pruned of the other threads
    int64_t pc = 0, pr = 0, mx = 0;
    for (int32_t j = threadIdx.x; j < p; j += blockDim.x) {
        const int64_t sz = (int64_t)part_off[j + 1] - part_off[j];
        mx = sz > mx ? sz : mx;
        if (pruned && pruned[j] && sz > 0) {
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
        for (int w = 1; w < (int)(blockDim.x / kWave); ++w) {
            pc += red[0][w];
            pr += red[1][w];
            mx = red[2][w] > mx ? red[2][w] : mx;
        }
        out[0] = pc;
        out[1] = pr;
        out[2] = mx;
    }
}

// ---- 2. partition offsets (one workgroup of 1024 threads, p <= 4096) --------------------------------
// (stats given: no pruning follows, so the partition statistics are taken here)
__global__ void __launch_bounds__(1024) part_offsets_kernel(const int32_t* __restrict__ pcount, int32_t p,
                                                            int64_t n, int32_t* __restrict__ part_off,
                                                            int64_t* __restrict__ stats) {
    __shared__ int32_t ws[1024 / kWave];
    const int per = (p + 1023) / 1024;  // at most 4
    int32_t loc[4];
    int32_t s = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int32_t j = threadIdx.x * per + e;
        loc[e] = (e < per && j < p) ? pcount[j] : 0;
        s += loc[e];
    }
    const int lane = (int)lane_id(), wave = threadIdx.x / kWave;
    int32_t x = s;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const int32_t t = __shfl_up(x, off, kWave);
        if (lane >= off) x += t;
    }
    if (lane == kWave - 1) ws[wave] = x;
    __syncthreads();
    int32_t run = x - s;
    for (int w = 0; w < wave; ++w) run += ws[w];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int32_t j = threadIdx.x * per + e;
        if (e < per && j < p) part_off[j] = run;
        run += loc[e];
    }
    if (threadIdx.x == 0) part_off[p] = (int32_t)n;
    if (stats) partition_stats_block(part_off, nullptr, p, stats);
}

// ---- Grid cell pruning (Def. 3) ------------------------------------------------------------------
// A[c] = "some non-empty cell lies in the closed lower orthant of c" via prefix-OR along every
// axis; cell h is pruned iff all its coordinates are >= 1 and A[h - (1,...,1)].
__global__ void __launch_bounds__(1024) grid_prune_kernel(const int32_t* __restrict__ part_off,
                                                           int32_t m, int32_t d, int32_t cells,
                                                           uint8_t* __restrict__ pruned,
                                                           int64_t* __restrict__ stats) {
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
    partition_stats_block(part_off, pruned, cells, stats);
}

// ---- 3. killers and the prefilter ----------------------------------------------------------------
// One thread per (partition, slot): the slot's row (-1: none, or a pruned partition) and its
// canonical values.
template <int D>
__global__ void __launch_bounds__(kBlock) kill_rows_kernel(const unsigned long long* __restrict__ kmin,
                                                            const uint8_t* __restrict__ pruned, int32_t p,
                                                            const float* __restrict__ x, int32_t d_rt, int64_t ld,
                                                            int32_t* __restrict__ krow, float* __restrict__ kval) {
    constexpr int RS = row_stride<D>();
    const int d = dget<D>(d_rt);
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= (int64_t)p * kKill) return;
    const int32_t j = (int32_t)(e / kKill);
    const unsigned long long key = kmin[e];
    const bool ok = key != ~0ull && !(pruned && pruned[j]);
    const int32_t r = ok ? (int32_t)(uint32_t)key : -1;
    krow[e] = r;
    float v[RS];
#pragma unroll
    for (int k = 0; k < RS; ++k) v[k] = (ok && k < d) ? canon(x[(int64_t)k * ld + r]) : 2.0f;
    float4* dst = reinterpret_cast<float4*>(kval + e * RS);
#pragma unroll
    for (int c = 0; c < RS / 4; ++c) dst[c] = make_float4(v[4 * c], v[4 * c + 1], v[4 * c + 2], v[4 * c + 3]);
}

struct FilterArgs {
    int64_t n; int32_t d; int64_t ld; int32_t p;
    const float* x;                   // the relation (SoA)
    const int32_t* part_of_row;       // null: one partition
    const uint8_t* pruned;            // null: nothing pruned
    const int32_t* krow; const float* kval;
    int32_t killers;                  // 0: every row is kept (no tests)
    uint8_t* alive;                   // [n] out
    float* xa;                        // [n][row stride] out: the canonical values of every kept row
    int32_t* blk;                     // [workgroups] out: rows kept per workgroup
    unsigned long long* seg_tests;    // [p] += the tests of the partition's rows
    unsigned long long* tests;        // += all tests
};

constexpr int kKillLds = 8192;   // floats of killer values a workgroup keeps in LDS (32 KB)

// Every row of an unpruned partition against the partition's killer rows (not itself), until
// one dominates it; the survivors' canonical values go to the staging copy. Killer values sit
// in LDS when the whole table fits, else they are read from the (L2-resident) table.
template <int D>
__global__ void __launch_bounds__(kPT) filter_kernel(FilterArgs a) {
    constexpr int RS = row_stride<D>();
    constexpr int DM = D > 0 ? D : SKY_MAX_D;
    extern __shared__ unsigned int fl[];  // [p] test counters, then (when it fits) the killer table
    __shared__ int32_t ws[kPT / kWave];
    const int d = dget<D>(a.d);
    const int64_t tab = (int64_t)a.p * kKill * RS;
    const bool in_lds = a.killers && tab <= kKillLds;
    unsigned int* ltests = fl;
    float* lk = reinterpret_cast<float*>(fl + ((a.p + 3) & ~3));  // 16-byte aligned
    // in LDS the partitions' killer blocks are padded (values by 4 floats, row ids by 1): the
    // lanes of a wave look up different partitions, and unpadded blocks 128 bytes apart would
    // all start in the same banks
    constexpr int kVS = kKill * RS + 4, kRS = kKill + 1;
    int32_t* lr = reinterpret_cast<int32_t*>(lk + (in_lds ? (int64_t)a.p * kVS : 0));
    if (a.killers) {
        for (int32_t j = threadIdx.x; j < a.p; j += kPT) ltests[j] = 0u;
        if (in_lds) {
            for (int64_t e = threadIdx.x; e < tab; e += kPT) lk[(e / (kKill * RS)) * kVS + e % (kKill * RS)] = a.kval[e];
            for (int64_t e = threadIdx.x; e < (int64_t)a.p * kKill; e += kPT) lr[(e / kKill) * kRS + e % kKill] = a.krow[e];
        }
        __syncthreads();
    }
    const float* ktab = in_lds ? lk : a.kval;
    const int32_t* rtab = in_lds ? lr : a.krow;
    const int64_t vstride = in_lds ? kVS : kKill * RS, rstride = in_lds ? kRS : kKill;
    int32_t kept = 0;
    const int64_t b0 = (int64_t)blockIdx.x * kPRows;
    {
        // the thread's rows, their loads issued together
        int32_t part[kPPer];
        float t[kPPer][DM];
#pragma unroll
        for (int u = 0; u < kPPer; ++u) {
            const int64_t i = b0 + (int64_t)u * kPT + threadIdx.x;
            const bool valid = i < a.n;
            part[u] = valid ? (a.part_of_row ? a.part_of_row[i] : 0) : -1;
#pragma unroll
            for (int k = 0; k < DM; ++k)
                if (k < d) t[u][k] = valid ? canon(a.x[(int64_t)k * a.ld + i]) : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < kPPer; ++u) {
            const int64_t i = b0 + (int64_t)u * kPT + threadIdx.x;
            const bool valid = i < a.n;
            bool live = valid;
            uint32_t nt = 0;
            if (valid && a.killers) {
                if (a.pruned && a.pruned[part[u]]) {
                    live = false;  // Def. 3: the rows of a pruned cell take no part
                } else {
#pragma unroll
                    for (int s = 0; s < kKill; ++s) {
                        const int32_t r = rtab[part[u] * rstride + s];
                        float sv[RS];
                        load_row<D>(ktab + part[u] * vstride + s * RS, sv);
                        if (live && r >= 0 && r != (int32_t)i) {
                            ++nt;
                            bool le = true, lt = false;
#pragma unroll
                            for (int k = 0; k < DM; ++k)
                                if (k < d) {
                                    le &= sv[k] <= t[u][k];
                                    lt |= sv[k] < t[u][k];
                                }
                            live = !(le && lt);
                        }
                    }
                    if (nt) atomicAdd(&ltests[part[u]], nt);
                }
            }
            if (valid) {
                a.alive[i] = live ? 1 : 0;
                if (live) {
                    float q[RS];
#pragma unroll
                    for (int k = 0; k < RS; ++k) q[k] = 0.0f;
#pragma unroll
                    for (int k = 0; k < DM; ++k)
                        if (k < d) q[k] = t[u][k];
                    float4* row = reinterpret_cast<float4*>(a.xa + i * RS);
#pragma unroll
                    for (int c = 0; c < RS / 4; ++c) row[c] = make_float4(q[4 * c], q[4 * c + 1], q[4 * c + 2], q[4 * c + 3]);
                }
            }
            kept += live ? 1 : 0;
        }
    }
    int32_t total = 0;
    (void)block_exscan_t<kPT>(kept, ws, &total);
    if (threadIdx.x == 0) a.blk[blockIdx.x] = total;
    if (a.killers) {
        __syncthreads();
        unsigned long long sum = 0;
        for (int32_t j = threadIdx.x; j < a.p; j += kPT) {
            const unsigned long long c = ltests[j];
            if (c) {
                atomicAdd(&a.seg_tests[j], c);
                sum += c;
            }
        }
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) sum += __shfl_xor(sum, off, kWave);
        if (lane_id() == 0 && sum) atomicAdd(a.tests, sum);
    }
}

// ---- 4. the kept rows with their sort keys ---------------------------------------------------------
struct CompactArgs {
    int64_t n; int32_t d;
    const uint8_t* alive;
    const int32_t* blk_off;           // exclusive offsets of the workgroups' kept rows
    const int32_t* part_of_row;       // null: one partition
    const float* xa;
    int32_t cbits;                    // curve bits per attribute
    int32_t pshift;                   // the partition's place in the key (cbits * d)
    uint32_t* keys; uint32_t* rows;   // out, at the kept rows' ranks
    int32_t* n_live;                  // out: rows kept (written by the last workgroup)
};

template <int D>
__global__ void __launch_bounds__(kPT) compact_kernel(CompactArgs a) {
    constexpr int RS = row_stride<D>();
    __shared__ int32_t ws[kPT / kWave];
    const int d = dget<D>(a.d);
    // thread t takes kPPer consecutive rows, so ranks follow row order
    const int64_t r0 = ((int64_t)blockIdx.x * kPT + threadIdx.x) * kPPer;
    const int32_t boff = a.blk_off[blockIdx.x];
    uint32_t flags = 0;
    if (r0 + kPPer <= a.n) {
        const uint32_t w = *reinterpret_cast<const uint32_t*>(a.alive + r0);
#pragma unroll
        for (int e = 0; e < kPPer; ++e) flags |= ((w >> (8 * e)) & 1u) << e;
    } else {
        for (int e = 0; e < kPPer; ++e)
            if (r0 + e < a.n) flags |= (uint32_t)(a.alive[r0 + e] & 1u) << e;
    }
    int32_t total = 0;
    int32_t o = boff + block_exscan_t<kPT>(__popc(flags), ws, &total);
    while (flags) {
        const int e = __ffs(flags) - 1;
        flags &= flags - 1;
        const int64_t i = r0 + e;
        float v[RS];
        load_row<D>(a.xa + i * RS, v);
        uint32_t key = hilbert_key(v, d, a.cbits);
        if (a.part_of_row) key |= (uint32_t)a.part_of_row[i] << a.pshift;
        a.keys[o] = key;
        a.rows[o] = (uint32_t)i;
        ++o;
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *a.n_live = boff + total;
}

// ---- 6. the partition-contiguous copy of the kept rows in key order --------------------------------
// Each wave copies one contiguous run of positions (lanes 64 apart, coalesced) and folds the
// scores of each partition it meets into that partition's range (smin / smax), which the
// skyline rounds then use instead of a pass of their own. One partition: each workgroup's range
// goes to one of the kRangeSlots slots, which the skyline run's first kernel folds.
template <int D>
__global__ void __launch_bounds__(kBlock) part_gather_kernel(
    const uint32_t* __restrict__ keys, const uint32_t* __restrict__ rows, const int32_t* __restrict__ n_live,
    int32_t d_rt, int32_t pshift, int32_t multi, const float* __restrict__ xa, float* __restrict__ xp,
    int64_t ldp, int32_t* __restrict__ rowid, int32_t* __restrict__ seg, float* __restrict__ fsum,
    uint32_t* __restrict__ smin, uint32_t* __restrict__ smax, int32_t* __restrict__ iota_out) {
    constexpr int RS = row_stride<D>();
    const int d = dget<D>(d_rt);
    const int lane = (int)lane_id();
    const int64_t m = *n_live;
    const int64_t nwaves = (int64_t)gridDim.x * (kBlock / kWave);
    const int64_t per = (m + nwaves * kWave - 1) / (nwaves * kWave);
    const int64_t q0 = ((int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave) * per * kWave;
    int32_t cs = -1;  // partition of the lane's current run of scores
    uint32_t cmin = 0xFFFFFFFFu, cmax = 0u;
    for (int64_t j = 0; j < per; ++j) {
        const int64_t q = q0 + j * kWave + lane;
        if (q >= m) break;
        const int64_t i = rows[q];
        float v[RS];
        load_row<D>(xa + i * RS, v);
        float f = 0.0f;
#pragma unroll
        for (int k = 0; k < (D > 0 ? D : SKY_MAX_D); ++k)
            if (k < d) {
                xp[(int64_t)k * ldp + q] = v[k];
                f = __fadd_rn(f, v[k]);
            }
        const int32_t sg = multi ? (int32_t)(keys[q] >> pshift) : 0;
        rowid[q] = (int32_t)i;
        seg[q] = sg;
        fsum[q] = f;
        if (iota_out) iota_out[q] = (int32_t)q;
        const uint32_t fb = fbits(f);  // f >= 0: bit order == value order
        if (!multi) {
            cmin = fb < cmin ? fb : cmin;
            cmax = fb > cmax ? fb : cmax;
            continue;
        }
        if (sg != cs) {
            if (cs >= 0) {
                atomicMin(&smin[cs], cmin);
                atomicMax(&smax[cs], cmax);
            }
            cs = sg;
            cmin = fb;
            cmax = fb;
        } else {
            cmin = fb < cmin ? fb : cmin;
            cmax = fb > cmax ? fb : cmax;
        }
    }
    if (!multi) {
        __shared__ uint32_t wr[2][kBlock / kWave];
        for (int off = kWave / 2; off > 0; off >>= 1) {
            const uint32_t x = __shfl_xor(cmin, off, kWave), y = __shfl_xor(cmax, off, kWave);
            cmin = x < cmin ? x : cmin;
            cmax = y > cmax ? y : cmax;
        }
        if (lane == 0) {
            wr[0][threadIdx.x / kWave] = cmin;
            wr[1][threadIdx.x / kWave] = cmax;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t a0 = wr[0][0], a1 = wr[1][0];
            for (int w = 1; w < kBlock / kWave; ++w) {
                a0 = wr[0][w] < a0 ? wr[0][w] : a0;
                a1 = wr[1][w] > a1 ? wr[1][w] : a1;
            }
            if (a0 <= a1) {  // the workgroup copied a row
                const int64_t at = (int64_t)(blockIdx.x % (uint32_t)kRangeSlots) * kRangeStride;
                atomicMin(&smin[at], a0);
                atomicMax(&smax[at], a1);
            }
        }
        return;
    }
    // the lanes' last runs, one pair of atomics per partition and wave
    const bool valid = cs >= 0;
    uint64_t act = __ballot(valid);
    while (act) {
        const int leader = __ffsll((unsigned long long)act) - 1;
        const int32_t sl = __shfl(cs, leader, kWave);
        const bool mine = valid && cs == sl;
        const uint64_t peers = __ballot(mine);
        uint32_t vmin = mine ? cmin : 0xFFFFFFFFu, vmax = mine ? cmax : 0u;
        for (int off = kWave / 2; off > 0; off >>= 1) {
            const uint32_t x = __shfl_xor(vmin, off, kWave), y = __shfl_xor(vmax, off, kWave);
            vmin = x < vmin ? x : vmin;
            vmax = y > vmax ? y : vmax;
        }
        if (lane == leader) {
            atomicMin(&smin[sl], vmin);
            atomicMax(&smax[sl], vmax);
        }
        act &= ~peers;
    }
}

// ---- Sliced: boundary keys by radix selection -----------------------------------------------------
// A row's place in the (value, row) order of the slicing attribute is the order of its key
// slice_key = canonical value bits << 30 | row (rows < 2^30). The row at rank q goes to partition
// floor(q p / n), so partition(row) = #{e in [1, p-1] : rank(row) >= r_e} with r_e = ceil(e n / p):
// the number of boundary keys (the keys at ranks r_e) at or below the row's key. The boundary
// keys are found digit by digit from the top (14 bits, then six of 8): a histogram pass over the
// rows whose key starts with some boundary's prefix found so far, then one workgroup that moves
// every boundary into its digit. No sort of the relation, and nothing read back.
constexpr int kSelBins0 = 16384;             // first digit: key bits 61..48
constexpr int kSelPasses = 6;                // then 8-bit digits at shifts 40, 32, ..., 0
constexpr int kSelLdsSlots = 64;             // boundary prefixes whose histograms fit LDS
enum { SEL_H = kSelBins0 };                  // int32 offsets in sel_i32: [SEL_H, +256 p) histograms,
                                             // then rem [p], slot [p], nact
__device__ __forceinline__ int64_t sel_rem_off(int32_t p) { return SEL_H + 256 * (int64_t)p; }
__device__ __forceinline__ int64_t sel_slot_off(int32_t p) { return sel_rem_off(p) + p; }
__device__ __forceinline__ int64_t sel_nact_off(int32_t p) { return sel_slot_off(p) + p; }

__global__ void __launch_bounds__(kBlock) sel_zero_kernel(int32_t* __restrict__ sel, int64_t cnt) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * kBlock)
        sel[i] = 0;
}

// The histogram passes: workgroups of 1024 threads over chunks of 4096 rows (grid-stride, about
// two workgroups per CU, so that each clears and flushes its LDS histogram once).
constexpr int kSelChunk = 4096;
constexpr int kSelBloomBits = 65536;

// 16-bit hash of a key prefix (multiplicative, top bits)
__device__ __forceinline__ uint32_t sel_hash(unsigned long long pre) {
    return (uint32_t)((pre * 0x9E3779B97F4A7C15ull) >> 48);
}

// first digit of every row's key, LDS-privatised
__global__ void __launch_bounds__(1024) sel_hist0_kernel(const float* __restrict__ x, int64_t n, int32_t dim,
                                                         int64_t ld, int32_t* __restrict__ sel) {
    __shared__ int32_t h[kSelBins0];
    for (int32_t b = threadIdx.x; b < kSelBins0; b += 1024) h[b] = 0;
    __syncthreads();
    const int64_t nch = (n + kSelChunk - 1) / kSelChunk;
    for (int64_t c = blockIdx.x; c < nch; c += gridDim.x) {
        const int64_t r0 = c * kSelChunk + threadIdx.x;
        float v[kSelChunk / 1024];
#pragma unroll
        for (int it = 0; it < kSelChunk / 1024; ++it) {
            const int64_t i = r0 + (int64_t)it * 1024;
            v[it] = i < n ? x[(int64_t)dim * ld + i] : 0.0f;
        }
#pragma unroll
        for (int it = 0; it < kSelChunk / 1024; ++it) {
            const int64_t i = r0 + (int64_t)it * 1024;
            if (i < n) atomicAdd(&h[(int32_t)(slice_key(canon(v[it]), i) >> 48)], 1);
        }
    }
    __syncthreads();
    for (int32_t b = threadIdx.x; b < kSelBins0; b += 1024)
        if (h[b]) atomicAdd(&sel[b], h[b]);
}

// the boundaries' active prefixes after a digit: slot[e] = index of bkey[e] among the distinct
// prefixes (in order; boundaries past the last row keep slot -1, resolved ones -2, their bkey
// the full key), act = those prefixes, nact
__device__ void sel_slots(unsigned long long* __restrict__ bkey, int32_t nb, int32_t* __restrict__ slot,
                          unsigned long long* __restrict__ act, int32_t* __restrict__ nact) {
    __shared__ int32_t wsum[1024 / kWave];
    __shared__ int32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int32_t base = 0; base < nb; base += 1024) {
        const int32_t e = base + (int32_t)threadIdx.x;
        const bool live = e < nb && slot[e] >= 0;
        const bool first = live && (e == 0 || slot[e - 1] < 0 || bkey[e - 1] != bkey[e]);
        // inclusive count of first flags (wave scan, then across waves)
        int32_t v = first ? 1 : 0;
        for (int off = 1; off < kWave; off <<= 1) {
            const int32_t o = __shfl_up(v, off, kWave);
            if ((int)lane_id() >= off) v += o;
        }
        if (lane_id() == kWave - 1) wsum[threadIdx.x / kWave] = v;
        __syncthreads();
        int32_t before = carry;
        for (int w = 0; w < (int)(threadIdx.x / kWave); ++w) before += wsum[w];
        const int32_t sl = before + v - 1;
        __syncthreads();
        if (live) {
            slot[e] = sl;
            if (first) act[sl] = bkey[e];
        }
        if (threadIdx.x == 1023) carry = before + v;
        __syncthreads();
    }
    if (threadIdx.x == 0) *nact = carry;
}

// after the first digit: each boundary's bin, its rank inside it, the active prefixes
__global__ void __launch_bounds__(1024) sel_find0_kernel(int64_t n, int32_t p, int32_t* __restrict__ sel,
                                                         unsigned long long* __restrict__ bkey) {
    __shared__ int32_t cum[kSelBins0];
    __shared__ int32_t wsum[1024 / kWave];
    // exclusive prefix of the histogram, 16 bins per thread
    constexpr int per = kSelBins0 / 1024;
    int32_t loc[per], t = 0;
#pragma unroll
    for (int k = 0; k < per; ++k) {
        loc[k] = t;
        t += sel[threadIdx.x * per + k];
    }
    int32_t v = t;
    for (int off = 1; off < kWave; off <<= 1) {
        const int32_t o = __shfl_up(v, off, kWave);
        if ((int)lane_id() >= off) v += o;
    }
    if (lane_id() == kWave - 1) wsum[threadIdx.x / kWave] = v;
    __syncthreads();
    int32_t before = 0;
    for (int w = 0; w < (int)(threadIdx.x / kWave); ++w) before += wsum[w];
    before += v - t;
#pragma unroll
    for (int k = 0; k < per; ++k) cum[threadIdx.x * per + k] = before + loc[k];
    __syncthreads();
    const int32_t nb = p - 1;
    int32_t* rem = sel + sel_rem_off(p);
    int32_t* slot = sel + sel_slot_off(p);
    for (int32_t e = threadIdx.x; e < nb; e += 1024) {
        const int64_t r = ((int64_t)(e + 1) * n + p - 1) / p;
        if (r >= n) {  // no row has this rank: above every key
            bkey[e] = ~0ull;
            slot[e] = -1;
            continue;
        }
        int32_t lo = 0, hi = kSelBins0 - 1;  // the last bin whose prefix count is <= r
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (cum[mid] <= r) lo = mid; else hi = mid - 1;
        }
        bkey[e] = (unsigned long long)lo;
        rem[e] = (int32_t)(r - cum[lo]);
        slot[e] = 0;
    }
    for (int32_t a = threadIdx.x; a < p; a += 1024) bkey[2 * p + a] = 0;  // per-prefix maxima
    __syncthreads();
    sel_slots(bkey, nb, slot, bkey + p, sel + sel_nact_off(p));
}

// one 8-bit digit at `shift` of the rows whose key prefix (the bits above it) is active, and per
// active prefix the key of one of its rows (the key itself when only one row has the prefix:
// then exactly one workgroup holds it; a key of 0 is the value left by the clearing);
// LDS-privatised for up to kSelLdsSlots prefixes
__global__ void __launch_bounds__(1024) sel_hist_kernel(const float* __restrict__ x, int64_t n, int32_t dim,
                                                        int64_t ld, int32_t p, int32_t shift,
                                                        int32_t* __restrict__ sel,
                                                        unsigned long long* __restrict__ bkey) {
    __shared__ unsigned long long lact[kSelLdsSlots], lmax[kSelLdsSlots];
    __shared__ int32_t h[kSelLdsSlots * 256];
    __shared__ uint32_t bloom[kSelBloomBits / 32];  // hash bits of the active prefixes
    const int32_t nact = sel[sel_nact_off(p)];
    if (nact == 0) return;  // every boundary resolved (uniform)
    const unsigned long long* act = bkey + p;
    unsigned long long* kmax = bkey + 2 * p;
    int32_t* gh = sel + SEL_H;
    const bool in_lds = nact <= kSelLdsSlots;
    for (int32_t w = threadIdx.x; w < kSelBloomBits / 32; w += 1024) bloom[w] = 0;
    if (in_lds) {
        for (int32_t a = threadIdx.x; a < nact; a += 1024) {
            lact[a] = act[a];
            lmax[a] = 0;
        }
        for (int32_t b = threadIdx.x; b < nact * 256; b += 1024) h[b] = 0;
    }
    __syncthreads();
    for (int32_t a = threadIdx.x; a < nact; a += 1024) {
        const uint32_t hb = sel_hash(act[a]);
        atomicOr(&bloom[hb >> 5], 1u << (hb & 31u));
    }
    __syncthreads();
    const unsigned long long* sact = in_lds ? lact : act;
    const unsigned long long lo_pre = sact[0], hi_pre = sact[nact - 1];
    int32_t top = 1;  // the largest power of two <= nact
    while (2 * top <= nact) top *= 2;
    const int64_t nch = (n + kSelChunk - 1) / kSelChunk;
    for (int64_t c = blockIdx.x; c < nch; c += gridDim.x) {
        const int64_t r0 = c * kSelChunk + threadIdx.x;
        float v[kSelChunk / 1024];
#pragma unroll
        for (int it = 0; it < kSelChunk / 1024; ++it) {
            const int64_t i = r0 + (int64_t)it * 1024;
            v[it] = i < n ? x[(int64_t)dim * ld + i] : 0.0f;
        }
#pragma unroll
        for (int it = 0; it < kSelChunk / 1024; ++it) {
            const int64_t i = r0 + (int64_t)it * 1024;
            const unsigned long long k = slice_key(canon(v[it]), i);
            const unsigned long long pre = k >> (shift + 8);
            if (i >= n || pre < lo_pre || pre > hi_pre) continue;
            const uint32_t hb = sel_hash(pre);  // most rows have no active prefix: one LDS read
            if (((bloom[hb >> 5] >> (hb & 31u)) & 1u) == 0) continue;
            // the last active prefix <= pre, in a fixed number of steps (the rows' searches
            // interleave); the active prefixes are strictly increasing
            int32_t pos = 0;
            for (int32_t step = top; step > 0; step >>= 1)
                if (pos + step < nact && sact[pos + step] <= pre) pos += step;
            if (sact[pos] != pre) continue;
            const int32_t b = pos * 256 + (int32_t)((k >> shift) & 255u);
            // the key of some row with the prefix: a plain store, the one row's key when only one
            // row has it (with several, the value is never used)
            if (in_lds) {
                atomicAdd(&h[b], 1);
                lmax[pos] = k;
            } else {
                atomicAdd(&gh[b], 1);
                kmax[pos] = k;
            }
        }
    }
    __syncthreads();
    if (in_lds) {
        for (int32_t b = threadIdx.x; b < nact * 256; b += 1024)
            if (h[b]) atomicAdd(&gh[b], h[b]);
        for (int32_t a = threadIdx.x; a < nact; a += 1024)
            if (lmax[a]) kmax[a] = lmax[a];
    }
}

// every boundary moves into its digit (one wave per boundary: prefix over the 256 bins of its
// slot), the histograms are cleared for the next digit, and the active prefixes recomputed
__global__ void __launch_bounds__(1024) sel_find_kernel(int32_t p, int32_t* __restrict__ sel,
                                                        unsigned long long* __restrict__ bkey) {
    const int32_t nb = p - 1;
    int32_t* rem = sel + sel_rem_off(p);
    int32_t* slot = sel + sel_slot_off(p);
    int32_t* gh = sel + SEL_H;
    const int lane = (int)lane_id();
    for (int32_t e = threadIdx.x / kWave; e < nb; e += 1024 / kWave) {
        const int32_t a = slot[e];
        if (a < 0) continue;  // (uniform per wave)
        const int32_t* hs = gh + (int64_t)a * 256;
        int32_t c[4], t = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            c[k] = hs[lane * 4 + k];
            t += c[k];
        }
        int32_t v = t;  // inclusive prefix of the lanes' sums
        for (int off = 1; off < kWave; off <<= 1) {
            const int32_t o = __shfl_up(v, off, kWave);
            if (lane >= off) v += o;
        }
        const int32_t r = rem[e];
        if (__shfl(v, kWave - 1, kWave) == 1) {  // one row has the prefix: the boundary is its key
            if (lane == 0) {
                bkey[e] = bkey[2 * p + a];
                slot[e] = -2;
            }
            continue;
        }
        // the digit: the last bin whose exclusive prefix is <= r
        int32_t ex = v - t, dig = -1, below = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (ex <= r) { dig = lane * 4 + k; below = ex; }
            ex += c[k];
        }
        // the highest lane with a digit holds the answer
        const uint64_t m = __ballot(dig >= 0);
        const int src = 63 - __clzll((long long)m);
        dig = __shfl(dig, src, kWave);
        below = __shfl(below, src, kWave);
        if (lane == 0) {
            bkey[e] = (bkey[e] << 8) | (unsigned long long)dig;
            rem[e] = r - below;
        }
    }
    __syncthreads();
    const int32_t nact = sel[sel_nact_off(p)];
    for (int32_t b = threadIdx.x; b < nact * 256; b += 1024) gh[b] = 0;
    for (int32_t a = threadIdx.x; a < nact; a += 1024) bkey[2 * p + a] = 0;
    __syncthreads();
    sel_slots(bkey, nb, slot, bkey + p, sel + sel_nact_off(p));
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

int64_t partition_blocks(int64_t n) { return ceil_div(n > 0 ? n : 1, kPRows); }

// Sort-key layout: the partition above the curve key, in as few 8-bit radix passes as the
// default curve resolution (curve_bits) needs, at most four; the curve takes what is left.
void partition_key_layout(int32_t p, int32_t d, int32_t* cbits, int32_t* key_bits) {
    const int pbits = p > 1 ? bits_for(p) : 0;
    // three 8-bit passes where they leave the curve at least 4 bits per attribute next to the
    // partition id (a partition is a small part of the data space; measured on 64 partitions
    // of 4 attributes: the fourth pass cost more than the finer order saved), else up to four
    // (with hundreds of relations of 8 attributes, 1 bit per attribute loses the order). One
    // partition: the fewest passes that keep 2 bits per attribute (measured on 1M x 6 and on
    // 10M and 10k x 4: each pass saved cost more than the coarser order added; 1 bit per
    // attribute doubled the tests)
    int passes = (pbits + curve_bits(d) * d + 7) / 8;
    if (passes > 4) passes = 4;
    if (passes == 4 && (24 - pbits) / d >= 4) passes = 3;
    if (p == 1 && (2 * d + 7) / 8 < passes) passes = (2 * d + 7) / 8;
    int cb = (8 * passes - pbits) / d;
    cb = cb > 16 ? 16 : (cb < 1 ? 1 : cb);
    *cbits = cb;
    *key_bits = pbits + cb * d;
}


sky_status launch_partition(const PartitionArgs& a, hipStream_t st) {
    const int64_t n = a.n;
    const uint32_t rblocks = (uint32_t)ceil_div(n, kBlock);
    const uint32_t pblocks = (uint32_t)partition_blocks(n);
    const bool multi = a.p > 1;
    int32_t* const part_of_row = multi ? a.part_of_row : nullptr;
    // 0. counters of this partition step
    hipLaunchKernelGGL(partition_init_kernel, dim3((uint32_t)ceil_div((int64_t)a.p * kKill, kBlock)), dim3(kBlock),
                       0, st, a.p, a.pcount, a.kmin, a.seg_tests, a.tests, a.smin, a.smax, a.pruned);
    SKY_HIP(hipGetLastError());
    if (a.scheme == SKY_ANGULAR) {
        hipLaunchKernelGGL(angular_table_kernel, dim3(1), dim3(256), 0, st, a.m, a.tan2);
        SKY_HIP(hipGetLastError());
    } else if (a.scheme == SKY_SLICED && multi) {
        // the keys at the boundary ranks of the (value, row) order of the slicing attribute
        const int64_t zc = slice_select_elems(a.p);
        hipLaunchKernelGGL(sel_zero_kernel, dim3((uint32_t)(ceil_div(zc, kBlock) < 1024 ? ceil_div(zc, kBlock) : 1024)),
                           dim3(kBlock), 0, st, a.sel_i32, zc);
        int dev = 0, cus = 0;
        SKY_HIP(hipGetDevice(&dev));
        SKY_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        const int64_t nch = ceil_div(n, kSelChunk);
        const uint32_t sblocks = (uint32_t)(nch < 1 ? 1 : (nch < 2 * (int64_t)cus ? nch : 2 * (int64_t)cus));
        hipLaunchKernelGGL(sel_hist0_kernel, dim3(sblocks), dim3(1024), 0, st, a.x, n, a.slice_dim, a.ld,
                           a.sel_i32);
        hipLaunchKernelGGL(sel_find0_kernel, dim3(1), dim3(1024), 0, st, n, a.p, a.sel_i32, a.sel_key);
        for (int k = 0; k < kSelPasses; ++k) {
            const int32_t shift = 8 * (kSelPasses - 1 - k);
            hipLaunchKernelGGL(sel_hist_kernel, dim3(sblocks), dim3(1024), 0, st, a.x, n, a.slice_dim, a.ld, a.p,
                               shift, a.sel_i32, a.sel_key);
            hipLaunchKernelGGL(sel_find_kernel, dim3(1), dim3(1024), 0, st, a.p, a.sel_i32, a.sel_key);
        }
        SKY_HIP(hipGetLastError());
    }
    // 1. classify
    ClassifyArgs ca{};
    ca.x = a.x; ca.n = n; ca.d = a.d; ca.ld = a.ld;
    ca.scheme = multi ? a.scheme : SKY_NONE; ca.p = a.p; ca.m = a.m;
    ca.tan2 = a.tan2; ca.seg_off = a.seg_off;
    ca.slice_dim = a.slice_dim; ca.bkey = a.sel_key;
    ca.part_of_row = part_of_row; ca.pcount = a.pcount; ca.kmin = a.kmin;
    ca.dev_status = a.dev_status;
    const size_t clds = (size_t)a.p * (sizeof(unsigned long long) + sizeof(int32_t)) +
                        (ca.scheme == SKY_SLICED ? (size_t)(a.p - 1) * sizeof(unsigned long long) : 0);
    SKY_DISPATCH_D(a.d, classify_kernel, dim3(pblocks), dim3(kPT), clds, st, ca);
    SKY_HIP(hipGetLastError());
    // 2. partition offsets; Grid pruning
    const bool prune = a.scheme == SKY_GRID && multi;
    hipLaunchKernelGGL(part_offsets_kernel, dim3(1), dim3(1024), 0, st, (const int32_t*)a.pcount, a.p, n,
                       a.part_off, prune ? nullptr : a.stats_out);
    if (prune)
        hipLaunchKernelGGL(grid_prune_kernel, dim3(1), dim3(1024), 0, st, (const int32_t*)a.part_off, a.m, a.d,
                           a.p, a.pruned, a.stats_out);
    SKY_HIP(hipGetLastError());
    // 3. killers and the prefilter (or every row kept)
    if (a.prefilter) {
        SKY_DISPATCH_D(a.d, kill_rows_kernel, dim3((uint32_t)ceil_div((int64_t)a.p * kKill, kBlock)), dim3(kBlock),
                       0, st, (const unsigned long long*)a.kmin, (const uint8_t*)(a.scheme == SKY_GRID ? a.pruned : nullptr),
                       a.p, a.x, a.d, a.ld, a.krow, a.kval);
        SKY_HIP(hipGetLastError());
    }
    FilterArgs fa{};
    fa.n = n; fa.d = a.d; fa.ld = a.ld; fa.p = a.p; fa.x = a.x;
    fa.part_of_row = part_of_row;
    fa.pruned = a.scheme == SKY_GRID && multi ? a.pruned : nullptr;
    fa.krow = a.krow; fa.kval = a.kval;
    fa.killers = a.prefilter ? 1 : 0;
    fa.alive = a.alive; fa.xa = a.xa; fa.blk = a.blk;
    fa.seg_tests = a.seg_tests; fa.tests = a.tests;
    // LDS: the per-partition test counters, then (when it fits) the killer values and rows
    const int64_t tab = (int64_t)a.p * kKill * partition_row_stride(a.d);
    size_t flds = 0;
    if (a.prefilter) {
        flds = sizeof(unsigned int) * (size_t)((a.p + 3) & ~3);
        if (tab <= kKillLds)  // padded blocks (filter_kernel)
            flds += sizeof(float) * (size_t)a.p * (size_t)(kKill * partition_row_stride(a.d) + 4) +
                    sizeof(int32_t) * (size_t)a.p * (kKill + 1);
    }
    SKY_DISPATCH_D(a.d, filter_kernel, dim3(pblocks), dim3(kPT), flds, st, fa);
    SKY_HIP(hipGetLastError());
    // 4. the kept rows with their keys
    SKY_TRY(launch_exclusive_scan(a.blk, a.blk, pblocks, a.scan_tmp, st));
    int32_t cbits = 1, key_bits = 1;
    partition_key_layout(a.p, a.d, &cbits, &key_bits);
    CompactArgs ka{};
    ka.n = n; ka.d = a.d; ka.alive = a.alive; ka.blk_off = a.blk;
    ka.part_of_row = part_of_row; ka.xa = a.xa;
    ka.cbits = cbits; ka.pshift = cbits * a.d;
    ka.keys = a.k0; ka.rows = a.v0; ka.n_live = a.n_live;
    SKY_DISPATCH_D(a.d, compact_kernel, dim3(pblocks), dim3(kPT), 0, st, ka);
    SKY_HIP(hipGetLastError());
    // 5. stable sort of the kept rows by (partition, curve key)
    const uint32_t* sorted_keys = nullptr;
    const uint32_t* order = nullptr;
    SKY_TRY(launch_radix_sort(a.k0, a.v0, a.k1, a.v1, n, key_bits, a.radix_tmp, st, &sorted_keys, &order,
                              a.n_live));
    // 6. the partition-contiguous copy (with several partitions, fewer and longer wave runs: each
    // wave adds its runs' score ranges to the partitions' with atomics, which queue when many
    // waves share a partition)
    const uint32_t gcap = multi ? 512u : 8192u;
    SKY_DISPATCH_D(a.d, part_gather_kernel, dim3(rblocks < gcap ? rblocks : gcap), dim3(kBlock), 0, st, sorted_keys, order,
                   (const int32_t*)a.n_live, a.d, cbits * a.d, multi ? 1 : 0, (const float*)a.xa, a.xp, a.ldp,
                   a.rowid, a.seg, a.fsum, a.smin, a.smax, a.iota_out);
    SKY_HIP(hipGetLastError());
    return SKY_OK;
}

}  // namespace sky
