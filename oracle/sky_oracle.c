/*
 * sky_oracle.c -- TEST INFRASTRUCTURE ONLY (the oracle).
 *
 * A plain, slow, obviously correct CPU implementation of what the skyline / grid-resistance
 * path computes, written from the definitions of
 *   "Parallelizing the Computation of Robustness for Measuring the Strength of Tuples"
 *   (Ciaccia, Martinenghi et al., arXiv 2412.02274).
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may load this
 * library. It shares no code, header, table or helper with the GPU library.
 *
 * Build: gcc -O2 -std=c11 -fno-fast-math -ffp-contract=off -fopenmp -shared -fPIC
 * (no FMA contraction, IEEE semantics; the only FP32 arithmetic is one multiply per key).
 *
 * Layout of every relation: structure of arrays, attribute k of row i at x[k*ld + i], ld >= n.
 *
 * Parity status of each function (what pins it, see the tests under tests/):
 *   orc_count_invalid       -- pinned (hand-made values).
 *   orc_skyline             -- pinned (brute force on tiny inputs, d=1 and d=2 closed forms).
 *   orc_skyline_sfs         -- pinned (equals orc_skyline on random inputs with ties).
 *   orc_local_skylines      -- pinned (each partition's local skyline equals the Python brute
 *                              force of Def. 1 over that partition's rows alone, for Grid with
 *                              a pruned cell, Angular and Sliced ids on data with duplicates;
 *                              union/final == orc_skyline for every scheme).
 *   orc_grid_part           -- pinned (paper's 3x3 worked example, cell bounds).
 *   orc_grid_pruned         -- pinned (paper's worked example: cell 1 prunes exactly 5 and 8).
 *   orc_angular_part        -- pinned (angles recomputed in closed form on special directions
 *                              and by arccos on random rows).
 *   orc_sliced_part         -- pinned (sizes floor/ceil(N/p), order on the slicing attribute).
 *   orc_gres, orc_gres_rows -- pinned (Python brute force of Def. 2 with set semantics, FP32
 *                              and exact rationals; the worked counterexample; invariants;
 *                              the two agree on sampled rows).
 *   orc_skyline_rows        -- pinned (equals orc_skyline on the sampled rows).
 *   orc_representatives     -- pinned (numpy lexsort of the FP32 scores for the selection, the
 *                              Python brute force of Def. 1 for the kept set).
 *   orc_dominated_by        -- pinned (brute force of Def. 1 on tiny inputs).
 *   orc_ell, orc_ell_sorted -- pinned (exact-rational brute force over pairs on tiny inputs, a
 *                              hand-worked lattice example, degenerate inputs; the two agree).
 *   orc_gbar                -- pinned (floor(1/ell) in exact rationals; on lattice data no exit
 *                              appears beyond g_bar, checked by the exact brute force).
 *   test counts (orc_skyline_sfs return value, orc_gres *tests) -- "parity unpinned": they
 *                              depend on the scan order; reported, never compared.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define X(x, ld, k, i) ((x)[(int64_t)(k) * (ld) + (i)])

/* ------------------------------------------------------------------------------------------ */
/* Domain (Sec. 2 and Sec. 4): values are non-negative reals; the synthetic data and the Grid  */
/* numbering assume [0, 1). Returns the number of values that are NaN/inf or outside [0, 1).    */
/* -0.0 compares equal to 0 and is accepted.                                                     */
/* ------------------------------------------------------------------------------------------ */
int64_t orc_count_invalid(const float* x, int64_t n, int32_t d, int64_t ld) {
    int64_t bad = 0;
    for (int32_t k = 0; k < d; ++k)
        for (int64_t i = 0; i < n; ++i) {
            float v = X(x, ld, k, i);
            if (!(v >= 0.0f && v < 1.0f)) ++bad; /* NaN fails both comparisons */
        }
    return bad;
}

/* ------------------------------------------------------------------------------------------ */
/* Def. 1 (Sec. 2): s dominates t iff s[A] <= t[A] for every attribute A and s[A'] < t[A'] for  */
/* some attribute A'. Smaller values are preferred.                                              */
/* ------------------------------------------------------------------------------------------ */
static int dominates(const float* x, int64_t ld, int32_t d, int64_t s, int64_t t) {
    int strict = 0;
    for (int32_t k = 0; k < d; ++k) {
        float a = X(x, ld, k, s), b = X(x, ld, k, t);
        if (a > b) return 0;
        if (a < b) strict = 1;
    }
    return strict;
}

/* Def. 1: Sky(r) = { t in r | no s in r dominates t }. member[i] = 1 iff row i is in Sky(r).
 * Nested loops over the definition; the inner search stops at the first dominator. */
void orc_skyline(const float* x, int64_t n, int32_t d, int64_t ld, uint8_t* member) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < n; ++t) {
        uint8_t in = 1;
        for (int64_t s = 0; s < n; ++s)
            if (s != t && dominates(x, ld, d, s, t)) { in = 0; break; }
        member[t] = in;
    }
}

/* ------------------------------------------------------------------------------------------ */
/* SFS (Sort-Filter-Skyline), the plain sequential algorithm the paper uses for its sequential */
/* timings (Sec. 4, execution times). Rows are presorted by a monotone scoring function f       */
/* (Sec. 2); then a single scan keeps a window of confirmed skyline rows: a row enters the      */
/* window iff no window row dominates it. Monotonicity makes every dominator of a row come     */
/* before it, so the window is exactly Sky(r).                                                  */
/* f = sum of the attributes in FP32, ascending attribute order; ties are broken               */
/* lexicographically on the attributes and then by row index, so that s dominates t implies s  */
/* sorts before t even when the FP32 sums are equal.                                            */
/* ------------------------------------------------------------------------------------------ */
typedef struct { const float* x; int64_t ld; int32_t d; const float* f; } sfs_ctx;
static sfs_ctx g_sfs; /* qsort has no context argument; the oracle is single-call at a time */

static int sfs_cmp(const void* pa, const void* pb) {
    int64_t a = *(const int64_t*)pa, b = *(const int64_t*)pb;
    if (g_sfs.f[a] < g_sfs.f[b]) return -1;
    if (g_sfs.f[a] > g_sfs.f[b]) return 1;
    for (int32_t k = 0; k < g_sfs.d; ++k) {
        float u = X(g_sfs.x, g_sfs.ld, k, a), v = X(g_sfs.x, g_sfs.ld, k, b);
        if (u < v) return -1;
        if (u > v) return 1;
    }
    return (a > b) - (a < b);
}

/* Returns the number of dominance tests made by the window scan (reported, not compared). */
int64_t orc_skyline_sfs(const float* x, int64_t n, int32_t d, int64_t ld, uint8_t* member) {
    float* f = (float*)malloc(sizeof(float) * (size_t)(n > 0 ? n : 1));
    int64_t* ord = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t* win = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        float acc = 0.0f;
        for (int32_t k = 0; k < d; ++k) acc += X(x, ld, k, i);
        f[i] = acc;
        ord[i] = i;
        member[i] = 0;
    }
    g_sfs.x = x; g_sfs.ld = ld; g_sfs.d = d; g_sfs.f = f;
    qsort(ord, (size_t)n, sizeof(int64_t), sfs_cmp);
    int64_t w = 0, tests = 0;
    for (int64_t j = 0; j < n; ++j) {
        int64_t t = ord[j];
        int dominated = 0;
        for (int64_t q = 0; q < w; ++q) {
            ++tests;
            if (dominates(x, ld, d, win[q], t)) { dominated = 1; break; }
        }
        if (!dominated) { win[w++] = t; member[t] = 1; }
    }
    free(f); free(ord); free(win);
    return tests;
}

/* ------------------------------------------------------------------------------------------ */
/* Two-phase parallel skyline (Sec. 3), phase 1: the local skyline of every partition, by the  */
/* definition restricted to the rows of that partition. Rows whose partition is flagged in      */
/* skip[] (Grid cells pruned by grid dominance, Def. 3) contribute no local skyline rows.       */
/* Phase 2 (the final skyline of the union) is orc_skyline over the union.                     */
/* ------------------------------------------------------------------------------------------ */
void orc_local_skylines(const float* x, int64_t n, int32_t d, int64_t ld, const int32_t* part,
                        const uint8_t* skip /* nullable, indexed by partition */, uint8_t* local) {
    /* rows grouped by partition (a counting sort; bookkeeping only) so that each row is
     * compared with the rows of its own partition */
    int32_t p = 0;
    for (int64_t i = 0; i < n; ++i) if (part[i] + 1 > p) p = part[i] + 1;
    int64_t* start = (int64_t*)calloc((size_t)p + 1, sizeof(int64_t));
    int64_t* rows = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) start[part[i] + 1]++;
    for (int32_t j = 0; j < p; ++j) start[j + 1] += start[j];
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(p > 0 ? p : 1));
    for (int32_t j = 0; j < p; ++j) fill[j] = start[j];
    for (int64_t i = 0; i < n; ++i) rows[fill[part[i]]++] = i;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < n; ++t) {
        int32_t pt = part[t];
        if (skip && skip[pt]) { local[t] = 0; continue; }
        uint8_t in = 1;
        for (int64_t q = start[pt]; q < start[pt + 1]; ++q) {
            int64_t s = rows[q];
            if (s != t && dominates(x, ld, d, s, t)) { in = 0; break; }
        }
        local[t] = in;
    }
    free(start); free(rows); free(fill);
}

/* ------------------------------------------------------------------------------------------ */
/* Grid partitioning (Sec. 3.1): with m slices per dimension, the partition of t is            */
/*   sum_i floor(t[A_i] * m) * m^(i-1),  i = 1..d  (first attribute varies fastest).            */
/* The coordinate floor(x*m) uses one FP32 multiply; it is clamped to m-1 defensively (it is   */
/* already < m for x < 1).                                                                      */
/* ------------------------------------------------------------------------------------------ */
void orc_grid_part(const float* x, int64_t n, int32_t d, int64_t ld, int32_t m, int32_t* part) {
    for (int64_t i = 0; i < n; ++i) {
        int64_t id = 0, w = 1;
        for (int32_t k = 0; k < d; ++k) {
            float prod = X(x, ld, k, i) * (float)m;
            int64_t c = (int64_t)floorf(prod);
            if (c > m - 1) c = m - 1;
            if (c < 0) c = 0;
            id += c * w;
            w *= m;
        }
        part[i] = (int32_t)id;
    }
}

/* Def. 3 (grid dominance): cell c_i grid-dominates c_h iff c_i[j] < c_h[j] in every dimension.
 * A non-empty cell that grid-dominates another lets the latter be disregarded (Sec. 3.1).
 * pruned[h] = 1 iff some non-empty cell grid-dominates cell h. Cells are numbered as in
 * orc_grid_part; coordinates are 0-based. */
void orc_grid_pruned(const uint8_t* nonempty, int32_t m, int32_t d, uint8_t* pruned) {
    int64_t cells = 1;
    for (int32_t k = 0; k < d; ++k) cells *= m;
    for (int64_t h = 0; h < cells; ++h) {
        pruned[h] = 0;
        for (int64_t c = 0; c < cells && !pruned[h]; ++c) {
            if (!nonempty[c]) continue;
            int64_t a = c, b = h, all_less = 1;
            for (int32_t k = 0; k < d; ++k) {
                if (!(a % m < b % m)) { all_less = 0; break; }
                a /= m; b /= m;
            }
            if (all_less) pruned[h] = 1;
        }
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Angle-based partitioning, Eq. (1) (Sec. 3.1): hyper-spherical angles phi_1..phi_{d-1} of t  */
/* (the standard conversion: phi_i = atan2( sqrt(sum_{j>i} t_j^2), t_i ), in [0, pi/2] for      */
/* non-negative data), and partition sum_{i=1}^{d-1} floor(2*phi_i*m/pi) * m^(i-1).             */
/* The bucket of phi_i = pi/2 exactly would be m; it is clamped to m-1. Computed in double.     */
/* A zero sub-vector (t_i = 0 and all later attributes 0) has atan2(0, 0) = 0, bucket 0.         */
/* near[i] has bit i-1 set when angle phi_i lies within 1e-9 (relative) of a bucket boundary:  */
/* there a different but equally faithful evaluation of the same formula may put the row in    */
/* the bucket on the other side of that boundary (and only there).                              */
/* ------------------------------------------------------------------------------------------ */
void orc_angular_part(const float* x, int64_t n, int32_t d, int64_t ld, int32_t m, int32_t* part,
                      int32_t* near) {
    const double pi = 3.14159265358979323846;
    for (int64_t i = 0; i < n; ++i) {
        int64_t id = 0, w = 1;
        int32_t nb = 0;
        for (int32_t a = 0; a + 1 < d; ++a) {
            double tail = 0.0;
            for (int32_t j = a + 1; j < d; ++j) {
                double v = (double)X(x, ld, j, i);
                tail += v * v;
            }
            /* + 0.0 turns an accepted -0.0 into +0.0, so that atan2 sees the value 0 */
            double phi = atan2(sqrt(tail), (double)X(x, ld, a, i) + 0.0);
            double q = 2.0 * phi * (double)m / pi;
            int64_t b = (int64_t)floor(q);
            if (b > m - 1) b = m - 1;
            if (b < 0) b = 0;
            double r = q - floor(q + 0.5);
            if (fabs(r) < 1e-9 * (q > 1.0 ? q : 1.0) && q > 0.5 && q < (double)m - 0.5) nb |= 1 << a;
            id += b * w;
            w *= m;
        }
        part[i] = (int32_t)id;
        if (near) near[i] = nb;
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Sliced partitioning (Sec. 3.1): sort on one chosen attribute, then the i-th row of the       */
/* ordering (1-based) goes to partition floor((i-1)*p/N). Equal values are ordered by row index. */
/* ------------------------------------------------------------------------------------------ */
static const float* g_slice_col;
static int slice_cmp(const void* pa, const void* pb) {
    int64_t a = *(const int64_t*)pa, b = *(const int64_t*)pb;
    float u = g_slice_col[a], v = g_slice_col[b];
    if (u < v) return -1;
    if (u > v) return 1;
    return (a > b) - (a < b);
}

void orc_sliced_part(const float* x, int64_t n, int32_t d, int64_t ld, int32_t dim, int32_t p,
                     int32_t* part) {
    (void)d;
    int64_t* ord = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) ord[i] = i;
    g_slice_col = x + (int64_t)dim * ld;
    qsort(ord, (size_t)n, sizeof(int64_t), slice_cmp);
    for (int64_t i = 0; i < n; ++i) part[ord[i]] = (int32_t)((i * (int64_t)p) / n);
    free(ord);
}

/* Closest achievable number of partitions (Sec. 4): Grid gives m^d and Angular m^(d-1)
 * partitions; pick m >= 2 minimising |m^e - target| (ties to the smaller m) so that the
 * resulting p is > 1. */
int32_t orc_closest_m(int64_t target, int32_t e) {
    if (e < 1) return -1;
    int32_t best = 2;
    double bestdiff = fabs(pow(2.0, e) - (double)target);
    for (int32_t m = 3; m <= 4096; ++m) {
        double v = pow((double)m, e);
        double diff = fabs(v - (double)target);
        if (diff < bestdiff) { best = m; bestdiff = diff; }
        if (v > (double)target) break;
    }
    return best;
}

/* ------------------------------------------------------------------------------------------ */
/* Grid projection (Sec. 2): gproj(t, g) = < floor(t[i]*g)/g >. Dominance between projections   */
/* is decided by the integer numerators floor(t[i]*g) (dividing every value by the same g > 0   */
/* keeps the order). The product is one IEEE FP32 multiply, rounded to nearest even.            */
/* ------------------------------------------------------------------------------------------ */
static int32_t key(float v, int32_t g) { return (int32_t)floorf(v * (float)g); }

static int proj_dominates(const float* x, int64_t ld, int32_t d, int64_t s, int64_t t, int32_t g) {
    int strict = 0;
    for (int32_t k = 0; k < d; ++k) {
        int32_t a = key(X(x, ld, k, s), g), b = key(X(x, ld, k, t), g);
        if (a > b) return 0;
        if (a < b) strict = 1;
    }
    return strict;
}

/* ------------------------------------------------------------------------------------------ */
/* Grid resistance, Def. 2 (Sec. 2): gres(t) = min { 1/g : gproj(t,g) is not in              */
/* Sky(gproj(r,g)) }, 1 when there is no such g; the levels are g = 2..g_max, the range Alg. 1 */
/* (Sec. 3.2) searches (g = 1 sends every value of [0, 1) to 0, so nothing leaves there).     */
/* The projection of t is outside the projected skyline iff some projected candidate dominates */
/* it, and the smallest 1/g is the largest such g, so each tuple scans g downwards from g_max   */
/* and stops at the first level where a candidate's projection dominates its own.              */
/* Candidates cand[0..s) are the skyline rows (gres is stable, Sec. 3.2: dominated rows never  */
/* change it); they are also the tuples whose gres is computed.                                */
/* g_exit_of returns that level, or 1; *tests counts the projected dominance tests made,       */
/* scanning candidates in the given order and stopping at the first dominator. This is also   */
/* the count of Alg. 1's level-by-level scan: both test the same (tuple, level) pairs against */
/* the same candidates in the same order (reported, not compared).                            */
/* ------------------------------------------------------------------------------------------ */
static int32_t g_exit_of(const float* x, int64_t ld, int32_t d, const int64_t* cand, int64_t s,
                         int64_t t, int32_t g_max, int64_t* tests) {
    for (int32_t g = g_max; g >= 2; --g)
        for (int64_t q = 0; q < s; ++q) {
            if (cand[q] == t) continue;
            ++*tests;
            if (proj_dominates(x, ld, d, cand[q], t, g)) return g;
        }
    return 1; /* no level at which the projection of t is dominated: gres(t) = 1 */
}

/* Output: g_exit[j] for t = cand[j]; gres = 1/g_exit. */
void orc_gres(const float* x, int64_t n, int32_t d, int64_t ld, const int64_t* cand, int64_t s,
              int32_t g_max, int32_t* g_exit, int64_t* tests) {
    (void)n;
    int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : total)
    for (int64_t j = 0; j < s; ++j) {
        int64_t c = 0;
        g_exit[j] = g_exit_of(x, ld, d, cand, s, cand[j], g_max, &c);
        total += c;
    }
    if (tests) *tests = total;
}

/* The same search for a subset of the tuples: targets[0..nt) (row ids) against the candidates
 * (lets full-size parity be checked on sampled tuples). */
void orc_gres_rows(const float* x, int64_t n, int32_t d, int64_t ld, const int64_t* cand,
                   int64_t s, const int64_t* targets, int64_t nt, int32_t g_max, int32_t* g_exit) {
    (void)n;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < nt; ++j) {
        int64_t c = 0;
        g_exit[j] = g_exit_of(x, ld, d, cand, s, targets[j], g_max, &c);
    }
}

/* Membership of single rows in Sky(r), by the definition (for sampled full-size parity). */
void orc_skyline_rows(const float* x, int64_t n, int32_t d, int64_t ld, const int64_t* rows,
                      int64_t nr, uint8_t* member) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < nr; ++j) {
        uint8_t in = 1;
        for (int64_t s = 0; s < n; ++s)
            if (s != rows[j] && dominates(x, ld, d, s, rows[j])) { in = 0; break; }
        member[j] = in;
    }
}

/* ------------------------------------------------------------------------------------------ */
/* The upper end of Alg. 1's level range (Sec. 3.2): ell is the smallest non-zero absolute      */
/* difference between two values of the same attribute, over every pair of rows and every      */
/* attribute, and g_bar = floor(1/ell); beyond g_bar no new dominance between grid projections  */
/* can appear. Each difference is taken in FP64 (the difference of two FP32 values, rounded to  */
/* nearest; exact whenever the two exponents are within 29 of each other). +inf when no        */
/* attribute holds two different values.                                                       */
/* orc_ell is the definition as nested loops over pairs.                                       */
/* ------------------------------------------------------------------------------------------ */
double orc_ell(const float* x, int64_t n, int32_t d, int64_t ld) {
    double best = INFINITY;
    for (int32_t k = 0; k < d; ++k) {
#pragma omp parallel for schedule(dynamic, 64) reduction(min : best)
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = i + 1; j < n; ++j) {
                double e = fabs((double)X(x, ld, k, i) - (double)X(x, ld, k, j));
                if (e > 0.0 && e < best) best = e;
            }
    }
    return best;
}

static int dbl_cmp(const void* pa, const void* pb) {
    double a = *(const double*)pa, b = *(const double*)pb;
    return (a > b) - (a < b);
}

/* The same minimum through a sort of each attribute (for sizes where pairs are too many): in   */
/* sorted order, the smallest non-zero difference is between neighbours.                       */
double orc_ell_sorted(const float* x, int64_t n, int32_t d, int64_t ld) {
    double best = INFINITY;
    double* v = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int32_t k = 0; k < d; ++k) {
        for (int64_t i = 0; i < n; ++i) v[i] = (double)X(x, ld, k, i);
        qsort(v, (size_t)n, sizeof(double), dbl_cmp);
        for (int64_t i = 1; i < n; ++i) {
            double e = v[i] - v[i - 1];
            if (e > 0.0 && e < best) best = e;
        }
    }
    free(v);
    return best;
}

/* g_bar = floor(1/ell), the quotient rounded to nearest in FP64; 1 when ell is +inf (no level  */
/* above 1 to search).                                                                         */
double orc_gbar(double ell) {
    if (!(ell < INFINITY)) return 1.0;
    return floor(1.0 / ell);
}

/* ------------------------------------------------------------------------------------------ */
/* Representative Filtering (Sec. 3.1): the representatives are the k tuples with the smallest  */
/* value of a monotone scoring function, here f = the FP32 sum of the attributes in ascending   */
/* attribute order (the SFS score); equal scores are taken in row order. Representatives       */
/* dominated by another representative add no pruning power and are dropped: kept[j] = 1 for    */
/* the ones no other representative dominates (Def. 1).                                         */
/* ------------------------------------------------------------------------------------------ */
typedef struct { float f; int64_t row; } rep_key;

static int rep_cmp(const void* pa, const void* pb) {
    const rep_key *a = (const rep_key*)pa, *b = (const rep_key*)pb;
    if (a->f < b->f) return -1;
    if (a->f > b->f) return 1;
    return (a->row > b->row) - (a->row < b->row);
}

int64_t orc_representatives(const float* x, int64_t n, int32_t d, int64_t ld, int64_t k,
                            int64_t* rows, uint8_t* kept) {
    if (k > n) k = n;
    rep_key* v = (rep_key*)malloc(sizeof(rep_key) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        float f = 0.0f;
        for (int32_t a = 0; a < d; ++a) f = f + X(x, ld, a, i);
        v[i].f = f;
        v[i].row = i;
    }
    qsort(v, (size_t)n, sizeof(rep_key), rep_cmp);
    for (int64_t j = 0; j < k; ++j) rows[j] = v[j].row;
    free(v);
    for (int64_t j = 0; j < k; ++j) {
        kept[j] = 1;
        for (int64_t q = 0; q < k && kept[j]; ++q)
            if (q != j && dominates(x, ld, d, rows[q], rows[j])) kept[j] = 0;
    }
    return k;
}

/* flags[i] = 1 when some row of by[0..nb) dominates row i (Def. 1). */
void orc_dominated_by(const float* x, int64_t n, int32_t d, int64_t ld, const int64_t* by,
                      int64_t nb, uint8_t* flags) {
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        uint8_t f = 0;
        for (int64_t q = 0; q < nb && !f; ++q)
            if (dominates(x, ld, d, by[q], i)) f = 1;
        flags[i] = f;
    }
}

/* Projected key of one value, exposed so that the quantisation rule itself can be pinned. */
int32_t orc_key(float v, int32_t g) { return key(v, g); }

int32_t orc_num_threads(void) {
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
