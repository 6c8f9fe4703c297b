/*
 * sky.h -- C ABI of libsky: skyline over partitioned data and grid resistance (gres) of the
 * skyline tuples, on one AMD Instinct MI355X (gfx950).
 *
 * Method: "Parallelizing the Computation of Robustness for Measuring the Strength of Tuples"
 * (arXiv 2412.02274). Definitions used below:
 *   Def. 1 (Sec. 2)   dominance s < t: s[A] <= t[A] for every attribute, < for at least one
 *                     (smaller is better); Sky(r) = tuples of r dominated by no tuple of r.
 *   Def. 2 (Sec. 2)   grid projection gproj(t,g) = < floor(t[i]*g)/g >; grid resistance
 *                     gres(t;r) = min { 1/g : gproj(t,g) not in Sky(gproj(r,g)) }, 1 if none.
 *   Sec. 3            two-phase parallel skyline: local skylines of partitions, then the
 *                     skyline of their union.
 *   Sec. 3.1          Grid (with grid dominance, Def. 3), Angle-based (Eq. (1)) and Sliced
 *                     partitioning; Sec. 4: Grid/Angular use the closest achievable p > 1.
 *   Alg. 1 (Sec. 3.2) gres of every skyline tuple, scanning g from g_max down to 2.
 *
 * Conventions shared by every entry point
 *   - Relations are FP32 in structure-of-arrays layout: attribute k of row i at x[k*ld + i],
 *     ld >= n. Row indices are 0-based. Values must be finite and in [0, 1) (the domain the
 *     paper assumes for its data and for Grid numbering); -0.0 is accepted and treated as 0.
 *   - Quantisation contract: the projected key of value v at level g is
 *     (int)floorf(v * (float)g) with ONE IEEE FP32 multiply rounded to nearest even (no FMA,
 *     no fast-math); dominance between projections compares these integer keys.
 *   - All pointers named dev_* / x / ws / outputs are DEVICE pointers; the caller owns them
 *     (typically torch tensors) and keeps them alive until the work on `stream` has finished
 *     (and, for a plan, until sky_plan_destroy). The library never allocates or frees device
 *     memory and never changes the current device.
 *   - Argument errors are returned synchronously with no device work queued. Data-dependent
 *     errors (a value outside the domain, an output capacity that is too small) are written
 *     to the device word *dev_status (first error wins; the caller zeroes it beforehand and
 *     reads it after synchronising the stream). Outputs are defined only when both are SKY_OK.
 *   - Work is queued on `stream` (a hipStream_t passed as void*; NULL = the null stream).
 *     The calls of the plain path -- sky_ingest, sky_build, sky_local_skylines, sky_merge,
 *     sky_gres, gres_compute, gres_prepare, gres_search -- never synchronise and never read
 *     anything back: every count they need stays on the device and every launch is sized by a
 *     bound known when the call is made, so a whole pass can be captured in a HIP graph and
 *     replayed. The inspection call sky_plan_info, and
 *     sky_batch_create, sky_batch_skylines and sky_batch_tune, read back or copy small host
 *     tables and synchronise.
 *   - Thread safety: plans and batches are independent; one must not be used by two threads
 *     at once.
 *     No global mutable state.
 */
#ifndef SKY_H
#define SKY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum sky_status {
    SKY_OK = 0,
    SKY_ERR_INVALID_ARG = 1, /* null pointer, bad size, bad option */
    SKY_ERR_DOMAIN = 2,      /* a value is NaN/inf or outside [0, 1) (device-side) */
    SKY_ERR_WORKSPACE = 3,   /* ws_bytes below the size returned by the *_workspace_bytes call */
    SKY_ERR_CAPACITY = 4,    /* output capacity too small (device-side; size in *dev_count) */
    SKY_ERR_HIP = 5,         /* a HIP runtime call failed */
    SKY_ERR_STATE = 6,       /* call out of order on a plan */
    SKY_ERR_UNSUPPORTED = 7  /* valid request outside the implemented limits */
} sky_status;

typedef enum sky_scheme {
    SKY_NONE = 0,    /* one partition: plain skyline */
    SKY_GRID = 1,    /* Sec. 3.1 Grid: p = m^d cells, cell pruning by grid dominance (Def. 3) */
    SKY_ANGULAR = 2, /* Sec. 3.1 Angle-based, Eq. (1): p = m^(d-1) */
    SKY_SLICED = 3   /* Sec. 3.1 Sliced: sort on one attribute, p equal-size slices */
} sky_scheme;

/* Limits of this implementation. */
#define SKY_MAX_D 16           /* attributes per tuple */
#define SKY_MAX_CELLS 4096     /* partitions of any scheme (Grid m^d, Angular m^(d-1), Sliced p) */
#define SKY_MAX_G 16777216     /* largest g_max accepted by gres_compute: 2^24, the largest level
                                  at which (float)g is exact, as the key contract needs */
#define SKY_MAX_REPS 1024      /* largest sky_params.reps */
#define SKY_KILLERS 8          /* rows per partition that sky_build's prefilter tests every row of
                                  the partition against (see sky_params.prefilter_off) */
#define SKY_NOALLOC_SCRATCH_BYTES 67108864 /* 64 MiB: the fixed device workspace of
                                              gres_compute_noalloc, per device */

/* gres_compute mapping choice (sky_gres_opts.mapping). */
#define SKY_GRES_AUTO 0         /* pick by shape */
#define SKY_GRES_TILES 1        /* one wave per tuple, lanes over candidate tiles */
#define SKY_GRES_LEVELS 2       /* one wave per tuple, lanes over 64 consecutive levels g */

typedef struct sky_params {
    int32_t scheme;    /* sky_scheme */
    int32_t target_p;  /* requested partitions; Grid/Angular take the closest m^e > 1 (Sec. 4),
                          Sliced takes exactly min(target_p, n); ignored for SKY_NONE */
    int32_t slice_dim; /* Sliced: attribute to sort on (0-based) */
    int32_t reps;      /* Representative Filtering (Sec. 3.1), 0 = off, at most SKY_MAX_REPS: the
                          reps rows with the smallest FP32 attribute sum (summed in attribute
                          order; equal sums in row order) are the representatives; those no
                          other representative dominates are shared with every partition, and
                          the rows they dominate leave the local skylines. The final skyline is
                          unchanged. */
    int32_t prefilter_off; /* 0 (default): before sorting, sky_build drops every row that one of
                          SKY_KILLERS rows of its own partition dominates (per partition, the
                          rows of smallest attribute sum among fixed blocks of rows); such a
                          row is in no skyline of its partition (Def. 1), so the local skylines,
                          the final skyline and gres are unchanged, and its tests are counted in
                          the local phase. 1: every row goes through the local phase. With
                          reps > 0 every row is kept either way. */
} sky_params;

typedef struct sky_info {
    int64_t n;                /* rows */
    int32_t d;                /* attributes */
    int32_t scheme;           /* sky_scheme */
    int32_t p;                /* actual number of partitions */
    int32_t m;                /* slices per (angular) dimension for Grid/Angular, else 0 */
    int32_t pruned_cells;     /* Grid: cells disregarded by grid dominance (after sky_local_skylines) */
    int32_t rounds_local;     /* filter rounds run by sky_local_skylines */
    int32_t rounds_merge;     /* filter rounds run by sky_merge */
    int32_t state;            /* 1 built, 2 local skylines done, 3 merged */
    int64_t pruned_rows;      /* Grid: rows inside pruned cells */
    int64_t local_count;      /* size of the union of the local skylines */
    int64_t sky_count;        /* size of the final skyline */
    int64_t tests_local;      /* row-against-row dominance tests evaluated in the local phase,
                                 the prefilter's (sky_params.prefilter_off) included (counted on
                                 device; tile-box tests are not counted) */
    int64_t tests_merge;      /* dominance tests evaluated in the final phase */
    int64_t max_partition;    /* rows in the largest partition */
    int32_t events_used;      /* timing-hook event pairs recorded (sky_plan_set_events) */
    int32_t reps_kept;        /* representatives no other representative dominates (0 when off);
                                 their tests against the rows are counted in tests_local */
    int64_t tests_local_max;  /* the largest local-phase test count of one partition: the cost
                                 of the parallel phase as Sec. 4 counts it (its tests plus the
                                 final phase's, tests_merge, are the method's count);
                                 equals tests_local when p = 1 */
    int64_t rows_kept;        /* rows the build kept for the local phase: n without the
                                 prefilter (sky_params.prefilter_off), else the rows of unpruned
                                 partitions that no killer row dominates */
    int64_t tests_prefilter;  /* of tests_local: the tests of the build's prefilter (rows against
                                 the killer rows of their partition) */
    int64_t tests_gres;       /* batched plans (sky_batch_info): the candidate tests the last
                                 sky_batch_gres evaluated; 0 for plain plans */
} sky_info;

typedef struct sky_gres_opts {
    int32_t mapping;   /* SKY_GRES_AUTO / SKY_GRES_TILES / SKY_GRES_LEVELS */
    int32_t reserved;  /* must be 0 */
    void* ev_begin;    /* optional hipEvent_t recorded on the stream just before the search kernel */
    void* ev_end;      /* optional hipEvent_t recorded just after it (both or neither) */
    unsigned long long* dev_tests; /* optional device counter: the candidate tests the search
                                      evaluates (one candidate against one tuple at one level;
                                      tile-box tests not counted) are added to it */
} sky_gres_opts;

typedef struct sky_plan sky_plan; /* opaque, host-side; refers to caller memory */

/* Human-readable name of a status code (static string). */
const char* sky_status_string(sky_status s);

/* Library version, as major*10000 + minor*100 + patch. */
int32_t sky_version(void);

/*
 * sky_ingest -- the input step: validate a row-major relation and write it as SoA.
 * x_rows: device float[n*d], row i at x_rows[i*d .. i*d+d). x_soa: device float[d*ld],
 * written as x_soa[k*ld + i] with -0.0 replaced by +0.0. Values that are NaN/inf or outside
 * [0, 1) raise SKY_ERR_DOMAIN in *dev_status (the copy is still written). n may be 0.
 * Returns SKY_ERR_INVALID_ARG for null pointers (when n > 0), d outside [1, SKY_MAX_D],
 * n < 0 or ld < n.
 */
sky_status sky_ingest(const float* x_rows, int64_t n, int32_t d, float* x_soa, int64_t ld,
                      int32_t* dev_status, void* stream);

/*
 * Workspace for sky_build / sky_local_skylines / sky_merge on one plan, in bytes (device
 * memory, any alignment >= 256). Returns 0 for invalid arguments.
 */
size_t sky_build_workspace_bytes(int64_t n, int32_t d, const sky_params* params);

/*
 * sky_build -- partition assignment (Sec. 3.1) and the partition-contiguous copy.
 * Validates the values (SKY_ERR_DOMAIN on device), computes the partition of every row
 * (Grid: sum floor(x_k*m) m^k; Angular: Eq. (1); Sliced: rank on slice_dim, ties by row
 * index, part = floor(rank*p/n); None: one partition), the Grid cells pruned by grid
 * dominance, and a stable partition-contiguous SoA copy in the workspace.
 * x_soa must stay valid until sky_merge returns. On success *out receives a new plan
 * (host memory owned by the library; release it with sky_plan_destroy).
 * n must be in [1, 2^30 - 2^20]; every scheme needs p <= SKY_MAX_CELLS (else SKY_ERR_UNSUPPORTED);
 * Angular needs d >= 2.
 */
sky_status sky_build(const float* x_soa, int64_t n, int32_t d, int64_t ld,
                     const sky_params* params, void* ws, size_t ws_bytes, int32_t* dev_status,
                     void* stream, sky_plan** out);

/*
 * sky_local_skylines -- Sec. 3, phase 1: the skyline of every partition, all partitions at
 * once. Rows of Grid cells pruned by grid dominance take no part. The result stays in the
 * plan's workspace. Queues a fixed number of filter rounds, chosen from n alone; rounds that
 * find no live row do no work. Never synchronises. SKY_ERR_STATE unless the plan is freshly
 * built.
 */
sky_status sky_local_skylines(sky_plan* plan, void* stream);

/*
 * sky_merge -- Sec. 3, phase 2: the skyline of the union of the local skylines, which is
 * Sky(r). Writes the row indices of Sky(r) in ascending order to sky_idx[0..count) (device
 * int64[cap]), the count to *dev_count (device int64), and, if member is non-null, member[i]
 * = 1 iff row i is in Sky(r) (device uint8[n]). If count > cap, SKY_ERR_CAPACITY goes to
 * *dev_status, *dev_count holds the required size and sky_idx is left undefined.
 * cap = 0 (sky_idx may then be null) only counts. Never synchronises. SKY_ERR_STATE unless
 * sky_local_skylines has run on the plan.
 */
sky_status sky_merge(sky_plan* plan, int64_t* sky_idx, int64_t cap, int64_t* dev_count,
                     uint8_t* member, void* stream);

/*
 * sky_plan_partitions -- inspection: part[i] = the partition of row i (device int32[n]),
 * as assigned by sky_build (Sec. 3.1). Any state >= built.
 */
sky_status sky_plan_partitions(const sky_plan* plan, int32_t* part, void* stream);

/*
 * sky_plan_local -- inspection: local[i] = 1 iff row i belongs to the skyline of its own
 * partition and its partition was not pruned (device uint8[n]). SKY_ERR_STATE before
 * sky_local_skylines.
 */
sky_status sky_plan_local(const sky_plan* plan, uint8_t* local, void* stream);

/*
 * sky_plan_partition_tests -- inspection: tests[j] = the dominance tests sky_local_skylines
 * evaluated for the rows of partition j (device int64[p], p as sky_plan_info reports; rows
 * against the prefilter's killer rows and the head rows of their own partition, plus rows
 * against the representatives when Representative Filtering is on). They sum to sky_info.tests_local and their maximum is
 * sky_info.tests_local_max; pruned Grid cells hold 0. Sec. 4 measures the parallel phase by
 * this maximum. SKY_ERR_STATE before sky_local_skylines.
 */
sky_status sky_plan_partition_tests(const sky_plan* plan, int64_t* tests, void* stream);

/*
 * sky_plan_set_events -- optional timing hooks, to measure the dominance-test kernels alone.
 * ev_begin/ev_end: host arrays of cap hipEvent_t handles (as void*) created by the caller.
 * sky_local_skylines and sky_merge then record ev_begin[i] / ev_end[i] on the stream around
 * their i-th dominance-test launch (i counted across both calls, at most cap pairs) and report
 * the number of pairs recorded in sky_info.events_used. Null arrays or cap = 0 disable it.
 */
sky_status sky_plan_set_events(sky_plan* plan, void* const* ev_begin, void* const* ev_end,
                               int32_t cap);

/*
 * Plan inspection: the counters listed in sky_info. Those the device computes (partition
 * statistics, rounds, counts, tests) are copied back on the stream of the plan's last call
 * that queued work, which this call waits for: do not call it while that stream is being
 * captured into a graph. Fields of a phase that has not run are 0.
 */
sky_status sky_plan_info(const sky_plan* plan, sky_info* out);

/* Releases a plan (host memory and its events). Null is accepted. */
void sky_plan_destroy(sky_plan* plan);

/*
 * sky_project -- the grid projection of Def. 2 as a relation of its own, for running the
 * skyline machinery on projected tuples (Alg. 1 as written recomputes Sky(gproj(s, g)) at every
 * level; gres_compute gives the same answer per tuple without it). For j < s and every attribute
 * k: out_soa[k*ld_out + j] = floor(fl32(x[k][rows[j]] * g)) * 2^-b, where 2^b is the smallest
 * power of two >= g. That is the key of the quantisation contract scaled by a power of two:
 * exact in FP32, in [0, 1), and ordered exactly like floor(t g) / g, so dominance between
 * projections is unchanged. rows: device int64[s] in [0, n) (SKY_ERR_INVALID_ARG in
 * *dev_status otherwise); values outside the domain raise SKY_ERR_DOMAIN. g in [1, SKY_MAX_G].
 * Never synchronises.
 */
sky_status sky_project(const float* x_soa, int64_t n, int32_t d, int64_t ld, const int64_t* rows,
                       int64_t s, int32_t g, float* out_soa, int64_t ld_out, int32_t* dev_status,
                       void* stream);

/*
 * sky_literal_level -- the exit bookkeeping of Alg. 1 as written (Sec. 3.2), for one level g,
 * after the skyline of the projected candidates at g has been computed (sky_project, then the
 * skyline path on the projected relation, whose sky_merge gives member[j] = 1 iff projected
 * candidate j is in it): for every j < s with g_exit[j] == 0 (no level yet) and member[j] == 0,
 * g_exit[j] = g. Call it for g = g_max, g_max - 1, ..., 2 on g_exit zeroed beforehand, then once
 * with g = 1 (member may be null): every tuple still at 0 gets 1, it never left the skyline.
 * The result equals gres_compute's g_exit for the same candidates. nil_left (device int32,
 * optional, zeroed by the caller) gets the number of tuples still without a level added to it,
 * for stopping early. member: device uint8[s]; g_exit: device int32[s]; g in [1, SKY_MAX_G].
 * Never synchronises.
 */
sky_status sky_literal_level(const uint8_t* member, int64_t s, int32_t g, int32_t* g_exit, int32_t* nil_left,
                             void* stream);

/*
 * Workspace for gres_compute, in bytes. Returns 0 for invalid arguments. For g_max <= 64 it
 * includes a table of every candidate's keys at every level, packed into one 64-bit word per
 * (level, candidate) when the d keys fit (d * (bit length of g_max + 1, plus one) <= 64, e.g.
 * d <= 10 at g_max 25): (g_max - 1) x (s rounded up, plus padding tiles) x 8 bytes.
 */
size_t gres_workspace_bytes(int64_t s, int32_t d, int32_t g_max);

/*
 * gres_compute -- Def. 2 through Alg. 1 for the tuples t = rows sky_idx[0..s) of x, with the
 * same rows as the candidate set (gres is stable: dominated tuples never change it, so
 * Sky(r) suffices; any superset gives the same answer).
 * For each j: g_exit[j] = the largest g in [2, g_max] such that the projection of some other
 * candidate dominates the projection of row sky_idx[j] at level g, or 1 if there is none;
 * gres[j] = 1.0f / (float)g_exit[j]. g_exit and gres are device arrays of s entries; either
 * may be null. sky_idx: device int64[s], each in [0, n) (checked on device:
 * SKY_ERR_INVALID_ARG in *dev_status). s may be 0. g_max in [2, SKY_MAX_G].
 * opts may be null (automatic mapping). Never synchronises.
 */
sky_status gres_compute(const float* x_soa, int64_t n, int32_t d, int64_t ld,
                        const int64_t* sky_idx, int64_t s, int32_t g_max, int32_t* g_exit,
                        float* gres, void* ws, size_t ws_bytes, int32_t* dev_status,
                        const sky_gres_opts* opts, void* stream);

/*
 * gres_compute_noalloc -- gres_compute without a workspace argument, for callers that cannot
 * allocate device memory (code under graph capture, tight serving loops, harnesses that forbid
 * allocation). Same arguments, results and errors as gres_compute, minus ws / ws_bytes: the
 * workspace is a fixed array of SKY_NOALLOC_SCRATCH_BYTES bytes inside this library, one per
 * device, held from the library's first use on that device until the process ends. Calls whose
 * workspace without the key table (gres_workspace_bytes(s, d, 65): no table above g_max 64)
 * exceeds it return SKY_ERR_UNSUPPORTED (with no work queued); at d = 6 that is about 700,000
 * tuples. The key table is used when the whole gres_workspace_bytes(s, d, g_max) fits (the
 * results are the same either way). The array of the CURRENT device is used, so `stream`
 * must belong to the current device. Every call on one device shares its array and leaves its
 * contents behind (the call itself depends on none of them): calls that overlap on one device,
 * on different streams or from different threads, race and give undefined results -- queue
 * them on one stream. The first call on a device looks up the array's address (a host-side
 * runtime query, no device work); the calls never allocate or free memory and never
 * synchronise.
 */
sky_status gres_compute_noalloc(const float* x_soa, int64_t n, int32_t d, int64_t ld,
                                const int64_t* sky_idx, int64_t s, int32_t g_max, int32_t* g_exit,
                                float* gres, int32_t* dev_status, const sky_gres_opts* opts,
                                void* stream);

/*
 * sky_gres -- gres_compute for the plan's own skyline, after sky_merge: the candidates and the
 * tuples are Sky(r) as sky_merge returned it, and g_exit[j] / gres[j] (device arrays of
 * min(count, cap) entries, cap being sky_merge's; either may be null) refer to sky_idx[j] of
 * that call. The result is the one gres_compute gives for (x, sky_idx, count, g_max), but the
 * candidates are read from the plan's partition-contiguous copy in its curve order, so no sort
 * is needed. The skyline size is read on the device: ws must hold at least
 * gres_workspace_bytes(c, d, g_max) bytes with c = max(1, min(cap, n)) (device,
 * caller-owned); a skyline larger than cap raises SKY_ERR_CAPACITY in *dev_status. The mapping
 * (SKY_GRES_AUTO included) and the work split are chosen on the device from the real size.
 * g_max in [2, SKY_MAX_G]; opts as for gres_compute. SKY_ERR_STATE before sky_merge. The
 * plan's skyline state is read, not changed (calls may repeat). Never synchronises.
 */
sky_status sky_gres(sky_plan* plan, int32_t g_max, int32_t* g_exit, float* gres, void* ws,
                    size_t ws_bytes, int32_t* dev_status, const sky_gres_opts* opts, void* stream);

/*
 * Workspace for gres_gbar, in bytes (independent of d). Returns 0 for invalid arguments.
 */
size_t gres_gbar_workspace_bytes(int64_t n);

/*
 * gres_gbar -- the upper end of Alg. 1's level range (Sec. 3.2): ell is the smallest non-zero
 * absolute difference between two values of the same attribute, over every pair of rows of x
 * and every attribute; g_bar = floor(1 / ell). Beyond g_bar, every difference within an
 * attribute spans more than one grid interval, so no new dominance between projections can
 * appear (exact arithmetic), and gres_compute with g_max = g_bar gives Def. 2's value.
 * Outputs (device, either may be null, not both):
 *   ell[0]   -- a double: each difference is taken in FP64 from the two FP32 values (rounded
 *               to nearest; exact unless the two exponents differ by more than 29); +inf when no
 *               attribute holds two different values (n < 2 included). -0.0 equals 0.0.
 *   g_bar[0] -- an int64: floor of the FP64 quotient 1/ell, saturated at 2^62; 1 when ell is +inf
 *               (no level above 1 to search). To search up to it, pass min(g_bar, SKY_MAX_G) as
 *               g_max; a g_bar above SKY_MAX_G means levels past 2^24 are not searched.
 * x_soa: [d][ld] device FP32, n in [0, 2^30 - 2^20), ld >= n. Values outside [0, 1) or NaN set
 * SKY_ERR_DOMAIN in *dev_status (outputs then undefined). ws: device, at least
 * gres_gbar_workspace_bytes(n) bytes, caller-owned, free again when the stream reaches the end
 * of this call's work. Never synchronises.
 */
sky_status gres_gbar(const float* x_soa, int64_t n, int32_t d, int64_t ld, double* ell,
                     int64_t* g_bar, void* ws, size_t ws_bytes, int32_t* dev_status,
                     void* stream);

/*
 * Two-phase form of gres_compute, for candidate sets that are queried many times (a resident
 * dataset serving requests): the candidates are prepared once, then any tuples are searched.
 *
 * gres_prepare -- orders the candidate rows cand_idx[0..s) of x (normally Sky(r)) for the
 * search and keeps them, with their tile boxes, in `prep` (device memory of
 * gres_prepare_bytes(s, d) bytes, owned by the caller; it stays valid as long as the caller
 * keeps it, independently of x). Checks indices (SKY_ERR_INVALID_ARG) and values
 * (SKY_ERR_DOMAIN) on device. Never synchronises.
 */
size_t gres_prepare_bytes(int64_t s, int32_t d);
sky_status gres_prepare(const float* x_soa, int64_t n, int32_t d, int64_t ld,
                        const int64_t* cand_idx, int64_t s, void* prep, size_t prep_bytes,
                        int32_t* dev_status, void* stream);

/*
 * gres_search -- Def. 2 via Alg. 1 for target tuples against a prepared candidate set (the
 * same s and d as given to gres_prepare). targets: device int64[nt] row indices into x (any
 * rows; their values are read from x, which must hold the same relation the candidates came
 * from for the result to be gres in that relation). targets == NULL means "every candidate"
 * (then nt must equal s and outputs are indexed like cand_idx, as in gres_compute); x may then
 * be NULL. g_exit[q], gres[q] (either may be NULL) refer to targets[q]. ws: device memory of
 * gres_search_bytes(nt, d) bytes. Requires s >= 1 when nt >= 1; nt at most 2^30 - 2^20 (the row
 * cap of a plan; gres_search_bytes returns 0 and gres_search SKY_ERR_INVALID_ARG above it; the
 * targets may repeat rows, so nt is not bounded by n). Never synchronises; distinct
 * searches on distinct streams may run concurrently on one prepared set.
 */
size_t gres_search_bytes(int64_t nt, int32_t d);
sky_status gres_search(const void* prep, int64_t s, int32_t d, const float* x_soa, int64_t n,
                       int64_t ld, const int64_t* targets, int64_t nt, int32_t g_max,
                       int32_t* g_exit, float* gres, void* ws, size_t ws_bytes,
                       int32_t* dev_status, const sky_gres_opts* opts, void* stream);

/*
 * ------------------------------------------------------------------ batched relations
 * Many independent relations with the same number of attributes d, one after the other in one
 * SoA buffer: relation j is rows [offsets[j], offsets[j+1]) of x_soa. Each relation gets its own
 * skyline (Def. 1) and the gres (Def. 2 via Alg. 1) of each of its skyline tuples with its own
 * skyline as the candidate set -- exactly what the plain calls give for that relation alone;
 * rows of different relations never meet. All relations advance together: each skyline round
 * serves all of them (one segment per relation), and the gres search of all of their skyline
 * tuples is ONE persistent launch whose waves take (tuple, level band) pairs of any relation.
 *
 * Sequence: sky_batch_workspace_bytes -> sky_batch_create -> (sky_batch_tune,
 * sky_batch_set_keys) -> sky_batch_skylines -> sky_batch_gres -> ... -> sky_batch_destroy. After sky_batch_create no
 * call synchronises or reads anything back (sky_batch_info aside): a step sky_batch_skylines +
 * sky_batch_gres, repeated on new values in x_soa, can be captured in one HIP graph and replayed.
 */
typedef struct sky_batch sky_batch; /* opaque, host-side; refers to caller memory */

typedef struct sky_tune {
    int32_t mapping;        /* SKY_GRES_AUTO (by the largest relation's skyline) / SKY_GRES_TILES /
                               SKY_GRES_LEVELS */
    int32_t near_first;     /* 1 = each tuple scans the candidate tiles next to its own place on
                               the curve first (default), 0 = tiles in curve order */
    int32_t lpt;            /* 1 = the tuples of the relations with the largest skylines are
                               searched first (default), 0 = relation order */
} sky_tune;

/*
 * Workspace for a batch: offsets is a HOST array of nbatch + 1 row offsets, non-decreasing,
 * offsets[0] = 0; the total offsets[nbatch] in [1, 2^30 - 2^20]; nbatch in [1, SKY_MAX_CELLS].
 * Relations may be empty. Returns 0 for invalid arguments.
 */
size_t sky_batch_workspace_bytes(const int64_t* offsets, int32_t nbatch, int32_t d);

/*
 * sky_batch_create -- validates the arguments and copies the offsets to the workspace (waiting
 * for that copy, so the host array may be released on return). No other device work. The batch
 * reads x_soa (device float[d*ld], ld >= offsets[nbatch]) at every sky_batch_skylines, which
 * raises SKY_ERR_DOMAIN in *dev_status for values outside the domain.
 */
sky_status sky_batch_create(const float* x_soa, int32_t d, int64_t ld, const int64_t* offsets,
                            int32_t nbatch, void* ws, size_t ws_bytes, int32_t* dev_status,
                            void* stream, sky_batch** out);

/*
 * sky_batch_skylines -- the skyline of every relation from the current values of x_soa (every
 * relation's rows ordered along a Hilbert curve as one segment, then the segmented skyline
 * rounds). Writes sky_idx (device int64[cap]): the skyline rows of all relations, ascending (so
 * grouped by relation), as rows of x_soa; and sky_off (device int64[nbatch+1]): relation j's
 * skyline is sky_idx[sky_off[j] .. sky_off[j+1]). Then prepares the candidate store of every
 * relation for the gres search. A total above cap raises SKY_ERR_CAPACITY in *dev_status (then
 * only the first cap rows are written and searched); cap = offsets[nbatch] always suffices.
 * Never synchronises; may be repeated (each call recomputes everything).
 */
sky_status sky_batch_skylines(sky_batch* batch, int64_t* sky_idx, int64_t cap, int64_t* sky_off,
                              void* stream);

/*
 * sky_batch_tune -- the search's choices for the next sky_batch_gres calls (tune may be NULL:
 * defaults). Host-side only. Results never depend on them.
 */
sky_status sky_batch_tune(sky_batch* batch, const sky_tune* tune, void* stream);

/*
 * sky_batch_gres -- gres of every skyline tuple of every relation: g_exit[j] and gres[j]
 * (device arrays of min(cap of sky_batch_skylines, offsets[nbatch]) entries; either may be
 * NULL) refer to sky_idx[j], with the same meaning as in gres_compute and relation j's
 * skyline as the candidate set. g_max in [2, SKY_MAX_G]. The counts, the mapping choice of AUTO
 * and the order of the relations are worked out on the device; ev_begin / ev_end (hipEvent_t,
 * optional, both or neither) are recorded around the search kernels. Never synchronises.
 * SKY_ERR_STATE before sky_batch_skylines.
 */
sky_status sky_batch_gres(sky_batch* batch, int32_t g_max, int32_t* g_exit, float* gres,
                          void* ev_begin, void* ev_end, void* stream);

/*
 * Workspace for the packed key tables of a batch's gres search (every candidate's keys at every
 * level g in [2, g_max_keys], one 64-bit word per (level, candidate), plus the tile and chunk
 * box corners), for skylines of up to sky_total tuples in all. Returns 0 when packed keys do
 * not apply: g_max_keys above 64, or the batch's d keys too wide for one word (see
 * gres_workspace_bytes), or invalid arguments.
 */
size_t sky_batch_keys_bytes(const sky_batch* batch, int64_t sky_total, int32_t g_max_keys);

/*
 * sky_batch_set_keys -- attaches a device workspace (caller-owned, at least
 * sky_batch_keys_bytes(batch, sky_total, g_max_keys) bytes, kept until detached or the batch
 * is destroyed) for the key tables; ws NULL detaches. Later sky_batch_gres calls with g_max <=
 * g_max_keys then search on packed keys when the batch's skyline total fits sky_total (checked
 * on the device; otherwise they search the values). The results are the same either way.
 * Host-side only; SKY_ERR_WORKSPACE when ws_bytes is too small.
 */
sky_status sky_batch_set_keys(sky_batch* batch, void* ws, size_t ws_bytes, int64_t sky_total,
                              int32_t g_max_keys);

/*
 * sky_batch_info -- n = total rows, d, scheme = SKY_NONE, p = nbatch, max_partition = rows of
 * the largest relation, state (1 created, 2 skylines queued); after sky_batch_skylines also
 * rounds_local / tests_local / tests_local_max / tests_prefilter / rows_kept of the skyline
 * rounds and local_count = sky_count = the total skyline size, read back on the stream of the
 * last sky_batch_skylines; after sky_batch_gres also tests_gres, read back on its stream (this
 * call waits for both).
 */
sky_status sky_batch_info(const sky_batch* batch, sky_info* out);

/* Releases a batch (host memory only). Null is accepted. */
void sky_batch_destroy(sky_batch* batch);

/* ------------------------------------------------------------------------------------------
 * Measurement aids (not part of the path): probes of the two device rates the kernels'
 * rooflines are priced against, so that a benchmark can report the rates it measured beside
 * the published ones.
 * ------------------------------------------------------------------------------------------ */

/*
 * sky_probe_valu -- one launch of `grid` workgroups of 256 threads, each thread running `iters`
 * iterations of four independent chains of 32-bit integer add / xor / max / min (the dominance
 * test's instruction mix), 24 VALU ops per iteration. *lane_ops (host) = the lane-ops the launch
 * executes. sink: device uint32[grid] (written, to keep the work live). ev_begin / ev_end:
 * optional hipEvent_t recorded around the launch (both or neither). SKY_ERR_INVALID_ARG for
 * iters < 1, grid < 1 or null pointers.
 */
sky_status sky_probe_valu(int64_t iters, int32_t grid, uint32_t* sink, void* ev_begin, void* ev_end,
                          void* stream, int64_t* lane_ops);

/*
 * sky_probe_copy -- a streaming copy of `bytes` device bytes from src to dst (16-byte
 * aligned, bytes a positive multiple of 16; the ranges must not overlap): every byte is read
 * once and written once. ev_begin / ev_end as for sky_probe_valu.
 */
sky_status sky_probe_copy(const void* src, void* dst, int64_t bytes, void* ev_begin, void* ev_end,
                          void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SKY_H */
