/*
 * td.h -- C ABI of the exact Tukey-depth library for AMD MI355X (gfx950).
 *
 * The library computes depth counts  counts[q] = n * D_n(Z_q),  where
 *     D_n(z) = min over unit u of  #{ i : u'X_i <= u'z } / n
 * is the sample Tukey depth (Section 1, equation (1)), with the paper's
 * first algorithm (Section 3): the depth of the origin after the shift
 * x_i = X_i - z equals, by Proposition 1 with r = p-2 (equation (8)), the
 * minimum over all (p-2)-subsets I of the observations of a bivariate depth,
 * obtained by projecting onto the 2-D complement of span(x_I) (Algorithm 1,
 * Step 1(a)-(b)) and running one angular sort and one circular sweep
 * (Algorithm 2); the count form of Algorithm 1, Step 2, is returned.
 *
 * The result is an exact integer for every finite input, not only in general
 * position: points inside span(x_I), exactly equal angles and dependent
 * subsets are decided with exact integer predicates (TD_PREC_FP32_FILTERED and
 * TD_PREC_EXACT).  TD_PREC_FP64_PLAIN follows the paper's steps in float64
 * without certification (ties are grouped only when the float64 keys are
 * equal, points inside span(x_I) are counted as in Algorithm 2, Step 2) and
 * can differ from the exact count on degenerate data.
 *
 * Conventions for every entry point below.
 *  - X (n x p) and Z (m x p) are row-major contiguous float64 arrays in
 *    DEVICE memory; counts (m int32) is DEVICE memory.  All three are owned by
 *    the caller; the library keeps no reference to them once the enqueued
 *    work has completed.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Calls are asynchronous on that stream: results are valid once the stream
 *    has completed the work.  Calls on the same stream are ordered; the
 *    library serialises its own workspace between calls.
 *  - Argument errors are reported synchronously by the return value and leave
 *    `counts` untouched.  Limits: 1 <= p <= TD_MAX_P, 1 <= n <= TD_MAX_N,
 *    m >= 0 (m = 0 is a no-op).
 *  - Data-dependent failures are reported per query: counts[q] = -1 and a bit
 *    in td_stats.device_status (see TD_DEV_*), readable after the stream has
 *    completed.
 *  - The library lazily creates a per-device workspace (device buffers, a
 *    binomial table, captured graphs); td_release() frees it.
 */
#ifndef TD_H
#define TD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TD_MAX_P 8
#define TD_MAX_N 1024

typedef enum {
    TD_OK = 0,
    TD_ERR_INVALID_ARG = 1,   /* null pointer, size out of range, bad option */
    TD_ERR_UNSUPPORTED = 2,   /* valid request the library does not handle */
    TD_ERR_OUT_OF_MEMORY = 3, /* workspace allocation failed */
    TD_ERR_HIP = 4,           /* a HIP runtime call failed */
    TD_ERR_DEVICE_STATUS = 5, /* td_get_stats: the last call flagged queries */
    TD_ERR_NO_DEVICE = 6,     /* no HIP device is visible */
    TD_ERR_TOO_LARGE = 7      /* td_depth_noalloc: the call needs more than its
                                 static workspace holds */
} td_status;

/* Per-query failure bits of td_stats.device_status (OR over the queries). */
#define TD_DEV_NONFINITE 1        /* NaN or Inf in X or in the query */
#define TD_DEV_NO_VALID_SUBSET 2  /* the centred points span <= p-3 dimensions */
#define TD_DEV_DEFER_OVERFLOW 4   /* more uncertain subsets than deferred_capacity */
#define TD_DEV_EXACT_RANGE 8      /* exact fallback needed but the integerised
                                     inputs exceed 126 bits */
#define TD_DEV_DEGENERACY_LIMIT 16/* exact fallback met a tie run or an in-span
                                     point set larger than the library handles */
#define TD_DEV_NOT_GENERAL 32     /* TD_METHOD_VERTEX: a point's side of some
                                     hyperplane through p-1 points is not
                                     certified in float64 (points not in
                                     general position, or too close to it) */

typedef enum {
    TD_PREC_FP64_PLAIN = 0,    /* float64 keys, no certification */
    TD_PREC_FP32_FILTERED = 1, /* float32 projection with forward error bounds,
                                  float64 re-check, exact fallback */
    TD_PREC_EXACT = 2          /* float64 projection with error bounds and
                                  exact fallback for every subset */
} td_precision;

/* Angular order of the filtered tier (Algorithm 2, Step 1(e)).  Both give the
 * same exact counts. */
typedef enum {
    TD_SWEEP_AUTO = 0,    /* counting sort into pseudo-angle buckets, exact
                             order only where the sweep minimum may lie (the
                             exact tier when that region is large); at p = 2,
                             one sweep per query, the full sort */
    TD_SWEEP_BITONIC = 1  /* full bitonic sort of every sweep */
} td_sweep;

/* Which of the paper's algorithms computes the count (td_depth, td_depth_ex
 * only; td_depth_batched and td_depth_noalloc return TD_ERR_UNSUPPORTED for
 * the methods other than RCOM). */
typedef enum {
    TD_METHOD_RCOM = 0,   /* Algorithm 1 with Algorithm 2 (Section 3): every
                             (p-2)-subset; the exact count */
    TD_METHOD_ADIA = 1,   /* Algorithm 3 (Section 4): a descent over critical
                             (p-1)-sets by Proposition 3 (Steps 2-4), then
                             Algorithm 1 over the subsets of the candidate
                             points only (Step 5), swept by the certified
                             tiers.  The paper reports the exact count in all
                             its experiments but proves no bound; the result
                             is a count attained by some subset, so it never
                             lies below the depth, and it equals the depth
                             whenever an optimal subset lies among the
                             candidates.  For p < 3 or n <= 2p, Algorithm 1
                             (the paper's advice). */
    TD_METHOD_VERTEX = 2  /* Proposition 1 with r = p-1 (Section 2, the
                             critical-direction route): the smaller side count
                             of every hyperplane through the query and p-1
                             sample points, O(n^p); an independent check of
                             RCOM.  Valid for points in general position (the
                             proposition's assumption): every side decision is
                             certified in float64 (cofactors with a
                             permanent-based error bound), and a query with an
                             undecided one returns -1 with TD_DEV_NOT_GENERAL.
                             n <= 512 at p >= 5, n <= 1024 at p <= 4
                             (TD_ERR_UNSUPPORTED beyond); a query
                             needs n' >= p-1 points apart from it
                             (TD_DEV_NO_VALID_SUBSET otherwise); p = 1 is the
                             closed form. */
} td_method;

typedef struct {
    int32_t precision;         /* td_precision (default TD_PREC_FP32_FILTERED) */
    int32_t autotune;          /* 1: use the tuned launch shape when cached */
    int32_t chunk;             /* subsets per work item (multiple of 64), 0 = auto (256, halved
                                  down to 64 while there are fewer than four items per
                                  resident wave) */
    int32_t grid_blocks;       /* persistent blocks, 0 = auto */
    double filter_scale;       /* scales the float32 error radius (error
                                  and rounding terms): 1 normal, above 1
                                  wider (still exact), +inf re-checks every
                                  float32 decision, 0 trusts float32 with
                                  no margin (negative control, results may
                                  be wrong) */
    int32_t force_exact;       /* 1: every subset goes through the exact tier */
    int32_t timing;            /* 1: record HIP events per stage (td_get_stats) */
    int64_t deferred_capacity; /* max deferred subsets per call, 0 = default */
    int32_t sweep;             /* td_sweep: how the filtered tier orders the
                                  projected points (default TD_SWEEP_AUTO) */
    int32_t prune;             /* 1 (default): before the subsets, bound the
                                  minimum by the closed halfspace counts of the
                                  2n directions +-(X_j - z) (Algorithm 3,
                                  Step 2(a)), let the bucketed sweep skip
                                  subsets that cannot go below it, and skip the
                                  remaining subsets of a query once a term of 0
                                  is reached; 0: sweep every subset.  The
                                  counts are the same either way.  Ignored by
                                  TD_PREC_FP64_PLAIN. */
    int32_t method;            /* td_method (default TD_METHOD_RCOM) */
} td_options;

typedef struct {
    uint64_t subsets_swept;      /* subsets processed by the main kernels */
    uint64_t fp64_rechecks;      /* float32 decisions re-checked in float64 */
    uint64_t deferred_subsets;   /* subsets sent to the exact tier */
    uint64_t exact_predicates;   /* exact integer predicates evaluated */
    uint64_t degenerate_subsets; /* subsets with extra points inside span(x_I) */
    uint64_t invalid_subsets;    /* subsets with linearly dependent points:
                                    found by the plain tier's basis, or by
                                    the exact tier among the deferred
                                    subsets (then also in deferred_subsets) */
    int32_t device_status;       /* OR of TD_DEV_* over the last call's queries */
    float prep_ms, subset_ms, exact_ms, finalize_ms, total_ms; /* if timing */
    uint64_t walked_sweeps;      /* bucketed sweeps whose bucket bounds did not
                                    settle the minimum and that were walked in
                                    exact order (TD_SWEEP_AUTO) */
    uint64_t pruned_subsets;     /* subsets skipped because the query's
                                    minimum had already reached 0 (prune) */
    uint64_t exact_subsets;      /* deferred subsets the exact tier took up:
                                    each deferred subset once, so this equals
                                    min(deferred_subsets, deferred_capacity) */
    uint64_t adia_evaluations;   /* TD_METHOD_ADIA: subsets evaluated on the
                                    device in the descent (Algorithm 3, Steps
                                    2-4), counting those of nodes taken off
                                    the queue ahead in a batch and then
                                    deleted by an earlier node */
    uint64_t adia_candidates;    /* TD_METHOD_ADIA: candidate points of Step 5,
                                    summed over the queries */
    uint64_t f64_items;          /* work items of the bucketed sweep (p >= 3)
                                    finished by its float64 pass: from the
                                    first sweep of the item that needed the
                                    float64 re-check or re-order on */
    uint64_t adia_rcom_queries;  /* TD_METHOD_ADIA: queries that Algorithm 1
                                    answered instead: n <= 2p or p < 3 (as
                                    Section 4 advises), no seed subset in
                                    Step 2(c), an evaluation with more than 32
                                    points next to its minimising states (the
                                    set T of Step 4(a)(ii)), or a descent of
                                    more than 4 C(n, p-2) + 4096 evaluations */
} td_stats;

/* One independent depth problem of a batch (pointers as for td_depth). */
typedef struct {
    const double* X;
    int64_t n;
    int32_t p;
    const double* Z;
    int64_t m;
    int32_t* counts;
} td_problem;

/* Fills *out with the defaults. */
td_status td_default_options(td_options* out);

/* Depth counts of the m queries Z w.r.t. X with the default options.
 * counts[q] = n * D_n(Z_q), the sample halfspace depth of Section 1,
 * equation (1), computed by Algorithm 1 (loop over the (p-2)-subsets, each
 * step the bivariate sort and sweep of Algorithm 2; Proposition 1 with
 * r = p-2, equation (8)); the integer count of Algorithm 1, Step 2.
 * X: n x p, Z: m x p, row-major float64, counts: m int32, all device memory
 * owned by the caller.  p = 1 uses the closed form of Section 3; p = 2 runs
 * Algorithm 2 once on the centred points.  Errors: TD_ERR_INVALID_ARG for a
 * null pointer, p outside [1, TD_MAX_P], n outside [1, TD_MAX_N] or m < 0
 * (synchronous, counts untouched); per-query failures as counts[q] = -1 with
 * a TD_DEV_* bit. */
td_status td_depth(const double* X, int64_t n, int32_t p, const double* Z, int64_t m,
                   int32_t* counts, void* stream);

/* As td_depth with explicit options (NULL = defaults): the arithmetic tier
 * (Algorithm 2 in float32 with certified error bounds, plain float64, or
 * exact), the order of the sweep, the bound of Algorithm 3, Step 2(a), and
 * the launch shape.  An invalid option returns TD_ERR_INVALID_ARG. */
td_status td_depth_ex(const double* X, int64_t n, int32_t p, const double* Z, int64_t m,
                      int32_t* counts, const td_options* opt, void* stream);

/* Many independent problems of uneven n and p (each as td_depth: Section 1,
 * equation (1), by Algorithm 1 with Algorithm 2) in one captured HIP graph
 * launch: one preparation kernel, one persistent subset kernel per (p,
 * points-per-lane) class pulling (query, subset-range) work items from a
 * device counter, the exact tier and the finalisation.  `probs` is a HOST
 * array of `num` problems read during the call; the pointers inside follow
 * the td_depth conventions.  TD_ERR_INVALID_ARG for num < 0, a null array or
 * an invalid problem; TD_ERR_UNSUPPORTED for more than 2^30 queries or a
 * query with more than 2^32 work items. */
td_status td_depth_batched(const td_problem* probs, int32_t num, const td_options* opt,
                           void* stream);

/* As td_depth_ex, for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * calls no hipMalloc, hipFree or other allocating routine.  Its workspace is
 * a static device array of 128 MiB (TD_NOALLOC_BYTES) that every device the
 * library runs on holds until the process ends; all calls on one device
 * share it, so calls that overlap on one device (different streams, host
 * threads) race, while calls ordered on one stream are safe.  The grid is
 * shrunk to fit the array; a call that does not fit even so (roughly
 * m * M * p * 36 bytes of per-query arrays, M the sort width >= n, plus the
 * deferred list and per-block scratch) returns TD_ERR_TOO_LARGE.  At most
 * 2^16 work items go to the float64 pass (marked subsets beyond that go to
 * the exact tier) and at most 2^18 subsets per call to the exact tier
 * (deferred_capacity is capped there); beyond that the query reports
 * TD_DEV_DEFER_OVERFLOW, which data far from general position can reach
 * (the td_depth_ex lists are 2^22 and 2^25 entries).  The tuned
 * launch shapes of td_autotune and the timing option are not used; counters
 * are available from td_get_stats.  Arguments and errors otherwise as
 * td_depth_ex. */
#define TD_NOALLOC_BYTES (128ull << 20)
td_status td_depth_noalloc(const double* X, int64_t n, int32_t p, const double* Z, int64_t m,
                           int32_t* counts, const td_options* opt, void* stream);

/* Counters and timings of the last call; synchronises the device. */
td_status td_get_stats(td_stats* out);

/* Times candidate launch shapes for (p, n) on synthetic data and caches the
 * fastest for later calls with autotune = 1; synchronises the device. */
td_status td_autotune(int32_t p, int64_t n, const td_options* base, void* stream);

/* The cache of td_autotune outlives the process only through these two
 * calls.  td_tuning_save writes the current device's tuned launch shapes to
 * the text file `path` (one line per (tier, p, points per lane): chunk and
 * grid); TD_ERR_INVALID_ARG when the file cannot be written.  td_tuning_load
 * reads such a file into the current device's cache: every line is checked
 * before any is applied and before any device is touched
 * (TD_ERR_INVALID_ARG for a missing or malformed file), and a file written
 * on a device with another number of compute units returns
 * TD_ERR_UNSUPPORTED. */
td_status td_tuning_save(const char* path);
td_status td_tuning_load(const char* path);

const char* td_status_string(td_status s);

/* Frees the workspace of every device (safe to call more than once). */
void td_release(void);

int32_t td_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TD_H */
