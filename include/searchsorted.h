/*
 * libsearchsorted -- batched search over small sorted float64 tables on
 * AMD Instinct MI355X (gfx950).
 *
 * THE OPERATION (paper Sec. 1 and Sec. 3): for a small sorted table a[0..n)
 * and many targets x, find the index of the largest table entry that is less
 * than the target.  This library fixes the comparison as strict and returns
 * -1 when no entry qualifies:
 *
 *     idx(x) = #{ i in [0, n) : a[i] < x } - 1        (int32, in [-1, n-1])
 *
 * Equivalently a[idx] < x <= a[idx+1] with a[-1] = -inf and a[n] = +inf.
 * (Sec. 3 states a "<=" variant clamped to [0, n-1]; the strict form above is
 * the one implemented.)  Consequences, all exact:
 *   - a target below the first entry gives -1, above the last gives n-1;
 *   - a target equal to a[i] gives the index of the last entry below it;
 *   - NaN targets give -1; -0.0 and +0.0 compare equal; denormals are
 *     compared exactly (no flush-to-zero anywhere);
 *   - -inf gives -1, +inf gives (number of entries below +inf) - 1.
 *
 * TABLE PRECONDITION: sorted non-decreasing (duplicates allowed), no NaN.
 * The search entry points do not check it (ss_validate_table does, on
 * request).  A table that violates it yields unspecified indices in
 * [-1, n-1] but never an out-of-bounds access.
 *
 * CONVENTIONS
 *   - Unless stated otherwise every pointer argument is a DEVICE pointer
 *     (hipMalloc'd or equivalent) owned by the caller; the library never
 *     frees caller memory and keeps no reference to it after a call returns,
 *     except where a plan or handle documents otherwise.
 *   - Calls are asynchronous on the calling thread's current library stream
 *     (ss_set_stream; default: the null stream) unless documented as
 *     synchronous.  Output buffers are valid once that stream reaches the
 *     call's work.
 *   - Every entry point returns SS_OK (0) or a negative ss_status.  No C++
 *     exception or abort crosses this interface.  On error, ss_last_error()
 *     returns a message for the calling thread, and no device work has been
 *     queued for argument errors.
 *   - Sizes are int64_t; a table holds at most INT32_MAX entries.
 *   - Outputs must not overlap inputs.
 */
#ifndef SEARCHSORTED_H
#define SEARCHSORTED_H

#include <stdint.h>

#ifndef SS_API
#define SS_API __attribute__((visibility("default")))
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SS_OK = 0,
    SS_ERR_INVALID_ARG = -1,    /* null pointer with a nonzero count, negative
                                   size, n > INT32_MAX, misaligned or
                                   overlapping buffers, bad option value */
    SS_ERR_NOT_DEVICE_PTR = -2, /* a buffer is not device-accessible memory */
    SS_ERR_NO_DEVICE = -3,      /* no usable GPU */
    SS_ERR_HIP = -4,            /* a HIP runtime call failed */
    SS_ERR_OOM = -5,            /* device or host allocation failed */
    SS_ERR_UNSUPPORTED = -6     /* valid request the library cannot serve */
} ss_status;

/* Search kernels (values of SS_OPT_FORCE_ALGO and of plan choices). */
typedef enum {
    SS_ALGO_AUTO = 0,
    SS_ALGO_BINARY = 1,      /* branchless bisection (Sec. 3.2) over the table
                                staged in LDS, fixed trip count */
    SS_ALGO_BALLOT = 2,      /* linear scan (Sec. 2.1) limited to the bracket
                                of the wavefront's smallest and largest
                                target, found with wavefront ballots */
    SS_ALGO_EXPHASH = 3,     /* exponent hash (Sec. 3.5): bin by the float64
                                exponent bits (plus optional leading fraction
                                bits), then a linear scan inside the bin */
    SS_ALGO_BINARY_GLOBAL = 4, /* bisection reading the table from global
                                memory (tables too large for LDS) */
    SS_ALGO_LEARNED = 5,     /* learned index (see ss_learned_build); in
                                plans, when SS_OPT_PLAN_LEARNED is set */
    SS_ALGO_LOGHASH = 6,     /* logarithm hash (Sec. 3.4, Eq. 1-3): |H| bins
                                of equal width in log x over [a[0], a[n-1]]
                                (|H| = SS_OPT_BUCKET_CAP, else 4n rounded up
                                to a power of two in 64..16384), a scan inside
                                the bin, a bracket check with bisection where
                                it fails; needs a normal 0 < a[0] < a[n-1] <
                                inf, else bisection */
    SS_ALGO_SKIPLIST = 7     /* skiplist (Sec. 3.3): bisection over every 8th
                                entry (a compact skip table in LDS), then a
                                count over the 8-entry block */
} ss_algo;

/* Process-wide tuning options (ss_set_option / ss_get_option). */
typedef enum {
    SS_OPT_FORCE_ALGO = 1,       /* ss_algo; default SS_ALGO_AUTO */
    SS_OPT_BUCKET_BITS = 2,      /* leading fraction bits s of the exponent
                                    hash, 0..20; -1 (default) = choose per
                                    table so the bin count fits the cap */
    SS_OPT_BUCKET_CAP = 3,       /* max bins of the exponent hash in the
                                    single-table path; 0 (default) = auto */
    SS_OPT_BLOCK_SIZE = 4,       /* threads per workgroup of single-table
                                    launches and of plans built afterwards:
                                    256, 512 or 1024; 0 (default) = auto */
    SS_OPT_GRID_BLOCKS = 5,      /* workgroups per single-table launch; 0
                                    (default) = a few tiles per workgroup,
                                    or for a small call one pass of the
                                    resident workgroups */
    SS_OPT_CHECK_POINTERS = 6,   /* 1 (default): verify that buffers are
                                    device memory before launching; 0: skip */
    SS_OPT_TARGETS_PER_LANE = 7, /* targets each lane of a single-table
                                    launch keeps in flight per tile: 4 or
                                    8; 0 (default) = 8, or 4 for a small
                                    call (at most three passes of the
                                    resident workgroups at 8).  Plans and
                                    learned searches use their own */
    SS_OPT_PLAN_TILES = 8,       /* tiles per workgroup of plans built
                                    afterwards; 0 (default) = tuner */
    SS_OPT_PLAN_LEARNED = 9,     /* learned models in plans built
                                    afterwards.  0 (default): the tuner
                                    decides per table (see the autotuner
                                    section); 1: every eligible table (2 <=
                                    n, 0 < a[0] < a[n-1] < inf) gets a model
                                    trained on the device at plan creation;
                                    2: none (exponent hash / bisection) */
    SS_OPT_LEARNED_STEPS = 10,   /* Adam steps of plan models; 0 (default)
                                    = 500 */
    SS_OPT_PLAN_XCD = 11,        /* workgroup-to-XCD mapping of plans built
                                    afterwards: the workgroup ranges are
                                    dealt to the 8 XCDs round robin in
                                    chunks of C consecutive ranges.  0
                                    (default): C = 1 (dispatch order) when
                                    the plan's segments average under 64
                                    tiles of 4096 targets, else C = 8; 1:
                                    dispatch order; 2..2^24: C = the value (a C of
                                    at least a 1/8 of the ranges gives each
                                    XCD one contiguous part) */
    SS_OPT_PAIR_JOINT = 12,      /* paired plans built afterwards: 0
                                    (default) = the density and temperature
                                    searches run as 2M independent segments
                                    of one launch, one table staged per
                                    workgroup; 1 = each workgroup searches
                                    both axes of its pairs with both of the
                                    material's tables staged */
    SS_OPT_CONVENTION = 13,      /* 0 (default): idx(x) = #{a < x} - 1, -1
                                    when no entry is below x.  1: the
                                    paper's convention (Sec. 3), the last
                                    index with a[i] <= x clamped to [0,
                                    n-1] (NaN gives 0; an empty table -1).
                                    Read by single-table and learned
                                    searches at each call and by plans at
                                    creation */
    SS_OPT_PLAN_ALGO = 14,       /* kernel of every table of plans built
                                    afterwards: SS_ALGO_AUTO (default) = the
                                    tuner's choice; SS_ALGO_BINARY = the
                                    bisection; SS_ALGO_EXPHASH = the
                                    exponent hash at the tuner's best bin
                                    bits wherever it applies (bisection
                                    elsewhere); SS_ALGO_BALLOT = the ballot
                                    scan.  Learned models follow
                                    SS_OPT_PLAN_LEARNED unless this is
                                    not SS_ALGO_AUTO, which implies none */
    SS_OPT_PLAN_ORDER = 15       /* tile order of plans built afterwards:
                                    each segment's tiles go to workgroups of
                                    at most k tiles; 1 = contiguous ranges
                                    of k tiles; 2 = strided (workgroup i of
                                    W takes tiles i, i + W, ..., so a
                                    segment's workgroups sweep it side by
                                    side); 0 (default) = 2 */
} ss_option;

/* Environment, read once when the library is loaded:
 *   SS_<NAME>=<value> sets option SS_OPT_<NAME> as ss_set_option would
 *   (SS_FORCE_ALGO, SS_BUCKET_BITS, SS_PLAN_ALGO, SS_CONVENTION, ... every
 *   option above); the values are integers, and the two algorithm options
 *   also take the names auto, binary, ballot, exphash, binary_global,
 *   learned, loghash and skiplist.  A value the option refuses is reported
 *   on stderr and ignored.  Calls to ss_set_option override them later.
 *   SS_LOG=1 writes one line per library decision to stderr, prefixed
 *   "[ss] ": options taken from the environment, every plan's per-table
 *   kernel counts, tile shape, grid, LDS and XCD mapping, a sampled plan's
 *   mean bracket, tuner calibrations and model loads, learned builds.
 *   SS_TUNER_CACHE: see the autotuner section below. */

/* Device bounds checks (the library built with -DSS_DEVICE_CHECKS=1, the
 * variant in _lib/checked/ that the package loads with SS_LIBRARY pointing
 * at it; slower, for tests).  Its kernels test every LDS index of the search
 * routines against the region it reads (the staged table and its +inf
 * padding, bin tables, model images), every full tile's target range and
 * every plan workgroup's staged layout and tile; a violation is counted and
 * the index clamped into its region, so the kernel never reads or writes
 * outside it.  ss_debug_violations (host out) returns the violations counted
 * since its last call on the current device and clears them; SYNCHRONOUS.
 * ss_debug_selftest runs a one-thread kernel that clamps one out-of-range
 * index (touching nothing outside a one-int buffer): afterwards
 * ss_debug_violations reports 1.  In the normal build both return
 * SS_ERR_UNSUPPORTED. */
SS_API int ss_debug_violations(int64_t *count);
SS_API int ss_debug_selftest(void);

/* Human-readable message for the calling thread's most recent error
 * (empty string if none).  The pointer stays valid until the next library
 * call on the same thread. */
SS_API const char *ss_last_error(void);

/* Library version as major*10000 + minor*100 + patch. */
SS_API int ss_version(void);

/* Selects the HIP stream (a hipStream_t, passed as void*) that subsequent
 * calls from the calling thread enqueue on.  NULL selects the null stream.
 * The stream is not retained: the caller keeps it alive while in use. */
SS_API int ss_set_stream(void *hip_stream);

/* Sets / reads a process-wide option (see ss_option).  Invalid option ids or
 * values return SS_ERR_INVALID_ARG and change nothing. */
SS_API int ss_set_option(int option, int64_t value);
SS_API int ss_get_option(int option, int64_t *value_out /* host */);

/* ---------------------------------------------------------------------------
 * Single table.
 * ------------------------------------------------------------------------- */

/* out_idx[k] = idx(targets[k]) for k in [0, m) (the operation defined at the
 * top of this header; paper Sec. 1, Sec. 3.2 and Sec. 3.5).
 *   table   : n float64 entries, device, sorted non-decreasing, 8-byte aligned
 *   n       : 0 <= n <= INT32_MAX; n == 0 makes every index -1
 *   targets : m float64 values, device, 8-byte aligned, any values
 *   m       : m >= 0; m == 0 is a no-op
 *   out_idx : m int32, device, 4-byte aligned, must not overlap the inputs
 * The kernel is the bisection over the table staged in LDS (or, for
 * tables over 64 KB, read from global memory) unless SS_OPT_FORCE_ALGO
 * names another: with one table per call the search is bound by HBM and a
 * hash's per-workgroup bin build costs more than it saves (plans, which
 * build each bin table once, choose per table).  Allocates
 * nothing; asynchronous; safe to capture in a HIP graph.  With
 * SS_OPT_CONVENTION = 1 the results follow the paper's convention. */
SS_API int search_sorted_batch(const double *table, int64_t n, const double *targets, int64_t m,
                        int32_t *out_idx);

/* Same as search_sorted_batch with an explicit kernel and bin bits (ignores
 * SS_OPT_FORCE_ALGO / SS_OPT_BUCKET_BITS).  algo = SS_ALGO_AUTO behaves like
 * search_sorted_batch; bucket_bits = -1 chooses automatically.  Used to
 * compare the kernels on one workload. */
SS_API int ss_search_with(const double *table, int64_t n, const double *targets, int64_t m,
                   int32_t *out_idx, int algo, int bucket_bits);

/* Checks the table precondition on the device and waits for the answer
 * (SYNCHRONOUS on the current stream).  *bad_index_out (host) receives -1 if
 * the table is sorted non-decreasing without NaN, else the smallest i with
 * a[i] NaN or a[i] > a[i+1]. */
SS_API int ss_validate_table(const double *table, int64_t n, int64_t *bad_index_out /* host */);

/* Exponent-hash bin table of a table, as the search builds it in LDS, written
 * to device memory for inspection (paper Sec. 3.5 with Eq. 3, prefix-count
 * form).  With key_s(v) = (IEEE-754 biased exponent of v) * 2^s + (leading
 * s fraction bits of v), kmin = key_s(a[0]) and nb = key_s(a[n-1]) - kmin + 1:
 *     counts[b] = #{ i : key_s(a[i]) - kmin < b },   b = 0 .. nb,
 * so bin b holds entries counts[b] .. counts[b+1]-1.
 *   bucket_bits : s in 0..20, or -1 to use the single-table path's automatic
 *                 choice for bin cap `cap`
 *   counts      : device, int32, room for `cap` entries
 *   info_out    : host, 4 int64: {s, kmin, nb, K} with K the most entries
 *                 in one bin, reported as 9 when 9 or more
 * Requires 1 <= n <= 65535 and a[0] with a clear sign bit.  If nb + 1 > cap
 * returns SS_ERR_INVALID_ARG.  For a table that violates the sort
 * precondition some entries of counts may be left unwritten.  SYNCHRONOUS. */
SS_API int ss_exphash_bins(const double *table, int64_t n, int bucket_bits, int32_t *counts,
                    int64_t cap, int64_t *info_out /* host, 4 entries */);

/* Logarithm-hash bin table of a table, as the search builds it in LDS,
 * written to device memory for inspection (paper Sec. 3.4, Eq. 1-3, in
 * prefix-count form).  Eq. 1 sets log2 b = (log2 a[n-1] - log2 a[0]) / nb;
 * Eq. 2's key floor(log_b x) - floor(log_b a[0]) is evaluated in FP32 as
 * floor(u(x) S + phi) with u(x) = log2 x - log2 a[0] (exact binary exponent
 * plus the FP32 log2 of the mantissa), S = 1 / log2 b, phi = frac(log_b
 * a[0]), clamped to [0, nb - 1]; then
 *     counts[i] = #{ j : key(a[j]) < i },   i = 0 .. nb.
 *   nb       : |H|, 1..65535
 *   counts   : device, int32, nb + 1 entries
 *   info_out : host, 6 doubles: {nb, K, e0, lm0, S, phi} with K the most
 *              entries in one bin (9 when 9 or more), e0 the biased exponent
 *              of a[0] and lm0 the FP32 log2 of its mantissa
 * Requires 2 <= n <= 65535 and a normal 0 < a[0] < a[n-1] < inf, else
 * SS_ERR_INVALID_ARG.  SYNCHRONOUS. */
SS_API int ss_loghash_bins(const double *table, int64_t n, int64_t nb, int32_t *counts,
                           double *info_out /* host, 6 entries */);

/* ---------------------------------------------------------------------------
 * Many tables in one launch (batched) and paired lookups.
 *
 * A plan is built once per set of tables (the setup the paper pays once per
 * table load, Sec. 5.3) and then searched many times.  Building it copies
 * the tables to the host once, lets the autotuner choose, per table, the
 * kernel (exponent hash or bisection) and the hash's bin bits, and the
 * number of consecutive target tiles a workgroup takes, builds the
 * exponent-hash bin tables on the device, and prepares a HIP graph whose
 * one kernel node searches the whole batch.  Plans own device memory; the tables
 * are referenced (not copied) and must stay valid and unchanged while the
 * plan is used.  A plan may be used from one thread at a time, and its
 * searches run in the order they are issued on the caller's stream; passing
 * new target or output pointers updates the graph's kernel parameters in
 * place, so searches of one plan must not be issued on two streams at once.
 * Destroy a plan only after its last search has completed (synchronise the
 * stream first).
 * ------------------------------------------------------------------------- */
typedef struct ss_plan ss_plan;
typedef struct ss_learned ss_learned; /* learned index handle (below) */

/* Plan for T tables stored back to back (CSR):
 *   tables    : device, float64; table t is tables[table_off[t] .. table_off[t+1])
 *   table_off : host, T+1 non-decreasing int64 offsets, table_off[0] == 0;
 *               each table must be sorted and is staged whole in LDS: at
 *               most 6136 entries (48 KB with its +inf padding), else
 *               SS_ERR_UNSUPPORTED (single-table calls take any size)
 *   T         : 1 <= T <= 2^20
 *   query_off : host, T+1 non-decreasing int64 offsets, query_off[0] == 0;
 *               the targets (and indices) of table t are positions
 *               query_off[t] .. query_off[t+1] of the arrays passed to
 *               ss_multi_search
 *   out       : host, receives the plan
 * SYNCHRONOUS (device work on the current stream, then waits). */
SS_API int ss_multi_plan_create(const double *tables, const int64_t *table_off, int32_t T,
                                const int64_t *query_off, ss_plan **out);

/* As ss_multi_plan_create, with learned models attached to chosen tables:
 * models (host, T handles) holds for table t either NULL (the tuner chooses
 * its kernel) or a handle built on exactly that table -- on the device
 * memory tables + table_off[t], with its entry count, on the current
 * device -- which then searches it (verified window, bisection fallback;
 * the plan counts fallbacks as with SS_OPT_PLAN_LEARNED).  The plan copies
 * each model's compiled form at creation, so the handles may be destroyed
 * afterwards.  SS_OPT_PLAN_LEARNED is ignored.  Returns SS_ERR_INVALID_ARG
 * for a handle built on other memory or another size.  SYNCHRONOUS. */
SS_API int ss_multi_plan_create_learned(const double *tables, const int64_t *table_off,
                                        int32_t T, const int64_t *query_off,
                                        ss_learned *const *models, ss_plan **out);

/* As ss_multi_plan_create, with sample targets that show how the searches'
 * targets are distributed (paper Sec. 5.2: the best method depends on the
 * data).  sample: device float64 [query_off[T]], laid out as the targets of
 * ss_multi_search (the first batch to be searched, say); it is read during
 * creation only.  For each table the plan measures, over 32 wave-sized
 * groups of sample targets spread over its tiles (the targets one wave of
 * the search kernel takes together), the mean number of table entries
 * between the group's smallest and largest target, and the autotuner adds
 * the ballot scan (SS_ALGO_BALLOT: a linear scan of that bracket, Sec. 2.1)
 * as a candidate at its modelled cost for that bracket, against the
 * bisection (tables the exponent hash does not take: negative entries, too
 * many bins); the hash is kept where it applies.  Close targets (sorted or
 * slowly varying streams) give narrow brackets; i.i.d. targets give
 * brackets near the table's size, where it is never chosen.  Later
 * searches may pass any targets: results are exact whatever the choice,
 * but a ballot table searched with spread-out targets is slow.
 * SS_PLAN_BRACKETS reports the measured brackets.  SYNCHRONOUS. */
SS_API int ss_multi_plan_create_sampled(const double *tables, const int64_t *table_off,
                                        int32_t T, const int64_t *query_off,
                                        const double *sample, ss_plan **out);

/* out_idx[k] = idx_t(targets[k]) for every k in [query_off[t], query_off[t+1]),
 * where idx_t is the operation defined at the top of this header applied to
 * table t.  targets: device float64 [query_off[T]]; out_idx: device int32,
 * same length, not overlapping.  Asynchronous on the current stream (one
 * graph launch). */
SS_API int ss_multi_search(ss_plan *plan, const double *targets, int32_t *out_idx);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, serving loops and harnesses that forbid hipMalloc -- the batched
 * search of ss_multi_search without a plan:
 *   out_idx[k] = idx_t(targets[k]) for k in [query_off[t], query_off[t+1])
 * with idx_t the operation at the top of this header over table t.
 *   tables    : device, float64, total_n entries; table t is
 *               tables[table_off[t] .. table_off[t+1]) (sorted, any length up
 *               to INT32_MAX; up to 6136 entries are staged in LDS, longer
 *               tables are searched in place)
 *   table_off : DEVICE, T+1 int64, non-decreasing, within [0, total_n]
 *   T         : 1 <= T <= 65536 (the limit of the device scratch below;
 *               larger T returns SS_ERR_INVALID_ARG)
 *   query_off : DEVICE, T+1 int64, non-decreasing, query_off[0] == 0 and
 *               query_off[T] == m
 *   targets   : device, m float64; out_idx: device, m int32, not overlapping
 *               any input
 * Every table is searched by bisection (no tuner, no bin tables); results
 * are those of ss_multi_search on the same tables, and follow
 * SS_OPT_CONVENTION as read at the call.  Offsets are read on the device and
 * not validated: offsets outside [0, total_n] / [0, m] are clamped into them
 * and decreasing ones are raised to the running maximum, so a violation
 * gives unspecified indices (or leaves targets outside every segment
 * unwritten) but no out-of-bounds access.
 * Allocates nothing and never synchronises: two kernels on the current
 * stream.  Working memory is a 1 MiB array of static device memory that each
 * GPU the library runs on holds until the process ends; every call on one GPU
 * shares it, so calls that overlap on one GPU (from two streams or two
 * threads) race and must be ordered by the caller.  Each call rewrites every
 * entry it reads.  Asynchronous. */
SS_API int ss_multi_search_noalloc(const double *tables, int64_t total_n,
                                   const int64_t *table_off, int32_t T,
                                   const int64_t *query_off, const double *targets, int64_t m,
                                   int32_t *out_idx);

/* Paired lookup (the density and temperature axes of EOS tables, Sec. 1):
 * M materials, each with a density table and a temperature table (CSR as
 * above, each at most 6136 entries; in the joint form, SS_OPT_PAIR_JOINT,
 * and in interpolation plans, which stage both axes at once, the largest
 * density table and the largest temperature table together at most 6128:
 * their two staged copies, each with 8 +inf entries and rounded up to 16
 * bytes, within 48 KB),
 * and pair_off (host, M+1) grouping the
 * query pairs by material.  ss_pair_search writes, for every pair k of
 * material j, out_rho[k] = idx over density table j of rho[k] and
 * out_t[k] = idx over temperature table j of temp[k], in one launch. */
SS_API int ss_pair_plan_create(const double *rho_tables, const int64_t *rho_off,
                               const double *t_tables, const int64_t *t_off, int32_t M,
                               const int64_t *pair_off, ss_plan **out);
SS_API int ss_pair_search(ss_plan *plan, const double *rho, const double *temp,
                          int32_t *out_rho, int32_t *out_t);

/* As ss_pair_plan_create, with sample pairs (device float64 [pair_off[M]]
 * each, laid out as the rho and temp arrays of ss_pair_search) from which
 * the autotuner measures every density and temperature table's ballot
 * bracket, as in ss_multi_plan_create_sampled.  SYNCHRONOUS. */
SS_API int ss_pair_plan_create_sampled(const double *rho_tables, const int64_t *rho_off,
                                       const double *t_tables, const int64_t *t_off, int32_t M,
                                       const int64_t *pair_off, const double *sample_rho,
                                       const double *sample_temp, ss_plan **out);

/* Interpolation after the paired search (the step EOSPAC takes after it,
 * Sec. 1): material j also has a value grid F_j over its two axes, stored
 * row-major over (density, temperature) -- F_j[a][b] at
 * values[voff_j + a * nT_j + b], with the grids back to back in material
 * order (voff_j = sum over k < j of nR_k nT_k).  For pair p of material j:
 *   i = clamp(idx_rho(rho[p]), 0, nR_j - 2),  k = clamp(idx_T(T[p]), 0, nT_j - 2)
 *   u = (rho - R[i]) / (R[i+1] - R[i]),       v = (T - T[k]) / (T[k+1] - T[k])
 *   out_f[p] = (1-u)(1-v) F[i][k] + u(1-v) F[i+1][k] + (1-u) v F[i][k+1] + u v F[i+1][k+1]
 * with idx the strict index of this header (outside the axes the edge cell
 * is extended linearly; NaN gives NaN).  Each workgroup stages both axes of
 * its material and reads the four corner values from the grid (L2).
 * Requirements beyond ss_pair_plan_create's: every axis has at least 2
 * finite, strictly increasing entries; values is a device array of
 * sum nR_j nT_j float64, referenced (must outlive the plan).  The plan
 * ignores SS_OPT_PLAN_LEARNED and SS_OPT_CONVENTION.  SYNCHRONOUS. */
SS_API int ss_interp_plan_create(const double *rho_tables, const int64_t *rho_off,
                                 const double *t_tables, const int64_t *t_off, int32_t M,
                                 const int64_t *pair_off, const double *values, ss_plan **out);

/* out_f: float64[m] (device); out_rho, out_t: both NULL, or int32[m] each
 * (device) to receive the two indices as well.  Asynchronous. */
SS_API int ss_interp_search(ss_plan *plan, const double *rho, const double *temp, double *out_f,
                            int32_t *out_rho, int32_t *out_t);

SS_API int ss_plan_destroy(ss_plan *plan);

/* Saves a plan's choices -- per table its kernel and exponent-hash bin
 * bits, and a learned table's 1153 model parameters -- with its form, tiles
 * per workgroup, tile order and convention, as a text file: the setup the
 * paper pays once per table load (Sec. 5.3), kept across runs.
 * Interpolation plans return SS_ERR_UNSUPPORTED.  Host file I/O only. */
SS_API int ss_plan_save(const ss_plan *plan, const char *path);

/* Rebuild a saved batched or paired plan (arguments as ss_multi_plan_create
 * and ss_pair_plan_create; the paired form comes from the file) for tables of
 * the same sizes, without tuning or training: each table takes its saved
 * kernel (an exponent hash's bin parameters are recomputed from the table;
 * a table whose saved bits no longer apply gets the tuner's choice), learned
 * tables get their saved models, and every model's error bound is measured
 * again on the device, so the plan is exact for any tables of these sizes.
 * The saved tiles per workgroup, tile order and convention replace the
 * options in force.  SS_ERR_INVALID_ARG for a missing or malformed file, a
 * plan of another form, or tables of other sizes.  SYNCHRONOUS. */
SS_API int ss_multi_plan_load(const char *path, const double *tables, const int64_t *table_off,
                              int32_t T, const int64_t *query_off, ss_plan **out);
SS_API int ss_pair_plan_load(const char *path, const double *rho_tables, const int64_t *rho_off,
                             const double *t_tables, const int64_t *t_off, int32_t M,
                             const int64_t *pair_off, ss_plan **out);

/* Targets of the most recent search of a plan with learned tables that
 * failed the window check and were answered by bisection (0 for plans
 * without learned tables).  SYNCHRONOUS (waits for the current stream). */
SS_API int ss_plan_fallbacks(ss_plan *plan, int64_t *count);

/* What the autotuner chose, for inspection (host output):
 *   SS_PLAN_ALGOS  : int32 per table (ss_algo: binary, exphash, ballot or
 *                    learned); paired plans list the density tables, then
 *                    the temperature tables
 *   SS_PLAN_BITS   : int32 per table (bin bits s, -1 for bisection)
 *   SS_PLAN_SUMMARY: 8 int64 {tables, tiles, tiles per workgroup, grid,
 *                    block, lds_bytes, longest bin (9 = 9 or more),
 *                    graph launches so far}; with cap >= 10 also the
 *                    targets per lane and the learned form of the search
 *                    kernel (0: no learned table, 1: clamped windows,
 *                    2: bounded staging)
 *   SS_PLAN_COSTS  : 2 doubles per table (cap >= 2 T): the autotuner's
 *                    modelled ns per query of its best plain kernel, and of
 *                    the table's trained learned model (-1 if none was
 *                    trained); in tuner mode a trained table is learned
 *                    exactly when the second is the smaller
 *   SS_PLAN_BRACKETS: 1 double per table: the mean ballot bracket measured
 *                    on the sample targets of a sampled plan (-1: not
 *                    sampled, or no targets)
 * `cap` is the number of elements `out` can hold. */
typedef enum {
    SS_PLAN_ALGOS = 1,
    SS_PLAN_BITS = 2,
    SS_PLAN_SUMMARY = 3,
    SS_PLAN_COSTS = 4,
    SS_PLAN_BRACKETS = 5
} ss_plan_query;
SS_API int ss_plan_info(const ss_plan *plan, int what, void *out, int64_t cap);

/* ---------------------------------------------------------------------------
 * Learned index (not in the paper; the nearest analogue is the logarithm
 * hash of Sec. 3.4, an analytic model of a table's position as a function
 * of log x).  A per-table model predicts where x falls; a verified, bounded
 * search corrects the prediction; the plain search is the fallback, so the
 * result is always exactly the operation defined at the top of this header.
 *
 * Model: an FP32 multilayer perceptron 1 -> 32 -> 32 -> 1 with ReLU hidden
 * layers.  Input z = (log2 x - log2 a[0]) / (log2 a[n-1] - log2 a[0]),
 * computed in FP32 from x rounded to FP32.  Output p estimates i / (n-1) for
 * x = a[i] (the table's CDF).  Parameters (1153 floats, in this order):
 *   w1[32], b1[32], W2[32][32] (row k holds the weights into hidden unit k
 *   of layer 2), b2[32], w3[32], b3.
 * Training: full-batch Adam on the mean squared error over the n table
 * entries, `steps` steps at learning rate `lr` (beta1 0.9, beta2 0.999,
 * eps 1e-8, cosine-decayed rate), parameters initialised from `seed`; run by
 * one workgroup with deterministic, fixed-order reductions.
 * Evaluation (search, E and ss_learned_predict): the trained model is
 * compiled once, exactly.  With one input z the network is a continuous
 * piecewise-linear function: its pieces end at layer 1's breakpoints
 * -b1_j / w1_j and, between those, where a layer-2 unit's pre-activation
 * changes sign.  The compiled form is the sorted list of piece boundaries
 * (at most 1088) and one (slope, intercept) per piece (at most 1089), both
 * formed in float64 and rounded to FP32: p(z) = slope_i z + intercept_i for
 * the piece i holding z, i = #{boundaries < z}.  i is found through a table
 * of equal cells over the boundaries' range (prefix counts plus a scan of
 * at most 8 boundaries), or by bisection when some cell would hold more.
 * This is the same function as the layered form, up to FP32 rounding.
 * Search: g = floor(p (n-1)) clamped to [-1, n-1]; the window
 * [L, R] = [g - E, g + E] clamped to [-1, n-1] is accepted if
 * (L == -1 or a[L] < x) and (R == n-1 or x <= a[R+1]); the index is then
 * found by bisection inside it, otherwise by bisection over the whole table.
 * A table staged in LDS with -inf entries before a[0] and +inf entries after
 * a[n-1] takes the window unclamped and widened at the top to
 * [g - E, g - E + 2s - 1], s the largest power of two <= 2E + 1 (the
 * bisection's 2s positions), with the same acceptance test.
 * E = 1 + the largest |g(x) - idx(x)| over the entries, their upward
 * neighbours and the log-midpoints between entries, measured on the device
 * with the search's own prediction code.
 * ------------------------------------------------------------------------- */

typedef struct {
    int32_t steps;     /* Adam steps; 0 keeps the initial parameters */
    float lr;          /* peak learning rate (> 0) */
    uint64_t seed;     /* initialisation seed */
} ss_mlp_opts;

#define SS_MLP_PARAMS 1153

/* Trains a model for the table (device, n entries, sorted, 2 <= n <= 65535,
 * a[0] > 0, all finite) and measures E.  opts may be NULL for the defaults
 * {steps 3000, lr 0.01, seed 1}.  The table is referenced, not copied, and
 * must stay valid while the handle is used.  SYNCHRONOUS. */
SS_API int ss_learned_build(const double *table, int64_t n, const ss_mlp_opts *opts,
                            ss_learned **out);

/* Same, with given parameters instead of training (weights: host, 1153
 * floats); E is measured for this table. */
SS_API int ss_learned_from_weights(const double *table, int64_t n, const float *weights,
                                   ss_learned **out);

/* Writes the model to a text file (JSON: format tag, n, E, steps, loss, the
 * normalisation and the 1153 parameters, each printed so that it reads back
 * bit-exactly).  SYNCHRONOUS (host file I/O only). */
SS_API int ss_learned_save(const ss_learned *h, const char *path);

/* Reads a model written by ss_learned_save and attaches it to a table of the
 * same size (the table the model was trained on, or any other: E is
 * measured again on the device for this table, so the search stays exact
 * for any stored model).  Returns SS_ERR_INVALID_ARG for a missing or
 * malformed file or a size mismatch.  SYNCHRONOUS. */
SS_API int ss_learned_load(const double *table, int64_t n, const char *path, ss_learned **out);

/* out_idx[k] = idx(targets[k]) through the learned index; asynchronous.
 * The table is staged in LDS with the compiled model when both fit in
 * 64 KB (n up to about 8000); larger tables are read in place from global
 * memory, with the same results. */
SS_API int ss_learned_search(ss_learned *h, const double *targets, int64_t m,
                             int32_t *out_idx);

/* Model outputs p(x) * (n-1) (the predicted fractional position) for each
 * target (device in, device out); asynchronous. */
SS_API int ss_learned_predict(ss_learned *h, const double *x, int64_t m, float *out_pos);

/* info (host, count >= 6 doubles): {E, n, steps, final training loss,
 * log2 a[0], 1 / (log2 a[n-1] - log2 a[0])}; with count >= 8 also the
 * compiled model's piece count and its padded boundary slots (a power of two,
 * at least pieces + 7); with count >= 10 also its cell count (0: the piece
 * is found by bisection) and the most boundaries in one cell.  SYNCHRONOUS
 * only in that it reads the handle's host copy. */
SS_API int ss_learned_info(const ss_learned *h, double *info, int count);

/* Targets of the most recent ss_learned_search that failed the window
 * check and were answered by the fallback.  SYNCHRONOUS (waits for the
 * current stream). */
SS_API int ss_learned_fallbacks(ss_learned *h, int64_t *count);

/* The model's error bound E (host out), as measured at build or load time:
 * every table entry's predicted index lies within E - 1 of its index. */
SS_API int ss_learned_error_bound(const ss_learned *h, int32_t *E);

/* Replaces the error bound the searches use (0 <= E <= 65535; plans built
 * afterwards with this handle take it too), to exercise the verification:
 * a bound below the measured one makes windows miss, and those targets are
 * answered by the fallback bisection (results stay exact, the fallback
 * count rises); a larger one widens every window.  ss_learned_error_bound
 * then reports the value in force, and ss_learned_save writes it. */
SS_API int ss_learned_set_error_bound(ss_learned *h, int32_t E);

/* Statistics of the most recent ss_learned_search: the targets answered by
 * the fallback (the same count as ss_learned_fallbacks).  SYNCHRONOUS. */
SS_API int ss_learned_stats(ss_learned *h, int64_t *fallbacks);

/* Copies the 1153 parameters (host out, cap >= 1153). */
SS_API int ss_learned_weights(const ss_learned *h, float *out, int64_t cap);

/* Full-batch gradient of the training loss at the given parameters (host
 * in, 1153 floats; host out, 1153 floats, same layout) for this table,
 * computed by the training kernel's code.  For checking the training
 * arithmetic.  SYNCHRONOUS. */
SS_API int ss_mlp_gradient(const double *table, int64_t n, const float *weights,
                           float *grad_out, double *loss_out);

SS_API int ss_learned_destroy(ss_learned *h);

/* ---------------------------------------------------------------------------
 * Autotuner (paper Sec. 5.1-5.2: the best method depends on the array sizes
 * and on the distribution of the data).  Plans choose each table's kernel
 * (exponent hash at some bin bits, bisection, or -- with SS_OPT_PLAN_LEARNED
 * 0 -- the learned index) and the number of consecutive target tiles a
 * workgroup takes, from a cost model in device-wide nanoseconds per query:
 * every kernel moves the same 12 bytes per query, so the choice minimises
 * compute:
 *   bisection      bin_base + bin_per_step * ceil(log2 n)
 *   exponent hash  hash_base + hash_per_k * K(s)   (K: the longest bin)
 *   learned index  learned_base + learned_per_step * (lookup + window(E)),
 *                  lookup = the model's piece lookup in LDS steps, window(E)
 *                  = floor(log2(2E + 1)) + 3 (bisection and its two checks)
 *   ballot scan    ballot_base + ballot_per_entry * (B + ceil((n + 1) / 64)),
 *                  B = the mean bracket measured on sample targets (sampled
 *                  plans only, against the bisection; otherwise the target
 *                  order is unknown and it is not a candidate)
 * In tuner mode a table is trained only when the learned cost at the best
 * possible bound (E = 1) undercuts its best plain kernel; after training the
 * measured E and lookup decide.  The model starts from built-in coefficients;
 * ss_tuner_calibrate measures them on the current device.  A model is saved
 * as JSON with the device architecture and HIP runtime version it was
 * measured with, and a file from another architecture or runtime is refused.
 * If the environment variable SS_TUNER_CACHE names a file, the first plan
 * (or tuner call) loads it; when it is missing or refused, the model is
 * calibrated on the current device once and written there (messages on
 * stderr).  Plans built earlier keep their choices.
 * ------------------------------------------------------------------------- */

/* Runs the calibration microbenchmarks on the current device and stream
 * (about 1.5 GiB of temporary device memory and a 300-step model training,
 * about a second).  SYNCHRONOUS. */
SS_API int ss_tuner_calibrate(void);

/* coeffs (host) receives, with count >= 8: {stream GB/s, hash fixed ns, hash
 * ns per scanned entry, bisection fixed ns, bisection ns per step, learned
 * index fixed ns, calibrated flag, most bins per table entry}; with count >=
 * 10 also {tiles per workgroup for segments averaging under 64 tiles of 4096
 * targets, for longer segments}; with count >= 11 also {learned index ns per
 * LDS step}; with count >= 13 also {ballot scan fixed ns, ballot scan ns per
 * entry}.  ss_tuner_set replaces the model with 8, 10, 11 or 13 such values
 * (all finite and non-negative; bandwidth and bins per entry positive; tiles
 * in 1..4096). */
SS_API int ss_tuner_get(double *coeffs, int count);
SS_API int ss_tuner_set(const double *coeffs, int count);

/* Saves / loads the model as JSON at a host file path.  Loading refuses
 * (SS_ERR_INVALID_ARG, model unchanged) a malformed file, or one measured on
 * another architecture than the current device (or, without a device, than
 * gfx950) or under another HIP runtime version. */
SS_API int ss_tuner_save(const char *path);
SS_API int ss_tuner_load(const char *path);

#ifdef __cplusplus
}
#endif

#endif /* SEARCHSORTED_H */
