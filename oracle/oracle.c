/*
 * CPU ORACLE -- test infrastructure only.
 *
 * Plain, slow, obviously correct reference for the batched sorted search.
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load this file's library; the product path never does.  It
 * shares no code, header or table with the device library.
 *
 * The search result (Sec. 1 of the paper: the index of the largest table
 * element that is less than a given target), read with a strict "<" and -1
 * when no element qualifies, has a plain definition:
 *
 *     idx(x) = #{ i in [0, n) : a[i] < x } - 1.
 *
 * Every method in the library (bisection, Sec. 3.2; the exponent hash with
 * an in-bin linear scan, Sec. 3.4-3.5; the learned index) must reach exactly
 * this number, so the oracle is the definition written out: one full pass
 * over the table per target, IEEE ordered compares, no early exit.  Special
 * targets need no special code: a NaN target compares false with every entry
 * (-> -1), -0.0 equals +0.0, denormals compare exactly, -inf -> -1 and
 * +inf -> (number of finite entries) - 1.
 *
 * Build: gcc -O2 -shared -fPIC -pthread, never with -ffast-math, -ffinite-math
 * or flush-to-zero flags (they would change the meaning of the compares).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <unistd.h>

/* ---- host threading: static chunks over the targets ----------------------- */

typedef void (*chunk_fn)(void *ctx, int64_t begin, int64_t end, int tid);

typedef struct {
    chunk_fn fn;
    void *ctx;
    int64_t begin, end;
    int tid;
} chunk_job;

static void *chunk_main(void *p) {
    chunk_job *j = (chunk_job *)p;
    j->fn(j->ctx, j->begin, j->end, j->tid);
    return NULL;
}

int oracle_default_threads(void) {
    long c = sysconf(_SC_NPROCESSORS_ONLN);
    if (c < 1) c = 1;
    const char *env = getenv("OMP_NUM_THREADS");
    if (env) {
        long e = strtol(env, NULL, 10);
        if (e > 0 && e < c) c = e;
    }
    return c > 256 ? 256 : (int)c;
}

/* Runs fn over [0, count) split into `threads` contiguous chunks; returns the
 * number of threads that actually ran. */
static int run_chunks(int threads, int64_t count, chunk_fn fn, void *ctx) {
    if (threads <= 0) threads = oracle_default_threads();
    if (threads > 256) threads = 256;
    if (count < threads) threads = count > 0 ? (int)count : 1;
    if (threads == 1) {
        fn(ctx, 0, count, 0);
        return 1;
    }
    pthread_t th[256];
    chunk_job job[256];
    int ran = 0;
    for (int t = 0; t < threads; ++t) {
        job[t].fn = fn;
        job[t].ctx = ctx;
        job[t].begin = count * t / threads;
        job[t].end = count * (t + 1) / threads;
        job[t].tid = t;
        if (pthread_create(&th[t], NULL, chunk_main, &job[t]) != 0) {
            fn(ctx, job[t].begin, job[t].end, t);
            job[t].fn = NULL;
        } else {
            ++ran;
        }
    }
    for (int t = 0; t < threads; ++t)
        if (job[t].fn) pthread_join(th[t], NULL);
    return ran > 0 ? ran : 1;
}

/* ---- the definition: idx(x) = #{a[i] < x} - 1 ----------------------------- */

typedef struct {
    const double *a;
    int64_t n;
    const double *x;
    int32_t *out;
} count_ctx;

static void count_chunk(void *p, int64_t b, int64_t e, int tid) {
    (void)tid;
    count_ctx *c = (count_ctx *)p;
    for (int64_t k = b; k < e; ++k) {
        const double xk = c->x[k];
        int64_t cnt = 0;
        for (int64_t i = 0; i < c->n; ++i) cnt += (c->a[i] < xk);
        c->out[k] = (int32_t)(cnt - 1);
    }
}

/* out[k] = #{i : a[i] < x[k]} - 1 for k in [0, m).  Returns threads used. */
int oracle_search_lt(const double *a, int64_t n, const double *x, int64_t m, int32_t *out,
                     int threads) {
    count_ctx c = {a, n, x, out};
    return run_chunks(threads, m, count_chunk, &c);
}

/* Same definition at selected positions only: out[j] = idx(x[pos[j]]). */
typedef struct {
    const double *a;
    int64_t n;
    const double *x;
    const int64_t *pos;
    int32_t *out;
} count_at_ctx;

static void count_at_chunk(void *p, int64_t b, int64_t e, int tid) {
    (void)tid;
    count_at_ctx *c = (count_at_ctx *)p;
    for (int64_t j = b; j < e; ++j) {
        const double xk = c->x[c->pos[j]];
        int64_t cnt = 0;
        for (int64_t i = 0; i < c->n; ++i) cnt += (c->a[i] < xk);
        c->out[j] = (int32_t)(cnt - 1);
    }
}

int oracle_search_lt_at(const double *a, int64_t n, const double *x, const int64_t *pos,
                        int64_t count, int32_t *out, int threads) {
    count_at_ctx c = {a, n, x, pos, out};
    return run_chunks(threads, count, count_at_chunk, &c);
}

/* Segmented form for batched workloads: segment s searches table
 * tables[toff[s] .. toff[s+1]) with targets x[qoff[s] .. qoff[s+1]). */
int oracle_search_lt_segments(const double *tables, const int64_t *toff, const double *x,
                              const int64_t *qoff, int32_t nseg, int32_t *out, int threads) {
    int used = 1;
    for (int32_t s = 0; s < nseg; ++s) {
        int64_t m = qoff[s + 1] - qoff[s];
        if (m <= 0) continue;
        int u = oracle_search_lt(tables + toff[s], toff[s + 1] - toff[s], x + qoff[s], m,
                                 out + qoff[s], threads);
        if (u > used) used = u;
    }
    return used;
}

/* ---- bracket check: a[i] < x <= a[i+1], with a[-1] = -inf, a[n] = +inf ----
 * For a table sorted non-decreasing this property holds for exactly one i
 * in [-1, n-1], which makes it an exact per-target check at any size.  A NaN
 * target must give -1.  Returns the number of violations; *first_bad gets the
 * smallest violating position (or -1). */
typedef struct {
    const double *a;
    int64_t n;
    const double *x;
    const int32_t *idx;
    int64_t bad[256];
    int64_t first[256];
} bracket_ctx;

static void bracket_chunk(void *p, int64_t b, int64_t e, int tid) {
    bracket_ctx *c = (bracket_ctx *)p;
    int64_t bad = 0, first = -1;
    for (int64_t k = b; k < e; ++k) {
        const double xk = c->x[k];
        const int64_t i = c->idx[k];
        int ok;
        if (xk != xk) {
            ok = (i == -1);
        } else if (i < -1 || i > c->n - 1) {
            ok = 0;
        } else {
            int lower_ok = (i == -1) || (c->a[i] < xk);
            int upper_ok = (i == c->n - 1) || (xk <= c->a[i + 1]);
            ok = lower_ok && upper_ok;
        }
        if (!ok) {
            if (first < 0) first = k;
            ++bad;
        }
    }
    c->bad[tid] = bad;
    c->first[tid] = first;
}

int64_t oracle_check_bracket(const double *a, int64_t n, const double *x, int64_t m,
                             const int32_t *idx, int64_t *first_bad, int threads) {
    bracket_ctx *c = (bracket_ctx *)calloc(1, sizeof(bracket_ctx));
    if (!c) return -1;
    c->a = a;
    c->n = n;
    c->x = x;
    c->idx = idx;
    for (int t = 0; t < 256; ++t) c->first[t] = -1;
    run_chunks(threads, m, bracket_chunk, c);
    int64_t bad = 0, first = -1;
    for (int t = 0; t < 256; ++t) {
        bad += c->bad[t];
        if (c->first[t] >= 0 && (first < 0 || c->first[t] < first)) first = c->first[t];
    }
    free(c);
    if (first_bad) *first_bad = first;
    return bad;
}

/* ---- exponent-hash bins (Sec. 3.5 with Eq. 3) ------------------------------
 * The paper's exponent hash bins a value by the base-2 exponent stored in its
 * IEEE 754 binary64 encoding.  With s extra leading fraction bits each binade
 * is split into 2^s equal sub-bins; s = 0 is the paper's hash.  Written out
 * from the encoding's definition (biased exponent E, 52-bit fraction F):
 *   normal v = 2^e (1 + f), f in [0,1):  E = e + 1023,  key = E 2^s + floor(f 2^s)
 *   subnormal v = F 2^-1074:             E = 0,         key = floor(F 2^(s-52))
 *   v = +0: key = 0;   v = +inf: key = 2047 2^s.
 * Defined for v >= +0 (sign bit clear) and s in [0, 20]. */
int64_t oracle_exponent_key(double v, int s) {
    if (v == 0.0) return 0;
    if (isinf(v)) return (int64_t)2047 << s;
    if (v < 0x1p-1022) {
        double F = ldexp(v, 1074); /* exact: the integer fraction field */
        return (int64_t)floor(ldexp(F, s - 52));
    }
    int E2;
    double mant = frexp(v, &E2); /* v = mant 2^E2, mant in [0.5, 1) */
    int e = E2 - 1;
    double f = 2.0 * mant - 1.0; /* exact */
    return ((int64_t)(e + 1023) << s) + (int64_t)floor(ldexp(f, s));
}

/* Prefix-count bin table of a sorted non-negative table:
 *   kmin = key(a[0]), nb = key(a[n-1]) - kmin + 1,
 *   C[b] = #{ i : key(a[i]) - kmin < b },  b = 0 .. nb.
 * Bin b holds entries C[b] .. C[b+1]-1 (the set Eq. 3 indexes by its
 * smallest member).  Returns nb, or -1 if C would need more than cap
 * entries, or -2 for an empty table. */
int64_t oracle_exponent_bins(const double *a, int64_t n, int s, int64_t *C, int64_t cap,
                             int64_t *kmin_out) {
    if (n <= 0) return -2;
    int64_t kmin = oracle_exponent_key(a[0], s);
    int64_t kmax = oracle_exponent_key(a[n - 1], s);
    int64_t nb = kmax - kmin + 1;
    if (kmin_out) *kmin_out = kmin;
    if (nb < 1 || nb + 1 > cap) return -1;
    for (int64_t b = 0; b <= nb; ++b) {
        int64_t cnt = 0;
        for (int64_t i = 0; i < n; ++i) cnt += (oracle_exponent_key(a[i], s) - kmin < b);
        C[b] = cnt;
    }
    return nb;
}

/* ---- logarithm-hash bins (Sec. 3.4, Eq. 1-3) --------------------------------
 * For a table with 0 < Xmin = a[0] < Xmax = a[n-1] < inf and |H| bins:
 *   base     b = 10^((log10 Xmax - log10 Xmin) / |H|)                 (Eq. 1)
 *   hash(x)    = floor(log_b x) - floor(log_b Xmin),  log_b x = ln x / ln b
 *                                                                      (Eq. 2)
 * Eq. 1 puts Xmax itself at hash |H| (outside 0 <= hash < |H|), and
 * targets outside [Xmin, Xmax] fall outside too, so keys are clamped to
 * [0, |H| - 1]; x <= 0 and NaN take bin 0.  The bin table is Eq. 3 in
 * prefix-count form:
 *   C[i] = #{ j : hash(a[j]) < i },  i = 0 .. |H|
 * (for a non-empty bin i, C[i] is Eq. 3's smallest index with hash i). */
double oracle_log_hash_base(double xmin, double xmax, int64_t H) {
    return pow(10.0, (log10(xmax) - log10(xmin)) / (double)H);
}

int64_t oracle_log_hash_raw(double x, double xmin, double base) {
    const double lb = log(base);
    return (int64_t)(floor(log(x) / lb) - floor(log(xmin) / lb));
}

int64_t oracle_log_hash_key(double x, double xmin, double base, int64_t H) {
    if (!(x > 0.0)) return 0;
    if (isinf(x)) return H - 1;
    int64_t k = oracle_log_hash_raw(x, xmin, base);
    if (k < 0) return 0;
    if (k > H - 1) return H - 1;
    return k;
}

void oracle_log_hash_keys(const double *x, int64_t m, double xmin, double base, int64_t H,
                          int64_t *out) {
    for (int64_t i = 0; i < m; ++i) out[i] = oracle_log_hash_key(x[i], xmin, base, H);
}

/* C[0..H] for a sorted table; returns H, -1 if the table does not satisfy
 * 0 < a[0] < a[n-1] < inf, -2 if it is empty or H < 1. */
int64_t oracle_log_hash_bins(const double *a, int64_t n, int64_t H, int64_t *C) {
    if (n < 1 || H < 1) return -2;
    if (!(a[0] > 0.0) || !(a[n - 1] > a[0]) || isinf(a[n - 1])) return -1;
    const double base = oracle_log_hash_base(a[0], a[n - 1], H);
    int64_t *key = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!key) return -3;
    for (int64_t j = 0; j < n; ++j) key[j] = oracle_log_hash_key(a[j], a[0], base, H);
    for (int64_t i = 0; i <= H; ++i) {
        int64_t cnt = 0;
        for (int64_t j = 0; j < n; ++j) cnt += key[j] < i;
        C[i] = cnt;
    }
    free(key);
    return H;
}

/* ---- the paper's convention (Sec. 3) -----------------------------------------
 * Sec. 3 states the problem as the index of the last element of X that is
 * less than or equal to the target, 0 when there is none, and n - 1 for a
 * target above the last element:
 *   idx_le(y) = min(max(#{ i : a[i] <= y } - 1, 0), n - 1)
 * (a NaN target has no element <= it, hence 0; an empty table gives -1). */
typedef struct {
    const double *a;
    int64_t n;
    const double *x;
    int32_t *out;
} le_ctx;

static void le_chunk(void *p, int64_t b, int64_t e, int tid) {
    (void)tid;
    le_ctx *c = (le_ctx *)p;
    for (int64_t k = b; k < e; ++k) {
        const double xk = c->x[k];
        int64_t cnt = 0;
        for (int64_t i = 0; i < c->n; ++i) cnt += (c->a[i] <= xk);
        int64_t r = cnt - 1;
        if (c->n > 0) {
            if (r < 0) r = 0;
            if (r > c->n - 1) r = c->n - 1;
        }
        c->out[k] = (int32_t)r;
    }
}

int oracle_search_le_clamped(const double *a, int64_t n, const double *x, int64_t m,
                             int32_t *out, int threads) {
    le_ctx c = {a, n, x, out};
    return run_chunks(threads, m, le_chunk, &c);
}

/* ---- bilinear interpolation after the paired search ------------------------
 * EOSPAC interpolates a material's table F over its density and temperature
 * axes after finding each target's cell (Sec. 1).  For a pair (r, t) of
 * material j with axes R[0..nr) and T[0..nt) (strictly increasing, nr, nt
 * >= 2) and grid F[a][b] = values[a nt + b]:
 *   i = min(max(#{R < r} - 1, 0), nr - 2),  k = min(max(#{T < t} - 1, 0), nt - 2)
 *   u = (r - R[i]) / (R[i+1] - R[i]),        v = (t - T[k]) / (T[k+1] - T[k])
 *   f = (1-u)(1-v) F[i][k] + u(1-v) F[i+1][k] + (1-u) v F[i][k+1] + u v F[i+1][k+1]
 * (outside the axes the edge cell is extended linearly; NaN gives NaN).
 * scale = |w00 F[i][k]| + |w10 F[i+1][k]| + |w01 F[i][k+1]| + |w11 F[i+1][k+1]|,
 * the four terms' magnitudes with the weights formed from the rounded u,
 * 1-u, v and 1-v.  Any evaluation order of the same four terms from the
 * same rounded factors (products, sums, fused multiply-adds) stays within a
 * few units of rounding of scale of the exact sum of those terms, however
 * much they cancel, so a small multiple of eps * scale bounds the
 * difference between two such orders. */
static int64_t count_lt(const double *a, int64_t n, double x) {
    int64_t c = 0;
    for (int64_t i = 0; i < n; ++i) c += a[i] < x;
    return c;
}

void oracle_interp_pairs(const double *rho_tables, const int64_t *rho_off, const double *t_tables,
                         const int64_t *t_off, const int64_t *pair_off, int32_t M,
                         const double *values, const double *rho, const double *temp,
                         double *out, double *scale) {
    int64_t voff = 0;
    for (int32_t j = 0; j < M; ++j) {
        const double *R = rho_tables + rho_off[j];
        const double *T = t_tables + t_off[j];
        const int64_t nr = rho_off[j + 1] - rho_off[j], nt = t_off[j + 1] - t_off[j];
        const double *F = values + voff;
        for (int64_t p = pair_off[j]; p < pair_off[j + 1]; ++p) {
            int64_t i = count_lt(R, nr, rho[p]) - 1, k = count_lt(T, nt, temp[p]) - 1;
            if (i < 0) i = 0;
            if (i > nr - 2) i = nr - 2;
            if (k < 0) k = 0;
            if (k > nt - 2) k = nt - 2;
            const double u = (rho[p] - R[i]) / (R[i + 1] - R[i]);
            const double v = (temp[p] - T[k]) / (T[k + 1] - T[k]);
            const double w00 = (1 - u) * (1 - v), w10 = u * (1 - v), w01 = (1 - u) * v,
                         w11 = u * v;
            const double f00 = F[i * nt + k], f10 = F[(i + 1) * nt + k],
                         f01 = F[i * nt + k + 1], f11 = F[(i + 1) * nt + k + 1];
            out[p] = w00 * f00 + w10 * f10 + w01 * f01 + w11 * f11;
            if (scale)
                scale[p] = fabs(w00 * f00) + fabs(w10 * f10) + fabs(w01 * f01) + fabs(w11 * f11);
        }
        voff += nr * nt;
    }
}
