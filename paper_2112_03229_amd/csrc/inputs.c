/*
 * Seeded synthetic input generators (host only).
 *
 * These stand in for the SESAME density and temperature axes and for the
 * target streams searched in them (Sec. 4, 5.1, 5.2 and 5.5 of the paper:
 * small sorted, roughly logarithmically distributed float64 tables, and many
 * more targets than table entries).  Nothing in this file performs any part
 * of the search method: it only draws numbers.  Both the device path and the
 * CPU oracle consume the exact bytes written here.
 *
 * Random numbers come from a counter-based generator: word k of stream s
 * under seed S is the SplitMix64 output function (Steele, Lea and Flood,
 * "Fast splittable pseudorandom number generators", OOPSLA 2014) applied to
 * a counter, so any element can be produced independently of the others and
 * the result never depends on the number of host threads.
 *
 * Build: gcc -O2 -shared -fPIC -pthread (no -ffast-math: the log-uniform
 * transform must be the same IEEE arithmetic on every run).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define GOLDEN 0x9e3779b97f4a7c15ULL

static inline uint64_t sm64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* Key of one stream: decorrelates (seed, stream) pairs. */
static inline uint64_t stream_key(uint64_t seed, uint64_t stream) {
    return sm64_mix(seed * GOLDEN + sm64_mix(stream + GOLDEN));
}

/* 64 random bits for counter k of a stream. */
static inline uint64_t word_at(uint64_t key, uint64_t k) {
    return sm64_mix(key + (k + 1) * GOLDEN);
}

/* Uniform double in [0, 1) with 53 random bits. */
static inline double u01_at(uint64_t key, uint64_t k) {
    return (double)(word_at(key, k) >> 11) * 0x1.0p-53;
}

uint64_t ssin_word(uint64_t seed, uint64_t stream, uint64_t k) {
    return word_at(stream_key(seed, stream), k);
}

double ssin_u01(uint64_t seed, uint64_t stream, uint64_t k) {
    return u01_at(stream_key(seed, stream), k);
}

/* ---- a minimal static-chunk parallel loop over [0, count) ---------------- */

typedef void (*range_fn)(void *ctx, int64_t begin, int64_t end);

typedef struct {
    range_fn fn;
    void *ctx;
    int64_t begin, end;
} range_job;

static void *range_thread(void *p) {
    range_job *j = (range_job *)p;
    j->fn(j->ctx, j->begin, j->end);
    return NULL;
}

static int resolve_threads(int threads) {
    if (threads > 0) return threads > 256 ? 256 : threads;
    long c = sysconf(_SC_NPROCESSORS_ONLN);
    if (c < 1) c = 1;
    const char *env = getenv("OMP_NUM_THREADS");
    if (env) {
        long e = strtol(env, NULL, 10);
        if (e > 0 && e < c) c = e;
    }
    return c > 256 ? 256 : (int)c;
}

/* Chunks are aligned to `grain` elements so that work which is only
 * reproducible per fixed block (the smooth walk) can use the same loop. */
static void parallel_range(int threads, int64_t count, int64_t grain, range_fn fn, void *ctx) {
    threads = resolve_threads(threads);
    if (count <= 0) return;
    int64_t blocks = (count + grain - 1) / grain;
    if (threads > blocks) threads = (int)blocks;
    if (threads <= 1) {
        fn(ctx, 0, count);
        return;
    }
    pthread_t tid[256];
    range_job job[256];
    int started = 0;
    for (int t = 0; t < threads; ++t) {
        int64_t b0 = blocks * t / threads, b1 = blocks * (t + 1) / threads;
        job[t].fn = fn;
        job[t].ctx = ctx;
        job[t].begin = b0 * grain;
        job[t].end = b1 * grain < count ? b1 * grain : count;
        if (pthread_create(&tid[t], NULL, range_thread, &job[t]) != 0) {
            /* fall back to running this chunk inline */
            fn(ctx, job[t].begin, job[t].end);
            job[t].fn = NULL;
        } else {
            ++started;
        }
    }
    for (int t = 0; t < threads; ++t)
        if (job[t].fn) pthread_join(tid[t], NULL);
    (void)started;
}

/* ---- uniform and log-uniform streams -------------------------------------- */

typedef struct {
    uint64_t key, k0;
    double l0, dl; /* log10 bounds */
    double *out;
} logu_ctx;

static void logu_body(void *p, int64_t b, int64_t e) {
    logu_ctx *c = (logu_ctx *)p;
    for (int64_t i = b; i < e; ++i)
        c->out[i] = pow(10.0, c->l0 + u01_at(c->key, c->k0 + (uint64_t)i) * c->dl);
}

/* out[i] = 10^(log10 lo + u_i (log10 hi - log10 lo)), u_i = u01(k0 + i). */
void ssin_log_uniform(uint64_t seed, uint64_t stream, uint64_t k0, double lo, double hi,
                      int64_t count, double *out, int threads) {
    logu_ctx c = {stream_key(seed, stream), k0, log10(lo), log10(hi) - log10(lo), out};
    parallel_range(threads, count, 1 << 16, logu_body, &c);
}

typedef struct {
    uint64_t key, k0;
    double *out;
} u01_ctx;

static void u01_body(void *p, int64_t b, int64_t e) {
    u01_ctx *c = (u01_ctx *)p;
    for (int64_t i = b; i < e; ++i) c->out[i] = u01_at(c->key, c->k0 + (uint64_t)i);
}

void ssin_uniform(uint64_t seed, uint64_t stream, uint64_t k0, int64_t count, double *out,
                  int threads) {
    u01_ctx c = {stream_key(seed, stream), k0, out};
    parallel_range(threads, count, 1 << 16, u01_body, &c);
}

/* ---- tables ---------------------------------------------------------------- */

static int cmp_double(const void *a, const void *b) {
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* n i.i.d. log-uniform draws on [lo, hi], sorted ascending; with pin_ends the
 * first and last entries are set to lo and hi exactly after sorting. */
void ssin_sorted_log_table(uint64_t seed, uint64_t stream, int64_t n, double lo, double hi,
                           int pin_ends, double *out) {
    if (n <= 0) return;
    ssin_log_uniform(seed, stream, 0, lo, hi, n, out, 1);
    qsort(out, (size_t)n, sizeof(double), cmp_double);
    if (pin_ends) {
        out[0] = lo;
        if (n > 1) out[n - 1] = hi;
    }
}

/* Log-spaced table with multiplicative jitter, then sorted:
 * a_i = 10^(e0 + (e1 - e0) i / (n - 1)) * (1 + jitter (2 u_i - 1)). */
void ssin_jittered_log_table(uint64_t seed, uint64_t stream, int64_t n, double e0, double e1,
                             double jitter, double *out) {
    if (n <= 0) return;
    uint64_t key = stream_key(seed, stream);
    for (int64_t i = 0; i < n; ++i) {
        double t = n > 1 ? (double)i / (double)(n - 1) : 0.0;
        double u = u01_at(key, (uint64_t)i);
        out[i] = pow(10.0, e0 + (e1 - e0) * t) * (1.0 + jitter * (2.0 * u - 1.0));
    }
    qsort(out, (size_t)n, sizeof(double), cmp_double);
}

/* ---- smooth (sorted random-walk) targets ----------------------------------- */

/* log10 x_k = L0 + (L1 - L0) S_k / S_m with S_k = sum_{j<=k} e_j and
 * e_j = -log(1 - u_j) ~ Exp(1).  The prefix sum is taken in fixed blocks of
 * WALK_BLOCK elements (block-local sums, then block offsets in order), so the
 * bytes do not depend on the thread count. */
#define WALK_BLOCK 65536

typedef struct {
    uint64_t key;
    double *out;
    double *block_sum;
    double l0, dl, total;
    int64_t m;
} walk_ctx;

static void walk_pass1(void *p, int64_t b, int64_t e) {
    walk_ctx *c = (walk_ctx *)p;
    for (int64_t blk = b / WALK_BLOCK; blk * WALK_BLOCK < e; ++blk) {
        int64_t i0 = blk * WALK_BLOCK, i1 = i0 + WALK_BLOCK < c->m ? i0 + WALK_BLOCK : c->m;
        double s = 0.0;
        for (int64_t i = i0; i < i1; ++i) {
            s += -log1p(-u01_at(c->key, (uint64_t)i));
            c->out[i] = s; /* block-local prefix */
        }
        c->block_sum[blk] = s;
    }
}

static void walk_pass2(void *p, int64_t b, int64_t e) {
    walk_ctx *c = (walk_ctx *)p;
    for (int64_t blk = b / WALK_BLOCK; blk * WALK_BLOCK < e; ++blk) {
        int64_t i0 = blk * WALK_BLOCK, i1 = i0 + WALK_BLOCK < c->m ? i0 + WALK_BLOCK : c->m;
        double off = c->block_sum[blk]; /* exclusive offset after the scan */
        for (int64_t i = i0; i < i1; ++i)
            c->out[i] = pow(10.0, c->l0 + c->dl * ((off + c->out[i]) / c->total));
    }
}

int ssin_smooth_walk(uint64_t seed, uint64_t stream, double lo, double hi, int64_t m, double *out,
                     int threads) {
    if (m <= 0) return 0;
    int64_t nblk = (m + WALK_BLOCK - 1) / WALK_BLOCK;
    double *bs = (double *)malloc((size_t)nblk * sizeof(double));
    if (!bs) return -1;
    walk_ctx c = {stream_key(seed, stream), out, bs, log10(lo), log10(hi) - log10(lo), 0.0, m};
    parallel_range(threads, m, WALK_BLOCK, walk_pass1, &c);
    double run = 0.0;
    for (int64_t b = 0; b < nblk; ++b) {
        double s = bs[b];
        bs[b] = run;
        run += s;
    }
    c.total = run;
    parallel_range(threads, m, WALK_BLOCK, walk_pass2, &c);
    free(bs);
    return 0;
}

/* ---- segmented log-uniform targets for batched workloads ------------------- */

typedef struct {
    uint64_t seed, stream;
    const int64_t *off;
    const double *lo, *hi;
    int32_t nseg;
    double *out;
} seg_ctx;

static void seg_body(void *p, int64_t b, int64_t e) {
    seg_ctx *c = (seg_ctx *)p;
    /* locate the first segment holding element b */
    int32_t lo = 0, hi = c->nseg;
    while (hi - lo > 1) {
        int32_t mid = (lo + hi) / 2;
        if (c->off[mid] <= b) lo = mid; else hi = mid;
    }
    for (int32_t s = lo; s < c->nseg && c->off[s] < e; ++s) {
        int64_t s0 = c->off[s], s1 = c->off[s + 1];
        int64_t i0 = b > s0 ? b : s0, i1 = e < s1 ? e : s1;
        if (i1 <= i0) continue;
        uint64_t key = stream_key(c->seed, c->stream * 1000003ULL + (uint64_t)s);
        double l0 = log10(c->lo[s]), dl = log10(c->hi[s]) - l0;
        for (int64_t i = i0; i < i1; ++i)
            c->out[i] = pow(10.0, l0 + u01_at(key, (uint64_t)(i - s0)) * dl);
    }
}

/* Segment s (elements off[s] .. off[s+1]-1) is log-uniform on [lo[s], hi[s]],
 * drawn from its own stream so segments are independent of one another. */
void ssin_log_uniform_segments(uint64_t seed, uint64_t stream, const int64_t *off,
                               const double *lo, const double *hi, int32_t nseg, double *out,
                               int threads) {
    if (nseg <= 0 || off[nseg] <= 0) return;
    seg_ctx c = {seed, stream, off, lo, hi, nseg, out};
    parallel_range(threads, off[nseg], 1 << 16, seg_body, &c);
}
