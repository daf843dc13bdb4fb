/*
 * oracle.c -- plain FP64 CPU oracle for filtered exact top-k vector search.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code with the GPU path.
 *
 * What it computes (Sanca & Ailamaki, "Efficient Data Access Paths for Mixed
 * Vector-Relational Search", Section 3):
 *
 *   selection with a query vector v and similarity predicate eps:
 *       sigma_{eps,v}(R) = { t in R : eps(t, v) }                 (eq. 1)
 *   brute force = cross product of v with the vector column     (eq. 2)
 *   with a relational predicate theta pushed down:
 *       sigma_{eps,v,theta}(R) = sigma_eps(v x sigma_theta(R))   (eq. 3)
 *
 * eps is instantiated as "the k rows of sigma_theta(R) with the smallest
 * distance to v", where ties in distance go to the lower row id.  The scan is
 * exact (Table 1: scans give exact results, indexes approximate ones), so the
 * result is the brute-force one: compute every qualifying distance, sort, cut.
 *
 * Readings where the paper is silent (each is also listed in the design
 * notes):
 *   - distance L2SQ = sum_j (q_j - x_j)^2 (squared L2; same ranking as L2);
 *     distance IP = -<q, x> (so "smaller is closer" for both metrics);
 *     cosine similarity is IP on row-normalised vectors (Section 3.1, the
 *     tensor formulation on normalised matrices);
 *   - FP64 arithmetic, j ascending, one fused multiply-add per element,
 *     accumulator starting at +0.0; a zero distance is stored as +0.0;
 *   - predicate = conjunction of half-open ranges lo <= A[col][i] < hi with
 *     int64 bounds, no terms = all rows;
 *   - fewer than k qualifying rows: the tail is padded with (id -1, +inf);
 *   - the returned float distance is the FP64 one rounded to nearest-even.
 *
 * Stored tables: float32 rows, bfloat16 rows, or FP8 (OCP e4m3fn) codes with
 * one float32 scale per row; the stored value of an FP8 element is
 * scale_i * decode(code).  For IP the FP64 sum runs over the codes and the
 * row scale multiplies the sum (dist = -(scale_i * acc)).
 *
 * Every function below is plain loops over the definition; the only library
 * primitives are fma, sqrt and qsort.
 */
#include <math.h>
#include <pthread.h>
#include <unistd.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OR_F32 = 0, OR_BF16 = 1, OR_FP8 = 2 };
enum { OR_L2SQ = 0, OR_IP = 1 };

int oracle_abi_version(void) { return 1; }

/* ------------------------------------------------------------------------ */
/* Value codecs                                                              */
/* ------------------------------------------------------------------------ */

/* bfloat16: the upper 16 bits of an IEEE binary32. */
double oracle_bf16_value(uint16_t h)
{
    uint32_t u = (uint32_t)h << 16;
    float f;
    memcpy(&f, &u, sizeof f);
    return (double)f;
}

/* OCP FP8 e4m3fn: 1 sign, 4 exponent (bias 7), 3 mantissa bits, no
 * infinities, S.1111.111 is NaN, subnormals are 2^-6 * m/8. */
double oracle_e4m3_value(uint8_t c)
{
    int s = c >> 7, e = (c >> 3) & 15, m = c & 7;
    double mag;
    if (e == 15 && m == 7)
        return NAN;
    if (e == 0)
        mag = ldexp((double)m, -9);
    else
        mag = ldexp(8.0 + (double)m, e - 10);
    return s ? -mag : mag;
}

/* float32 -> bfloat16, round to nearest, ties to even.  The two bfloat16
 * neighbours of |x| are compared in exact FP64 arithmetic.  Returns 1 if the
 * result is an infinity produced from a finite input (overflow), else 0. */
int oracle_bf16_from_f32(float x, uint16_t *out)
{
    uint32_t u;
    memcpy(&u, &x, sizeof u);
    uint32_t sign = u & 0x80000000u, mag = u & 0x7fffffffu;
    if (mag >= 0x7f800000u) { /* inf or NaN: carried through (NaN kept quiet) */
        *out = (uint16_t)(u >> 16) | (mag > 0x7f800000u ? 0x40 : 0);
        return 0;
    }
    uint32_t lo = mag & 0xffff0000u;  /* bfloat16 neighbour towards zero */
    if (lo == mag) {
        *out = (uint16_t)((sign | lo) >> 16);
        return 0;
    }
    uint32_t hi = lo + 0x00010000u;   /* neighbour away from zero */
    float flo, fhi, fx;
    memcpy(&flo, &lo, 4);
    memcpy(&fhi, &hi, 4);
    memcpy(&fx, &mag, 4);
    /* With an unbounded exponent the step above the largest finite value
     * lands on 2^128; rounding there means overflow to infinity. */
    double vhi = (hi == 0x7f800000u) ? ldexp(1.0, 128) : (double)fhi;
    double dlo = (double)fx - (double)flo, dhi = vhi - (double)fx;
    uint32_t pick;
    if (dlo < dhi)
        pick = lo;
    else if (dhi < dlo)
        pick = hi;
    else
        pick = (((lo >> 16) & 1) == 0) ? lo : hi;
    *out = (uint16_t)((sign | pick) >> 16);
    return pick == 0x7f800000u;
}

/* |value| of the non-negative finite e4m3 codes 0x00..0x7e, ascending. */
static double e4m3_pos(int c) { return oracle_e4m3_value((uint8_t)c); }

/* FP64 value -> e4m3fn code, round to nearest, ties to even code (the
 * mantissa's last bit), saturating at +-448; the sign bit is the sign of v
 * (so -0.0 and tiny negatives give 0x80). */
uint8_t oracle_e4m3_from_f64(double v)
{
    uint8_t sign = signbit(v) ? 0x80 : 0x00;
    double a = fabs(v);
    if (!(a < 448.0))
        return sign | 0x7e;
    /* largest code with value <= a (binary search over the ascending table) */
    int lo = 0, hi = 0x7e;
    while (lo < hi) {
        int mid = (lo + hi + 1) / 2;
        if (e4m3_pos(mid) <= a)
            lo = mid;
        else
            hi = mid - 1;
    }
    if (e4m3_pos(lo) == a)
        return sign | (uint8_t)lo;
    int up = lo + 1;
    double dlo = a - e4m3_pos(lo), dup = e4m3_pos(up) - a;
    int pick;
    if (dlo < dup)
        pick = lo;
    else if (dup < dlo)
        pick = up;
    else
        pick = (lo & 1) == 0 ? lo : up;
    return sign | (uint8_t)pick;
}

/* Bulk codecs (used by the tests on whole tables).  Rows are independent,
 * so large tables are split into contiguous row ranges over a few threads;
 * every row is computed exactly as in the serial loop. */
typedef struct {
    void (*fn)(void *ctx, int64_t i0, int64_t i1);
    void *ctx;
    int64_t n, per;
    int t;
} rows_job_t;

static void *rows_worker(void *arg)
{
    rows_job_t *J = (rows_job_t *)arg;
    int64_t i0 = (int64_t)J->t * J->per, i1 = i0 + J->per;
    if (i1 > J->n)
        i1 = J->n;
    if (i0 < i1)
        J->fn(J->ctx, i0, i1);
    return NULL;
}

static void for_rows(int64_t n, void (*fn)(void *, int64_t, int64_t), void *ctx)
{
    long nt = sysconf(_SC_NPROCESSORS_ONLN);
    if (nt < 1)
        nt = 1;
    if (nt > 32)
        nt = 32;
    if (n < 65536 || nt == 1) {
        fn(ctx, 0, n);
        return;
    }
    rows_job_t J[32];
    pthread_t th[32];
    int ok[32];
    int64_t per = (n + nt - 1) / nt;
    for (int t = 0; t < nt; t++) {
        J[t] = (rows_job_t){fn, ctx, n, per, t};
        ok[t] = pthread_create(&th[t], NULL, rows_worker, &J[t]) == 0;
        if (!ok[t])
            rows_worker(&J[t]);
    }
    for (int t = 0; t < nt; t++)
        if (ok[t])
            pthread_join(th[t], NULL);
}

typedef struct {
    const float *x;
    uint16_t *out;
    int64_t overflow[32];
    int64_t per;
} bf16_ctx_t;

static void bf16_rows(void *c, int64_t i0, int64_t i1)
{
    bf16_ctx_t *C = (bf16_ctx_t *)c;
    int64_t ov = 0;
    for (int64_t i = i0; i < i1; i++)
        ov += oracle_bf16_from_f32(C->x[i], &C->out[i]);
    C->overflow[i0 / C->per] = ov;
}

int64_t oracle_encode_bf16(const float *x, int64_t n, uint16_t *out)
{
    long nt = sysconf(_SC_NPROCESSORS_ONLN);
    if (nt < 1)
        nt = 1;
    if (nt > 32)
        nt = 32;
    bf16_ctx_t C = {x, out, {0}, n < 65536 || nt == 1 ? (n > 0 ? n : 1) : (n + nt - 1) / nt};
    for_rows(n, bf16_rows, &C);
    int64_t overflow = 0;
    for (int t = 0; t < 32; t++)
        overflow += C.overflow[t];
    return overflow;
}

/* Row-wise FP8 quantisation: scale_i = max_j |x_ij| / 448 (one float32
 * division), 1 for an all-zero row; code_ij = e4m3(x_ij / scale_i) with the
 * quotient taken in FP64. */
typedef struct {
    const float *x;
    int32_t d;
    uint8_t *codes;
    float *scale;
} fp8_ctx_t;

static void fp8_rows(void *c, int64_t i0, int64_t i1)
{
    fp8_ctx_t *C = (fp8_ctx_t *)c;
    const int32_t d = C->d;
    for (int64_t i = i0; i < i1; i++) {
        const float *row = C->x + i * (int64_t)d;
        float m = 0.0f;
        for (int32_t j = 0; j < d; j++) {
            float a = fabsf(row[j]);
            if (a > m)
                m = a;
        }
        volatile float s = (m == 0.0f) ? 1.0f : m / 448.0f;
        C->scale[i] = s;
        for (int32_t j = 0; j < d; j++)
            C->codes[i * (int64_t)d + j] = oracle_e4m3_from_f64((double)row[j] / (double)s);
    }
}

void oracle_encode_fp8_rows(const float *x, int64_t n, int32_t d, uint8_t *codes, float *scale)
{
    fp8_ctx_t C = {x, d, codes, scale};
    for_rows(n, fp8_rows, &C);
}

/* Row L2 normalisation for the cosine metric: ||x|| = sqrt(sum_j x_j^2) in
 * FP64 (j ascending, fma), then x_j / ||x|| in FP64 rounded to float32.  An
 * all-zero row is left as is. */
typedef struct {
    const float *x;
    int32_t d;
    float *out;
} norm_ctx_t;

static void norm_rows(void *c, int64_t i0, int64_t i1)
{
    norm_ctx_t *C = (norm_ctx_t *)c;
    const int32_t d = C->d;
    for (int64_t i = i0; i < i1; i++) {
        const float *row = C->x + i * (int64_t)d;
        double acc = 0.0;
        for (int32_t j = 0; j < d; j++)
            acc = fma((double)row[j], (double)row[j], acc);
        double nrm = sqrt(acc);
        for (int32_t j = 0; j < d; j++)
            C->out[i * (int64_t)d + j] = (nrm == 0.0) ? row[j] : (float)((double)row[j] / nrm);
    }
}

void oracle_normalize_rows(const float *x, int64_t n, int32_t d, float *out)
{
    norm_ctx_t C = {x, d, out};
    for_rows(n, norm_rows, &C);
}

/* ------------------------------------------------------------------------ */
/* Relational predicate (the selection sigma_theta(R) of eq. 3)             */
/* ------------------------------------------------------------------------ */

static int qualifies(const int32_t *attr, int64_t n, int64_t i, int32_t nterms,
                     const int32_t *cols, const int64_t *lo, const int64_t *hi)
{
    for (int32_t t = 0; t < nterms; t++) {
        int64_t a = (int64_t)attr[(int64_t)cols[t] * n + i];
        if (!(lo[t] <= a && a < hi[t]))
            return 0;
    }
    return 1;
}

/* Ascending ids of the qualifying rows; returns their count. */
int64_t oracle_select(const int32_t *attr, int64_t n, int32_t nterms, const int32_t *cols,
                      const int64_t *lo, const int64_t *hi, int32_t *ids_out)
{
    int64_t c = 0;
    for (int64_t i = 0; i < n; i++)
        if (qualifies(attr, n, i, nterms, cols, lo, hi))
            ids_out[c++] = (int32_t)i;
    return c;
}

/* ------------------------------------------------------------------------ */
/* Distance (the similarity part of eps)                                     */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t dtype, d;
    int64_t n;
    const float *f32;     /* [n][d] when dtype == OR_F32 */
    const uint16_t *bf16; /* [n][d] when dtype == OR_BF16 */
    const uint8_t *fp8;   /* [n][d] when dtype == OR_FP8 */
    const float *scale;   /* [n]    when dtype == OR_FP8 */
} table_t;

/* the element as the sum over codes sees it (unscaled for FP8) */
static double code_value(const table_t *T, int64_t i, int32_t j)
{
    int64_t o = i * (int64_t)T->d + j;
    switch (T->dtype) {
    case OR_BF16: return oracle_bf16_value(T->bf16[o]);
    case OR_FP8: return oracle_e4m3_value(T->fp8[o]);
    default: return (double)T->f32[o];
    }
}

static double row_scale(const table_t *T, int64_t i)
{
    return T->dtype == OR_FP8 ? (double)T->scale[i] : 1.0;
}

static double dist64(const table_t *T, const float *q, int64_t i, int32_t metric)
{
    double acc = 0.0;
    if (metric == OR_L2SQ) {
        double s = row_scale(T, i);
        for (int32_t j = 0; j < T->d; j++) {
            double t = (double)q[j] - s * code_value(T, i, j);
            acc = fma(t, t, acc);
        }
    } else {
        for (int32_t j = 0; j < T->d; j++)
            acc = fma((double)q[j], code_value(T, i, j), acc);
        acc = -(row_scale(T, i) * acc);
    }
    return acc == 0.0 ? 0.0 : acc;
}

/* Distances of one query to a list of rows (no predicate). */
void oracle_distances(int32_t dtype, int64_t n, int32_t d, const void *rows, const float *scale,
                      const float *q, const int64_t *ids, int64_t count, int32_t metric, double *out)
{
    table_t T = {dtype, d, n, (const float *)rows, (const uint16_t *)rows, (const uint8_t *)rows, scale};
    for (int64_t c = 0; c < count; c++)
        out[c] = dist64(&T, q, ids[c], metric);
}

/* ------------------------------------------------------------------------ */
/* Exact top-k (eq. 3 with eps = k smallest (distance, id))                  */
/* ------------------------------------------------------------------------ */

typedef struct {
    double dist;
    int64_t id;
} pair_t;

static int pair_cmp(const void *a, const void *b)
{
    const pair_t *x = (const pair_t *)a, *y = (const pair_t *)b;
    if (x->dist < y->dist) return -1;
    if (x->dist > y->dist) return 1;
    return (x->id > y->id) - (x->id < y->id);
}

typedef struct {
    const table_t *T;
    const int32_t *attr;
    const float *q;            /* [B][d] */
    int32_t B;
    int32_t nterms_max;        /* per-query term arrays are [B][nterms_max] */
    const int32_t *nterms;     /* [B] */
    const int32_t *cols;
    const int64_t *lo, *hi;
    const int32_t *ks;         /* [B] */
    int32_t out_stride;        /* columns of the output arrays */
    int32_t metric;
    int64_t *out_idx;
    float *out_dist;
    double *out_dist64;
    int64_t *out_nvalid;
    /* threshold selection (range_mode = 1): thr[b], at most out_stride ids
     * per query, counts[b] = number of qualifying rows below the threshold */
    int32_t range_mode;
    const double *thr;
    int64_t *out_count;
    int64_t next;              /* next query to take (guarded by mu) */
    pthread_mutex_t mu;
    int failed;
} job_t;

static int one_query(job_t *J, int32_t b)
{
    const table_t *T = J->T;
    const float *q = J->q + (int64_t)b * T->d;
    const int32_t nt = J->nterms[b];
    const int32_t *cols = J->cols + (int64_t)b * J->nterms_max;
    const int64_t *lo = J->lo + (int64_t)b * J->nterms_max;
    const int64_t *hi = J->hi + (int64_t)b * J->nterms_max;
    int64_t cnt = 0;
    for (int64_t i = 0; i < T->n; i++)
        cnt += qualifies(J->attr, T->n, i, nt, cols, lo, hi);
    pair_t *p = (pair_t *)malloc((size_t)(cnt > 0 ? cnt : 1) * sizeof(pair_t));
    if (!p)
        return -1;
    int64_t c = 0;
    for (int64_t i = 0; i < T->n; i++) {
        if (qualifies(J->attr, T->n, i, nt, cols, lo, hi)) {
            p[c].dist = dist64(T, q, i, J->metric);
            p[c].id = i;
            c++;
        }
    }
    qsort(p, (size_t)cnt, sizeof(pair_t), pair_cmp);
    int64_t k = J->ks[b];
    int64_t m = cnt < k ? cnt : k;
    int64_t *oi = J->out_idx + (int64_t)b * J->out_stride;
    float *od = J->out_dist + (int64_t)b * J->out_stride;
    double *od64 = J->out_dist64 ? J->out_dist64 + (int64_t)b * J->out_stride : NULL;
    for (int64_t r = 0; r < J->out_stride; r++) {
        if (r < m) {
            oi[r] = p[r].id;
            od[r] = (float)p[r].dist;
            if (od64) od64[r] = p[r].dist;
        } else {
            oi[r] = -1;
            od[r] = INFINITY;
            if (od64) od64[r] = INFINITY;
        }
    }
    if (J->out_nvalid)
        J->out_nvalid[b] = m;
    free(p);
    return 0;
}

/* Threshold selection for query b: the qualifying rows i, ascending, whose
 * FP64 distance is below thr[b]; the first out_stride of them are written,
 * the rest of the row is padded with (-1, +inf); out_count[b] counts all. */
static int one_query_range(job_t *J, int32_t b)
{
    const table_t *T = J->T;
    const float *q = J->q + (int64_t)b * T->d;
    const int32_t nt = J->nterms[b];
    const int32_t *cols = J->cols + (int64_t)b * J->nterms_max;
    const int64_t *lo = J->lo + (int64_t)b * J->nterms_max;
    const int64_t *hi = J->hi + (int64_t)b * J->nterms_max;
    int64_t *oi = J->out_idx + (int64_t)b * J->out_stride;
    float *od = J->out_dist + (int64_t)b * J->out_stride;
    double *od64 = J->out_dist64 ? J->out_dist64 + (int64_t)b * J->out_stride : NULL;
    int64_t c = 0;
    for (int64_t i = 0; i < T->n; i++) {
        if (!qualifies(J->attr, T->n, i, nt, cols, lo, hi))
            continue;
        double dv = dist64(T, q, i, J->metric);
        if (!(dv < J->thr[b]))
            continue;
        if (c < J->out_stride) {
            oi[c] = i;
            od[c] = (float)dv;
            if (od64) od64[c] = dv;
        }
        c++;
    }
    for (int64_t r = c; r < J->out_stride; r++) {
        oi[r] = -1;
        od[r] = INFINITY;
        if (od64) od64[r] = INFINITY;
    }
    J->out_count[b] = c;
    return 0;
}

static void *worker(void *arg)
{
    job_t *J = (job_t *)arg;
    for (;;) {
        pthread_mutex_lock(&J->mu);
        int64_t b = J->next++;
        pthread_mutex_unlock(&J->mu);
        if (b >= J->B)
            break;
        if ((J->range_mode ? one_query_range(J, (int32_t)b) : one_query(J, (int32_t)b)) != 0) {
            pthread_mutex_lock(&J->mu);
            J->failed = 1;
            pthread_mutex_unlock(&J->mu);
        }
    }
    return NULL;
}

/* Run J's queries on nthreads threads (the caller's thread included). */
static int run_job(job_t *J, int32_t nthreads)
{
    pthread_mutex_init(&J->mu, NULL);
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > J->B)
        nthreads = J->B > 0 ? J->B : 1;
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
    char *ok = (char *)calloc((size_t)nthreads, 1);
    for (int t = 1; t < nthreads; t++)
        ok[t] = pthread_create(&th[t], NULL, worker, J) == 0;
    worker(J); /* the calling thread takes part too */
    for (int t = 1; t < nthreads; t++)
        if (ok[t])
            pthread_join(th[t], NULL);
    free(ok);
    free(th);
    pthread_mutex_destroy(&J->mu);
    return J->failed ? -1 : 0;
}

/*
 * Exact filtered top-k for B queries, each with its own predicate and k.
 *   rows/scale : stored table (see table_t), n rows of d elements
 *   attr       : int32 attributes, column-major [n_attr][n]
 *   nterms[b], cols/lo/hi[b][nterms_max] : query b's conjunction
 *   ks[b]      : query b's k (<= out_stride)
 *   outputs    : [B][out_stride] ids (int64), float32 and FP64 distances,
 *                and nvalid[b] = min(k_b, |S_b|); out_dist64/out_nvalid may
 *                be NULL.
 * Returns 0, or -1 if memory ran out.
 */
int oracle_scan_topk(int32_t dtype, int64_t n, int32_t d, const void *rows, const float *scale,
                     const int32_t *attr, const float *q, int32_t B, int32_t nterms_max,
                     const int32_t *nterms, const int32_t *cols, const int64_t *lo, const int64_t *hi,
                     const int32_t *ks, int32_t out_stride, int32_t metric, int32_t nthreads,
                     int64_t *out_idx, float *out_dist, double *out_dist64, int64_t *out_nvalid)
{
    table_t T = {dtype, d, n, (const float *)rows, (const uint16_t *)rows, (const uint8_t *)rows, scale};
    job_t J;
    memset(&J, 0, sizeof J);
    J.T = &T;
    J.attr = attr;
    J.q = q;
    J.B = B;
    J.nterms_max = nterms_max;
    J.nterms = nterms;
    J.cols = cols;
    J.lo = lo;
    J.hi = hi;
    J.ks = ks;
    J.out_stride = out_stride;
    J.metric = metric;
    J.out_idx = out_idx;
    J.out_dist = out_dist;
    J.out_dist64 = out_dist64;
    J.out_nvalid = out_nvalid;
    return run_job(&J, nthreads);
}

/* ------------------------------------------------------------------------ */
/* Threshold selection (eq. 1 and eq. 3 with eps = "distance below a         */
/* threshold"; the evaluation's similarity predicate is a cosine-similarity  */
/* threshold, Section 5 "Dataset": on normalised rows and a normalised query */
/* cosine similarity > t is IP distance < -t)                                */
/* ------------------------------------------------------------------------ */

/*
 * For B queries, each with its own predicate and threshold thr[b]: the
 * qualifying rows whose FP64 distance is below thr[b], ascending by row id.
 *   outputs : [B][cap] ids (int64), float32 and FP64 distances (the first
 *             cap rows; the rest padded with -1 / +inf), counts[b] = number
 *             of rows selected (may exceed cap).
 * Returns 0.
 */
int oracle_scan_range(int32_t dtype, int64_t n, int32_t d, const void *rows, const float *scale,
                      const int32_t *attr, const float *q, int32_t B, int32_t nterms_max,
                      const int32_t *nterms, const int32_t *cols, const int64_t *lo, const int64_t *hi,
                      const double *thr, int32_t cap, int32_t metric, int32_t nthreads,
                      int64_t *out_idx, float *out_dist, double *out_dist64, int64_t *out_count)
{
    table_t T = {dtype, d, n, (const float *)rows, (const uint16_t *)rows, (const uint8_t *)rows, scale};
    job_t J;
    memset(&J, 0, sizeof J);
    J.T = &T;
    J.attr = attr;
    J.q = q;
    J.B = B;
    J.nterms_max = nterms_max;
    J.nterms = nterms;
    J.cols = cols;
    J.lo = lo;
    J.hi = hi;
    J.out_stride = cap;
    J.metric = metric;
    J.out_idx = out_idx;
    J.out_dist = out_dist;
    J.out_dist64 = out_dist64;
    J.range_mode = 1;
    J.thr = thr;
    J.out_count = out_count;
    return run_job(&J, nthreads);
}
