/*
 * CPU oracle for exact fixed-radius nearest-neighbour search.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The GPU library never
 * calls it, links it or shares code with it.
 *
 * It is the plain definition written out, by brute force over every pair:
 *
 *   N_r(i) = { j : ||x_i - x_j||_2 <= r }                      (Sec. 1, Eq. 1)
 *
 * optionally cut to the K nearest "in distance order" (Sec. 1, the sentence
 * after Eq. 1).  The paper states the relation over the reals and insists that
 * float32 membership be reproduced exactly (Sec. 4.2: reordered accumulation
 * changed float32 membership near the radius).  The float32 reading fixed here:
 *
 *   r2        = fl32(r * r)                    one rounded float32 multiply
 *   s(i, j)   = +0;  for d = 0 .. D-1:  t = fl32(q_d - x_d);  u = fl32(t * t);
 *               s = fl32(s + u)                three separately rounded ops
 *   j in row i  <=>  s(i, j) <= r2             inclusive boundary
 *   row order:  ascending (s, j), s compared as a float, j as an integer
 *   K > 0:      keep the first min(|row|, K) entries of that order
 *
 * Built with -ffp-contract=off and without fast-math, so there is no fused
 * multiply-add, no flush of subnormals and no reassociation.  Rows are
 * independent, so threads split the queries; each pair is evaluated in the
 * order above by one thread.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define ORACLE_OK 0
#define ORACLE_ERR_ARG (-1)
#define ORACLE_ERR_NONFINITE (-2)
#define ORACLE_ERR_OOM (-3)

typedef struct {
    int64_t M;
    int64_t nnz;
    int64_t *offsets;  /* M + 1 */
    int32_t *indices;  /* nnz */
    float *dist2;      /* nnz */
    int64_t *degree;   /* M: number of in-radius references before the cap */
} oracle_csr;

/* r2 := fl32(r * r).  Storing through a float forces the rounding. */
float oracle_r2(float r) {
    volatile float rr = r * r;
    return rr;
}

/* Squared distance in the canonical order, three rounded ops per axis. */
float oracle_dist2(const float *q, const float *x, int32_t D) {
    float s = 0.0f;
    for (int32_t d = 0; d < D; ++d) {
        float t = q[d] - x[d];
        float u = t * t;
        s = s + u;
    }
    return s;
}

typedef struct {
    float s;
    int32_t j;
} hit_t;

static int hit_cmp(const void *a, const void *b) {
    const hit_t *x = (const hit_t *)a, *y = (const hit_t *)b;
    if (x->s < y->s) return -1;
    if (x->s > y->s) return 1;
    return (x->j > y->j) - (x->j < y->j);
}

typedef struct {
    /* shared, read-only */
    const float *Q, *X;
    int64_t M, N;
    int32_t D, K;
    float r2;
    const int64_t *self_ids;
    int want_rows;
    /* shared work counter */
    int64_t *next;
    pthread_mutex_t *lock;
    /* shared outputs indexed by query */
    int64_t *degree;
    int64_t *rowlen;
    /* this thread's rows, in the order it processed them */
    hit_t *buf;
    int64_t buf_len, buf_cap;
    int64_t *done_q;    /* queries this thread processed */
    int64_t *done_at;   /* start of each processed row in buf */
    int64_t n_done, done_cap, done_at_cap;
    int status;
} worker_t;

#define GRAB 16

static int grow(void **p, int64_t *cap, int64_t need, size_t elt) {
    if (need <= *cap) return 0;
    int64_t nc = *cap ? *cap : 1024;
    while (nc < need) nc *= 2;
    void *np = realloc(*p, (size_t)nc * elt);
    if (!np) return -1;
    *p = np;
    *cap = nc;
    return 0;
}

static void *worker_main(void *arg) {
    worker_t *w = (worker_t *)arg;
    hit_t *row = NULL;
    int64_t row_cap = 0;
    for (;;) {
        pthread_mutex_lock(w->lock);
        int64_t q0 = *w->next;
        *w->next = q0 + GRAB;
        pthread_mutex_unlock(w->lock);
        if (q0 >= w->M) break;
        int64_t q1 = q0 + GRAB < w->M ? q0 + GRAB : w->M;
        for (int64_t i = q0; i < q1; ++i) {
            const float *q = w->Q + i * (int64_t)w->D;
            int64_t self = w->self_ids ? w->self_ids[i] : -1;
            int64_t n = 0;
            for (int64_t j = 0; j < w->N; ++j) {
                if (j == self) continue;
                float s = oracle_dist2(q, w->X + j * (int64_t)w->D, w->D);
                if (s <= w->r2) {
                    if (w->want_rows) {
                        if (grow((void **)&row, &row_cap, n + 1, sizeof(hit_t))) {
                            w->status = ORACLE_ERR_OOM;
                            free(row);
                            return NULL;
                        }
                        row[n].s = s;
                        row[n].j = (int32_t)j;
                    }
                    ++n;
                }
            }
            w->degree[i] = n;
            if (!w->want_rows) continue;
            qsort(row, (size_t)n, sizeof(hit_t), hit_cmp);
            int64_t keep = (w->K > 0 && n > w->K) ? w->K : n;
            w->rowlen[i] = keep;
            if (grow((void **)&w->buf, &w->buf_cap, w->buf_len + keep, sizeof(hit_t)) ||
                grow((void **)&w->done_q, &w->done_cap, w->n_done + 1, sizeof(int64_t)) ||
                grow((void **)&w->done_at, &w->done_at_cap, w->n_done + 1, sizeof(int64_t))) {
                w->status = ORACLE_ERR_OOM;
                free(row);
                return NULL;
            }
            memcpy(w->buf + w->buf_len, row, (size_t)keep * sizeof(hit_t));
            w->done_q[w->n_done] = i;
            w->done_at[w->n_done] = w->buf_len;
            w->n_done++;
            w->buf_len += keep;
        }
    }
    free(row);
    return NULL;
}

static int all_finite(const float *a, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(a[i])) return 0;
    return 1;
}

static int run(const float *Q, int64_t M, const float *X, int64_t N, int32_t D,
               float r, int32_t K, const int64_t *self_ids, int nthreads,
               int want_rows, int64_t *degree_out, oracle_csr *out) {
    if (M < 0 || N < 0 || D < 1 || (M > 0 && !Q) || (N > 0 && !X) || N > INT32_MAX)
        return ORACLE_ERR_ARG;
    if (!isfinite(r) || r < 0.0f) return ORACLE_ERR_ARG;
    if (!all_finite(Q, M * (int64_t)D) || !all_finite(X, N * (int64_t)D))
        return ORACLE_ERR_NONFINITE;
    if (nthreads <= 0) nthreads = (int)sysconf(_SC_NPROCESSORS_ONLN);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;

    int64_t *degree = degree_out ? degree_out : (int64_t *)calloc((size_t)(M ? M : 1), sizeof(int64_t));
    int64_t *rowlen = (int64_t *)calloc((size_t)(M ? M : 1), sizeof(int64_t));
    worker_t *ws = (worker_t *)calloc((size_t)nthreads, sizeof(worker_t));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!degree || !rowlen || !ws || !th) return ORACLE_ERR_OOM;

    int64_t next = 0;
    pthread_mutex_t lock;
    pthread_mutex_init(&lock, NULL);
    float r2 = oracle_r2(r);
    for (int t = 0; t < nthreads; ++t) {
        worker_t *w = &ws[t];
        w->Q = Q; w->X = X; w->M = M; w->N = N; w->D = D; w->K = K; w->r2 = r2;
        w->self_ids = self_ids; w->want_rows = want_rows;
        w->next = &next; w->lock = &lock;
        w->degree = degree; w->rowlen = rowlen;
        pthread_create(&th[t], NULL, worker_main, w);
    }
    int status = ORACLE_OK;
    for (int t = 0; t < nthreads; ++t) {
        pthread_join(th[t], NULL);
        if (ws[t].status) status = ws[t].status;
    }
    pthread_mutex_destroy(&lock);

    if (status == ORACLE_OK && want_rows) {
        memset(out, 0, sizeof(*out));
        out->M = M;
        out->offsets = (int64_t *)malloc((size_t)(M + 1) * sizeof(int64_t));
        out->degree = (int64_t *)malloc((size_t)(M ? M : 1) * sizeof(int64_t));
        if (!out->offsets || !out->degree) status = ORACLE_ERR_OOM;
        if (status == ORACLE_OK) {
            out->offsets[0] = 0;
            for (int64_t i = 0; i < M; ++i) out->offsets[i + 1] = out->offsets[i] + rowlen[i];
            out->nnz = out->offsets[M];
            memcpy(out->degree, degree, (size_t)M * sizeof(int64_t));
            out->indices = (int32_t *)malloc((size_t)(out->nnz ? out->nnz : 1) * sizeof(int32_t));
            out->dist2 = (float *)malloc((size_t)(out->nnz ? out->nnz : 1) * sizeof(float));
            if (!out->indices || !out->dist2) status = ORACLE_ERR_OOM;
        }
        if (status == ORACLE_OK) {
            for (int t = 0; t < nthreads; ++t) {
                worker_t *w = &ws[t];
                for (int64_t k = 0; k < w->n_done; ++k) {
                    int64_t i = w->done_q[k];
                    const hit_t *src = w->buf + w->done_at[k];
                    int64_t o = out->offsets[i];
                    for (int64_t e = 0; e < rowlen[i]; ++e) {
                        out->indices[o + e] = src[e].j;
                        out->dist2[o + e] = src[e].s;
                    }
                }
            }
        }
    }
    for (int t = 0; t < nthreads; ++t) {
        free(ws[t].buf);
        free(ws[t].done_q);
        free(ws[t].done_at);
    }
    free(ws);
    free(th);
    free(rowlen);
    if (!degree_out) free(degree);
    return status;
}

/* Full CSR rows for every query.  self_ids (may be NULL) gives, per query, a
 * reference index to leave out (self-exclusion in a self-join). */
int oracle_frnn(const float *Q, int64_t M, const float *X, int64_t N, int32_t D,
                float r, int32_t K, const int64_t *self_ids, int nthreads,
                oracle_csr *out) {
    if (!out) return ORACLE_ERR_ARG;
    memset(out, 0, sizeof(*out));
    return run(Q, M, X, N, D, r, K, self_ids, nthreads, 1, NULL, out);
}

/* In-radius counts only (before any cap); no rows are kept. */
int oracle_degrees(const float *Q, int64_t M, const float *X, int64_t N, int32_t D,
                   float r, const int64_t *self_ids, int nthreads, int64_t *degree) {
    if (!degree && M > 0) return ORACLE_ERR_ARG;
    return run(Q, M, X, N, D, r, 0, self_ids, nthreads, 0, degree, NULL);
}

void oracle_csr_free(oracle_csr *c) {
    if (!c) return;
    free(c->offsets);
    free(c->indices);
    free(c->dist2);
    free(c->degree);
    memset(c, 0, sizeof(*c));
}

int oracle_threads_default(void) { return (int)sysconf(_SC_NPROCESSORS_ONLN); }
