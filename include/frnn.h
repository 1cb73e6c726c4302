/*
 * frnn.h — C ABI of libfrnn, exact fixed-radius nearest-neighbour search on
 * AMD Instinct MI355X (gfx950).
 *
 * The operation (Sec. 1, Eq. 1): for query x_i and reference points x_j,
 *
 *     N_r(i) = { j : ||x_i - x_j||_2 <= r }
 *
 * optionally keeping at most K neighbours in distance order (Sec. 1, the
 * sentence after Eq. 1).  Membership is decided in float32 exactly as follows
 * (the paper requires float32 membership to be reproduced exactly, Sec. 4.2):
 *
 *     r2      = fl32(r * r)                          one rounded multiply
 *     s(i,j)  = +0; for d = 0..D-1: t = fl32(q_d - x_d); u = fl32(t*t);
 *               s = fl32(s + u)                      no fused multiply-add
 *     j is a neighbour of i  <=>  s(i,j) <= r2      inclusive boundary
 *
 * Each row is ordered by (s, j) ascending (s as a float, j as an integer) and,
 * when K > 0, cut to its first min(|row|, K) entries.  Subnormals are kept.
 * The result is unique; the GPU output is bit-identical to a brute force.
 *
 * Conventions for every call:
 *  - Point arrays are row-major [n][D] float32.  Pointers marked "device" are
 *    HIP device pointers owned by the caller; the library only reads them,
 *    and only during the call's stream work.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *    device work of a call is ordered on that stream.  Calls that must learn
 *    a size (the number of output pairs) synchronise that stream once.
 *  - Every call returns a status and never aborts; no C++ exception crosses
 *    this boundary.  On error, outputs are zeroed and frnn_last_error()
 *    (thread-local) holds a message.
 *  - Output CSR buffers are device memory owned by the library until
 *    frnn_csr_release().  offsets are int64 [M+1], indices int32 [nnz]
 *    (reference ids local to their event, 0-based), dist2 float32 [nnz].
 *  - Sizes: 1 <= D <= 32; N, M < 2^31; r finite and >= 0.
 */
#ifndef FRNN_H
#define FRNN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FRNN_OK = 0,
    FRNN_ERR_INVALID_ARG = 1, /* bad size, pointer, radius or flag */
    FRNN_ERR_NONFINITE = 2,   /* a coordinate is NaN or infinite */
    FRNN_ERR_OOM = 3,         /* device allocation failed */
    FRNN_ERR_BUDGET = 4,      /* request larger than the server's HBM budget */
    FRNN_ERR_RADIUS = 5,      /* query radius larger than the index radius */
    FRNN_ERR_HIP = 6,         /* a HIP runtime call failed */
    FRNN_ERR_INTERNAL = 7,    /* an internal consistency check failed */
    FRNN_ERR_NOT_READY = 8    /* server ticket still in flight (poll only) */
} frnn_status;

/* Query flags. */
enum {
    FRNN_WANT_DIST2 = 1,   /* also return dist2 (the s values) */
    FRNN_SELF_QUERY = 2,   /* queries are the indexed points (queries = NULL) */
    FRNN_EXCLUDE_SELF = 4  /* with FRNN_SELF_QUERY: leave j == i out of row i */
};

typedef struct frnn_index_s *frnn_index;   /* opaque, immutable after build */
typedef struct frnn_server_s *frnn_server; /* opaque */

/* CSR neighbour lists.  Device pointers; library-owned until released. */
typedef struct {
    int64_t M;        /* number of rows (queries) */
    int64_t nnz;      /* number of (query, reference) pairs */
    int64_t *offsets; /* [M+1], offsets[0] = 0, row i is [offsets[i], offsets[i+1]) */
    int32_t *indices; /* [nnz] reference ids, each row ordered by (dist2, id) */
    float *dist2;     /* [nnz] s(i, j), or NULL without FRNN_WANT_DIST2 */
    void *owner_;     /* library-private */
} frnn_csr;

/* Kernel and grid parameters.  Every setting gives the same output; they
 * only change speed.  Fill with frnn_opts_default() and override fields. */
typedef struct {
    int32_t grid_axes_max;    /* most coordinates the cell grid may use (0..6) */
    float cells_per_point;    /* cap on grid cells per indexed point */
    int32_t cell_multiple;    /* m: cell width about r/m, reach +-m cells (1..3) */
    int32_t cells_per_item;   /* grid cells along the first grid axis per work item (1..8; default 2) */
    int32_t queries_per_item; /* queries evaluated per work item (1..64) */
    int32_t persistent;       /* count and fill passes as persistent kernels whose resident waves
                                 drain a device work queue of windows (runs of cell blocks of one
                                 event), costliest events first: 0 never, 1 always, 2 (default)
                                 when the windows are at most twice the resident waves */
    int32_t blocks_per_cu;    /* cap on resident blocks per CU of a persistent pass (1..16) */
    int32_t row_cap_lds;      /* rows longer than this sort in global memory (1..512) */
    int32_t stash_cap;        /* hits per query kept by the count pass (0, 8, 16, 32, 64, 128, 256;
                                 default 64; 8 bytes per query each);
                                 the fill pass only re-evaluates rows longer than this */
    int32_t graphs;           /* batched calls: 1 replays each launch sequence as a HIP graph
                                 (recorded once per context), 0 (default) launches the kernels
                                 one by one, which reached the first kernel sooner here */
    int32_t adapt;            /* batched calls with stash_cap, cells_per_item and queries_per_item at
                                 their defaults: 1 (default) lets a capacity class whose run had
                                 long rows (keys of rows longer than the stash at least an eighth
                                 of the stash slots) use, from its next batch on, a 256-key stash
                                 (128 or 64 when the stash would exceed 4 GiB), one cell per work
                                 item and windows of 16 queries; 0 keeps the options as given */
} frnn_opts;

void frnn_opts_default(frnn_opts *opts);

/* Build an index (cell grid, sorted copy of the points) over N points of
 * dimension D for queries of radius at most r.  points: device [N][D].
 * Grid cell keys are computed in float64 with cell width above r, so that no
 * pair whose float32 s is <= fl32(r*r) can lie in non-adjacent cells (the
 * "roundoff-safe grid" of Sec. 4.2).  opts may be NULL.  Synchronises the
 * stream once (to report non-finite input).
 * Errors: INVALID_ARG, NONFINITE, OOM, HIP. */
frnn_status frnn_build(const float *points, int64_t N, int32_t D, float r,
                       const frnn_opts *opts, void *stream, frnn_index *out);

/* Query an index.  queries: device [M][D], or NULL with FRNN_SELF_QUERY (then
 * M must equal N).  r <= the build radius (else FRNN_ERR_RADIUS).  K <= 0:
 * every neighbour; K > 0: the first min(deg, K) of each row.  Counting pass,
 * exact-size allocation, then fill (the count-first allocation of Sec. 4.2).
 * Synchronises the stream once (to learn nnz).
 * Errors: INVALID_ARG, NONFINITE, RADIUS, OOM, HIP. */
frnn_status frnn_query(frnn_index idx, const float *queries, int64_t M, float r,
                       int32_t K, uint32_t flags, void *stream, frnn_csr *out);

void frnn_index_destroy(frnn_index idx);

/* Grid chosen for an index (for reports and tests). */
typedef struct {
    int64_t N;
    int32_t D;
    int32_t grid_axes;        /* G */
    int32_t axis[8];          /* coordinate used by each grid axis */
    int32_t cells_per_axis[8];
    int64_t cells;            /* product of cells_per_axis */
    double cell_width;
    int32_t cell_multiple;
} frnn_index_info;

frnn_status frnn_index_get_info(frnn_index idx, frnn_index_info *info);

/* One event of a batch: its own reference points and, unless the batch is a
 * self-query, its own queries.  Device pointers. */
typedef struct {
    const float *points;
    int64_t N;
    const float *queries; /* NULL with FRNN_SELF_QUERY */
    int64_t M;            /* ignored with FRNN_SELF_QUERY */
} frnn_event;

/* Many independent events, one pipeline: the events are binned, counted and
 * filled by single launches over all events (work items are windows of
 * sorted queries, i.e. runs of cell blocks of one event; with
 * opts->persistent the resident waves drain them from a per-XCD queue,
 * costliest events first), the fixed launch sequence of a capacity class is
 * launched kernel by kernel or, with opts->graphs, recorded once as HIP
 * graphs and replayed when the same capacity recurs (with opts->adapt, a
 * class whose rows outgrew the stash runs its later batches with the
 * dense-row setting), and outs[e] is bit-identical to querying event e
 * alone.
 * All events share D, r, K and flags.  The host waits once, for the counts
 * (published by the device into host-mapped memory); the fill may still be
 * running on the stream when the call returns, so the outputs are ready in
 * stream order (frnn_csr_copy to the host synchronises the stream).
 * The outs[] share one allocation; release each of them.
 * Errors: INVALID_ARG, NONFINITE, OOM, HIP. */
frnn_status frnn_query_batch(const frnn_event *events, int32_t E, int32_t D,
                             float r, int32_t K, uint32_t flags,
                             const frnn_opts *opts, void *stream, frnn_csr *outs);

/* Copy a CSR into caller buffers (device, or host when to_host != 0); any of
 * the three destinations may be NULL to skip it.  Synchronous when to_host;
 * a host copy also reports FRNN_ERR_INTERNAL when the output came from a run
 * whose fill pass recounted a row longer than the stash differently from
 * the count pass (an internal consistency check of the device code). */
frnn_status frnn_csr_copy(const frnn_csr *csr, int64_t *offsets, int32_t *indices,
                          float *dist2, int32_t to_host, void *stream);

/* Return a CSR's buffers to the library's pool; the struct is zeroed. */
void frnn_csr_release(frnn_csr *csr);

/* ------------------------------------------------------- host-array calls
 * Synchronous search on host arrays (the paper's public host interface,
 * Secs. 4.1 and 4.2): the points (and queries) are copied to the device through pinned
 * staging buffers, the host copy of one chunk overlapping the DMA of the
 * previous one; the batched device path runs on a library stream; the CSR
 * comes back compact, in pinned host memory owned by the library until
 * frnn_host_csr_release.  points: host [N][D] float32; queries: host [M][D],
 * or NULL with FRNN_SELF_QUERY (then M must equal N).  Errors as for
 * frnn_query_batch (the output is zeroed). */
typedef struct {
    int64_t M;        /* rows */
    int64_t nnz;      /* pairs */
    int64_t *offsets; /* host [M+1] */
    int32_t *indices; /* host [nnz] */
    float *dist2;     /* host [nnz], or NULL without FRNN_WANT_DIST2 */
    void *owner_;     /* library-private */
} frnn_host_csr;

frnn_status frnn_query_host(const float *points, int64_t N, const float *queries, int64_t M, int32_t D,
                            float r, int32_t K, uint32_t flags, const frnn_opts *opts,
                            frnn_host_csr *out);

/* Free a host CSR's pinned buffers; the struct is zeroed. */
void frnn_host_csr_release(frnn_host_csr *csr);

/* ------------------------------------------------------------ edge export
 * Undirected edge lists for graph construction (Sec. 1: the neighbour graph
 * of a particle-tracking pipeline, built from the fixed-radius relation of
 * Eq. 1).  The CSR must come from a self-query (row i is point i, every index
 * < M); self pairs (j == i) are never exported.
 *   FRNN_EDGES_UPPER       (i, j) for every j in row i with i < j.  For an
 *                          uncapped self-join the relation is symmetric, so
 *                          this lists every undirected edge once.
 *   FRNN_EDGES_SYMMETRIZED every pair present in either direction, once, as
 *                          (min, max): (i, j) with i < j from row i, and (j, i)
 *                          from row i when j < i and i is not in row j (a K
 *                          cap can keep one direction only).
 * Edges come in row order, and within a row in the CSR's order.  Device
 * pointers, library-owned until frnn_edges_release.  Errors: NULL arguments
 * or an unknown mode give FRNN_ERR_INVALID_ARG, and so does an index outside
 * 0..M-1 found on the device (the output is then zeroed). */
enum { FRNN_EDGES_UPPER = 0, FRNN_EDGES_SYMMETRIZED = 1 };

typedef struct {
    int64_t n;        /* number of edges */
    int32_t *src;     /* [n] smaller endpoint */
    int32_t *dst;     /* [n] larger endpoint */
    void *owner_;     /* library-private */
} frnn_edges;

frnn_status frnn_csr_edges(const frnn_csr *csr, int32_t mode, void *stream, frnn_edges *out);

/* Copy an edge list into caller buffers (device, or host when to_host != 0);
 * either destination may be NULL to skip it.  Synchronous when to_host. */
frnn_status frnn_edges_copy(const frnn_edges *edges, int32_t *src, int32_t *dst, int32_t to_host,
                            void *stream);

/* Return an edge list's buffers to the library's pool; the struct is zeroed. */
void frnn_edges_release(frnn_edges *edges);

/* ------------------------------------------------- no device allocation
 * For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid allocation): the single-event self-query of
 * frnn_query_batch (FRNN_SELF_QUERY required) with every work buffer taken
 * from one device array of FRNN_NOALLOC_SCRATCH_BYTES that the library holds
 * on each GPU it runs on until the process ends, and the output written into
 * caller buffers.  The call makes no device (or pinned host) allocation.
 *   points   device [N][D] float32, read during the call's stream work
 *   offsets  device int64 [N+1] (caller-owned)
 *   indices  device int32 [cap_pairs], dist2 device float32 [cap_pairs] (or
 *            NULL without FRNN_WANT_DIST2); the CSR is that of
 *            frnn_query_batch, bit for bit
 *   *nnz     host: the number of pairs (also on FRNN_ERR_BUDGET)
 * Synchronises the stream once (after counting); the outputs are complete
 * when the stream's work is.  Errors: INVALID_ARG (also when the event's
 * work buffers exceed the array: about 4*ceil(D/4)*4 + 8*stash_cap + 70 bytes
 * per point), NONFINITE, BUDGET (cap_pairs below the pair count, or the
 * rows longer than the stash exceed the rest of the array), HIP.  Calls on
 * one GPU share its array: calls that overlap in time race and must be
 * ordered by the caller. */
#define FRNN_NOALLOC_SCRATCH_BYTES (256LL << 20)

frnn_status frnn_query_noalloc(const float *points, int64_t N, int32_t D, float r, int32_t K,
                               uint32_t flags, const frnn_opts *opts, int64_t *offsets, int32_t *indices,
                               float *dist2, int64_t cap_pairs, int64_t *nnz, void *stream);

/* ---------------------------------------------------------------- serving
 * A request loop on its own host thread and streams.  Submitted events are
 * admitted against an HBM budget, batched with whatever else is queued into
 * the batched pipeline, and their results stay in device memory.  Batches
 * overlap on the device: a new batch is binned and counted while earlier
 * ones are still being filled.  Each result is bit-identical to the same
 * event queried alone. */
typedef struct {
    int32_t D;
    float r;
    int32_t K;
    uint32_t flags;            /* FRNN_SELF_QUERY is implied */
    int64_t hbm_budget_bytes;  /* device bytes the server may hold at once (frnn_server_memory) */
    int32_t max_batch_events;  /* cap on events per batch (1..1024) */
    int32_t max_inflight;      /* batches on the device at once (1..8) */
    frnn_opts opts;
} frnn_server_opts;

typedef struct {
    double submit_s;    /* host clock, seconds: submission */
    double admit_s;     /* admitted against the budget */
    double start_s;     /* its batch was launched */
    double done_s;      /* result complete on the device and observed */
    int32_t batch_id;
    int32_t batch_events;
} frnn_timing;

void frnn_server_opts_default(frnn_server_opts *o);
frnn_status frnn_server_create(const frnn_server_opts *o, frnn_server *out);
/* points: host [N][D] float32, copied before the call returns. */
frnn_status frnn_server_submit(frnn_server s, const float *points, int64_t N,
                               uint64_t *ticket);
/* Blocks until the ticket completes (timeout_s < 0: forever; 0: poll and
 * return FRNN_ERR_NOT_READY).  Hands the result to the caller (release it). */
frnn_status frnn_server_wait(frnn_server s, uint64_t ticket, double timeout_s,
                             frnn_csr *out, frnn_timing *timing);
/* Device bytes the server holds for its work, now and at the peak, as the
 * pool hands them out (size classes): input copies of admitted events, each
 * worker's batch context, and outputs not yet released.  Admission keeps
 * this within hbm_budget_bytes, except that the oldest running batch may
 * always reserve its output (so the excess is at most one output per batch
 * in flight); the pool's free blocks are not counted. */
frnn_status frnn_server_memory(frnn_server s, int64_t *held_bytes, int64_t *peak_bytes);
void frnn_server_destroy(frnn_server s);

/* ---------------------------------------------------------------- tuning
 * Times candidate frnn_opts on the given input (a batched self-query with K)
 * by coordinate descent (a second pass when the first changed anything)
 * over the grid axes, cells per point, cells and queries per work item,
 * stash size, persistent launch, blocks per CU and graph replay, and
 * returns the fastest whose output is bit-identical to the
 * default's.  The result is cached per (device, D, K, density class) in the
 * JSON file named by FRNN_TUNE_CACHE, if set; the density class is the pair
 * of half-octaves of the mean candidates and mean neighbours per query of
 * the default run, so inputs of one class share a setting whatever their
 * size.  Errors as frnn_query_batch. */
typedef struct {
    int32_t candidates_tried;
    int32_t candidates_rejected; /* output differed from the default's */
    double best_ms;
    double default_ms;
    int32_t from_cache;          /* 1: the class was found in the cache (nothing timed beyond the default) */
    char density_class[96];      /* the cache key */
} frnn_tune_report;

frnn_status frnn_tune(const float *points, int64_t N, int32_t D, float r, int32_t K,
                      uint32_t flags, void *stream, frnn_opts *best,
                      frnn_tune_report *report);

/* ------------------------------------------------------- instrumentation
 * When enabled, every launch is bracketed by HIP events on its own stream and
 * per-kernel totals accumulate until read. */
typedef struct {
    char name[48];
    int64_t launches;
    double total_ms;
} frnn_kernel_time;

void frnn_profile_enable(int32_t on);
int32_t frnn_profile_read(frnn_kernel_time *out, int32_t cap, int32_t reset);

/* Measured rate (operations per second, whole device) of the distance
 * evaluation's operation mix: float32 subtract, multiply and add, each
 * rounded on its own (no fused multiply-add, no packed FP32), run by every
 * resident wave with independent chains (a microkernel of ~25 ms).  The
 * roofline denominator of the distance kernels. */
frnn_status frnn_measure_valu_rate(void *stream, double *ops_per_s);

/* Work counters of the most recent query or batch on this thread. */
typedef struct {
    int64_t candidates;   /* (query, reference) pairs whose distance was evaluated */
    int64_t work_items;
    int64_t pairs;        /* output pairs (after the cap) */
    int64_t long_row_keys; /* keys of the rows longer than the stash (scratch rows of the fill pass) */
    int32_t stash_cap;    /* the stash size the run used */
    int32_t adapted;      /* 1 when frnn_opts.adapt chose the run's dense-row setting */
} frnn_stats;

frnn_status frnn_last_stats(frnn_stats *out);

/* Device bytes held by the pools (current and peak). */
void frnn_memory_stats(int64_t *current_bytes, int64_t *peak_bytes);

const char *frnn_status_str(frnn_status s);
const char *frnn_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FRNN_H */
