// Shared layout of the device-resident descriptors of one pipeline run.
//
// A run processes E independent events.  Every size a kernel needs is read
// from device memory (the batch descriptor, the chunk tables and the
// counters), never baked into a launch, so one launch sequence serves any
// batch that fits the buffers and can be replayed as a HIP graph.
#pragma once

#include <stdint.h>

namespace frnn {

constexpr int kWave = 64;        // CDNA wavefront width
constexpr int kGMax = 6;         // most grid axes
constexpr int kDMax = 32;        // most coordinates per point
constexpr int kRunsMax = 256;    // neighbour runs per work item (LDS table size)
constexpr int kCandLds = 512;    // candidate positions listed in LDS per work item
constexpr int kRowLds = 512;     // longest row one wave sorts on chip (8 keys per lane in registers)
constexpr int kChunkRows = 256;  // rows per chunk of the per-point kernels
constexpr int kWavesPerBlock = 4;

// Cell grid of one event, chosen on the device from the event's extent.
// A point x has grid coordinates c_a = clamp(floor((x[axis[a]] - lo[a]) *
// inv_h), 0, n[a]-1) and cell key sum_a c_a * stride[a] (stride[0] = 1, so
// cells adjacent along grid axis 0 have adjacent keys).
struct GridDesc {
    int32_t G;             // grid axes in use (0 = one cell)
    int32_t m;             // reach in cells: neighbours lie within +-m cells
    int32_t runs;          // (2m+1)^(G-1): key runs scanned per work item
    uint32_t C;            // cells
    int32_t axis[kGMax];
    int32_t n[kGMax];
    uint32_t stride[kGMax];
    double lo[kGMax];
    double inv_h;
    double h;
};

// Host-written description of one event.
struct EventDev {
    const float *pts;      // caller's [n_pts][D]
    const float *qry;      // caller's [n_q][D] (unused for self-queries)
    int64_t n_pts, pt_off; // rows, offset in the concatenated point arrays
    int64_t n_q, q_off;    // queries, offset in the concatenated query arrays
    int64_t cell_cap;      // most cells the plan may give this event
};

// Rows [r0, r1) of the concatenated point (or query) arrays, all in event ev.
struct Chunk {
    int32_t ev;
    int32_t pad;
    int64_t r0, r1;
};

// Host-written scalars of a run.
struct BatchDesc {
    int32_t E;
    int32_t D, Dp;         // dimension and padded row length (multiple of 4)
    int32_t n_pchunks, n_qchunks;
    int32_t grid_axes_max, cell_multiple;
    float cells_per_point;
    float r_build;
    uint32_t run_id;       // the host's number of this run (echoed in the counters)
    int64_t total_pts, total_q;
};

// Device-written counters, copied to the host once per run.
struct Counters {
    uint64_t total_cells;  // sum of the events' cell counts
    uint64_t nnz;          // output pairs (after the cap)
    uint64_t long_total;   // keys in the scratch rows (rows longer than the stash)
    uint64_t candidates;   // distance evaluations of the count pass
    uint32_t n_groups;     // cell-block groups evaluated by the count pass
    uint32_t n_long;       // rows sorted in global memory
    uint32_t status;       // kStatus* bits
    uint32_t n_fill;       // windows listed for the fill pass
    uint32_t plan_done;    // plan blocks finished (the last one scans the cell counts)
    uint32_t n_fill_light; // windows listed for the fill pass from the back of the list (lighter ones)
    uint32_t run_id;       // BatchDesc::run_id of the run that wrote them (batched path)
    uint32_t pad[5];
};

// One neighbour key run of a work group: offsets o[a] (a = 1..G-1) of the
// neighbour cell on the grid axes other than axis 0, and the key offset
// sum_a o[a] * stride[a].
struct RunEntry {
    int32_t koff;
    int8_t o[kGMax];
    int8_t pad[6];
};

constexpr uint32_t kStatusNonfinitePts = 1u;
constexpr uint32_t kStatusNonfiniteQry = 2u;
constexpr uint32_t kStatusInternal = 4u;

// Where the fill pass writes (device-resident so graphs need not change).
// An output may be allocated before the pair count is known, at a capacity
// guessed from earlier runs: when the run's pairs or long-row keys exceed
// the capacities below, the fill kernels write nothing and the host fills
// again into an output of the exact size.
struct OutDesc {
    int64_t *offsets;      // per-event offsets, event e at q_off + e
    int32_t *indices;      // [cap_pairs]
    float *dist2;          // [cap_pairs] or null
    uint64_t *long_keys;   // [cap_long] scratch rows of the fill pass
    int64_t cap_pairs;
    int64_t cap_long;
    uint32_t *status;      // written by the long-row pass: kStatusInternal when the fill's
                           // recount of a row differed from the count pass
};

// The read-back of a run's counts (passed by value to the kernel that
// performs it): n16 16-byte words from src (the counters first, then the
// event bases) to dst, device-mapped host memory, then the counters' run
// number into *flag.  All 16-byte aligned; flag null: no read-back.
struct Publish {
    const void *src;
    void *dst;
    int64_t n16;
    uint32_t *flag;
};

// Per-run scalars passed by value.
struct Knobs {
    float r2;              // fl32(r*r), computed on the host
    int32_t K;             // <= 0: no cap
    int32_t self_query;    // queries are the sorted points
    int32_t exclude_self;
    int32_t window;        // sorted queries per work window (divides kChunkRows)
    int32_t cells_per_item;
    int32_t long_cap;      // rows longer than this sort in global memory
    int32_t persistent;
    int32_t stash_cap;     // hits per query kept by the count pass (0 = none)
    uint32_t fill_cap;     // entries of fill_list
};

// Layout of the persistent count pass's work order for E events (words):
//   order[E]       events by decreasing estimated cost per window
//   chunk0[E]      first query chunk of each event
//   nwin[E]        windows of each event
//   pre[8][E + 1]  per XCD: exclusive prefix of the event slices in that order
constexpr int64_t lpt_words(int64_t E) { return 3 * E + 8 * (E + 1); }
// most events the work order is built for (one block, in LDS); larger
// batches take the non-persistent launch
constexpr int kLptMaxEvents = 1024;

// A listed window whose fill work (queries with rows longer than the stash
// times the candidates of their group) reaches this many distance
// evaluations goes to the front of the fill list.
constexpr uint32_t kFillHeavy = 1u << 15;

// Device buffers of a run.
struct Bufs {
    const BatchDesc *bd;
    const EventDev *ev;
    const Chunk *pchunks;
    const Chunk *qchunks;
    Counters *ctr;
    int64_t *bases;        // [E+1] first output pair of each event
    GridDesc *grid;        // [E]
    RunEntry *runs;        // [E][kRunsMax]
    int64_t *cell_off;     // [E+1]
    uint32_t *ext;         // [E][2][D] order-preserving min / max bits
    // points, concatenated over events
    float *xs;             // [total_pts][Dp] sorted by cell
    int32_t *perm;         // sorted slot -> local original index
    uint32_t *key, *rank;  // per original point
    uint32_t *skey;        // per sorted slot
    uint32_t *cells;       // [total_cells+1] counts, then exclusive scan
    // queries (for self-queries these alias the point arrays)
    float *qs;
    int32_t *qperm;
    uint32_t *qkey, *qrank, *sqkey, *qcells;
    // rows
    uint32_t *deg;         // in-radius count per query (global row)
    int64_t *offs;         // [total_q+1] exclusive scan of capped counts
    int64_t *lofs;         // [total_q+1] exclusive scan of the lengths of rows longer than the stash
    uint32_t *long_rows;   // [total_q] length of each row listed for the row sort
    int64_t *long_at;      // [2*total_q] its scratch offset and output offset
    uint64_t *stash;       // [total_q][stash_cap] first hit keys per query (global row)
    uint32_t *fill_list;   // windows holding rows longer than the stash: heavier ones from the
                           // front, lighter ones from the back (fill_cap entries)
    uint32_t *lpt;         // persistent count pass: work order (see k_lpt), lpt_words(E) words
    uint64_t *scan_part;   // scan block partials (2 x kScanBlocks)
    OutDesc *out;
};

constexpr int kScanBlocks = 1024;
constexpr int kExtentRows = 1024;  // rows per extent block (per-unit slots)
constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;

}  // namespace frnn
