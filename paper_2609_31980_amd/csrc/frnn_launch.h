// Host-side launchers of the pipeline kernels (frnn_kernels.hip).  Each
// returns the launch error, if any; grid sizes are capacities, the kernels
// read the actual sizes from device memory.
#pragma once

#include <hip/hip_runtime_api.h>

#include "frnn_device.h"

namespace frnn {

// Graph recording.  While a thread has a recorder set, the launchers below
// append kernel nodes to its graph instead of launching, each node depending
// on the one before (the order of launches on one stream).  Building the
// graph this way involves no stream capture, so nothing another thread does
// meanwhile (allocations, synchronisations, work on other streams or the
// null stream) can spoil it.
struct GraphRecorder {
    hipGraph_t graph = nullptr;
    hipGraphNode_t last = nullptr;
    hipError_t err = hipSuccess;  // first failure to add a node
};
void set_recorder(GraphRecorder *r);  // this thread's; null: launch again

// zeroes b.ctr (and `also`, when given); with src, also copies `bytes` of
// descriptors from device-mapped host memory src to device memory dst (both
// 16-byte aligned, bytes rounded up to 16)
hipError_t launch_init(const Bufs &b, hipStream_t s, Counters *also = nullptr, const void *src = nullptr,
                       void *dst = nullptr, int64_t bytes = 0);
// one block per chunk (per-chunk extent slots for the points); also clears
// zero_n cells of the (point or query) cell histogram
hipError_t launch_extent(const Bufs &b, int nchunks, int E_cap, bool queries, int64_t zero_n, hipStream_t s);
// with lpt (a persistent count pass's knobs), the plan's last block also
// builds that pass's work order, as launch_lpt does
hipError_t launch_plan(const Bufs &b, int E_cap, hipStream_t s, const Knobs *lpt = nullptr);
hipError_t launch_keys(const Bufs &b, int nchunks, bool queries, hipStream_t s);
hipError_t launch_scan_cells(const Bufs &b, int64_t cells_cap, bool queries, hipStream_t s);
hipError_t launch_scatter(const Bufs &b, int nchunks, bool queries, hipStream_t s);
// blocks: plain mode, enough for every window (rounded up to a multiple of
// 8); persistent mode, the resident grid.
hipError_t launch_count(const Bufs &b, const Knobs &kn, int D, int blocks, hipStream_t s);
hipError_t launch_scan_rows(const Bufs &b, const Knobs &kn, int64_t total_q, hipStream_t s);
// rows of at most stash_cap pairs, and every row's per-event offset: one
// block per query chunk; with pub, its first block also performs that
// read-back of the counts (in place of launch_publish)
hipError_t launch_short_rows(const Bufs &b, const Knobs &kn, int nqchunks, hipStream_t s,
                             const Publish *pub = nullptr);
// the windows listed by the count pass; any grid size is correct
hipError_t launch_fill(const Bufs &b, const Knobs &kn, int D, int blocks, hipStream_t s);
hipError_t launch_long_sort(const Bufs &b, const Knobs &kn, int blocks, hipStream_t s);
// blocks of the persistent count kernel resident on the whole device
int count_resident_blocks(const Knobs &kn, int D);
// work order of the persistent count pass (needs the grids and b.lpt)
hipError_t launch_lpt(const Bufs &b, const Knobs &kn, hipStream_t s);
hipError_t launch_set_out(const Bufs &b, const OutDesc &v, hipStream_t s);
// the read-back (one block): see Publish
hipError_t launch_publish(const Publish &p, hipStream_t s);

}  // namespace frnn
