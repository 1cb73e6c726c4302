// Batched pipeline: many events through one launch sequence.
//
// A BatchContext owns device buffers sized for a capacity class (events,
// points, queries, cells, chunks; rounded up so that similar batches share a
// class).  Its launch sequence has fixed grid sizes and reads every actual
// size from device memory, so it is launched kernel by kernel (the default)
// or, with the graphs option, recorded once as HIP graphs (built node by
// node, no stream capture) and replayed for any batch of its class:
//   phase A: bin the points of every event, count every query's neighbours,
//            scan the capped counts, and publish the counters and event
//            bases to a host-mapped block (then a flag the host polls)
//   phase B: short rows and per-event offsets; then, only when some row is
//            longer than the stash, the fill pass and the long-row sort
// Run exactly, A and B are separated by the read-back that sizes the output.
// Once a context has run, its next batch is run speculatively instead: the
// output is allocated at a capacity guessed from the previous run, and A
// and B are launched together (one graph when replayed; the first block of
// the short-row pass then publishes the counts, one launch less), so the
// host checks the counts while B runs; the fill kernels write nothing when
// the run does not fit, and only then does the host allocate the exact size
// and run B again.
// The count and fill kernels take windows of sorted queries (runs of cell
// blocks of one event) as work items: one wave per window from the
// hardware's dispatch, or, persistent (frnn_opts.persistent), a resident
// grid dealing per-XCD queues built costliest event first (by the plan
// kernel's last block).
#pragma once

#include <condition_variable>
#include <cstdint>
#include <memory>
#include <mutex>
#include <vector>

#include "frnn_runtime.h"

namespace frnn {

struct BatchCounts {
    Counters ctr;
    uint32_t build_status;
    std::vector<int64_t> bases;  // [E+1]
};

class BatchContext {
public:
    struct Shape {
        int D;
        uint32_t flags;
        int K;
        float r;
        int E_cap;
        int64_t pts_cap, q_cap, cells_cap;
        int pch_cap, qch_cap;
        frnn_opts o;
        bool operator==(const Shape &x) const;
    };

    BatchContext(const Shape &sh, hipStream_t s);
    ~BatchContext();
    const Shape &shape() const { return sh_; }
    static Shape shape_for(const frnn_event *ev, int E, int D, float r, int K, uint32_t flags,
                           const Opts &o);
    bool fits(const Shape &need) const;
    // device bytes a context of this shape holds (pool size classes), and
    // those this one holds now (its long-row scratch included)
    static int64_t bytes_for(const Shape &sh);
    int64_t device_bytes() const;

    // 1. descriptors of this batch; prepare writes them to the context's
    //    pinned, device-mapped stage, upload adds the output descriptor when
    //    given; the first kernel of phase A copies the stage to the device
    void set_inputs(const frnn_event *ev, int E, hipStream_t s);
    void prepare(const frnn_event *ev, int E);
    void upload(hipStream_t s, const OutDesc *od);
    // 2. bin + count + scan, and the counters and event bases written to
    //    the host-mapped read-back block (phase A)
    void phase_a(hipStream_t s);
    // 2+4. phase A followed by the short rows (and the long rows) in one
    //    sequence, for a run whose output was allocated from a guess
    void phase_ab(bool with_long, hipStream_t s);
    // 3. wait for phase A's read-back and read the counters (fetch_counts
    //    notes the stream, wait_counts polls the block's run number)
    BatchCounts read_counts(hipStream_t s);
    void fetch_counts(hipStream_t s);
    BatchCounts wait_counts();
    // 4. fill into the given output (phase B: the short rows, then, when
    //    some row is longer than the stash, the long rows); the parts alone
    //    fill into the output descriptor given to upload
    void phase_b(const OutDesc &od, bool long_rows, hipStream_t s);
    void phase_b_short(hipStream_t s);
    void phase_b_long(hipStream_t s);
    // whether the previous run had rows longer than the stash
    bool expect_long() const { return seen_long_ > 0; }

    // Output capacities for a speculative run (false before the first run).
    bool guess(int64_t *pairs, int64_t *long_keys) const;
    void learn(const BatchCounts &c);

    // Make every buffer's stream-ordered release follow stream s (the
    // stream of the current user, or null once the device work is done).
    void retarget(hipStream_t s);
    // every buffer's use is complete (its stream synchronised): their
    // release then records nothing on any stream
    void retire();

    // recorded on the stream of the last run when the context is returned
    hipEvent_t done() const { return done_; }
    // long-row key scratch of speculative runs, grown to at least n keys
    uint64_t *long_scratch(int64_t n, hipStream_t s);
    int E() const { return E_; }
    const std::vector<int64_t> &q_off() const { return qoff_; }
    const std::vector<int64_t> &n_q() const { return nq_; }
    int64_t total_q() const { return totq_; }
    bool graphs_enabled = false;  // the shape's graphs option (cleared if recording fails)
    int replays = 0;

private:
    void launch_a(hipStream_t s, bool publish = true);
    void launch_b_short(hipStream_t s, bool publish = false);
    Publish publish_args();
    void launch_b_long(hipStream_t s);
    void launch_ab(hipStream_t s);
    void launch_abl(hipStream_t s);
    bool replay(hipGraphExec_t *ge, hipGraph_t *g, void (*fn)(void *, hipStream_t), hipStream_t s);
    Shape sh_;
    int Dp_ = 0;
    int E_ = 0;
    int64_t totq_ = 0;
    std::vector<int64_t> qoff_, nq_;
    Knobs kn_{};
    Bufs bb_{}, bq_{};  // build run and query run
    size_t o_ev_ = 0, o_pc_ = 0, o_qc_ = 0;
    DevBuf desc, hv, grid, cell_off, ext, xs, perm, key, rank,
        skey, cells, qs, qperm, qkey, qrank, sqkey, qcells, runs, deg, offs, lofs, lrows, lat, stash, flist, part,
        lpt;
    MappedHost back_;  // read-back block, written by the last kernel of phase A
    size_t hv16_ = 0;  // its size in 16-byte words
    MappedHost stage_;            // descriptors, host side, read by the first kernel
    size_t stage_cap_ = 0;        // bytes, the capacity of the descriptor block
    int64_t seen_pairs_ = -1, seen_long_ = 0;  // the previous run's output
    uint32_t run_seq_ = 0;          // number of the latest run (BatchDesc::run_id)
    hipStream_t last_s_ = nullptr;  // stream of the latest run
    hipEvent_t done_ = nullptr;
    DevBuf lk_;
    hipGraphExec_t ga_ = nullptr, gbs_ = nullptr, gbl_ = nullptr, gab_ = nullptr, gabl_ = nullptr;
    hipGraph_t gra_ = nullptr, grbs_ = nullptr, grbl_ = nullptr, grab_ = nullptr, grabl_ = nullptr;
};

// Check a context of a fitting class out of the shared cache (or make one);
// give it back when done.  Contexts are never used by two runs at once.
std::unique_ptr<BatchContext> acquire_context(const BatchContext::Shape &need, hipStream_t s);
void return_context(std::unique_ptr<BatchContext> ctx, hipStream_t s);

// One batch end to end: acquire, run, hand out per-event CSRs.
frnn_status batch_run(const frnn_event *ev, int E, int D, float r, int K, uint32_t flags,
                      const Opts &o, hipStream_t s, frnn_csr *outs);

// Output allocation of a batch (offsets | indices | dist2 | long scratch).
struct BatchOutput {
    OutputOwner *own = nullptr;
    OutDesc od{};
    DevBuf long_keys;
};
// Capacities: pairs (indices and dist2) and long-row keys (in long_scratch
// when given, else in a buffer of the output's own).
BatchOutput alloc_output(const BatchContext &ctx, int64_t pairs, int64_t long_keys, bool want_d2,
                         hipStream_t s, uint64_t *long_scratch = nullptr);
BatchOutput alloc_output(const BatchContext &ctx, const BatchCounts &c, bool want_d2, hipStream_t s);
// device bytes (pool size classes) of the output alloc_output makes
int64_t output_bytes(const BatchContext &ctx, int64_t pairs, int64_t long_keys, bool want_d2);
void hand_out(const BatchContext &ctx, const BatchCounts &c, BatchOutput &bo, frnn_csr *outs);

}  // namespace frnn
