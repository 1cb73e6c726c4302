// Host runtime of libfrnn: device memory pool, pipeline runs, instrumentation.
// Shared by the C ABI, the batcher, the server and the tuner.
#pragma once

#include <hip/hip_runtime_api.h>

#include <atomic>
#include <functional>
#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/frnn.h"
#include "frnn_device.h"

namespace frnn {

// ----------------------------------------------------------------- errors
struct Fail {
    frnn_status st;
    std::string msg;
};

void set_error(const std::string &msg);
frnn_status fail(frnn_status st, const std::string &msg);

#define FRNN_HIP(call)                                                              \
    do {                                                                            \
        hipError_t e_ = (call);                                                     \
        if (e_ != hipSuccess)                                                       \
            throw ::frnn::Fail{FRNN_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
    } while (0)

// ------------------------------------------------------------------- pool
// Caching device allocator.  Blocks are kept in size classes (2^k times
// 1, 1.25, 1.5, 1.75) and reused: on the stream that freed them at once
// (stream order), on another stream once the work before the free point is
// complete (no host synchronisation, no cross-stream wait).
class Pool {
public:
    static Pool &get();
    void *alloc(size_t bytes, hipStream_t s);
    void free(void *p, hipStream_t s);
    // return a block whose every use is already complete (no stream order)
    void free_complete(void *p);
    void trim();
    int64_t held() const { return held_.load(); }
    int64_t in_use() const { return in_use_.load(); }
    int64_t peak() const { return peak_.load(); }
    // test hook: the k-th allocation from now fails (0 = off)
    void fail_after(int64_t k) { fail_at_ = k; }
    // bytes the pool holds for a request of `bytes` (its size class)
    static int64_t class_bytes(size_t bytes) { return (int64_t)size_class(bytes ? bytes : 16); }

private:
    struct Block {
        void *p;
        size_t cls;
        hipEvent_t ready;   // recorded at free; null: every use is complete
        hipStream_t stream; // stream of the free
    };
    static size_t size_class(size_t bytes);
    void *take_free(size_t cls, hipStream_t s);
    size_t unlive(void *p);
    // free blocks' events are recycled (creating one costs a runtime call)
    hipEvent_t take_event();
    void give_event(hipEvent_t e);
    std::mutex mu_;
    std::vector<Block> free_;
    std::vector<hipEvent_t> spare_;
    std::vector<std::pair<void *, size_t>> live_;
    std::atomic<int64_t> held_{0}, in_use_{0}, peak_{0};
    std::atomic<int64_t> fail_at_{0};
};

// Owner of one pool block, returned on the stream it was last used on.
class DevBuf {
public:
    DevBuf() = default;
    DevBuf(size_t bytes, hipStream_t s) { reset(bytes, s); }
    ~DevBuf() { release(); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept { *this = std::move(o); }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) {
            release();
            p_ = o.p_;
            bytes_ = o.bytes_;
            s_ = o.s_;
            done_ = o.done_;
            o.p_ = nullptr;
            o.bytes_ = 0;
        }
        return *this;
    }
    void reset(size_t bytes, hipStream_t s) {
        release();
        s_ = s;
        done_ = false;
        bytes_ = bytes;
        p_ = Pool::get().alloc(bytes ? bytes : 16, s);
    }
    void release() {
        if (p_) {
            if (done_) Pool::get().free_complete(p_);
            else Pool::get().free(p_, s_);
        }
        p_ = nullptr;
        bytes_ = 0;
    }
    void set_stream(hipStream_t s) {
        s_ = s;
        done_ = false;
    }
    // Every use of the block is complete (the caller has synchronised its
    // stream): its release then records nothing on any stream, so it may
    // come from any thread after that stream is gone.
    void mark_complete() { done_ = true; }
    template <class T>
    T *as() const { return reinterpret_cast<T *>(p_); }
    void *get() const { return p_; }
    size_t bytes() const { return bytes_; }

private:
    void *p_ = nullptr;
    size_t bytes_ = 0;
    hipStream_t s_ = nullptr;
    bool done_ = false;
};

// Pinned host staging buffer (grows, never shrinks).
class Pinned {
public:
    ~Pinned();
    void *ensure(size_t bytes);
    template <class T>
    T *as() { return reinterpret_cast<T *>(p_); }

private:
    void *p_ = nullptr;
    size_t bytes_ = 0;
};

// Pinned host memory mapped into the device's address space, coherent (the
// device reads and writes it without caching), of a fixed size.
class MappedHost {
public:
    MappedHost() = default;
    ~MappedHost();
    MappedHost(const MappedHost &) = delete;
    MappedHost &operator=(const MappedHost &) = delete;
    void reset(size_t bytes);  // zero-filled; throws on failure
    char *host() const { return h_; }
    void *dev() const { return d_; }

private:
    char *h_ = nullptr;
    void *d_ = nullptr;
};

// ---------------------------------------------------------- instrumentation
void prof_begin(const char *name, hipStream_t s, bool capturing);
void prof_end(hipStream_t s, bool capturing);
bool prof_enabled();

// ------------------------------------------------------------- pipeline
struct Opts {
    frnn_opts o;
    static Opts from(const frnn_opts *p);
    frnn_status validate(std::string *why) const;
};

// Reference points of E events, binned (device-resident, immutable).
struct Index {
    int E = 0, D = 0, Dp = 0;
    float r = 0.f;
    Opts opts;
    int64_t total_pts = 0, cells_cap = 0;
    int n_pchunks = 0;
    std::vector<int64_t> n_pts, pt_off;
    std::vector<const float *> pts;
    DevBuf desc, grid, runs, cell_off, ext, xs, perm, skey, cells, ctr;
    size_t o_ev = 0, o_ch = 0;        // offsets of the event and chunk tables in desc
    bool status_checked = false;      // non-finite input already ruled out
    std::vector<GridDesc> grid_host;  // valid after a synchronised build
    Pinned stage;                     // descriptor staging of the build copies
    hipStream_t stream = nullptr;
};

struct OutputOwner {
    DevBuf buf;                     // offsets | indices | dist2 | status word
    std::atomic<int> refs{0};
    uint32_t *status = nullptr;     // device word written by the long-row pass
    bool long_ran = false;          // the long-row pass wrote into this output
    // Reads the status word when the long-row pass ran (synchronises s):
    // FRNN_ERR_INTERNAL when the fill's recount of a row differed.
    frnn_status check(hipStream_t s);
    std::function<void()> on_release;  // e.g. return the bytes to a budget
    ~OutputOwner() {
        if (on_release) on_release();
    }
};

// Build an index over E events (points[e] is device [n[e]][D]).  With sync,
// waits for the build and reports non-finite input; without, the status is
// checked by the first query run on the same stream.
frnn_status build_index(Index &ix, const float *const *points, const int64_t *n, int E, int D,
                        float r, const Opts &opts, hipStream_t s, bool sync);

// Query an index: queries[e] device [m[e]][D], or the indexed points when
// self_query.  Produces E CSRs sharing one allocation.
struct QueryArgs {
    const float *const *queries = nullptr;
    const int64_t *m = nullptr;
    float r = 0.f;
    int K = 0;
    uint32_t flags = 0;
};
frnn_status run_query(Index &ix, const QueryArgs &qa, hipStream_t s, frnn_csr *outs,
                      frnn_stats *stats);

// Last run's counters (thread-local).
void record_stats(const frnn_stats &st);
frnn_stats last_stats();
const char *last_error_cstr();
void prof_set(bool on);
int prof_read(frnn_kernel_time *out, int cap, bool reset);

float r2_of(float r);
int query_blocks(const frnn_opts &o, int64_t nqchunks, bool persistent);
bool use_persistent(const frnn_opts &o, int E, int64_t nqchunks, const Knobs &kn, int D);
// grid of the fill pass over `windows` listed windows (it strides past 4096 blocks)
int fill_blocks(int64_t windows);

// Graph recording in progress on this thread (per-launch timing is skipped).
void set_capturing(bool on);
bool capturing();

#define LAUNCH(name, stream, call)                                                     \
    do {                                                                               \
        ::frnn::prof_begin(name, stream, ::frnn::capturing());                         \
        hipError_t e_ = (call);                                                        \
        ::frnn::prof_end(stream, ::frnn::capturing());                                 \
        if (e_ != hipSuccess)                                                          \
            throw ::frnn::Fail{FRNN_ERR_HIP, std::string("launch ") + name + ": " + hipGetErrorString(e_)}; \
    } while (0)

}  // namespace frnn
