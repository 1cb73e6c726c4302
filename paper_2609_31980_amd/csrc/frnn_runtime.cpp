// Host runtime: pool, instrumentation, index build and query runs.
#include "frnn_runtime.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>

#include "frnn_launch.h"

namespace frnn {

// ----------------------------------------------------------------- errors
static thread_local std::string t_err;
static thread_local frnn_stats t_stats{};

void set_error(const std::string &msg) { t_err = msg; }

frnn_status fail(frnn_status st, const std::string &msg) {
    t_err = msg;
    return st;
}

const char *last_error_cstr() { return t_err.c_str(); }

void record_stats(const frnn_stats &st) { t_stats = st; }
frnn_stats last_stats() { return t_stats; }

float r2_of(float r) {
    volatile float rr = r * r;  // one float32 rounding
    return rr;
}

frnn_status OutputOwner::check(hipStream_t s) {
    if (!long_ran || !status) return FRNN_OK;
    uint32_t v = 0;
    FRNN_HIP(hipMemcpyAsync(&v, status, sizeof(v), hipMemcpyDeviceToHost, s));
    FRNN_HIP(hipStreamSynchronize(s));
    if (v & kStatusInternal) return fail(FRNN_ERR_INTERNAL, "the fill pass recounted a row differently");
    return FRNN_OK;
}

// ------------------------------------------------------------------- pool
Pool &Pool::get() {
    static Pool *p = new Pool();  // never destroyed: blocks live to exit
    return *p;
}

size_t Pool::size_class(size_t bytes) {
    if (bytes <= 256) return 256;
    size_t p = 256;
    while (p * 2 <= bytes) p *= 2;
    // p <= bytes < 2p: quarter steps
    for (size_t q = 0; q <= 4; ++q) {
        size_t c = p + p * q / 4;
        if (c >= bytes) return (c + 255) / 256 * 256;
    }
    return 2 * p;
}

// A free block of class cls that stream s may use now: one freed on s is
// reused at once (stream order); one freed on another stream only once its
// last use there is complete (no cross-stream wait: that would tie this
// stream's later work to the other stream's).
void *Pool::take_free(size_t cls, hipStream_t s) {
    Block got{nullptr, 0, nullptr, nullptr};
    {
        std::lock_guard<std::mutex> g(mu_);
        for (size_t i = 0; i < free_.size(); ++i) {
            if (free_[i].cls != cls) continue;
            if (free_[i].ready && free_[i].stream != s && hipEventQuery(free_[i].ready) != hipSuccess) {
                (void)hipGetLastError();
                continue;
            }
            got = free_[i];
            free_[i] = free_.back();
            free_.pop_back();
            break;
        }
    }
    if (got.ready) give_event(got.ready);
    return got.p;
}

void *Pool::alloc(size_t bytes, hipStream_t s) {
    if (fail_at_.load() > 0 && --fail_at_ == 0)
        throw Fail{FRNN_ERR_OOM, "device allocation failed (test hook)"};
    const size_t cls = size_class(bytes);
    void *p = take_free(cls, s);
    if (!p) {
        hipError_t e = hipMalloc(&p, cls);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            trim();  // give cached blocks back and retry once
            e = hipMalloc(&p, cls);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                throw Fail{FRNN_ERR_OOM, "hipMalloc of " + std::to_string(cls) + " bytes failed"};
            }
        }
        held_ += (int64_t)cls;
    }
    {
        std::lock_guard<std::mutex> g(mu_);
        live_.push_back({p, cls});
    }
    int64_t now = (in_use_ += (int64_t)cls);
    int64_t pk = peak_.load();
    while (now > pk && !peak_.compare_exchange_weak(pk, now)) {
    }
    return p;
}

size_t Pool::unlive(void *p) {
    std::lock_guard<std::mutex> g(mu_);
    for (size_t i = 0; i < live_.size(); ++i) {
        if (live_[i].first == p) {
            const size_t cls = live_[i].second;
            live_[i] = live_.back();
            live_.pop_back();
            return cls;
        }
    }
    return 0;
}

void Pool::free(void *p, hipStream_t s) {
    if (!p) return;
    const size_t cls = unlive(p);
    if (!cls) return;
    hipEvent_t ev = take_event();
    if (ev && hipEventRecord(ev, s) != hipSuccess) {
        (void)hipGetLastError();
        give_event(ev);
        ev = nullptr;
    }
    if (!ev) {
        // the reuse cannot be ordered by an event: wait here instead
        (void)hipStreamSynchronize(s);
        (void)hipGetLastError();
    }
    in_use_ -= (int64_t)cls;
    std::lock_guard<std::mutex> g(mu_);
    free_.push_back({p, cls, ev, s});
}

void Pool::free_complete(void *p) {
    if (!p) return;
    const size_t cls = unlive(p);
    if (!cls) return;
    in_use_ -= (int64_t)cls;
    std::lock_guard<std::mutex> g(mu_);
    free_.push_back({p, cls, nullptr, nullptr});
}

hipEvent_t Pool::take_event() {
    {
        std::lock_guard<std::mutex> g(mu_);
        if (!spare_.empty()) {
            hipEvent_t e = spare_.back();
            spare_.pop_back();
            return e;
        }
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

// A recorded event may be re-recorded at once: waits already queued on it
// keep the state they captured.
void Pool::give_event(hipEvent_t e) {
    std::lock_guard<std::mutex> g(mu_);
    spare_.push_back(e);
}

void Pool::trim() {
    std::vector<Block> blocks;
    {
        std::lock_guard<std::mutex> g(mu_);
        blocks.swap(free_);
    }
    for (auto &b : blocks) {
        if (b.ready) {
            (void)hipEventSynchronize(b.ready);
            (void)hipEventDestroy(b.ready);
        }
        (void)hipFree(b.p);
        held_ -= (int64_t)b.cls;
    }
}

MappedHost::~MappedHost() {
    if (h_) (void)hipHostFree(h_);
}

void MappedHost::reset(size_t bytes) {
    if (h_) (void)hipHostFree(h_);
    h_ = nullptr;
    d_ = nullptr;
    if (hipHostMalloc((void **)&h_, bytes ? bytes : 16, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
        h_ = nullptr;
        (void)hipGetLastError();
        throw Fail{FRNN_ERR_OOM, "hipHostMalloc failed"};
    }
    std::memset(h_, 0, bytes ? bytes : 16);
    if (hipHostGetDevicePointer(&d_, h_, 0) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipHostFree(h_);
        h_ = nullptr;
        throw Fail{FRNN_ERR_HIP, "hipHostGetDevicePointer failed"};
    }
}

Pinned::~Pinned() {
    if (p_) (void)hipHostFree(p_);
}

void *Pinned::ensure(size_t bytes) {
    if (bytes <= bytes_) return p_;
    if (p_) (void)hipHostFree(p_);
    p_ = nullptr;
    size_t nb = std::max<size_t>(bytes, 2 * bytes_);
    if (hipHostMalloc(&p_, nb, hipHostMallocDefault) != hipSuccess) {
        p_ = nullptr;
        bytes_ = 0;
        throw Fail{FRNN_ERR_OOM, "hipHostMalloc failed"};
    }
    bytes_ = nb;
    return p_;
}

// ---------------------------------------------------------- instrumentation
namespace {
struct ProfRec {
    std::string name;
    hipEvent_t a, b;
};
std::mutex g_prof_mu;
std::atomic<bool> g_prof_on{false};
std::vector<ProfRec> &g_prof_pending = *new std::vector<ProfRec>();
std::map<std::string, std::pair<int64_t, double>> &g_prof_total =
    *new std::map<std::string, std::pair<int64_t, double>>();
thread_local ProfRec t_open{"", nullptr, nullptr};
}  // namespace

bool prof_enabled() { return g_prof_on.load(); }

void prof_begin(const char *name, hipStream_t s, bool capturing) {
    if (!g_prof_on.load() || capturing) return;
    t_open.name = name;
    (void)hipEventCreate(&t_open.a);
    (void)hipEventCreate(&t_open.b);
    (void)hipEventRecord(t_open.a, s);
}

void prof_end(hipStream_t s, bool capturing) {
    if (!g_prof_on.load() || capturing || !t_open.a) return;
    (void)hipEventRecord(t_open.b, s);
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_prof_pending.push_back(t_open);
    t_open = ProfRec{"", nullptr, nullptr};
}

static void prof_collect() {
    std::vector<ProfRec> recs;
    {
        std::lock_guard<std::mutex> g(g_prof_mu);
        recs.swap(g_prof_pending);
    }
    for (auto &r : recs) {
        float ms = 0.f;
        (void)hipEventSynchronize(r.b);
        (void)hipEventElapsedTime(&ms, r.a, r.b);
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
        std::lock_guard<std::mutex> g(g_prof_mu);
        auto &t = g_prof_total[r.name];
        t.first += 1;
        t.second += ms;
    }
}

void prof_set(bool on) { g_prof_on = on; }

int prof_read(frnn_kernel_time *out, int cap, bool reset) {
    prof_collect();
    std::lock_guard<std::mutex> g(g_prof_mu);
    int n = 0;
    for (auto &kv : g_prof_total) {
        if (n < cap && out) {
            std::memset(&out[n], 0, sizeof(frnn_kernel_time));
            std::strncpy(out[n].name, kv.first.c_str(), sizeof(out[n].name) - 1);
            out[n].launches = kv.second.first;
            out[n].total_ms = kv.second.second;
        }
        ++n;
    }
    if (reset) g_prof_total.clear();
    return n;
}

// ------------------------------------------------------------- options
Opts Opts::from(const frnn_opts *p) {
    Opts o;
    if (p) {
        o.o = *p;
    } else {
        frnn_opts_default(&o.o);
    }
    return o;
}

frnn_status Opts::validate(std::string *why) const {
    auto bad = [&](const char *m) {
        *why = m;
        return FRNN_ERR_INVALID_ARG;
    };
    if (o.grid_axes_max < 0 || o.grid_axes_max > kGMax) return bad("grid_axes_max out of 0..6");
    if (!(o.cells_per_point > 0.f) || !std::isfinite(o.cells_per_point)) return bad("cells_per_point must be > 0");
    if (o.cell_multiple < 1 || o.cell_multiple > 3) return bad("cell_multiple out of 1..3");
    if (o.cells_per_item < 1 || o.cells_per_item > 8) return bad("cells_per_item out of 1..8");
    if (o.queries_per_item < 1 || o.queries_per_item > 64 || (o.queries_per_item & (o.queries_per_item - 1)))
        return bad("queries_per_item must be a power of two in 1..64");
    if (o.blocks_per_cu < 1 || o.blocks_per_cu > 16) return bad("blocks_per_cu out of 1..16");
    if (o.persistent < 0 || o.persistent > 2) return bad("persistent must be 0, 1 or 2");
    if (o.row_cap_lds < 1 || o.row_cap_lds > kRowLds) return bad("row_cap_lds out of 1..512");
    if (o.stash_cap != 0 && o.stash_cap != 8 && o.stash_cap != 16 && o.stash_cap != 32 && o.stash_cap != 64 &&
        o.stash_cap != 128 && o.stash_cap != 256)
        return bad("stash_cap must be 0, 8, 16, 32, 64, 128 or 256");
    if (o.graphs != 0 && o.graphs != 1) return bad("graphs must be 0 or 1");
    if (o.adapt != 0 && o.adapt != 1) return bad("adapt must be 0 or 1");
    return FRNN_OK;
}

// ------------------------------------------------------------- pipeline
static thread_local bool t_capturing = false;
// never freed: thread-local destructors may run after the HIP runtime is gone
static thread_local Pinned &t_stage = *new Pinned();
static thread_local Pinned &t_back = *new Pinned();

void set_capturing(bool on) { t_capturing = on; }
bool capturing() { return t_capturing; }

static int64_t pad4(int64_t d) { return (d + 3) & ~int64_t(3); }

static void make_chunks(const std::vector<int64_t> &n, const std::vector<int64_t> &off,
                        std::vector<Chunk> &out) {
    out.clear();
    for (size_t e = 0; e < n.size(); ++e)
        for (int64_t r = 0; r < n[e]; r += kChunkRows)
            out.push_back(Chunk{(int32_t)e, 0, off[e] + r, off[e] + std::min<int64_t>(n[e], r + kChunkRows)});
}

static int64_t cell_cap_of(int64_t n, float cpp) {
    double c = std::floor((double)cpp * (double)std::max<int64_t>(n, 1));
    c = std::max(1.0, std::min(c, (double)(1 << 30)));
    return (int64_t)c;
}

// Workgroups of the fill kernel: one wave per listed window, at most 4096
// blocks (the waves stride over the rest).
int fill_blocks(int64_t windows) {
    return (int)std::min<int64_t>(std::max<int64_t>(8, (windows + kWavesPerBlock - 1) / kWavesPerBlock), 4096);
}

// Workgroups of the count kernel: the resident grid when persistent, else
// one wave per window of sorted queries.
int query_blocks(const frnn_opts &o, int64_t nqchunks, bool persistent) {
    if (persistent) return 256 * o.blocks_per_cu;
    const int64_t windows = nqchunks * (kChunkRows / o.queries_per_item);
    return (int)std::max<int64_t>(8, (windows + kWavesPerBlock - 1) / kWavesPerBlock);
}

// Whether the count and fill passes run persistent.  Automatic: when the
// windows are at most twice the waves that stay resident (a single event of
// a few hundred thousand queries), where the dealt queue measured faster
// than the hardware's dispatch of one block per four windows; with many
// windows per wave (a large batch) the dealt queue's tail measured longer.
bool use_persistent(const frnn_opts &o, int E, int64_t nqchunks, const Knobs &kn, int D) {
    if (o.persistent == 0 || E > kLptMaxEvents) return false;
    if (o.persistent == 1) return true;
    const int64_t windows = nqchunks * (kChunkRows / o.queries_per_item);
    const int64_t waves = (int64_t)std::min(count_resident_blocks(kn, D), 256 * o.blocks_per_cu) * kWavesPerBlock;
    return windows <= 2 * waves;
}

frnn_status build_index(Index &ix, const float *const *points, const int64_t *n, int E, int D,
                        float r, const Opts &opts, hipStream_t s, bool sync) {
    ix.E = E;
    ix.D = D;
    ix.Dp = (int)pad4(D);
    ix.r = r;
    ix.opts = opts;
    ix.stream = s;
    ix.n_pts.assign(n, n + E);
    ix.pts.assign(points, points + E);
    ix.pt_off.resize(E);
    int64_t tot = 0, ccap = 0;
    std::vector<EventDev> evh(E);
    for (int e = 0; e < E; ++e) {
        ix.pt_off[e] = tot;
        evh[e] = EventDev{points[e], nullptr, n[e], tot, 0, 0, cell_cap_of(n[e], opts.o.cells_per_point)};
        tot += n[e];
        ccap += evh[e].cell_cap;
    }
    ix.total_pts = tot;
    ix.cells_cap = ccap;
    std::vector<Chunk> ch;
    make_chunks(ix.n_pts, ix.pt_off, ch);
    ix.n_pchunks = (int)ch.size();

    BatchDesc bd{};
    bd.E = E;
    bd.D = D;
    bd.Dp = ix.Dp;
    bd.n_pchunks = ix.n_pchunks;
    bd.n_qchunks = 0;
    bd.grid_axes_max = opts.o.grid_axes_max;
    bd.cell_multiple = opts.o.cell_multiple;
    bd.cells_per_point = opts.o.cells_per_point;
    bd.r_build = r;
    bd.total_pts = tot;
    bd.total_q = 0;

    // descriptors: one pinned staging block, copied in three pieces
    const size_t o_ev = 256, o_ch = o_ev + sizeof(EventDev) * E;
    const size_t stage = o_ch + sizeof(Chunk) * std::max<size_t>(1, ch.size());
    // staging owned by the index: the copies may still be pending on return
    char *h = (char *)ix.stage.ensure(stage);
    std::memcpy(h, &bd, sizeof(bd));
    std::memcpy(h + o_ev, evh.data(), sizeof(EventDev) * E);
    if (!ch.empty()) std::memcpy(h + o_ch, ch.data(), sizeof(Chunk) * ch.size());

    // descriptors: one device block, one copy
    ix.desc.reset(stage, s);
    ix.grid.reset(sizeof(GridDesc) * E, s);
    ix.runs.reset(sizeof(RunEntry) * kRunsMax * E, s);
    ix.cell_off.reset(sizeof(int64_t) * (E + 1), s);
    ix.ext.reset(sizeof(uint32_t) * 2 * std::max(1, ix.n_pchunks) * D, s);  // per-chunk extent slots
    ix.xs.reset(sizeof(float) * std::max<int64_t>(1, tot) * ix.Dp, s);
    ix.perm.reset(sizeof(int32_t) * std::max<int64_t>(1, tot), s);
    ix.skey.reset(sizeof(uint32_t) * std::max<int64_t>(1, tot), s);
    ix.cells.reset(sizeof(uint32_t) * (ccap + 1), s);
    ix.ctr.reset(sizeof(Counters), s);
    DevBuf key(sizeof(uint32_t) * std::max<int64_t>(1, tot), s);
    DevBuf rank(sizeof(uint32_t) * std::max<int64_t>(1, tot), s);
    DevBuf part(sizeof(uint64_t) * 2 * kScanBlocks, s);

    FRNN_HIP(hipMemcpyAsync(ix.desc.get(), h, stage, hipMemcpyHostToDevice, s));

    Bufs b{};
    b.bd = ix.desc.as<BatchDesc>();
    b.ev = reinterpret_cast<const EventDev *>(ix.desc.as<char>() + o_ev);
    b.pchunks = reinterpret_cast<const Chunk *>(ix.desc.as<char>() + o_ch);
    ix.o_ev = o_ev;
    ix.o_ch = o_ch;
    b.ctr = ix.ctr.as<Counters>();
    b.grid = ix.grid.as<GridDesc>();
    b.runs = ix.runs.as<RunEntry>();
    b.cell_off = ix.cell_off.as<int64_t>();
    b.ext = ix.ext.as<uint32_t>();
    b.xs = ix.xs.as<float>();
    b.perm = ix.perm.as<int32_t>();
    b.key = key.as<uint32_t>();
    b.rank = rank.as<uint32_t>();
    b.skey = ix.skey.as<uint32_t>();
    b.cells = ix.cells.as<uint32_t>();
    b.scan_part = part.as<uint64_t>();

    LAUNCH("init", s, launch_init(b, s));
    LAUNCH("extent", s, launch_extent(b, ix.n_pchunks, E, false, ccap + 1, s));
    LAUNCH("plan", s, launch_plan(b, E, s));
    LAUNCH("keys", s, launch_keys(b, ix.n_pchunks, false, s));
    LAUNCH("scan_cells", s, launch_scan_cells(b, ccap, false, s));
    LAUNCH("scatter", s, launch_scatter(b, ix.n_pchunks, false, s));

    if (sync) {
        char *p = (char *)t_back.ensure(sizeof(Counters) + sizeof(GridDesc) * E);
        FRNN_HIP(hipMemcpyAsync(p, ix.ctr.get(), sizeof(Counters), hipMemcpyDeviceToHost, s));
        FRNN_HIP(hipMemcpyAsync(p + sizeof(Counters), ix.grid.get(), sizeof(GridDesc) * E,
                                hipMemcpyDeviceToHost, s));
        FRNN_HIP(hipStreamSynchronize(s));
        Counters c;
        std::memcpy(&c, p, sizeof(c));
        ix.grid_host.resize(E);
        std::memcpy(ix.grid_host.data(), p + sizeof(Counters), sizeof(GridDesc) * E);
        if (c.status & kStatusNonfinitePts) return fail(FRNN_ERR_NONFINITE, "non-finite coordinate in the points");
        ix.status_checked = true;
    }
    return FRNN_OK;
}

frnn_status run_query(Index &ix, const QueryArgs &qa, hipStream_t s, frnn_csr *outs,
                      frnn_stats *stats) {
    const int E = ix.E, D = ix.D, Dp = ix.Dp;
    const bool selfq = (qa.flags & FRNN_SELF_QUERY) != 0;
    const bool excl = selfq && (qa.flags & FRNN_EXCLUDE_SELF);
    const bool want_d2 = (qa.flags & FRNN_WANT_DIST2) != 0;
    const Opts &op = ix.opts;

    std::vector<int64_t> nq(E), qoff(E);
    int64_t totq = 0;
    for (int e = 0; e < E; ++e) {
        nq[e] = selfq ? ix.n_pts[e] : qa.m[e];
        qoff[e] = totq;
        totq += nq[e];
    }
    std::vector<EventDev> evh(E);
    for (int e = 0; e < E; ++e)
        evh[e] = EventDev{ix.pts[e], selfq ? nullptr : qa.queries[e], ix.n_pts[e], ix.pt_off[e],
                          nq[e], qoff[e], cell_cap_of(ix.n_pts[e], op.o.cells_per_point)};
    std::vector<Chunk> qch;
    make_chunks(nq, qoff, qch);
    const int nqc = (int)qch.size();

    BatchDesc bd{};
    bd.E = E;
    bd.D = D;
    bd.Dp = Dp;
    bd.n_pchunks = ix.n_pchunks;
    bd.n_qchunks = nqc;
    bd.grid_axes_max = op.o.grid_axes_max;
    bd.cell_multiple = op.o.cell_multiple;
    bd.cells_per_point = op.o.cells_per_point;
    bd.r_build = ix.r;
    bd.total_pts = ix.total_pts;
    bd.total_q = totq;

    const size_t o_ev = 256, o_ch = o_ev + sizeof(EventDev) * E;
    const size_t stage = o_ch + sizeof(Chunk) * std::max<size_t>(1, qch.size());
    // thread-local staging: this call synchronises after all its copies
    char *h = (char *)t_stage.ensure(stage);
    std::memcpy(h, &bd, sizeof(bd));
    std::memcpy(h + o_ev, evh.data(), sizeof(EventDev) * E);
    if (!qch.empty()) std::memcpy(h + o_ch, qch.data(), sizeof(Chunk) * qch.size());

    const int64_t tq1 = std::max<int64_t>(1, totq);
    DevBuf desc(stage, s);
    DevBuf hv(sizeof(Counters) + sizeof(int64_t) * (E + 1), s);
    DevBuf deg(sizeof(uint32_t) * tq1, s),
        offs(sizeof(int64_t) * (tq1 + 1), s), lofs(sizeof(int64_t) * (tq1 + 1), s),
        lrows(sizeof(uint32_t) * tq1, s), lat(sizeof(int64_t) * 2 * tq1, s),
        part(sizeof(uint64_t) * 2 * kScanBlocks, s),
        stash(sizeof(uint64_t) * tq1 * std::max(1, op.o.stash_cap), s),
        flist(sizeof(uint32_t) * std::max<int64_t>(1, (int64_t)nqc * (kChunkRows / op.o.queries_per_item)), s),
        outd(sizeof(OutDesc), s), lpt(sizeof(uint32_t) * lpt_words(E), s);
    DevBuf qs, qperm, qkey, qrank, sqkey, qcells;
    if (!selfq) {
        qs.reset(sizeof(float) * tq1 * Dp, s);
        qperm.reset(sizeof(int32_t) * tq1, s);
        qkey.reset(sizeof(uint32_t) * tq1, s);
        qrank.reset(sizeof(uint32_t) * tq1, s);
        sqkey.reset(sizeof(uint32_t) * tq1, s);
        qcells.reset(sizeof(uint32_t) * (ix.cells_cap + 1), s);
    }
    FRNN_HIP(hipMemcpyAsync(desc.get(), h, stage, hipMemcpyHostToDevice, s));

    Bufs b{};
    b.bd = desc.as<BatchDesc>();
    b.ev = reinterpret_cast<const EventDev *>(desc.as<char>() + o_ev);
    b.pchunks = reinterpret_cast<const Chunk *>(ix.desc.as<char>() + ix.o_ch);
    b.qchunks = reinterpret_cast<const Chunk *>(desc.as<char>() + o_ch);
    b.ctr = hv.as<Counters>();
    b.bases = reinterpret_cast<int64_t *>(hv.as<char>() + sizeof(Counters));
    b.grid = ix.grid.as<GridDesc>();
    b.runs = ix.runs.as<RunEntry>();
    b.cell_off = ix.cell_off.as<int64_t>();
    b.ext = ix.ext.as<uint32_t>();
    b.xs = ix.xs.as<float>();
    b.perm = ix.perm.as<int32_t>();
    b.skey = ix.skey.as<uint32_t>();
    b.cells = ix.cells.as<uint32_t>();
    b.qs = selfq ? ix.xs.as<float>() : qs.as<float>();
    b.qperm = selfq ? ix.perm.as<int32_t>() : qperm.as<int32_t>();
    b.qkey = qkey.as<uint32_t>();
    b.qrank = qrank.as<uint32_t>();
    b.sqkey = selfq ? ix.skey.as<uint32_t>() : sqkey.as<uint32_t>();
    b.qcells = selfq ? ix.cells.as<uint32_t>() : qcells.as<uint32_t>();
    b.deg = deg.as<uint32_t>();
    b.offs = offs.as<int64_t>();
    b.lofs = lofs.as<int64_t>();
    b.long_rows = lrows.as<uint32_t>();
    b.long_at = lat.as<int64_t>();
    b.stash = stash.as<uint64_t>();
    b.fill_list = flist.as<uint32_t>();
    b.lpt = lpt.as<uint32_t>();
    b.scan_part = part.as<uint64_t>();
    b.out = outd.as<OutDesc>();

    Knobs kn{};
    kn.r2 = r2_of(qa.r);
    kn.K = qa.K;
    kn.self_query = selfq;
    kn.exclude_self = excl;
    kn.window = op.o.queries_per_item;
    kn.cells_per_item = op.o.cells_per_item;
    kn.long_cap = op.o.row_cap_lds;
    kn.stash_cap = op.o.stash_cap;
    kn.fill_cap = (uint32_t)std::max<int64_t>(1, (int64_t)nqc * (kChunkRows / op.o.queries_per_item));
    kn.persistent = use_persistent(op.o, E, nqc, kn, D);
    const int qblocks = query_blocks(op.o, nqc, kn.persistent);

    LAUNCH("init", s, launch_init(b, s));
    if (!selfq) {
        LAUNCH("extent_q", s, launch_extent(b, nqc, E, true, ix.cells_cap + 1, s));
        LAUNCH("keys_q", s, launch_keys(b, nqc, true, s));
        LAUNCH("scan_cells_q", s, launch_scan_cells(b, ix.cells_cap, true, s));
        LAUNCH("scatter_q", s, launch_scatter(b, nqc, true, s));
    }
    if (kn.persistent) LAUNCH("lpt", s, launch_lpt(b, kn, s));
    LAUNCH("count", s, launch_count(b, kn, D, qblocks, s));
    LAUNCH("scan_rows", s, launch_scan_rows(b, kn, totq, s));

    // one synchronisation: counters, event bases and the build's status
    const size_t hvb = sizeof(Counters) + sizeof(int64_t) * (E + 1);
    char *p = (char *)t_back.ensure(hvb + sizeof(Counters));
    FRNN_HIP(hipMemcpyAsync(p, hv.get(), hvb, hipMemcpyDeviceToHost, s));
    // an index built without a synchronisation reports its status here
    if (!ix.status_checked)
        FRNN_HIP(hipMemcpyAsync(p + hvb, ix.ctr.get(), sizeof(Counters), hipMemcpyDeviceToHost, s));
    FRNN_HIP(hipStreamSynchronize(s));
    Counters c, cb{};
    std::memcpy(&c, p, sizeof(c));
    if (!ix.status_checked) std::memcpy(&cb, p + hvb, sizeof(cb));
    std::vector<int64_t> bases(E + 1);
    std::memcpy(bases.data(), p + sizeof(Counters), sizeof(int64_t) * (E + 1));
    if (cb.status & kStatusNonfinitePts) return fail(FRNN_ERR_NONFINITE, "non-finite coordinate in the points");
    if (c.status & kStatusNonfiniteQry) return fail(FRNN_ERR_NONFINITE, "non-finite coordinate in the queries");
    const int64_t nnz = (int64_t)c.nnz;
    if (bases[E] != nnz) return fail(FRNN_ERR_INTERNAL, "pair count mismatch");

    // exact-size output: per-event offsets | indices | dist2
    auto *own = new OutputOwner();
    const size_t b_off = sizeof(int64_t) * (totq + E);
    const size_t b_idx = (sizeof(int32_t) * nnz + 255) / 256 * 256;
    const size_t b_d2 = want_d2 ? sizeof(float) * nnz : 0;
    try {
        own->buf.reset(b_off + b_idx + (b_d2 + 15) / 16 * 16 + 16, s);
    } catch (...) {
        delete own;
        throw;
    }
    char *ob = own->buf.as<char>();
    own->status = reinterpret_cast<uint32_t *>(ob + b_off + b_idx + b_d2);
    DevBuf lkeys(sizeof(uint64_t) * std::max<uint64_t>(1, c.long_total), s);
    OutDesc od{reinterpret_cast<int64_t *>(ob), reinterpret_cast<int32_t *>(ob + b_off),
               want_d2 ? reinterpret_cast<float *>(ob + b_off + b_idx) : nullptr, lkeys.as<uint64_t>(),
               nnz, (int64_t)c.long_total, own->status};
    LAUNCH("set_out", s, launch_set_out(b, od, s));
    LAUNCH("short_rows", s, launch_short_rows(b, kn, nqc, s));
    const uint32_t n_fill = c.n_fill + c.n_fill_light;
    if (n_fill) LAUNCH("fill", s, launch_fill(b, kn, D, fill_blocks(n_fill), s));
    if (c.long_total) {
        LAUNCH("long_sort", s, launch_long_sort(b, kn, 1536, s));
        own->long_ran = true;
    }

    own->refs = E;
    for (int e = 0; e < E; ++e) {
        frnn_csr &o = outs[e];
        o.M = nq[e];
        o.nnz = bases[e + 1] - bases[e];
        o.offsets = od.offsets + qoff[e] + e;
        o.indices = od.indices + bases[e];
        o.dist2 = od.dist2 ? od.dist2 + bases[e] : nullptr;
        o.owner_ = own;
    }
    frnn_stats st{};
    st.candidates = (int64_t)c.candidates;
    st.work_items = c.n_groups;
    st.pairs = nnz;
    st.long_row_keys = (int64_t)c.long_total;
    st.stash_cap = op.o.stash_cap;
    if (stats) *stats = st;
    record_stats(st);
    return FRNN_OK;
}

}  // namespace frnn
