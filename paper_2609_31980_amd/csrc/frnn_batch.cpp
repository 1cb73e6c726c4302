// Batched pipeline, launched kernel by kernel or replayed as HIP graphs (see
// frnn_batch.h).
#include "frnn_batch.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <atomic>
#include <thread>
#include <chrono>

#include "frnn_launch.h"

namespace frnn {

// offset of the output descriptor in the descriptor block (after BatchDesc)
constexpr size_t kOutOff = 128;

static int64_t round_class(int64_t n) {
    // 2^k x {1, 1.25, 1.5, 1.75}, at least 4096
    int64_t p = 4096;
    if (n <= p) return p;
    while (p * 2 <= n) p *= 2;
    for (int q = 0; q <= 4; ++q) {
        int64_t c = p + p * q / 4;
        if (c >= n) return c;
    }
    return 2 * p;
}

static int next_pow2(int n) {
    int p = 1;
    while (p < n) p <<= 1;
    return p;
}

bool BatchContext::Shape::operator==(const Shape &x) const {
    return D == x.D && flags == x.flags && K == x.K && r == x.r && E_cap == x.E_cap &&
           pts_cap == x.pts_cap && q_cap == x.q_cap && cells_cap == x.cells_cap &&
           pch_cap == x.pch_cap && qch_cap == x.qch_cap && std::memcmp(&o, &x.o, sizeof(o)) == 0;
}

BatchContext::Shape BatchContext::shape_for(const frnn_event *ev, int E, int D, float r, int K,
                                            uint32_t flags, const Opts &o) {
    Shape sh{};
    sh.D = D;
    sh.flags = flags;
    sh.K = K;
    sh.r = r;
    sh.o = o.o;
    const bool selfq = flags & FRNN_SELF_QUERY;
    int64_t tp = 0, tq = 0;
    for (int e = 0; e < E; ++e) {
        tp += ev[e].N;
        tq += selfq ? ev[e].N : ev[e].M;
    }
    sh.E_cap = next_pow2(E);
    sh.pts_cap = round_class(tp);
    sh.q_cap = selfq ? sh.pts_cap : round_class(tq);
    sh.cells_cap = (int64_t)std::ceil((double)o.o.cells_per_point * (double)sh.pts_cap) + sh.E_cap;
    sh.pch_cap = (int)(sh.pts_cap / kChunkRows + sh.E_cap);
    sh.qch_cap = (int)(sh.q_cap / kChunkRows + sh.E_cap);
    return sh;
}

bool BatchContext::fits(const Shape &n) const {
    return sh_.D == n.D && sh_.flags == n.flags && sh_.K == n.K && sh_.r == n.r &&
           std::memcmp(&sh_.o, &n.o, sizeof(n.o)) == 0 && sh_.E_cap >= n.E_cap &&
           sh_.pts_cap >= n.pts_cap && sh_.q_cap >= n.q_cap && sh_.cells_cap >= n.cells_cap &&
           sh_.pch_cap >= n.pch_cap && sh_.qch_cap >= n.qch_cap;
}

namespace {
// Sizes of a context's device buffers, in the order the constructor makes
// them (0: not allocated).
struct BufSizes {
    size_t desc, hv, grid, runs, cell_off, ext, xs, perm, key, rank, skey, cells, qs, qperm, qkey, qrank, sqkey,
        qcells, deg, offs, lofs, lrows, lat, stash, flist, part, lpt;
    size_t o_ev, o_pc, o_qc;
};

BufSizes buf_sizes(const BatchContext::Shape &sh) {
    BufSizes z{};
    const int D = sh.D, Dp = (D + 3) & ~3, Ec = sh.E_cap;
    const bool selfq = sh.flags & FRNN_SELF_QUERY;
    z.o_ev = 256;
    z.o_pc = z.o_ev + sizeof(EventDev) * Ec;
    z.o_qc = z.o_pc + sizeof(Chunk) * sh.pch_cap;
    z.desc = (z.o_qc + sizeof(Chunk) * sh.qch_cap + 15) / 16 * 16;
    z.hv = (2 * sizeof(Counters) + sizeof(int64_t) * (Ec + 1) + 15) / 16 * 16;
    z.grid = sizeof(GridDesc) * Ec;
    z.runs = sizeof(RunEntry) * kRunsMax * Ec;
    z.cell_off = sizeof(int64_t) * (Ec + 1);
    z.ext = sizeof(uint32_t) * 2 * sh.pch_cap * D;  // per-chunk extent slots
    z.xs = sizeof(float) * sh.pts_cap * Dp;
    z.perm = z.key = z.rank = z.skey = sizeof(uint32_t) * sh.pts_cap;
    z.cells = sizeof(uint32_t) * (sh.cells_cap + 1);
    if (!selfq) {
        z.qs = sizeof(float) * sh.q_cap * Dp;
        z.qperm = z.qkey = z.qrank = z.sqkey = sizeof(uint32_t) * sh.q_cap;
        z.qcells = sizeof(uint32_t) * (sh.cells_cap + 1);
    }
    z.deg = sizeof(uint32_t) * sh.q_cap;
    z.offs = z.lofs = sizeof(int64_t) * (sh.q_cap + 1);
    z.lrows = sizeof(uint32_t) * sh.q_cap;
    z.lat = sizeof(int64_t) * 2 * sh.q_cap;
    z.stash = sizeof(uint64_t) * sh.q_cap * std::max(1, sh.o.stash_cap);
    z.flist = sizeof(uint32_t) * std::max<int64_t>(1, (int64_t)sh.qch_cap * (kChunkRows / sh.o.queries_per_item));
    z.part = sizeof(uint64_t) * 2 * kScanBlocks;
    z.lpt = sizeof(uint32_t) * lpt_words(Ec);
    return z;
}
}  // namespace

int64_t BatchContext::bytes_for(const Shape &sh) {
    const BufSizes z = buf_sizes(sh);
    int64_t t = 0;
    for (size_t v : {z.desc, z.hv, z.grid, z.runs, z.cell_off, z.ext, z.xs, z.perm, z.key, z.rank, z.skey, z.cells,
                     z.qs, z.qperm, z.qkey, z.qrank, z.sqkey, z.qcells, z.deg, z.offs, z.lofs, z.lrows, z.lat,
                     z.stash, z.flist, z.part, z.lpt})
        if (v) t += Pool::class_bytes(v);
    return t;
}

int64_t BatchContext::device_bytes() const {
    int64_t t = 0;
    for (const DevBuf *d : {&desc, &hv, &grid, &cell_off, &ext, &xs, &perm, &key, &rank, &skey, &cells, &qs, &qperm,
                            &qkey, &qrank, &sqkey, &qcells, &runs, &deg, &offs, &lofs, &lrows, &lat, &stash, &flist,
                            &part, &lpt, &lk_})
        if (d->get()) t += Pool::class_bytes(d->bytes());
    return t;
}

BatchContext::BatchContext(const Shape &sh, hipStream_t s) : sh_(sh) {
    graphs_enabled = sh.o.graphs != 0;
    const int D = sh.D;
    Dp_ = (D + 3) & ~3;
    const bool selfq = sh.flags & FRNN_SELF_QUERY;
    const int Ec = sh.E_cap;
    // descriptors (one block, one copy per batch): batch | output | events |
    // point chunks | query chunks, each region sized for the capacity
    static_assert(sizeof(BatchDesc) <= kOutOff && kOutOff + sizeof(OutDesc) <= 256, "descriptor head");
    const BufSizes z = buf_sizes(sh);
    o_ev_ = z.o_ev;
    o_pc_ = z.o_pc;
    o_qc_ = z.o_qc;
    stage_cap_ = z.desc;
    desc.reset(stage_cap_, s);
    // the host writes each batch's descriptors here and the first kernel of
    // phase A reads them (coherent: no stale copy in a GPU cache)
    stage_.reset(stage_cap_);
    // read-back block: query counters | build counters | event bases
    hv.reset(z.hv, s);
    // its host-mapped copy, written by the last kernel of phase A (coherent:
    // the host reads it after the stream's mark, no copy command needed)
    back_.reset(z.hv + 16);  // and the flag word after it
    hv16_ = z.hv / 16;
    grid.reset(z.grid, s);
    runs.reset(z.runs, s);
    cell_off.reset(z.cell_off, s);
    ext.reset(z.ext, s);
    xs.reset(z.xs, s);
    perm.reset(z.perm, s);
    key.reset(z.key, s);
    rank.reset(z.rank, s);
    skey.reset(z.skey, s);
    cells.reset(z.cells, s);
    if (!selfq) {
        qs.reset(z.qs, s);
        qperm.reset(z.qperm, s);
        qkey.reset(z.qkey, s);
        qrank.reset(z.qrank, s);
        sqkey.reset(z.sqkey, s);
        qcells.reset(z.qcells, s);
    }
    deg.reset(z.deg, s);
    offs.reset(z.offs, s);
    lofs.reset(z.lofs, s);
    lrows.reset(z.lrows, s);
    lat.reset(z.lat, s);
    stash.reset(z.stash, s);
    const int64_t fill_cap = (int64_t)(z.flist / sizeof(uint32_t));
    flist.reset(z.flist, s);
    part.reset(z.part, s);
    lpt.reset(z.lpt, s);

    Bufs b{};
    b.bd = desc.as<BatchDesc>();
    b.ev = reinterpret_cast<const EventDev *>(desc.as<char>() + o_ev_);
    b.pchunks = reinterpret_cast<const Chunk *>(desc.as<char>() + o_pc_);
    b.qchunks = reinterpret_cast<const Chunk *>(desc.as<char>() + o_qc_);
    b.grid = grid.as<GridDesc>();
    b.runs = runs.as<RunEntry>();
    b.cell_off = cell_off.as<int64_t>();
    b.ext = ext.as<uint32_t>();
    b.xs = xs.as<float>();
    b.perm = perm.as<int32_t>();
    b.key = key.as<uint32_t>();
    b.rank = rank.as<uint32_t>();
    b.skey = skey.as<uint32_t>();
    b.cells = cells.as<uint32_t>();
    b.qs = selfq ? xs.as<float>() : qs.as<float>();
    b.qperm = selfq ? perm.as<int32_t>() : qperm.as<int32_t>();
    b.qkey = qkey.as<uint32_t>();
    b.qrank = qrank.as<uint32_t>();
    b.sqkey = selfq ? skey.as<uint32_t>() : sqkey.as<uint32_t>();
    b.qcells = selfq ? cells.as<uint32_t>() : qcells.as<uint32_t>();
    b.deg = deg.as<uint32_t>();
    b.offs = offs.as<int64_t>();
    b.lofs = lofs.as<int64_t>();
    b.long_rows = lrows.as<uint32_t>();
    b.long_at = lat.as<int64_t>();
    b.stash = stash.as<uint64_t>();
    b.fill_list = flist.as<uint32_t>();
    b.lpt = lpt.as<uint32_t>();
    b.scan_part = part.as<uint64_t>();
    b.out = reinterpret_cast<OutDesc *>(desc.as<char>() + kOutOff);
    b.bases = reinterpret_cast<int64_t *>(hv.as<char>() + 2 * sizeof(Counters));
    bb_ = b;
    bb_.ctr = reinterpret_cast<Counters *>(hv.as<char>() + sizeof(Counters));
    bq_ = b;
    bq_.ctr = hv.as<Counters>();

    kn_.r2 = r2_of(sh.r);
    kn_.K = sh.K;
    kn_.self_query = selfq;
    kn_.exclude_self = selfq && (sh.flags & FRNN_EXCLUDE_SELF);
    kn_.window = sh.o.queries_per_item;
    kn_.cells_per_item = sh.o.cells_per_item;
    kn_.long_cap = sh.o.row_cap_lds;
    kn_.stash_cap = sh.o.stash_cap;
    kn_.fill_cap = (uint32_t)fill_cap;
    kn_.persistent = use_persistent(sh.o, Ec, sh.qch_cap, kn_, D);
    FRNN_HIP(hipEventCreateWithFlags(&done_, hipEventDisableTiming));
}

void BatchContext::retarget(hipStream_t s) {
    DevBuf *all[] = {&desc, &hv, &grid, &cell_off, &ext,
                     &xs, &perm, &key, &rank, &skey, &cells, &qs, &qperm, &qkey, &qrank, &sqkey,
                     &qcells, &runs, &deg, &offs, &lofs, &lrows, &lat, &stash, &flist, &part, &lpt, &lk_};
    for (DevBuf *d : all) d->set_stream(s);
}

void BatchContext::retire() {
    DevBuf *all[] = {&desc, &hv, &grid, &cell_off, &ext,
                     &xs, &perm, &key, &rank, &skey, &cells, &qs, &qperm, &qkey, &qrank, &sqkey,
                     &qcells, &runs, &deg, &offs, &lofs, &lrows, &lat, &stash, &flist, &part, &lpt, &lk_};
    for (DevBuf *d : all) d->mark_complete();
}

uint64_t *BatchContext::long_scratch(int64_t n, hipStream_t s) {
    const size_t need = sizeof(uint64_t) * (size_t)std::max<int64_t>(1, n);
    if (lk_.bytes() < need) lk_.reset(need, s);
    return lk_.as<uint64_t>();
}

BatchContext::~BatchContext() {
    for (hipGraphExec_t ge : {ga_, gbs_, gbl_, gab_, gabl_})
        if (ge) (void)hipGraphExecDestroy(ge);
    for (hipGraph_t g : {gra_, grbs_, grbl_, grab_, grabl_})
        if (g) (void)hipGraphDestroy(g);
    if (done_) (void)hipEventDestroy(done_);
}

void BatchContext::set_inputs(const frnn_event *ev, int E, hipStream_t s) {
    prepare(ev, E);
    upload(s, nullptr);
}

void BatchContext::prepare(const frnn_event *ev, int E) {
    const bool selfq = sh_.flags & FRNN_SELF_QUERY;
    E_ = E;
    std::vector<int64_t> np(E), poff(E);
    nq_.assign(E, 0);
    qoff_.assign(E, 0);
    int64_t tp = 0, tq = 0;
    std::vector<EventDev> evh(E);
    for (int e = 0; e < E; ++e) {
        np[e] = ev[e].N;
        poff[e] = tp;
        nq_[e] = selfq ? ev[e].N : ev[e].M;
        qoff_[e] = tq;
        double c = std::floor((double)sh_.o.cells_per_point * (double)std::max<int64_t>(np[e], 1));
        c = std::max(1.0, std::min(c, (double)(1 << 30)));
        evh[e] = EventDev{ev[e].points, selfq ? nullptr : ev[e].queries, np[e], tp, nq_[e], tq, (int64_t)c};
        tp += np[e];
        tq += nq_[e];
    }
    totq_ = tq;
    std::vector<Chunk> pc, qc;
    for (int e = 0; e < E; ++e) {
        for (int64_t r = 0; r < np[e]; r += kChunkRows)
            pc.push_back(Chunk{e, 0, poff[e] + r, poff[e] + std::min<int64_t>(np[e], r + kChunkRows)});
        for (int64_t r = 0; r < nq_[e]; r += kChunkRows)
            qc.push_back(Chunk{e, 0, qoff_[e] + r, qoff_[e] + std::min<int64_t>(nq_[e], r + kChunkRows)});
    }
    if ((int64_t)pc.size() > sh_.pch_cap || (int64_t)qc.size() > sh_.qch_cap || tp > sh_.pts_cap ||
        tq > sh_.q_cap || E > sh_.E_cap)
        throw Fail{FRNN_ERR_INTERNAL, "batch does not fit its context"};
    BatchDesc bd{};
    bd.run_id = ++run_seq_;
    bd.E = E;
    bd.D = sh_.D;
    bd.Dp = Dp_;
    bd.n_pchunks = (int)pc.size();
    bd.n_qchunks = (int)qc.size();
    bd.grid_axes_max = sh_.o.grid_axes_max;
    bd.cell_multiple = sh_.o.cell_multiple;
    bd.cells_per_point = sh_.o.cells_per_point;
    bd.r_build = sh_.r;
    bd.total_pts = tp;
    bd.total_q = tq;
    // the previous batch's phase A has read the stage: its counts were read
    // back before this context was handed out again
    char *h = stage_.host();
    std::memset(h, 0, o_ev_);
    std::memcpy(h, &bd, sizeof(bd));
    std::memcpy(h + o_ev_, evh.data(), sizeof(EventDev) * E);
    if (!pc.empty()) std::memcpy(h + o_pc_, pc.data(), sizeof(Chunk) * pc.size());
    if (!qc.empty()) std::memcpy(h + o_qc_, qc.data(), sizeof(Chunk) * qc.size());
}

void BatchContext::upload(hipStream_t, const OutDesc *od) {
    if (od) std::memcpy(stage_.host() + kOutOff, od, sizeof(OutDesc));
}

Publish BatchContext::publish_args() {
    return Publish{hv.get(), back_.dev(), (int64_t)hv16_, reinterpret_cast<uint32_t *>(back_.dev()) + 4 * hv16_};
}

void BatchContext::launch_a(hipStream_t s, bool publish) {
    const bool selfq = sh_.flags & FRNN_SELF_QUERY;
    const int D = sh_.D;
    // build and query counters in one launch
    LAUNCH("init", s, launch_init(bb_, s, bq_.ctr, stage_.dev(), desc.get(), (int64_t)stage_cap_));
    LAUNCH("extent", s, launch_extent(bb_, sh_.pch_cap, sh_.E_cap, false, sh_.cells_cap + 1, s));
    // the persistent count pass's work order is built by the plan's last block
    LAUNCH("plan", s, launch_plan(bb_, sh_.E_cap, s, kn_.persistent ? &kn_ : nullptr));
    LAUNCH("keys", s, launch_keys(bb_, sh_.pch_cap, false, s));
    LAUNCH("scan_cells", s, launch_scan_cells(bb_, sh_.cells_cap, false, s));
    LAUNCH("scatter", s, launch_scatter(bb_, sh_.pch_cap, false, s));
    if (!selfq) {
        LAUNCH("extent_q", s, launch_extent(bq_, sh_.qch_cap, sh_.E_cap, true, sh_.cells_cap + 1, s));
        LAUNCH("keys_q", s, launch_keys(bq_, sh_.qch_cap, true, s));
        LAUNCH("scan_cells_q", s, launch_scan_cells(bq_, sh_.cells_cap, true, s));
        LAUNCH("scatter_q", s, launch_scatter(bq_, sh_.qch_cap, true, s));
    }
    LAUNCH("count", s, launch_count(bq_, kn_, D, query_blocks(sh_.o, sh_.qch_cap, kn_.persistent), s));
    LAUNCH("scan_rows", s, launch_scan_rows(bq_, kn_, sh_.q_cap, s));
    if (publish) LAUNCH("publish", s, launch_publish(publish_args(), s));
}

// (the host reads the counts as soon as they are published, while the
// fill runs)
// (the short-row pass, launched right after the row scan, performs the
// read-back in its first block: one launch less)
void BatchContext::launch_ab(hipStream_t s) {
    launch_a(s, false);
    launch_b_short(s, true);
}

void BatchContext::launch_abl(hipStream_t s) {
    launch_a(s, false);
    launch_b_short(s, true);
    launch_b_long(s);
}

void BatchContext::launch_b_short(hipStream_t s, bool publish) {
    const Publish p = publish_args();
    LAUNCH("short_rows", s, launch_short_rows(bq_, kn_, sh_.qch_cap, s, publish ? &p : nullptr));
}

void BatchContext::launch_b_long(hipStream_t s) {
    LAUNCH("fill", s, launch_fill(bq_, kn_, sh_.D, fill_blocks(sh_.qch_cap * (kChunkRows / sh_.o.queries_per_item)), s));
    LAUNCH("long_sort", s, launch_long_sort(bq_, kn_, 1536, s));
}

// Builds the graph of fn's launches node by node (no stream capture) and
// instantiates it; false on any failure (the caller then launches eagerly).
static bool record(hipStream_t s, hipGraph_t *g, hipGraphExec_t *ge, void (*fn)(void *, hipStream_t), void *arg) {
    GraphRecorder rec;
    if (hipGraphCreate(&rec.graph, 0) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    set_recorder(&rec);
    set_capturing(true);
    bool ok = true;
    try {
        fn(arg, s);
    } catch (...) {
        ok = false;
    }
    set_capturing(false);
    set_recorder(nullptr);
    if (!ok || rec.err != hipSuccess || hipGraphInstantiate(ge, rec.graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipGraphDestroy(rec.graph);
        *ge = nullptr;
        return false;
    }
    *g = rec.graph;
    return true;
}

// Replays graph *ge, recording it from fn first; false when graphs are off
// or recording fails (the caller then launches eagerly).
bool BatchContext::replay(hipGraphExec_t *ge, hipGraph_t *g, void (*fn)(void *, hipStream_t), hipStream_t s) {
    if (!graphs_enabled || prof_enabled()) return false;
    if (!*ge && !record(s, g, ge, fn, this)) {
        graphs_enabled = false;
        return false;
    }
    FRNN_HIP(hipGraphLaunch(*ge, s));
    ++replays;
    return true;
}

void BatchContext::phase_a(hipStream_t s) {
    if (!replay(&ga_, &gra_, [](void *p, hipStream_t st) { ((BatchContext *)p)->launch_a(st); }, s))
        launch_a(s);
}

BatchCounts BatchContext::read_counts(hipStream_t s) {
    fetch_counts(s);
    return wait_counts();
}

void BatchContext::phase_ab(bool with_long, hipStream_t s) {
    last_s_ = s;
    if (with_long) {
        if (!replay(&gabl_, &grabl_, [](void *p, hipStream_t st) { ((BatchContext *)p)->launch_abl(st); }, s))
            launch_abl(s);
    } else {
        if (!replay(&gab_, &grab_, [](void *p, hipStream_t st) { ((BatchContext *)p)->launch_ab(st); }, s))
            launch_ab(s);
    }
}

void BatchContext::fetch_counts(hipStream_t s) { last_s_ = s; }

// Waits until the read-back block carries this run's number: polls the
// flag word (the last store of phase A) for a while, then also asks the
// stream, which fails on a device error and goes idle without the flag
// only if the run did not publish.
BatchCounts BatchContext::wait_counts() {
    const volatile uint32_t *flag = reinterpret_cast<const volatile uint32_t *>(back_.host() + 16 * hv16_);
    const auto t0 = std::chrono::steady_clock::now();
    for (uint32_t n = 0; *flag != run_seq_; ++n) {
        if ((n & 63u) != 63u || std::chrono::steady_clock::now() - t0 < std::chrono::milliseconds(1)) continue;
        const hipError_t q = hipStreamQuery(last_s_);
        if (*flag == run_seq_) break;
        if (q == hipSuccess) throw Fail{FRNN_ERR_INTERNAL, "the run finished without publishing its counters"};
        if (q != hipErrorNotReady) {
            (void)hipGetLastError();
            throw Fail{FRNN_ERR_HIP, std::string("count pass: ") + hipGetErrorString(q)};
        }
        std::this_thread::yield();
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    const char *p = back_.host();
    BatchCounts c;
    std::memcpy(&c.ctr, p, sizeof(Counters));
    Counters cb;
    std::memcpy(&cb, p + sizeof(Counters), sizeof(Counters));
    c.build_status = cb.status;
    c.bases.resize(E_ + 1);
    std::memcpy(c.bases.data(), p + 2 * sizeof(Counters), sizeof(int64_t) * (E_ + 1));
    return c;
}

void BatchContext::phase_b(const OutDesc &od, bool long_rows, hipStream_t s) {
    LAUNCH("set_out", s, launch_set_out(bq_, od, s));
    phase_b_short(s);
    if (long_rows) phase_b_long(s);
}

void BatchContext::phase_b_short(hipStream_t s) {
    if (!replay(&gbs_, &grbs_, [](void *p, hipStream_t st) { ((BatchContext *)p)->launch_b_short(st); }, s))
        launch_b_short(s);
}

void BatchContext::phase_b_long(hipStream_t s) {
    if (!replay(&gbl_, &grbl_, [](void *p, hipStream_t st) { ((BatchContext *)p)->launch_b_long(st); }, s))
        launch_b_long(s);
}

bool BatchContext::guess(int64_t *pairs, int64_t *long_keys) const {
    if (seen_pairs_ < 0) return false;
    // a quarter more than the previous run (batches of one class differ in
    // size by less than that), plus a floor for tiny outputs
    *pairs = seen_pairs_ + seen_pairs_ / 4 + 4096;
    *long_keys = seen_long_ + seen_long_ / 4 + 4096;
    return true;
}

void BatchContext::learn(const BatchCounts &c) {
    seen_pairs_ = (int64_t)c.ctr.nnz;
    seen_long_ = (int64_t)c.ctr.long_total;
}

// ---------------------------------------------------------------- cache
namespace {
struct Cached {
    std::unique_ptr<BatchContext> ctx;
    hipStream_t stream;  // stream of its last run (its done event is recorded there)
};
std::mutex g_cache_mu;
// never destroyed: no HIP call may run from a static destructor at exit
std::vector<Cached> &g_cache = *new std::vector<Cached>();
constexpr size_t kCacheMax = 8;
}  // namespace

std::unique_ptr<BatchContext> acquire_context(const BatchContext::Shape &need, hipStream_t s) {
    {
        std::lock_guard<std::mutex> g(g_cache_mu);
        int best = -1;
        for (size_t i = 0; i < g_cache.size(); ++i) {
            if (!g_cache[i].ctx->fits(need)) continue;
            if (best < 0 || g_cache[i].ctx->shape().pts_cap < g_cache[best].ctx->shape().pts_cap) best = (int)i;
        }
        if (best >= 0) {
            Cached c = std::move(g_cache[best]);
            g_cache.erase(g_cache.begin() + best);
            // the previous run of this context may still be on another stream:
            // wait for it on the host (no cross-stream dependency is left
            // behind in either stream)
            if (c.stream != s) FRNN_HIP(hipEventSynchronize(c.ctx->done()));
            c.ctx->retarget(s);
            return std::move(c.ctx);
        }
    }
    return std::unique_ptr<BatchContext>(new BatchContext(need, s));
}

void return_context(std::unique_ptr<BatchContext> ctx, hipStream_t s) {
    if (hipEventRecord(ctx->done(), s) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipStreamSynchronize(s);
        ctx->retire();
        return;  // drop the context
    }
    std::lock_guard<std::mutex> g(g_cache_mu);
    g_cache.push_back(Cached{std::move(ctx), s});
    if (g_cache.size() > kCacheMax) {
        Cached old = std::move(g_cache.front());
        g_cache.erase(g_cache.begin());
        (void)hipEventSynchronize(old.ctx->done());
        old.ctx->retire();  // its work is done; its stream may be gone
    }
}

int64_t output_bytes(const BatchContext &ctx, int64_t pairs, int64_t long_keys, bool want_d2) {
    const size_t b_off = sizeof(int64_t) * (ctx.total_q() + ctx.E());
    const size_t b_idx = (sizeof(int32_t) * pairs + 255) / 256 * 256;
    const size_t b_d2 = want_d2 ? (sizeof(float) * pairs + 15) / 16 * 16 : 0;
    return Pool::class_bytes(b_off + b_idx + b_d2 + 16) +
           Pool::class_bytes(sizeof(uint64_t) * std::max<int64_t>(1, long_keys));
}

BatchOutput alloc_output(const BatchContext &ctx, int64_t pairs, int64_t long_keys, bool want_d2,
                         hipStream_t s, uint64_t *long_scratch) {
    BatchOutput bo;
    const int E = ctx.E();
    const size_t b_off = sizeof(int64_t) * (ctx.total_q() + E);
    const size_t b_idx = (sizeof(int32_t) * pairs + 255) / 256 * 256;
    const size_t b_d2 = want_d2 ? (sizeof(float) * pairs + 15) / 16 * 16 : 0;
    std::unique_ptr<OutputOwner> own(new OutputOwner());
    own->buf.reset(b_off + b_idx + b_d2 + 16, s);
    own->status = reinterpret_cast<uint32_t *>(own->buf.as<char>() + b_off + b_idx + b_d2);
    if (!long_scratch) {
        bo.long_keys.reset(sizeof(uint64_t) * std::max<int64_t>(1, long_keys), s);
        long_scratch = bo.long_keys.as<uint64_t>();
    }
    char *ob = own->buf.as<char>();
    bo.od = OutDesc{reinterpret_cast<int64_t *>(ob), reinterpret_cast<int32_t *>(ob + b_off),
                    want_d2 ? reinterpret_cast<float *>(ob + b_off + b_idx) : nullptr,
                    long_scratch, pairs, long_keys, own->status};
    bo.own = own.release();
    return bo;
}

BatchOutput alloc_output(const BatchContext &ctx, const BatchCounts &c, bool want_d2, hipStream_t s) {
    return alloc_output(ctx, (int64_t)c.ctr.nnz, (int64_t)c.ctr.long_total, want_d2, s);
}

void hand_out(const BatchContext &ctx, const BatchCounts &c, BatchOutput &bo, frnn_csr *outs) {
    const int E = ctx.E();
    bo.own->refs = E;
    for (int e = 0; e < E; ++e) {
        frnn_csr &o = outs[e];
        o.M = ctx.n_q()[e];
        o.nnz = c.bases[e + 1] - c.bases[e];
        o.offsets = bo.od.offsets + ctx.q_off()[e] + e;
        o.indices = bo.od.indices + c.bases[e];
        o.dist2 = bo.od.dist2 ? bo.od.dist2 + c.bases[e] : nullptr;
        o.owner_ = bo.own;
    }
    bo.own = nullptr;
}

// Dense-row adaptation (frnn_opts.adapt): capacity classes, keyed by their
// shape under the options as given, whose run had long rows.  Their later
// batches use a larger stash, one cell per work item and windows of 16
// queries (every setting gives the same output; measured faster on inputs
// whose rows outgrow the default stash, slower on short rows).
namespace {
std::mutex g_dense_mu;
std::vector<BatchContext::Shape> g_dense;
constexpr size_t kDenseMax = 64;          // classes remembered (oldest dropped)
constexpr int64_t kDenseStashMax = 4ll << 30;  // bytes of stash a class may take

bool adapt_eligible(const Opts &o) {
    frnn_opts d;
    frnn_opts_default(&d);
    return o.o.adapt && o.o.stash_cap == d.stash_cap && o.o.cells_per_item == d.cells_per_item &&
           o.o.queries_per_item == d.queries_per_item;
}

bool is_dense(const BatchContext::Shape &sh) {
    std::lock_guard<std::mutex> g(g_dense_mu);
    return std::find(g_dense.begin(), g_dense.end(), sh) != g_dense.end();
}

void mark_dense(const BatchContext::Shape &sh) {
    std::lock_guard<std::mutex> g(g_dense_mu);
    if (std::find(g_dense.begin(), g_dense.end(), sh) != g_dense.end()) return;
    if (g_dense.size() >= kDenseMax) g_dense.erase(g_dense.begin());
    g_dense.push_back(sh);
}

Opts dense_opts(const Opts &o, int64_t q_cap) {
    Opts a = o;
    a.o.stash_cap = 64;
    for (int sc : {256, 128})
        if (q_cap * sc * (int64_t)sizeof(uint64_t) <= kDenseStashMax) {
            a.o.stash_cap = sc;
            break;
        }
    a.o.cells_per_item = 1;
    a.o.queries_per_item = 16;
    return a;
}
}  // namespace

frnn_status batch_run(const frnn_event *ev, int E, int D, float r, int K, uint32_t flags,
                      const Opts &o, hipStream_t s, frnn_csr *outs) {
    const BatchContext::Shape base = BatchContext::shape_for(ev, E, D, r, K, flags, o);
    const bool eligible = adapt_eligible(o);
    const bool adapted = eligible && is_dense(base);
    const BatchContext::Shape need =
        adapted ? BatchContext::shape_for(ev, E, D, r, K, flags, dense_opts(o, base.q_cap)) : base;
    std::unique_ptr<BatchContext> ctx = acquire_context(need, s);
    const bool want_d2 = flags & FRNN_WANT_DIST2;
    frnn_status st = FRNN_OK;
    try {
        ctx->prepare(ev, E);
        int64_t cap_pairs = 0, cap_long = 0;
        BatchOutput bo;
        const bool spec = ctx->guess(&cap_pairs, &cap_long);
        if (spec) {
            bo = alloc_output(*ctx, cap_pairs, cap_long, want_d2, s, ctx->long_scratch(cap_long, s));
            ctx->upload(s, &bo.od);
        } else {
            ctx->upload(s, nullptr);
        }
        // the output owner is freed here unless handed out
        std::unique_ptr<OutputOwner> own(bo.own);
        bo.own = nullptr;
        // with a guessed output the fill is launched with the count
        // (its long-row part only when the previous run had long rows; else
        // after the counts, if needed: the two parts write different rows);
        // a fill whose output turns out too small writes nothing
        bool long_queued = false;
        if (spec) {
            long_queued = ctx->expect_long();
            ctx->phase_ab(long_queued, s);
            if (long_queued) own->long_ran = true;
        } else {
            ctx->phase_a(s);
        }
        ctx->fetch_counts(s);
        BatchCounts c = ctx->wait_counts();
        if (c.build_status & kStatusNonfinitePts) {
            st = fail(FRNN_ERR_NONFINITE, "non-finite coordinate in the points");
        } else if (c.ctr.status & kStatusNonfiniteQry) {
            st = fail(FRNN_ERR_NONFINITE, "non-finite coordinate in the queries");
        } else if (c.bases[E] != (int64_t)c.ctr.nnz) {
            st = fail(FRNN_ERR_INTERNAL, "pair count mismatch");
        } else {
            ctx->learn(c);
            const bool long_rows = c.ctr.long_total > 0;
            // long-row keys at least an eighth of the stash slots: the
            // class's later batches take the dense-row setting
            if (eligible && !adapted &&
                (int64_t)c.ctr.long_total * 8 >= ctx->total_q() * (int64_t)std::max(1, need.o.stash_cap))
                mark_dense(base);
            if (!spec || (int64_t)c.ctr.nnz > cap_pairs || (int64_t)c.ctr.long_total > cap_long) {
                // exact size; a speculative fill (if any) wrote nothing
                own.reset();
                bo = alloc_output(*ctx, c, want_d2, s);
                own.reset(bo.own);
                bo.own = nullptr;
                ctx->phase_b(bo.od, long_rows, s);
                own->long_ran = long_rows;
            } else if (long_rows && !long_queued) {
                ctx->phase_b_long(s);
                own->long_ran = true;
            }
            bo.own = own.release();
            hand_out(*ctx, c, bo, outs);
            frnn_stats stt{};
            stt.candidates = (int64_t)c.ctr.candidates;
            stt.work_items = c.ctr.n_groups;
            stt.pairs = (int64_t)c.ctr.nnz;
            stt.long_row_keys = (int64_t)c.ctr.long_total;
            stt.stash_cap = need.o.stash_cap;
            stt.adapted = adapted ? 1 : 0;
            record_stats(stt);
        }
    } catch (...) {
        return_context(std::move(ctx), s);
        throw;
    }
    return_context(std::move(ctx), s);
    return st;
}

}  // namespace frnn
