// Host side of the edge export (frnn_csr_edges, frnn_edges_release): count
// per row, the library's int64 row scan, one read-back of the edge count,
// an exact-size output allocation, fill.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstring>
#include <new>

#include "frnn_edges.h"
#include "frnn_launch.h"
#include "frnn_runtime.h"

using namespace frnn;

namespace {

thread_local Pinned &t_edge_back = *new Pinned();  // leaked: outlives every stream

frnn_status edges_impl(const frnn_csr *csr, int32_t mode, hipStream_t s, frnn_edges *out) {
    if (!csr || !out) return fail(FRNN_ERR_INVALID_ARG, "null csr or output");
    if (mode != FRNN_EDGES_UPPER && mode != FRNN_EDGES_SYMMETRIZED)
        return fail(FRNN_ERR_INVALID_ARG, "unknown edge mode");
    const int64_t M = csr->M;
    if (M < 0 || M >= ((int64_t)1 << 31)) return fail(FRNN_ERR_INVALID_ARG, "row count out of range");
    if (M == 0) return FRNN_OK;
    if (!csr->offsets || (csr->nnz > 0 && !csr->indices)) return fail(FRNN_ERR_INVALID_ARG, "csr without buffers");

    // scan descriptor: one event of M rows
    const size_t o_ev = 256, desc_bytes = o_ev + sizeof(EventDev);
    DevBuf desc(desc_bytes, s), hv(sizeof(Counters) + 2 * sizeof(int64_t), s), deg(sizeof(uint32_t) * M, s),
        offs(sizeof(int64_t) * (M + 1), s), lofs(sizeof(int64_t) * (M + 1), s),
        part(sizeof(uint64_t) * 2 * kScanBlocks, s);
    char *h = (char *)t_edge_back.ensure(desc_bytes + sizeof(Counters));
    std::memset(h, 0, desc_bytes);
    BatchDesc bd{};
    bd.E = 1;
    bd.total_q = M;
    std::memcpy(h, &bd, sizeof(bd));
    EventDev ev{};
    ev.n_q = M;
    std::memcpy(h + o_ev, &ev, sizeof(ev));
    FRNN_HIP(hipMemcpyAsync(desc.get(), h, desc_bytes, hipMemcpyHostToDevice, s));
    FRNN_HIP(hipMemsetAsync(hv.get(), 0, sizeof(Counters), s));

    Bufs b{};
    b.bd = desc.as<BatchDesc>();
    b.ev = reinterpret_cast<const EventDev *>(desc.as<char>() + o_ev);
    b.ctr = hv.as<Counters>();
    b.bases = reinterpret_cast<int64_t *>(hv.as<char>() + sizeof(Counters));
    b.deg = deg.as<uint32_t>();
    b.offs = offs.as<int64_t>();
    b.lofs = lofs.as<int64_t>();
    b.scan_part = part.as<uint64_t>();
    Knobs kn{};
    kn.K = 0;
    kn.long_cap = INT_MAX;
    kn.stash_cap = INT_MAX;  // the row scan's second sum stays zero

    EdgeArgs a{};
    a.off = csr->offsets;
    a.idx = csr->indices;
    a.M = M;
    a.mode = mode;
    a.deg = b.deg;
    a.eoff = b.offs;
    a.status = &b.ctr->status;
    LAUNCH("edge_count", s, launch_edge_count(a, s));
    LAUNCH("edge_scan", s, launch_scan_rows(b, kn, M, s));
    Counters c;
    FRNN_HIP(hipMemcpyAsync(h + desc_bytes, hv.get(), sizeof(Counters), hipMemcpyDeviceToHost, s));
    FRNN_HIP(hipStreamSynchronize(s));
    std::memcpy(&c, h + desc_bytes, sizeof(c));
    if (c.status) return fail(FRNN_ERR_INVALID_ARG, "csr index outside 0..M-1 (not a self-query CSR)");
    const int64_t n = (int64_t)c.nnz;
    if (n == 0) return FRNN_OK;

    auto *own = new OutputOwner();
    const size_t half = (sizeof(int32_t) * n + 255) / 256 * 256;
    try {
        own->buf.reset(2 * half, s);
    } catch (...) {
        delete own;
        throw;
    }
    a.src = own->buf.as<int32_t>();
    a.dst = reinterpret_cast<int32_t *>(own->buf.as<char>() + half);
    try {
        LAUNCH("edge_fill", s, launch_edge_fill(a, s));
    } catch (...) {
        delete own;
        throw;
    }
    own->refs = 1;
    out->n = n;
    out->src = a.src;
    out->dst = a.dst;
    out->owner_ = own;
    return FRNN_OK;
}

}  // namespace

extern "C" {

frnn_status frnn_csr_edges(const frnn_csr *csr, int32_t mode, void *stream, frnn_edges *out) {
    if (out) std::memset(out, 0, sizeof(*out));
    try {
        return edges_impl(csr, mode, (hipStream_t)stream, out);
    } catch (const Fail &e) {
        set_error(e.msg);
        return e.st;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return FRNN_ERR_OOM;
    } catch (const std::exception &e) {
        set_error(e.what());
        return FRNN_ERR_INTERNAL;
    } catch (...) {
        set_error("unknown internal error");
        return FRNN_ERR_INTERNAL;
    }
}

frnn_status frnn_edges_copy(const frnn_edges *e, int32_t *src, int32_t *dst, int32_t to_host, void *stream) {
    try {
        if (!e) return fail(FRNN_ERR_INVALID_ARG, "null edge list");
        hipStream_t s = (hipStream_t)stream;
        const hipMemcpyKind k = to_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
        if (e->n > 0) {
            if (src) FRNN_HIP(hipMemcpyAsync(src, e->src, sizeof(int32_t) * e->n, k, s));
            if (dst) FRNN_HIP(hipMemcpyAsync(dst, e->dst, sizeof(int32_t) * e->n, k, s));
        }
        if (to_host) FRNN_HIP(hipStreamSynchronize(s));
        return FRNN_OK;
    } catch (const Fail &f) {
        set_error(f.msg);
        return f.st;
    }
}

void frnn_edges_release(frnn_edges *e) {
    if (!e) return;
    try {
        auto *own = static_cast<OutputOwner *>(e->owner_);
        if (own && --own->refs == 0) delete own;
    } catch (...) {
    }
    std::memset(e, 0, sizeof(*e));
}

}  // extern "C"
