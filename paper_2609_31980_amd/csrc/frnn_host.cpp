// Synchronous host-array interface (frnn_query_host): pinned staging in
// chunks (host copy of chunk k+1 overlaps the DMA of chunk k), the batched
// device path on a library stream, compact host CSR in pinned memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>

#include "frnn_runtime.h"

using namespace frnn;

namespace {

constexpr size_t kStageBytes = (size_t)8 << 20;  // per staging buffer

// Per host thread: a stream and two pinned staging buffers with their events
// (leaked on purpose: they must outlive every call made from the thread).
struct HostStage {
    hipStream_t s = nullptr;
    void *buf[2] = {nullptr, nullptr};
    hipEvent_t done[2] = {nullptr, nullptr};
    void init() {
        if (s) return;
        FRNN_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        for (int k = 0; k < 2; ++k) {
            FRNN_HIP(hipHostMalloc(&buf[k], kStageBytes, hipHostMallocDefault));
            FRNN_HIP(hipEventCreateWithFlags(&done[k], hipEventDisableTiming));
            FRNN_HIP(hipEventRecord(done[k], s));
        }
    }
};
thread_local HostStage &t_host = *new HostStage();

// Copy n bytes from pageable host memory to the device through the staging
// ring; returns once every chunk is enqueued (the caller's later work on the
// same stream is ordered after the copies).
void stage_to_device(void *dst, const void *src, size_t n) {
    HostStage &h = t_host;
    size_t off = 0;
    int k = 0;
    while (off < n) {
        const size_t len = std::min(kStageBytes, n - off);
        FRNN_HIP(hipEventSynchronize(h.done[k]));  // the DMA that last used this buffer is over
        std::memcpy(h.buf[k], (const char *)src + off, len);
        FRNN_HIP(hipMemcpyAsync((char *)dst + off, h.buf[k], len, hipMemcpyHostToDevice, h.s));
        FRNN_HIP(hipEventRecord(h.done[k], h.s));
        off += len;
        k ^= 1;
    }
}

struct HostOwner {
    void *p = nullptr;
    ~HostOwner() {
        if (p) (void)hipHostFree(p);
    }
};

frnn_status host_impl(const float *points, int64_t N, const float *queries, int64_t M, int32_t D, float r,
                      int32_t K, uint32_t flags, const frnn_opts *opts, frnn_host_csr *out) {
    if (!out) return fail(FRNN_ERR_INVALID_ARG, "null output");
    if (D < 1 || D > kDMax) return fail(FRNN_ERR_INVALID_ARG, "D must be in 1..32");
    if (N < 0 || M < 0) return fail(FRNN_ERR_INVALID_ARG, "negative size");
    const bool selfq = flags & FRNN_SELF_QUERY;
    if (selfq && (queries || M != N)) return fail(FRNN_ERR_INVALID_ARG, "self-query: no query array and M == N");
    if ((N > 0 && !points) || (!selfq && M > 0 && !queries)) return fail(FRNN_ERR_INVALID_ARG, "null input");
    HostStage &h = t_host;
    h.init();
    hipStream_t s = h.s;
    DevBuf dp(sizeof(float) * std::max<int64_t>(1, N * D), s), dq;
    if (N > 0) stage_to_device(dp.get(), points, sizeof(float) * N * D);
    if (!selfq) {
        dq.reset(sizeof(float) * std::max<int64_t>(1, M * D), s);
        if (M > 0) stage_to_device(dq.get(), queries, sizeof(float) * M * D);
    }
    frnn_event ev{};
    ev.points = dp.as<float>();
    ev.N = N;
    ev.queries = selfq ? nullptr : dq.as<float>();
    ev.M = selfq ? 0 : M;
    frnn_csr c{};
    frnn_status st = frnn_query_batch(&ev, 1, D, r, K, flags, opts, s, &c);
    if (st) return st;  // the error text is already set
    // exact-size pinned output: offsets | indices | dist2
    auto *own = new HostOwner();
    const size_t b_off = sizeof(int64_t) * (c.M + 1);
    const size_t b_idx = (sizeof(int32_t) * c.nnz + 63) / 64 * 64;
    const size_t b_d2 = c.dist2 ? sizeof(float) * c.nnz : 0;
    if (hipHostMalloc(&own->p, b_off + b_idx + b_d2, hipHostMallocDefault) != hipSuccess) {
        own->p = nullptr;
        delete own;
        frnn_csr_release(&c);
        return fail(FRNN_ERR_OOM, "pinned host allocation failed");
    }
    char *p = (char *)own->p;
    st = frnn_csr_copy(&c, (int64_t *)p, c.nnz ? (int32_t *)(p + b_off) : nullptr,
                       c.dist2 && c.nnz ? (float *)(p + b_off + b_idx) : nullptr, 1, s);
    const int64_t rows = c.M, pairs = c.nnz;
    frnn_csr_release(&c);  // zeroes c
    if (st) {
        delete own;
        return st;
    }
    out->M = rows;
    out->nnz = pairs;
    out->offsets = (int64_t *)p;
    out->indices = (int32_t *)(p + b_off);
    out->dist2 = b_d2 ? (float *)(p + b_off + b_idx) : nullptr;
    out->owner_ = own;
    return FRNN_OK;
}

}  // namespace

extern "C" {

frnn_status frnn_query_host(const float *points, int64_t N, const float *queries, int64_t M, int32_t D,
                            float r, int32_t K, uint32_t flags, const frnn_opts *opts,
                            frnn_host_csr *out) {
    if (out) std::memset(out, 0, sizeof(*out));
    try {
        return host_impl(points, N, queries, M, D, r, K, flags, opts, out);
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

void frnn_host_csr_release(frnn_host_csr *c) {
    if (!c) return;
    try {
        delete static_cast<HostOwner *>(c->owner_);
    } catch (...) {
    }
    std::memset(c, 0, sizeof(*c));
}

}  // extern "C"
