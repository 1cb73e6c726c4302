// extern "C" entry points of libfrnn (include/frnn.h).  Every call catches
// every exception and turns it into a status; nothing is thrown across the ABI.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "frnn_batch.h"
#include "frnn_runtime.h"

using namespace frnn;

struct frnn_index_s {
    Index ix;
};

namespace {

template <class F>
frnn_status guarded(F &&f) {
    try {
        return f();
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

bool bad_radius(float r) { return !std::isfinite(r) || r < 0.f; }

frnn_status check_common(int64_t n, int32_t D, float r, const void *p, std::string *why) {
    if (D < 1 || D > kDMax) {
        *why = "D must be in 1..32";
        return FRNN_ERR_INVALID_ARG;
    }
    if (n < 0 || n >= ((int64_t)1 << 31)) {
        *why = "point count must be in 0..2^31-1";
        return FRNN_ERR_INVALID_ARG;
    }
    if (n > 0 && !p) {
        *why = "null point pointer";
        return FRNN_ERR_INVALID_ARG;
    }
    if (bad_radius(r)) {
        *why = "radius must be finite and >= 0";
        return FRNN_ERR_INVALID_ARG;
    }
    return FRNN_OK;
}

void zero_csr(frnn_csr *o) {
    if (o) std::memset(o, 0, sizeof(*o));
}

}  // namespace

extern "C" {

void frnn_opts_default(frnn_opts *o) {
    if (!o) return;
    o->grid_axes_max = 6;
    o->cells_per_point = 2.0f;
    o->cell_multiple = 1;
    o->cells_per_item = 2;
    o->queries_per_item = 32;
    o->persistent = 2;
    o->blocks_per_cu = 8;
    o->row_cap_lds = kRowLds;
    o->stash_cap = 64;
    o->graphs = 0;
    o->adapt = 1;
}

const char *frnn_status_str(frnn_status s) {
    switch (s) {
    case FRNN_OK: return "ok";
    case FRNN_ERR_INVALID_ARG: return "invalid argument";
    case FRNN_ERR_NONFINITE: return "non-finite input";
    case FRNN_ERR_OOM: return "out of device memory";
    case FRNN_ERR_BUDGET: return "over the memory budget";
    case FRNN_ERR_RADIUS: return "query radius above the index radius";
    case FRNN_ERR_HIP: return "HIP runtime error";
    case FRNN_ERR_INTERNAL: return "internal error";
    case FRNN_ERR_NOT_READY: return "not ready";
    }
    return "unknown status";
}

const char *frnn_last_error(void) { return last_error_cstr(); }

frnn_status frnn_build(const float *points, int64_t N, int32_t D, float r, const frnn_opts *opts,
                       void *stream, frnn_index *out) {
    if (out) *out = nullptr;
    return guarded([&]() -> frnn_status {
        std::string why;
        if (!out) return fail(FRNN_ERR_INVALID_ARG, "null output handle");
        frnn_status st = check_common(N, D, r, points, &why);
        if (st) return fail(st, why);
        Opts o = Opts::from(opts);
        if ((st = o.validate(&why))) return fail(st, why);
        auto *h = new frnn_index_s();
        const float *pp[1] = {points};
        int64_t nn[1] = {N};
        try {
            st = build_index(h->ix, pp, nn, 1, D, r, o, (hipStream_t)stream, true);
        } catch (...) {
            delete h;
            throw;
        }
        if (st) {
            delete h;
            return st;
        }
        *out = h;
        return FRNN_OK;
    });
}

frnn_status frnn_query(frnn_index idx, const float *queries, int64_t M, float r, int32_t K,
                       uint32_t flags, void *stream, frnn_csr *out) {
    zero_csr(out);
    return guarded([&]() -> frnn_status {
        std::string why;
        if (!idx || !out) return fail(FRNN_ERR_INVALID_ARG, "null index or output");
        if (flags & ~(uint32_t)(FRNN_WANT_DIST2 | FRNN_SELF_QUERY | FRNN_EXCLUDE_SELF))
            return fail(FRNN_ERR_INVALID_ARG, "unknown flag");
        const bool selfq = flags & FRNN_SELF_QUERY;
        if ((flags & FRNN_EXCLUDE_SELF) && !selfq)
            return fail(FRNN_ERR_INVALID_ARG, "FRNN_EXCLUDE_SELF needs FRNN_SELF_QUERY");
        Index &ix = idx->ix;
        if (selfq) {
            if (queries) return fail(FRNN_ERR_INVALID_ARG, "self-query takes no query pointer");
            if (M != ix.n_pts[0]) return fail(FRNN_ERR_INVALID_ARG, "self-query: M must equal N");
        }
        frnn_status st = check_common(M, ix.D, r, selfq ? (const void *)1 : queries, &why);
        if (st) return fail(st, why);
        if (r > ix.r) return fail(FRNN_ERR_RADIUS, "query radius above the index radius");
        const float *qq[1] = {queries};
        int64_t mm[1] = {M};
        QueryArgs qa;
        qa.queries = qq;
        qa.m = mm;
        qa.r = r;
        qa.K = K;
        qa.flags = flags;
        return run_query(ix, qa, (hipStream_t)stream, out, nullptr);
    });
}

void frnn_index_destroy(frnn_index idx) {
    try {
        delete idx;
    } catch (...) {
    }
}

frnn_status frnn_index_get_info(frnn_index idx, frnn_index_info *info) {
    return guarded([&]() -> frnn_status {
        if (!idx || !info) return fail(FRNN_ERR_INVALID_ARG, "null argument");
        std::memset(info, 0, sizeof(*info));
        const Index &ix = idx->ix;
        info->N = ix.n_pts.empty() ? 0 : ix.n_pts[0];
        info->D = ix.D;
        if (ix.grid_host.empty()) return fail(FRNN_ERR_INTERNAL, "grid not available");
        const GridDesc &g = ix.grid_host[0];
        info->grid_axes = g.G;
        int64_t cells = 1;
        for (int a = 0; a < g.G; ++a) {
            info->axis[a] = g.axis[a];
            info->cells_per_axis[a] = g.n[a];
            cells *= g.n[a];
        }
        info->cells = cells;
        info->cell_width = g.h;
        info->cell_multiple = g.m;
        return FRNN_OK;
    });
}

frnn_status frnn_query_batch(const frnn_event *events, int32_t E, int32_t D, float r, int32_t K,
                             uint32_t flags, const frnn_opts *opts, void *stream, frnn_csr *outs) {
    if (outs && E > 0)
        for (int e = 0; e < E; ++e) zero_csr(&outs[e]);
    return guarded([&]() -> frnn_status {
        std::string why;
        if (E < 1 || !events || !outs) return fail(FRNN_ERR_INVALID_ARG, "need E >= 1 events and outputs");
        if (flags & ~(uint32_t)(FRNN_WANT_DIST2 | FRNN_SELF_QUERY | FRNN_EXCLUDE_SELF))
            return fail(FRNN_ERR_INVALID_ARG, "unknown flag");
        const bool selfq = flags & FRNN_SELF_QUERY;
        if ((flags & FRNN_EXCLUDE_SELF) && !selfq)
            return fail(FRNN_ERR_INVALID_ARG, "FRNN_EXCLUDE_SELF needs FRNN_SELF_QUERY");
        int64_t tp = 0, tq = 0;
        for (int e = 0; e < E; ++e) {
            frnn_status st = check_common(events[e].N, D, r, events[e].points, &why);
            if (st) return fail(st, why);
            if (!selfq) {
                st = check_common(events[e].M, D, r, events[e].queries, &why);
                if (st) return fail(st, why);
            } else if (events[e].queries) {
                return fail(FRNN_ERR_INVALID_ARG, "self-query events take no query pointer");
            }
            tp += events[e].N;
            tq += selfq ? events[e].N : events[e].M;
        }
        if (tp >= ((int64_t)1 << 31) || tq >= ((int64_t)1 << 31))
            return fail(FRNN_ERR_INVALID_ARG, "batch too large (2^31 points or queries)");
        Opts o = Opts::from(opts);
        frnn_status st = o.validate(&why);
        if (st) return fail(st, why);
        return batch_run(events, E, D, r, K, flags, o, (hipStream_t)stream, outs);
    });
}

frnn_status frnn_csr_copy(const frnn_csr *c, int64_t *offsets, int32_t *indices, float *dist2,
                          int32_t to_host, void *stream) {
    return guarded([&]() -> frnn_status {
        if (!c) return fail(FRNN_ERR_INVALID_ARG, "null csr");
        hipStream_t s = (hipStream_t)stream;
        hipMemcpyKind k = to_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
        if (offsets && c->offsets)
            FRNN_HIP(hipMemcpyAsync(offsets, c->offsets, sizeof(int64_t) * (c->M + 1), k, s));
        if (indices && c->nnz) FRNN_HIP(hipMemcpyAsync(indices, c->indices, sizeof(int32_t) * c->nnz, k, s));
        if (dist2 && c->nnz) {
            if (!c->dist2) return fail(FRNN_ERR_INVALID_ARG, "csr holds no dist2");
            FRNN_HIP(hipMemcpyAsync(dist2, c->dist2, sizeof(float) * c->nnz, k, s));
        }
        if (to_host) {
            FRNN_HIP(hipStreamSynchronize(s));
            // a row whose fill-pass recount differed from its count is reported here
            if (auto *own = static_cast<OutputOwner *>(c->owner_)) return own->check(s);
        }
        return FRNN_OK;
    });
}

void frnn_csr_release(frnn_csr *c) {
    if (!c) return;
    try {
        auto *own = static_cast<OutputOwner *>(c->owner_);
        if (own && --own->refs == 0) delete own;
    } catch (...) {
    }
    zero_csr(c);
}

void frnn_profile_enable(int32_t on) { prof_set(on != 0); }

int32_t frnn_profile_read(frnn_kernel_time *out, int32_t cap, int32_t reset) {
    try {
        return prof_read(out, cap, reset != 0);
    } catch (...) {
        return -1;
    }
}

frnn_status frnn_last_stats(frnn_stats *out) {
    if (!out) return FRNN_ERR_INVALID_ARG;
    *out = last_stats();
    return FRNN_OK;
}

void frnn_memory_stats(int64_t *current_bytes, int64_t *peak_bytes) {
    if (current_bytes) *current_bytes = Pool::get().in_use();
    if (peak_bytes) *peak_bytes = Pool::get().peak();
}

// Test hook (not in the public header): make the k-th device allocation from
// now fail, to exercise the out-of-memory paths.
void frnn_test_fail_alloc_after(int64_t k) { Pool::get().fail_after(k); }

}  // extern "C"
