// Autotuner: picks grid and kernel parameters for one input class.
//
// Coordinate descent from the defaults: each parameter in turn takes each of
// its candidate values with the others held, and the fastest setting is
// kept; a second pass runs when the first changed anything.  A candidate is timed as one batched self-query of the event (the
// graph-replayed path, the user's wall time including the count read-back)
// over a few repetitions, and its CSR must be bit-identical to the default
// setting's; a mismatch is counted as rejected and never chosen.  Winners
// are cached in a JSON file (FRNN_TUNE_CACHE) under a key of device, D, K
// and the input's density class: half-octaves of the mean candidates and of
// the mean neighbours per query, measured by the default run (inputs of one
// class share their cost structure whatever their size).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "frnn_runtime.h"

using namespace frnn;

namespace {

struct HostCSR {
    std::vector<int64_t> off;
    std::vector<int32_t> idx;
    std::vector<float> d2;
    bool operator==(const HostCSR &o) const {
        return off == o.off && idx == o.idx && d2.size() == o.d2.size() &&
               (d2.empty() || std::memcmp(d2.data(), o.d2.data(), d2.size() * 4) == 0);
    }
};

// One timed batched self-query; returns milliseconds (and the CSR when asked).
double run_once(const float *pts, int64_t N, int D, float r, int K, uint32_t flags,
                const frnn_opts &o, hipStream_t s, HostCSR *keep) {
    auto t0 = std::chrono::steady_clock::now();
    const frnn_event ev{pts, N, nullptr, 0};
    frnn_csr c{};
    frnn_status st = frnn_query_batch(&ev, 1, D, r, K, flags, &o, s, &c);
    if (st) throw Fail{st, frnn_last_error()};
    FRNN_HIP(hipStreamSynchronize(s));
    auto t1 = std::chrono::steady_clock::now();
    if (keep) {
        keep->off.resize(c.M + 1);
        keep->idx.resize(c.nnz);
        keep->d2.resize(c.dist2 ? c.nnz : 0);
        st = frnn_csr_copy(&c, keep->off.data(), c.nnz ? keep->idx.data() : nullptr,
                           (c.dist2 && c.nnz) ? keep->d2.data() : nullptr, 1, s);
    }
    frnn_csr_release(&c);
    if (st) throw Fail{st, frnn_last_error()};
    return std::chrono::duration<double, std::milli>(t1 - t0).count();
}

double time_opts(const float *pts, int64_t N, int D, float r, int K, uint32_t flags,
                 const frnn_opts &o, hipStream_t s, HostCSR *out) {
    run_once(pts, N, D, r, K, flags, o, s, out);  // warm-up (and the output)
    double best = 1e300;
    for (int i = 0; i < 3; ++i) best = std::min(best, run_once(pts, N, D, r, K, flags, o, s, nullptr));
    return best;
}

std::string device_name() {
    int dev = 0;
    hipDeviceProp_t p{};
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
    return p.gcnArchName;
}

// Density class of an input: half-octaves of the mean candidates and of the
// mean (capped) neighbours per query of the default run.
std::string cache_key(int D, int K, double cand_per_query, double pairs_per_query) {
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s|D%d|K%d|cand2^%.1f|nbr2^%.1f", device_name().c_str(), D, K,
                  std::round(2.0 * std::log2(1.0 + cand_per_query)) / 2.0,
                  std::round(2.0 * std::log2(1.0 + pairs_per_query)) / 2.0);
    return buf;
}

const char *kFields[] = {"grid_axes_max", "cells_per_point", "cell_multiple", "cells_per_item",
                         "queries_per_item", "persistent", "blocks_per_cu", "row_cap_lds",
                         "stash_cap", "graphs", "adapt"};

std::string opts_json(const frnn_opts &o) {
    char buf[512];
    std::snprintf(buf, sizeof buf,
                  "{\"grid_axes_max\": %d, \"cells_per_point\": %.9g, \"cell_multiple\": %d, "
                  "\"cells_per_item\": %d, \"queries_per_item\": %d, \"persistent\": %d, "
                  "\"blocks_per_cu\": %d, \"row_cap_lds\": %d, \"stash_cap\": %d, \"graphs\": %d, "
                  "\"adapt\": %d}",
                  o.grid_axes_max, (double)o.cells_per_point, o.cell_multiple, o.cells_per_item,
                  o.queries_per_item, o.persistent, o.blocks_per_cu, o.row_cap_lds, o.stash_cap, o.graphs,
                  o.adapt);
    return buf;
}

// Minimal reader for the cache file written below: {"key": {...}, ...}.
std::map<std::string, frnn_opts> read_cache(const std::string &path) {
    std::map<std::string, frnn_opts> m;
    std::ifstream f(path);
    if (!f) return m;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    size_t p = 0;
    while (true) {
        size_t k0 = s.find('"', p);
        if (k0 == std::string::npos) break;
        size_t k1 = s.find('"', k0 + 1);
        if (k1 == std::string::npos) break;
        size_t b0 = s.find('{', k1), b1 = s.find('}', k1);
        if (b0 == std::string::npos || b1 == std::string::npos || b0 > b1) break;
        const std::string key = s.substr(k0 + 1, k1 - k0 - 1);
        const std::string body = s.substr(b0, b1 - b0 + 1);
        frnn_opts o;
        frnn_opts_default(&o);
        bool ok = true;
        for (const char *fld : kFields) {
            size_t q = body.find(std::string("\"") + fld + "\"");
            if (q == std::string::npos) {
                ok = false;
                break;
            }
            double v = std::atof(body.c_str() + body.find(':', q) + 1);
            if (!std::strcmp(fld, "grid_axes_max")) o.grid_axes_max = (int)v;
            else if (!std::strcmp(fld, "cells_per_point")) o.cells_per_point = (float)v;
            else if (!std::strcmp(fld, "cell_multiple")) o.cell_multiple = (int)v;
            else if (!std::strcmp(fld, "cells_per_item")) o.cells_per_item = (int)v;
            else if (!std::strcmp(fld, "queries_per_item")) o.queries_per_item = (int)v;
            else if (!std::strcmp(fld, "persistent")) o.persistent = (int)v;
            else if (!std::strcmp(fld, "blocks_per_cu")) o.blocks_per_cu = (int)v;
            else if (!std::strcmp(fld, "row_cap_lds")) o.row_cap_lds = (int)v;
            else if (!std::strcmp(fld, "stash_cap")) o.stash_cap = (int)v;
            else if (!std::strcmp(fld, "graphs")) o.graphs = (int)v;
            else if (!std::strcmp(fld, "adapt")) o.adapt = (int)v;
        }
        if (ok) m[key] = o;
        p = b1 + 1;
    }
    return m;
}

void write_cache(const std::string &path, const std::map<std::string, frnn_opts> &m) {
    std::ofstream f(path + ".tmp");
    f << "{\n";
    size_t i = 0;
    for (auto &kv : m) {
        f << "  \"" << kv.first << "\": " << opts_json(kv.second) << (++i < m.size() ? ",\n" : "\n");
    }
    f << "}\n";
    f.close();
    std::rename((path + ".tmp").c_str(), path.c_str());
}

std::mutex g_cache_mu;

}  // namespace

extern "C" frnn_status frnn_tune(const float *points, int64_t N, int32_t D, float r, int32_t K,
                                 uint32_t flags, void *stream, frnn_opts *best,
                                 frnn_tune_report *report) {
    if (report) std::memset(report, 0, sizeof(*report));
    try {
        if (!best || D < 1 || D > kDMax || N < 1 || !points || !std::isfinite(r) || r < 0.f)
            return fail(FRNN_ERR_INVALID_ARG, "bad tuning input");
        hipStream_t s = (hipStream_t)stream;
        flags = (flags | FRNN_SELF_QUERY) & ~(uint32_t)FRNN_EXCLUDE_SELF;
        const char *cpath = std::getenv("FRNN_TUNE_CACHE");
        frnn_opts cur;
        frnn_opts_default(&cur);
        cur.adapt = 0;  // every candidate runs as given
        HostCSR ref;
        const double t_def = time_opts(points, N, D, r, K, flags, cur, s, &ref);
        const frnn_stats st0 = last_stats();
        const std::string key =
            cache_key(D, K, (double)st0.candidates / (double)N, (double)st0.pairs / (double)N);
        if (report) std::snprintf(report->density_class, sizeof report->density_class, "%s", key.c_str());
        if (cpath) {
            std::lock_guard<std::mutex> g(g_cache_mu);
            auto m = read_cache(cpath);
            auto it = m.find(key);
            if (it != m.end()) {
                *best = it->second;
                if (report) {
                    report->candidates_tried = 1;
                    report->default_ms = report->best_ms = t_def;
                    report->from_cache = 1;
                }
                return FRNN_OK;
            }
        }
        double t_best = t_def;
        int tried = 1, rejected = 0;
        // candidate values per parameter, tried in this order
        const int axes[] = {3, 4, 5, 6};
        const float cpps[] = {0.5f, 1.f, 2.f, 4.f, 16.f, 32.f};
        const int cpis[] = {1, 2, 4};
        const int qpis[] = {8, 16, 32, 64};
        const int stashes[] = {0, 8, 16, 32, 64, 128, 256};
        const int pers[] = {0, 1, 2};
        const int bpcs[] = {4, 8, 16};
        const int graphs[] = {0, 1};
        auto consider = [&](frnn_opts cand) {
            if (std::memcmp(&cand, &cur, sizeof cand) == 0) return;
            Opts oo = Opts::from(&cand);
            std::string why;
            if (oo.validate(&why)) return;
            HostCSR out;
            double t = time_opts(points, N, D, r, K, flags, cand, s, &out);
            ++tried;
            if (!(out == ref)) {
                ++rejected;
                return;
            }
            if (t < t_best) {
                t_best = t;
                cur = cand;
            }
        };
        // two passes over the parameters (the second only when the first
        // moved): a setting that pays only beside another one (a larger
        // stash with smaller windows, say) is reached from either side
        for (int pass = 0; pass < 2; ++pass) {
            const frnn_opts start = cur;
            for (int v : axes) {
                frnn_opts c = cur;
                c.grid_axes_max = std::min<int>(v, D);
                consider(c);
            }
            for (float v : cpps) {
                frnn_opts c = cur;
                c.cells_per_point = v;
                consider(c);
            }
            for (int v : cpis) {
                frnn_opts c = cur;
                c.cells_per_item = v;
                consider(c);
            }
            for (int v : qpis) {
                frnn_opts c = cur;
                c.queries_per_item = v;
                consider(c);
            }
            for (int v : stashes) {
                frnn_opts c = cur;
                c.stash_cap = v;
                consider(c);
            }
            for (int v : pers) {
                frnn_opts c = cur;
                c.persistent = v;
                consider(c);
            }
            for (int v : bpcs) {
                frnn_opts c = cur;
                c.blocks_per_cu = v;
                consider(c);
            }
            for (int v : graphs) {
                frnn_opts c = cur;
                c.graphs = v;
                consider(c);
            }
            if (std::memcmp(&start, &cur, sizeof cur) == 0) break;
        }
        *best = cur;
        if (report) {
            report->candidates_tried = tried;
            report->candidates_rejected = rejected;
            report->best_ms = t_best;
            report->default_ms = t_def;
        }
        if (cpath) {
            std::lock_guard<std::mutex> g(g_cache_mu);
            auto m = read_cache(cpath);
            m[key] = cur;
            write_cache(cpath, m);
        }
        if (rejected) return fail(FRNN_ERR_INTERNAL, "a candidate setting changed the output");
        return FRNN_OK;
    } catch (const Fail &f) {
        return fail(f.st, f.msg);
    } catch (const std::exception &x) {
        return fail(FRNN_ERR_INTERNAL, x.what());
    }
}
