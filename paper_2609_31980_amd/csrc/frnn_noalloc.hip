// frnn_query_noalloc: the single-event self-query of frnn_query_batch for
// callers that cannot allocate device memory.  Every work buffer of the
// pipeline is carved out of one file-scope device array (`scratch`, one copy
// per GPU, held until the process ends); the caller passes the points and
// the output arrays.  The call allocates nothing: no hipMalloc, hipFree,
// pool or host-pinned allocation, and the launches are the library's own
// kernels with pointers into that array.
//
// Calls that overlap on one GPU share its array and race: they must be
// ordered (one stream, or synchronised streams).  Every buffer a kernel
// expects at zero is cleared by the first kernel of each call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "../../include/frnn.h"
#include "frnn_device.h"
#include "frnn_launch.h"
#include "frnn_runtime.h"

namespace frnn {
namespace {

constexpr int64_t kScratchBytes = FRNN_NOALLOC_SCRATCH_BYTES;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char *g_ptr[kMaxDevices] = {};

// The array's device address on the current device (looked up once per
// device; host code never uses the symbol itself as an address).
unsigned char *scratch_ptr(int dev) {
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_ptr[dev] = static_cast<unsigned char *>(p);
    }
    return g_ptr[dev];
}

// Writes the run's descriptors (batch, the one event, the chunk table of its
// rows) from kernel arguments and clears both counter blocks.
__global__ void __launch_bounds__(256) k_noalloc_setup(Bufs b, Counters *ctr2, BatchDesc bd, EventDev ev,
                                                       int32_t nch, int64_t n) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0) {
        *const_cast<BatchDesc *>(b.bd) = bd;
        const_cast<EventDev *>(b.ev)[0] = ev;
    }
    if (t < (int)(sizeof(Counters) / 4)) {
        reinterpret_cast<uint32_t *>(b.ctr)[t] = 0u;
        reinterpret_cast<uint32_t *>(ctr2)[t] = 0u;
    }
    for (int c = t; c < nch; c += gridDim.x * blockDim.x) {
        Chunk ch;
        ch.ev = 0;
        ch.pad = 0;
        ch.r0 = (int64_t)c * kChunkRows;
        ch.r1 = std::min<int64_t>(n, ch.r0 + kChunkRows);
        const_cast<Chunk *>(b.pchunks)[c] = ch;
    }
}

// Sequential carving of the array into 256-byte aligned regions.
struct Carve {
    unsigned char *base;
    int64_t off = 0;
    template <class T>
    T *take(int64_t count) {
        T *p = reinterpret_cast<T *>(base + off);
        off += (int64_t)((sizeof(T) * (uint64_t)std::max<int64_t>(count, 1) + 255) / 256 * 256);
        return p;
    }
};

}  // namespace
}  // namespace frnn

using namespace frnn;

extern "C" frnn_status frnn_query_noalloc(const float *points, int64_t N, int32_t D, float r, int32_t K,
                                          uint32_t flags, const frnn_opts *opts, int64_t *offsets,
                                          int32_t *indices, float *dist2, int64_t cap_pairs, int64_t *nnz,
                                          void *stream) {
    if (nnz) *nnz = 0;
    try {
        hipStream_t s = (hipStream_t)stream;
        if (!nnz || !offsets) return fail(FRNN_ERR_INVALID_ARG, "null output");
        if (D < 1 || D > kDMax) return fail(FRNN_ERR_INVALID_ARG, "D must be in 1..32");
        if (N < 0 || N >= ((int64_t)1 << 31) || (N > 0 && !points)) return fail(FRNN_ERR_INVALID_ARG, "bad points");
        if (!std::isfinite(r) || r < 0.f) return fail(FRNN_ERR_INVALID_ARG, "radius must be finite and >= 0");
        if (!(flags & FRNN_SELF_QUERY)) return fail(FRNN_ERR_INVALID_ARG, "frnn_query_noalloc is a self-query");
        if (flags & ~(uint32_t)(FRNN_WANT_DIST2 | FRNN_SELF_QUERY | FRNN_EXCLUDE_SELF))
            return fail(FRNN_ERR_INVALID_ARG, "unknown flag");
        const bool want_d2 = flags & FRNN_WANT_DIST2;
        if (cap_pairs < 0 || (cap_pairs > 0 && (!indices || (want_d2 && !dist2))))
            return fail(FRNN_ERR_INVALID_ARG, "null index or dist2 output");
        Opts o = Opts::from(opts);
        std::string why;
        if (frnn_status st = o.validate(&why)) return fail(st, why);
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
            return fail(FRNN_ERR_HIP, "no current device");
        unsigned char *base = scratch_ptr(dev);
        if (!base) return fail(FRNN_ERR_HIP, "hipGetSymbolAddress of the scratch array failed");

        // sizes as a one-event batch of capacity N
        const int Dp = (D + 3) & ~3, SC = o.o.stash_cap;
        const int64_t n1 = std::max<int64_t>(N, 1);
        const int nch = (int)((N + kChunkRows - 1) / kChunkRows);
        const int ch_cap = nch + 1;
        const int64_t cells_cap = (int64_t)std::ceil((double)o.o.cells_per_point * (double)n1) + 1;
        const int wpc = kChunkRows / o.o.queries_per_item;
        const int64_t fill_cap = std::max<int64_t>(1, (int64_t)ch_cap * wpc);

        Carve cv{base};
        Bufs b{};
        char *desc = cv.take<char>(256);  // BatchDesc | OutDesc
        b.bd = reinterpret_cast<const BatchDesc *>(desc);
        b.out = reinterpret_cast<OutDesc *>(desc + 128);
        b.ev = cv.take<EventDev>(1);
        b.pchunks = b.qchunks = cv.take<Chunk>(ch_cap);
        Counters *ctr_q = cv.take<Counters>(1), *ctr_b = cv.take<Counters>(1);
        b.bases = cv.take<int64_t>(2);
        b.grid = cv.take<GridDesc>(1);
        b.runs = cv.take<RunEntry>(kRunsMax);
        b.cell_off = cv.take<int64_t>(2);
        b.ext = cv.take<uint32_t>(2 * (int64_t)ch_cap * D);
        b.xs = b.qs = cv.take<float>(n1 * Dp);
        b.perm = b.qperm = cv.take<int32_t>(n1);
        b.key = b.qkey = cv.take<uint32_t>(n1);
        b.rank = b.qrank = cv.take<uint32_t>(n1);
        b.skey = b.sqkey = cv.take<uint32_t>(n1);
        b.cells = b.qcells = cv.take<uint32_t>(cells_cap + 1);
        b.deg = cv.take<uint32_t>(n1);
        b.offs = cv.take<int64_t>(n1 + 1);
        b.lofs = cv.take<int64_t>(n1 + 1);
        b.long_rows = cv.take<uint32_t>(n1);
        b.long_at = cv.take<int64_t>(2 * n1);
        b.stash = cv.take<uint64_t>(n1 * std::max(1, SC));
        b.fill_list = cv.take<uint32_t>(fill_cap);
        b.scan_part = cv.take<uint64_t>(2 * kScanBlocks);
        b.lpt = cv.take<uint32_t>(lpt_words(1));
        uint32_t *status = cv.take<uint32_t>(4);
        const int64_t fixed = cv.off;
        if (fixed > kScratchBytes)
            return fail(FRNN_ERR_INVALID_ARG, "event too large for the no-allocation scratch array");
        // the rest of the array holds the long-row keys
        uint64_t *long_keys = reinterpret_cast<uint64_t *>(base + fixed);
        const int64_t cap_long = (kScratchBytes - fixed) / 8;

        Bufs bb = b, bq = b;
        bb.ctr = ctr_b;
        bq.ctr = ctr_q;

        BatchDesc bd{};
        bd.E = 1;
        bd.D = D;
        bd.Dp = Dp;
        bd.n_pchunks = bd.n_qchunks = nch;
        bd.grid_axes_max = o.o.grid_axes_max;
        bd.cell_multiple = o.o.cell_multiple;
        bd.cells_per_point = o.o.cells_per_point;
        bd.r_build = r;
        bd.total_pts = bd.total_q = N;
        double cc = std::floor((double)o.o.cells_per_point * (double)n1);
        cc = std::max(1.0, std::min(cc, (double)(1 << 30)));
        const EventDev ev{points, nullptr, N, 0, N, 0, (int64_t)cc};

        Knobs kn{};
        kn.r2 = r2_of(r);
        kn.K = K;
        kn.self_query = 1;
        kn.exclude_self = (flags & FRNN_EXCLUDE_SELF) ? 1 : 0;
        kn.window = o.o.queries_per_item;
        kn.cells_per_item = o.o.cells_per_item;
        kn.long_cap = o.o.row_cap_lds;
        kn.persistent = 0;  // the plain launch needs no occupancy query
        kn.stash_cap = SC;
        kn.fill_cap = (uint32_t)fill_cap;

        auto ck = [](hipError_t e) {
            if (e != hipSuccess) throw Fail{FRNN_ERR_HIP, hipGetErrorString(e)};
        };
        const int sblocks = std::max(1, std::min(256, (nch + 255) / 256));
        hipLaunchKernelGGL(k_noalloc_setup, dim3(sblocks), dim3(256), 0, s, bb, ctr_q, bd, ev, nch, N);
        ck(hipGetLastError());
        ck(launch_extent(bb, ch_cap, 1, false, cells_cap + 1, s));
        ck(launch_plan(bb, 1, s));
        ck(launch_keys(bb, ch_cap, false, s));
        ck(launch_scan_cells(bb, cells_cap, false, s));
        ck(launch_scatter(bb, ch_cap, false, s));
        ck(launch_count(bq, kn, D, query_blocks(o.o, ch_cap, false), s));
        ck(launch_scan_rows(bq, kn, n1, s));

        // the one synchronisation: both counter blocks and the event bases
        struct {
            Counters q, bld;
            int64_t bases[2];
        } back;
        ck(hipMemcpyAsync(&back.q, ctr_q, sizeof(Counters), hipMemcpyDeviceToHost, s));
        ck(hipMemcpyAsync(&back.bld, ctr_b, sizeof(Counters), hipMemcpyDeviceToHost, s));
        ck(hipMemcpyAsync(back.bases, b.bases, 16, hipMemcpyDeviceToHost, s));
        ck(hipStreamSynchronize(s));
        if (back.bld.status & kStatusNonfinitePts) return fail(FRNN_ERR_NONFINITE, "non-finite coordinate in the points");
        const int64_t pairs = (int64_t)back.q.nnz;
        *nnz = pairs;
        if (back.bases[1] != pairs) return fail(FRNN_ERR_INTERNAL, "pair count mismatch");
        if (pairs > cap_pairs) return fail(FRNN_ERR_BUDGET, "output capacity below the pair count (*nnz holds it)");
        if ((int64_t)back.q.long_total > cap_long)
            return fail(FRNN_ERR_BUDGET, "rows longer than the stash exceed the scratch array");

        const OutDesc od{offsets, indices, want_d2 ? dist2 : nullptr, long_keys, cap_pairs, cap_long, status};
        ck(launch_set_out(bq, od, s));
        ck(launch_short_rows(bq, kn, ch_cap, s));
        if (back.q.long_total > 0) {
            ck(launch_fill(bq, kn, D, fill_blocks(fill_cap), s));
            ck(launch_long_sort(bq, kn, 1536, s));
        }
        return FRNN_OK;
    } catch (const Fail &f) {
        return fail(f.st, f.msg);
    } catch (...) {
        return fail(FRNN_ERR_INTERNAL, "unknown internal error");
    }
}
