// HIP kernels of the exact fixed-radius neighbour pipeline, written for
// gfx950 (CDNA4, 64-lane wavefronts).
//
// Pipeline (every size is read from device memory, see frnn_device.h):
//   binning    k_init, k_extent (+ clears cells), k_plan, k_keys, scan, k_scatter
//   counting   k_query<count> over windows of sorted queries, scan of the
//              capped counts (and the events' first output pairs)
//   filling    k_set_out, k_short_rows (per-event offsets, rows the stash
//              holds), k_query<fill> (hit keys of longer rows into scratch
//              rows, for the windows the count pass listed), k_long_sort
//              (those rows sorted, one wave per row)
//
// Exactness: the squared distance is computed in float32 as
//   s = +0; for d in 0..D-1: t = q_d - x_d; u = t*t; s = s + u
// with every operation rounded on its own.  The file is compiled with
// -ffp-contract=off and the pragma below, so no fused multiply-add can
// replace t*t followed by s+u (a reassociated or fused sum changes float32
// membership near the radius, Sec. 4.2).  Subnormals are not flushed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

#include "frnn_device.h"
#include "frnn_launch.h"

#pragma clang fp contract(off)

namespace frnn {

// ------------------------------------------------------------ wave helpers
__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Writes value into lane `lane` (wave-uniform) of old and returns the rest
// of old unchanged: one v_writelane (the compiler's own intrinsic, reached
// by name, so its wait states are handled as for any other instruction).
extern "C" __device__ int frnn_writelane_i32(int value, int lane, int old) __asm("llvm.amdgcn.writelane.i32");

// global address space (a pointer made from an integer is otherwise generic)
#define FRNN_GLOBAL __attribute__((address_space(1)))

__device__ __forceinline__ int64_t readlane64(int64_t v, int t) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, t);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), t);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint32_t uniform(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

// Orders LDS writes of a wave before its later LDS reads by other lanes.
// s_waitcnt immediate that waits for every vector memory access (vmcnt 0)
// and for nothing else (expcnt 7, lgkmcnt 15)
constexpr int kWaitVmcnt0 = 0x0F70;

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Inclusive prefix sum over the wave with DPP lane moves (no LDS traffic):
// shifts by 1, 2, 4, 8 inside each row of 16 lanes (lanes whose source lies
// outside the row read 0), then the last lane of row 0 and of row 2 is added
// to rows 1 and 3, and the last lane of row 1 to rows 2 and 3.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, true);  // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, true);  // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, true);  // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, true);  // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false); // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false); // row_bcast:31
    return v;
}

// Float bits mapped so that unsigned order is float order (for atomics).
__device__ __forceinline__ uint32_t f2ord(float f) {
    uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float ord2f(uint32_t o) {
    uint32_t b = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
    return __uint_as_float(b);
}

__device__ __forceinline__ bool finite32(float f) {
    return (__float_as_uint(f) & 0x7f800000u) != 0x7f800000u;
}

// ------------------------------------------------------------------ init
// Clears the counters (block 0) and, when src is given, copies n16 16-byte
// words of descriptors from device-mapped host memory to dst, every block
// taking a contiguous part with kFetchUnroll loads in flight per thread.
constexpr int kFetchUnroll = 1;

__global__ void __launch_bounds__(256) k_init(Bufs b, Counters *ctr2, const uint4 *src, uint4 *dst, int64_t n16) {
    if (blockIdx.x == 0) {
        if (threadIdx.x < sizeof(Counters) / 4) {
            reinterpret_cast<uint32_t *>(b.ctr)[threadIdx.x] = 0u;
            if (ctr2) reinterpret_cast<uint32_t *>(ctr2)[threadIdx.x] = 0u;
        }
        // the run's number, from the descriptors at the head of the stage
        // (the host checks it in the read-back)
        __syncthreads();
        if (src && threadIdx.x == 0) {
            const uint32_t id = reinterpret_cast<const BatchDesc *>(src)->run_id;
            b.ctr->run_id = id;
            if (ctr2) ctr2->run_id = id;
        }
    }
    if (!src) return;
    const int64_t per = (int64_t)blockDim.x * kFetchUnroll;
    for (int64_t base = (int64_t)blockIdx.x * per; base < n16; base += (int64_t)gridDim.x * per) {
        uint4 v[kFetchUnroll];
#pragma unroll
        for (int u = 0; u < kFetchUnroll; ++u) {
            const int64_t i = base + (int64_t)u * blockDim.x + threadIdx.x;
            if (i < n16) v[u] = src[i];
        }
#pragma unroll
        for (int u = 0; u < kFetchUnroll; ++u) {
            const int64_t i = base + (int64_t)u * blockDim.x + threadIdx.x;
            if (i < n16) dst[i] = v[u];
        }
    }
}

// ---------------------------------------------------------------- extent
// Per-unit per-axis min / max of the points and a finiteness check
// (queries: finiteness only).  A unit is kExtentRows consecutive rows of one
// event (the events' units in order, ceil(n / kExtentRows) each); one block
// per unit, and the block's result goes to its own slot ext[unit][2][D] (no
// atomics on shared addresses: the plan reduces the slots of each event).
// Rows are read as 16-byte vectors when the event's array is 16-byte aligned:
// thread t takes vector t + k*T4 of the unit, and since 4*T4 is a multiple of
// D each of its four lanes always
// holds the same axis.  The same launch clears the cell histogram for the
// capacity of the run.
__global__ void __launch_bounds__(256) k_extent(Bufs b, int32_t queries, int64_t zero_n) {
    __shared__ uint32_t smin[kDMax], smax[kDMax];
    __shared__ int sbad;
    const BatchDesc bd = *b.bd;
    const int D = bd.D;
    const int stride = (256 / D) * D;
    int L = 4;  // lcm(4, D) floats
    while (L % D) L += 4;
    const int T4 = (256 / (L / 4)) * (L / 4);  // threads of the 16-byte path; 4*T4 is a multiple of D
    const int t = threadIdx.x;
    // clear the cell histogram (zero_n cells, the capacity)
    uint32_t *cells = queries ? b.qcells : b.cells;
    {
        const int64_t gt = (int64_t)blockIdx.x * blockDim.x + t, gs = (int64_t)gridDim.x * blockDim.x;
        const int64_t n4 = zero_n / 4;
        for (int64_t i = gt; i < n4; i += gs) reinterpret_cast<uint4 *>(cells)[i] = make_uint4(0u, 0u, 0u, 0u);
        for (int64_t i = 4 * n4 + gt; i < zero_n; i += gs) cells[i] = 0u;
    }
    if (t < kDMax) {
        smin[t] = 0xffffffffu;
        smax[t] = 0u;
    }
    if (t == 0) sbad = 0;
    __syncthreads();
    // this block's unit: rows [u*kExtentRows, ...) of event ev_u, found by
    // walking the events' unit counts ceil(n / kExtentRows)
    __shared__ int s_ev;
    __shared__ long long s_u;
    if (t == 0) {
        long long u = blockIdx.x;
        int e = 0;
        for (; e < bd.E; ++e) {
            const int64_t n = queries ? b.ev[e].n_q : b.ev[e].n_pts;
            const long long ne = (n + kExtentRows - 1) / kExtentRows;
            if (u < ne) break;
            u -= ne;
        }
        s_ev = e;
        s_u = u;
    }
    __syncthreads();
    const int c = blockIdx.x;
    const int ue = s_ev;
    bool bad = false;
    if (ue < bd.E) {
        uint32_t mn[4] = {0xffffffffu, 0xffffffffu, 0xffffffffu, 0xffffffffu}, mx[4] = {0u, 0u, 0u, 0u};
        auto fold = [&](uint32_t &lo, uint32_t &hi, float x) {
            bad |= !finite32(x);
            const uint32_t o = f2ord(x);
            lo = o < lo ? o : lo;
            hi = o > hi ? o : hi;
        };
        const EventDev ev = b.ev[ue];
        const float *src = queries ? ev.qry : ev.pts;
        const int64_t n = queries ? ev.n_q : ev.n_pts;
        const int64_t r0 = (int64_t)s_u * kExtentRows, r1 = r0 + kExtentRows < n ? r0 + kExtentRows : n;
        const int64_t f0 = r0 * D, nf = (r1 - r0) * D;
        if ((reinterpret_cast<uintptr_t>(src) & 15u) == 0) {
            // units start at multiples of kExtentRows rows, so src + f0 is aligned too
            const float4 *s4 = reinterpret_cast<const float4 *>(src + f0);
            const int64_t nv = nf / 4;
            if (t < T4) {
                int64_t i = t;
                for (; i + 3 * T4 < nv; i += 4 * T4) {
                    float4 v[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) v[u] = s4[i + u * T4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        fold(mn[0], mx[0], v[u].x);
                        fold(mn[1], mx[1], v[u].y);
                        fold(mn[2], mx[2], v[u].z);
                        fold(mn[3], mx[3], v[u].w);
                    }
                }
                for (; i < nv; i += T4) {
                    const float4 v0 = s4[i];
                    fold(mn[0], mx[0], v0.x);
                    fold(mn[1], mx[1], v0.y);
                    fold(mn[2], mx[2], v0.z);
                    fold(mn[3], mx[3], v0.w);
                }
                if (!queries) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        atomicMin(&smin[(4 * t + j) % D], mn[j]);
                        atomicMax(&smax[(4 * t + j) % D], mx[j]);
                    }
                }
            }
            // fewer than 4 trailing floats (only in an event's last chunk)
            if (t < nf - 4 * nv) {
                const int64_t f = 4 * nv + t;
                uint32_t lo = 0xffffffffu, hi = 0u;
                fold(lo, hi, src[f0 + f]);
                if (!queries) {
                    atomicMin(&smin[f % D], lo);
                    atomicMax(&smax[f % D], hi);
                }
            }
        } else if (t < stride) {
            for (int64_t f = t; f < nf; f += stride) fold(mn[0], mx[0], src[f0 + f]);
            if (!queries) {
                atomicMin(&smin[t % D], mn[0]);
                atomicMax(&smax[t % D], mx[0]);
            }
        }
    }
    if (bad) sbad = 1;
    __syncthreads();
    if (!queries && ue < bd.E && t < D) {
        b.ext[((int64_t)c * 2 + 0) * D + t] = smin[t];
        b.ext[((int64_t)c * 2 + 1) * D + t] = smax[t];
    }
    if (t == 0 && sbad) atomicOr(&b.ctr->status, queries ? kStatusNonfiniteQry : kStatusNonfinitePts);
}

// ------------------------------------------------------------------ plan
// Slot words per thread that the plan loads together (one batch covers 8,192
// words, the slots of about 524,000 points at D = 8).
constexpr int kPlanBatch = 32;

// Lane src's value (src wave-uniform), read through scalar registers.
__device__ __forceinline__ double lane_f64(double v, int src) {
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, src);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), src);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// One wave per event.  Grid axes = the coordinates of largest extent; cell
// width h = r_h / m with r_h = r (1 + 2^-16) + 2^-60 (float64); the most
// axes (up to the limit) whose cell count stays within the cap.
//
// Why no neighbour is lost (the roundoff-safe grid): float32 rounding is
// monotone and every u_d is >= 0, so s <= r2 implies fl32(t_a^2) <= r2 on
// each axis a, hence |x_a - y_a| <= r (1 + 2^-21) + 2^-73 in real numbers.
// Cell coordinates v = fl64(fl64(x - lo) * inv_h) carry a relative error
// below 2^-51, far less than the 2^-16 margin in h, so |v(x) - v(y)| < m and
// the floors differ by at most m; clamping to [0, n-1] cannot widen the gap.

__device__ void plan_offsets(Bufs &b, int E);

__device__ void plan_event(Bufs &b, const BatchDesc &bd, int e, int lane, uint32_t emin, uint32_t emax);

// One block per event: the block reduces the event's per-chunk extent slots
// (its units follow those of the earlier events, ceil(n / kExtentRows) each;
// slot layout [unit][min, max][D]),
// then its first wave plans the grid.  The last block to finish (a ticket
// counter) scans the events' cell counts into the cell offsets.
__device__ void lpt_order(Bufs &b, const Knobs &kn);

// with_lpt: the block that plans last also orders the persistent count
// pass's work (see lpt_order), which needs every event's grid
__global__ void __launch_bounds__(256) k_plan(Bufs b, Knobs kn, int32_t with_lpt) {
    __shared__ uint32_t s_last;
    __shared__ uint32_t rmin[256];
    __shared__ long long s_c0[256];
    const BatchDesc bd = *b.bd;
    const int e = blockIdx.x, D = bd.D, t = threadIdx.x;
    if (e < bd.E) {
        long long part = 0;
        for (int e2 = t; e2 < e; e2 += blockDim.x) part += (b.ev[e2].n_pts + kExtentRows - 1) / kExtentRows;
        s_c0[t] = part;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (t < o) s_c0[t] += s_c0[t + o];
            __syncthreads();
        }
        const int64_t c0 = s_c0[0];
        const int64_t nch = (b.ev[e].n_pts + kExtentRows - 1) / kExtentRows;
        // the event's slots are one contiguous block of nch * 2D words; thread
        // t < T reads words t + k*T, all in the same column (T is a multiple of
        // 2D), eight loads in flight at a time
        const int W = 2 * D, T = (256 / W) * W;
        const int64_t nw = nch * W;
        const uint32_t *slot = b.ext + c0 * W;
        const bool is_min = (t % W) < D;
        uint32_t acc = is_min ? 0xffffffffu : 0u;
        if (t < T) {
            // batches of kPlanBatch words per thread, all loads of a batch in
            // flight at once (the slots were written by other XCDs, so each
            // round trip goes past this XCD's L2); a position past the end
            // reads word i again, of the same column, which min / max ignore
            for (int64_t i = t; i < nw; i += kPlanBatch * T) {
                uint32_t v[kPlanBatch];
#pragma unroll
                for (int u = 0; u < kPlanBatch; ++u) v[u] = slot[i + u * T < nw ? i + u * T : i];
#pragma unroll
                for (int u = 0; u < kPlanBatch; ++u)
                    acc = is_min ? (v[u] < acc ? v[u] : acc) : (v[u] > acc ? v[u] : acc);
            }
        }
        rmin[t] = acc;
        __syncthreads();
        if (t < 64) {
            uint32_t emin = 0xffffffffu, emax = 0u;
            if (t < D) {
                for (int s = 0; s < T / W; ++s) {
                    const uint32_t lo = rmin[s * W + t], hi = rmin[s * W + D + t];
                    emin = lo < emin ? lo : emin;
                    emax = hi > emax ? hi : emax;
                }
            }
            plan_event(b, bd, e, t, emin, emax);
        }
    }
    if (gridDim.x == 1) {  // every event in this block: no ticket needed
        __syncthreads();
        plan_offsets(b, bd.E);
        if (with_lpt) {
            __syncthreads();
            lpt_order(b, kn);
        }
        return;
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) s_last = atomicAdd(&b.ctr->plan_done, 1u) == gridDim.x - 1 ? 1u : 0u;
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    plan_offsets(b, bd.E);
    if (with_lpt) {
        __syncthreads();
        lpt_order(b, kn);
    }
}

__device__ void plan_event(Bufs &b, const BatchDesc &bd, int e, int lane, uint32_t emin, uint32_t emax) {
    const int D = bd.D;
    const EventDev ev = b.ev[e];
    // lane d < D: extent and lower bound of coordinate d; a non-finite
    // input (reported to the host as an error) must still give an
    // in-bounds grid, so its extent counts as empty
    double x = -1.0, lo = 0.0;
    if (lane < D) {
        const float flo = ord2f(emin);
        const float fhi = ord2f(emax);
        x = ev.n_pts > 0 ? (double)fhi - (double)flo : 0.0;
        if (!(x >= 0.0 && x <= 1.0e39)) x = 0.0;
        lo = ev.n_pts > 0 ? (double)flo : 0.0;
        if (!(lo >= -3.5e38 && lo <= 3.5e38)) lo = 0.0;
    }
    // rank by decreasing extent, ties by coordinate index
    int rank = 0;
    for (int d2 = 0; d2 < D; ++d2) {
        const double x2 = lane_f64(x, d2);
        rank += (x2 > x || (x2 == x && d2 < lane)) ? 1 : 0;
    }
    GridDesc g;
    for (int a = 0; a < kGMax; ++a) {
        g.axis[a] = 0;
        g.n[a] = 1;
        g.stride[a] = 0;
        g.lo[a] = 0.0;
    }
    const int m = bd.cell_multiple;
    g.m = m;
    const double rh = (double)bd.r_build * (1.0 + 0x1p-16) + 0x1p-60;
    double inv_h = 1.0 / (rh / (double)m);
    int64_t cap = (int64_t)((double)bd.cells_per_point * (double)(ev.n_pts > 0 ? ev.n_pts : 1));
    if (cap < 1) cap = 1;
    if (cap > ((int64_t)1 << 30)) cap = (int64_t)1 << 30;
    if (cap > ev.cell_cap) cap = ev.cell_cap;
    const int gmax = min(bd.grid_axes_max, min(D, kGMax));
    // (every per-axis loop below runs over all kGMax axes with a guard, so
    // the arrays are indexed by constants and stay in registers)
    double cext[kGMax];
#pragma unroll
    for (int a = 0; a < kGMax; ++a) {
        cext[a] = 0.0;
        if (a < gmax) {
            const uint64_t hit = ballot(lane < D && rank == a);
            const int ax = __ffsll((unsigned long long)hit) - 1;
            g.axis[a] = ax;
            cext[a] = lane_f64(x, ax);
            g.lo[a] = lane_f64(lo, ax);
        }
    }
    int G = 0;
    const int W = 2 * m + 1;
    for (int gg = gmax; gg >= 1; --gg) {
        int64_t runs = 1;
        double C = 1.0;
#pragma unroll
        for (int a = 0; a < kGMax; ++a) {
            if (a < gg) {
                if (a >= 1) runs *= W;
                C *= floor(cext[a] * inv_h) + 1.0;
            }
        }
        if (runs > kRunsMax) continue;
        if (C <= (double)cap) {
            G = gg;
            break;
        }
    }
    if (G == 0 && gmax >= 1) {
        // even one axis at width r_h/m has too many cells: widen the cells
        // (wider cells never lose a neighbour)
        G = 1;
        if (cext[0] > 0.0) {
            const double w = (double)(cap - 1) / cext[0];
            inv_h = w < inv_h ? w : inv_h;
        }
    }
    g.G = G;
    g.inv_h = inv_h;
    g.h = inv_h > 0.0 ? 1.0 / inv_h : 0.0;
    uint32_t C = 1;
    int runs = 1;
#pragma unroll
    for (int a = 0; a < kGMax; ++a) {
        if (a < G) {
            double na = floor(cext[a] * inv_h) + 1.0;
            if (na > (double)cap) na = (double)cap;
            g.n[a] = (int32_t)na;
            g.stride[a] = C;
            C *= (uint32_t)g.n[a];
            if (a >= 1) runs *= W;
        }
    }
    g.C = C;
    g.runs = runs;
    if (lane == 0) b.grid[e] = g;
    // neighbour runs: offsets in -m..m on grid axes 1..G-1 (base 2m+1
    // digits of the run index) and their key offsets
    for (int s = lane; s < runs; s += 64) {
        RunEntry re;
        re.koff = 0;
#pragma unroll
        for (int a = 0; a < kGMax; ++a) re.o[a] = 0;
#pragma unroll
        for (int a = 0; a < 6; ++a) re.pad[a] = 0;
        int t = s;
#pragma unroll
        for (int a = 1; a < kGMax; ++a) {
            if (a < G) {
                const int o = t % W - m;
                t /= W;
                re.o[a] = (int8_t)o;
                re.koff += o * (int32_t)g.stride[a];
            }
        }
        b.runs[(int64_t)e * kRunsMax + s] = re;
    }
}

// Exclusive scan of the events' cell counts -> cell offsets (one block of
// 256 threads; run by the last block of the plan grid to finish).
__device__ void plan_offsets(Bufs &b, int E) {
    __shared__ int64_t ssum[256];
    const int per = (E + 255) / 256;
    const int e0 = threadIdx.x * per;
    const int e1 = min(E, e0 + per);
    int64_t local = 0;
    for (int e = e0; e < e1; ++e) local += b.grid[e].C;
    ssum[threadIdx.x] = local;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        int64_t v = threadIdx.x >= (unsigned)o ? ssum[threadIdx.x - o] : 0;
        __syncthreads();
        ssum[threadIdx.x] += v;
        __syncthreads();
    }
    int64_t run = ssum[threadIdx.x] - local;
    for (int e = e0; e < e1; ++e) {
        b.cell_off[e] = run;
        run += b.grid[e].C;
    }
    if (threadIdx.x == 255) {
        b.cell_off[E] = ssum[255];
        b.ctr->total_cells = (uint64_t)ssum[255];
    }
}

// ------------------------------------------------------------------ lpt
// Work order of the persistent count pass (one block).  The work items are
// the windows of sorted queries (each a run of cell blocks of one event).
// A window's cost is estimated from its event's grid: points per cell times
// the cells a work group scans, (R + 2m)(2m + 1)^(G-1).  Events are ranked
// by decreasing cost (ties by index: longest processing time first), and
// each of the 8 XCD queues takes an eighth of every event's windows in that
// order, so each XCD's L2 sees contiguous windows and every queue starts
// with the costliest work.
__device__ void lpt_order(Bufs &b, const Knobs &kn) {
    __shared__ float s_cost[kLptMaxEvents];
    __shared__ uint32_t s_nwin[kLptMaxEvents], s_order[kLptMaxEvents];
    if (b.bd->E > kLptMaxEvents) return;  // the host never asks for it then
    const BatchDesc &bd = *b.bd;
    const int E = bd.E, t = threadIdx.x;
    const uint32_t wpc = kChunkRows / kn.window;
    uint32_t *order = b.lpt, *chunk0 = b.lpt + E, *nwin = b.lpt + 2 * E, *pre = b.lpt + 3 * E;
    for (int e = t; e < E; e += blockDim.x) {
        const GridDesc g = b.grid[e];
        const int64_t np = b.ev[e].n_pts, nq = b.ev[e].n_q;
        float nb = 1.0f;
        for (int a = 0; a < g.G; ++a) nb *= (a == 0 ? (float)(kn.cells_per_item + 2 * g.m) : (float)(2 * g.m + 1));
        s_cost[e] = g.G > 0 ? (float)np / (float)max(1u, g.C) * nb : (float)np;
        s_nwin[e] = (uint32_t)((nq + kChunkRows - 1) / kChunkRows) * wpc;
    }
    __syncthreads();
    for (int e = t; e < E; e += blockDim.x) {
        const float c = s_cost[e];
        int rank = 0;
        for (int e2 = 0; e2 < E; ++e2) rank += (s_cost[e2] > c || (s_cost[e2] == c && e2 < e)) ? 1 : 0;
        s_order[rank] = (uint32_t)e;
    }
    __syncthreads();
    for (int e = t; e < E; e += blockDim.x) {
        order[e] = s_order[e];
        nwin[e] = s_nwin[e];
    }
    if (t == 8) {  // chunks of an event are contiguous, events in input order
        uint32_t c = 0;
        for (int e = 0; e < E; ++e) {
            chunk0[e] = c;
            c += s_nwin[e] / wpc;
        }
    }
    if (t < 8) {
        uint32_t acc = 0;
        for (int k = 0; k < E; ++k) {
            pre[t * (E + 1) + k] = acc;
            const uint64_t n = s_nwin[s_order[k]];
            acc += (uint32_t)(n * (t + 1) / 8 - n * t / 8);
        }
        pre[t * (E + 1) + E] = acc;
    }
}

__global__ void __launch_bounds__(256) k_lpt(Bufs b, Knobs kn) { lpt_order(b, kn); }

// ------------------------------------------------------------------ keys
__device__ __forceinline__ uint32_t cell_key(const GridDesc &g, const float *row) {
    uint32_t key = 0;
    for (int a = 0; a < g.G; ++a) {
        double v = ((double)row[g.axis[a]] - g.lo[a]) * g.inv_h;
        v = v > 0.0 ? v : 0.0;
        double top = (double)(g.n[a] - 1);
        v = v < top ? v : top;
        key += (uint32_t)v * g.stride[a];
    }
    return key;
}

__global__ void __launch_bounds__(256) k_keys(Bufs b, int32_t queries) {
    __shared__ GridDesc sg;
    const BatchDesc bd = *b.bd;
    const int D = bd.D;
    const int nch = queries ? bd.n_qchunks : bd.n_pchunks;
    const Chunk *chunks = queries ? b.qchunks : b.pchunks;
    uint32_t *cells = queries ? b.qcells : b.cells;
    uint32_t *keys = queries ? b.qkey : b.key;
    uint32_t *ranks = queries ? b.qrank : b.rank;
    for (int c = blockIdx.x; c < nch; c += gridDim.x) {
        const Chunk ch = chunks[c];
        __syncthreads();
        if (threadIdx.x == 0) sg = b.grid[ch.ev];
        __syncthreads();
        const EventDev ev = b.ev[ch.ev];
        const float *src = queries ? ev.qry : ev.pts;
        const int64_t off = queries ? ev.q_off : ev.pt_off;
        const int64_t coff = b.cell_off[ch.ev];
        for (int64_t i = ch.r0 + threadIdx.x; i < ch.r1; i += blockDim.x) {
            uint32_t k = cell_key(sg, src + (i - off) * D);
            keys[i] = k;
            ranks[i] = atomicAdd(&cells[coff + k], 1u);
        }
    }
}

// Sorted slot of every point: start of its cell plus its rank in the cell.
// Rows are stored padded to Dp floats (zeros), 16-byte aligned.
__global__ void __launch_bounds__(256) k_scatter(Bufs b, int32_t queries) {
    const BatchDesc bd = *b.bd;
    const int D = bd.D, Dp = bd.Dp;
    const int nch = queries ? bd.n_qchunks : bd.n_pchunks;
    const Chunk *chunks = queries ? b.qchunks : b.pchunks;
    const uint32_t *cells = queries ? b.qcells : b.cells;
    const uint32_t *keys = queries ? b.qkey : b.key;
    const uint32_t *ranks = queries ? b.qrank : b.rank;
    float *dst = queries ? b.qs : b.xs;
    int32_t *perm = queries ? b.qperm : b.perm;
    uint32_t *skey = queries ? b.sqkey : b.skey;
    for (int c = blockIdx.x; c < nch; c += gridDim.x) {
        const Chunk ch = chunks[c];
        const EventDev ev = b.ev[ch.ev];
        const float *src = queries ? ev.qry : ev.pts;
        const int64_t off = queries ? ev.q_off : ev.pt_off;
        const int64_t coff = b.cell_off[ch.ev];
        // rows of a multiple of 4 floats from a 16-byte aligned array are
        // read as float4 (the same for every row of the event)
        const bool vec = D == Dp && (reinterpret_cast<uintptr_t>(src) & 15u) == 0;
        for (int64_t i = ch.r0 + threadIdx.x; i < ch.r1; i += blockDim.x) {
            const uint32_t k = keys[i];
            const uint32_t p = cells[coff + k] + ranks[i];
            const float *row = src + (i - off) * D;
            float4 *out = reinterpret_cast<float4 *>(dst + (int64_t)p * Dp);
            if (vec) {
                for (int d4 = 0; d4 < Dp; d4 += 4) out[d4 / 4] = *reinterpret_cast<const float4 *>(row + d4);
            } else {
                for (int d4 = 0; d4 < Dp; d4 += 4) {
                    float4 v;
                    v.x = d4 + 0 < D ? row[d4 + 0] : 0.0f;
                    v.y = d4 + 1 < D ? row[d4 + 1] : 0.0f;
                    v.z = d4 + 2 < D ? row[d4 + 2] : 0.0f;
                    v.w = d4 + 3 < D ? row[d4 + 3] : 0.0f;
                    out[d4 / 4] = v;
                }
            }
            perm[p] = (int32_t)(i - off);
            skey[p] = k;
        }
    }
}

// ------------------------------------------------------------------ scan
// Exclusive scan of pairs of 64-bit values in two launches with a fixed
// grid (block partials; then each block adds its predecessors' partials and
// scans its range).  Modes:
//   0: point cells   (in place, 32-bit)
//   1: query cells   (in place, 32-bit)
//   2: row offsets   deg -> (min(deg, K), deg if the row is long else 0)
enum { kScanCells = 0, kScanQCells = 1, kScanRows = 2 };

template <int MODE>
__device__ __forceinline__ uint64_t scan_n(const Bufs &b) {
    if (MODE == kScanRows) return (uint64_t)b.bd->total_q + 1;
    return (uint64_t)b.cell_off[b.bd->E] + 1;
}

template <int MODE>
__device__ __forceinline__ ulonglong2 scan_load(const Bufs &b, const Knobs &kn, uint64_t i,
                                                uint64_t n) {
    ulonglong2 v;
    v.x = 0;
    v.y = 0;
    if (i >= n) return v;
    if (MODE == kScanCells) {
        v.x = b.cells[i];
    } else if (MODE == kScanQCells) {
        v.x = b.qcells[i];
    } else {
        if (i + 1 < n) {
            uint32_t d = b.deg[i];
            v.x = (kn.K > 0 && d > (uint32_t)kn.K) ? (uint32_t)kn.K : d;
            v.y = d > (uint32_t)kn.stash_cap ? d : 0;
        }
    }
    return v;
}

template <int MODE>
__device__ __forceinline__ void scan_store(const Bufs &b, uint64_t i, ulonglong2 v) {
    if (MODE == kScanCells) {
        b.cells[i] = (uint32_t)v.x;
    } else if (MODE == kScanQCells) {
        b.qcells[i] = (uint32_t)v.x;
    } else {
        b.offs[i] = (int64_t)v.x;
        b.lofs[i] = (int64_t)v.y;
        if (i == (uint64_t)b.bd->total_q) {  // the appended zero: its prefix is the total
            b.ctr->nnz = v.x;
            b.ctr->long_total = v.y;
        }
    }
}

__device__ __forceinline__ ulonglong2 add2(ulonglong2 a, ulonglong2 c) {
    ulonglong2 r;
    r.x = a.x + c.x;
    r.y = a.y + c.y;
    return r;
}

__device__ __forceinline__ ulonglong2 shfl_up2(ulonglong2 v, int o) {
    ulonglong2 r;
    r.x = (unsigned long long)__shfl_up((long long)v.x, o);
    r.y = (unsigned long long)__shfl_up((long long)v.y, o);
    return r;
}

// Block-wide exclusive scan over blockDim.x (<= 1024) threads; returns the
// exclusive prefix and writes the block total.
__device__ ulonglong2 block_excl_scan(ulonglong2 v, ulonglong2 *total) {
    __shared__ ulonglong2 swave[17];  // 16 wave prefixes + the total
    const int l = lane_id(), w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    ulonglong2 inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        ulonglong2 t = shfl_up2(inc, o);
        if (l >= o) inc = add2(inc, t);
    }
    if (l == 63) swave[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        ulonglong2 run;
        run.x = 0;
        run.y = 0;
        for (int i = 0; i < nw; ++i) {
            ulonglong2 t = swave[i];
            swave[i] = run;
            run = add2(run, t);
        }
        swave[16] = run;
    }
    __syncthreads();
    ulonglong2 base = swave[w];
    *total = swave[16];
    __syncthreads();
    ulonglong2 ex;
    ex.x = base.x + inc.x - v.x;
    ex.y = base.y + inc.y - v.y;
    return ex;
}

template <int MODE>
__device__ __forceinline__ void scan_range(const Bufs &b, uint64_t n, uint64_t *lo, uint64_t *hi) {
    const uint64_t tile = (uint64_t)kScanThreads * kScanItems;
    uint64_t per = (n + gridDim.x - 1) / gridDim.x;
    per = (per + tile - 1) / tile * tile;
    *lo = per * blockIdx.x;
    *hi = *lo + per < n ? *lo + per : n;
}

template <int MODE>
__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(Bufs b, Knobs kn) {
    const uint64_t n = scan_n<MODE>(b);
    uint64_t lo, hi;
    scan_range<MODE>(b, n, &lo, &hi);
    ulonglong2 s;
    s.x = 0;
    s.y = 0;
    for (uint64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) s = add2(s, scan_load<MODE>(b, kn, i, n));
    ulonglong2 tot;
    block_excl_scan(s, &tot);
    if (threadIdx.x == 0) {
        b.scan_part[2 * blockIdx.x] = tot.x;
        b.scan_part[2 * blockIdx.x + 1] = tot.y;
    }
}

// Each block adds up the partials of the blocks before it (at most
// kScanBlocks of them), then scans its own range.
template <int MODE>
__global__ void __launch_bounds__(kScanThreads) k_scan_apply(Bufs b, Knobs kn) {
    const uint64_t n = scan_n<MODE>(b);
    uint64_t lo, hi;
    scan_range<MODE>(b, n, &lo, &hi);
    ulonglong2 pre;
    pre.x = 0;
    pre.y = 0;
    for (unsigned j = threadIdx.x; j < blockIdx.x; j += blockDim.x) {
        pre.x += b.scan_part[2 * j];
        pre.y += b.scan_part[2 * j + 1];
    }
    ulonglong2 run;
    block_excl_scan(pre, &run);
    for (uint64_t t0 = lo; t0 < hi; t0 += (uint64_t)kScanThreads * kScanItems) {
        const uint64_t i0 = t0 + (uint64_t)threadIdx.x * kScanItems;
        ulonglong2 v[kScanItems];
        ulonglong2 s;
        s.x = 0;
        s.y = 0;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            v[k] = (i0 + k < hi) ? scan_load<MODE>(b, kn, i0 + k, n) : ulonglong2{0, 0};
            s = add2(s, v[k]);
        }
        ulonglong2 tot;
        ulonglong2 ex = block_excl_scan(s, &tot);
        ex = add2(ex, run);
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            if (i0 + k < hi) scan_store<MODE>(b, i0 + k, ex);
            ex = add2(ex, v[k]);
        }
        run = add2(run, tot);
    }
    if (MODE == kScanRows) {
        // first output pair of every event whose first row this block holds
        // (the host reads these with the counters)
        __syncthreads();
        const BatchDesc &bd = *b.bd;
        for (int e = threadIdx.x; e <= bd.E; e += blockDim.x) {
            const int64_t q = e < bd.E ? b.ev[e].q_off : bd.total_q;
            if ((uint64_t)q >= lo && (uint64_t)q < hi) b.bases[e] = b.offs[q];
        }
    }
}

// ---------------------------------------------------- count and fill pass
template <int DT>
struct QueryRow {
    float q[DT];
};

template <int DT>
struct CandRow {
    float x[(DT + 3) & ~3];
};

// Loads one padded point row (float4 pieces up to D).
template <int DT, bool EXACT_D>
__device__ __forceinline__ void load_row(CandRow<DT> &c, const float *xrow, int D) {
    constexpr int DP = (DT + 3) & ~3;
#pragma unroll
    for (int d4 = 0; d4 < DP; d4 += 4) {
        if (EXACT_D || d4 < D) {
            float4 v = *reinterpret_cast<const float4 *>(xrow + d4);
            c.x[d4] = v.x;
            c.x[d4 + 1] = v.y;
            c.x[d4 + 2] = v.z;
            c.x[d4 + 3] = v.w;
        } else {
            c.x[d4] = c.x[d4 + 1] = c.x[d4 + 2] = c.x[d4 + 3] = 0.0f;
        }
    }
}

// Squared distance in the canonical order: three rounded operations per
// axis, axes 0..D-1, starting from +0.
template <int DT, bool EXACT_D>
__device__ __forceinline__ float dist2(const QueryRow<DT> &qr, const CandRow<DT> &c, int D) {
    float s = 0.0f;
#pragma unroll
    for (int d = 0; d < DT; ++d) {
        if (EXACT_D || d < D) {
            float t = qr.q[d] - c.x[d];
            float u = t * t;
            s = s + u;
        }
    }
    return s;
}

struct WaveLds {
    uint32_t run_base[kRunsMax];
    uint32_t run_pref[kRunsMax + 1];
    unsigned long long starts;  // run starts inside the current chunk (bit per lane); zero between uses
    int32_t cw[kGMax - 1][64];  // grid coordinates 1.. of each window query's cell
};

// Lane (lane ^ j)'s 32-bit value, j a power of two below 64 (a constant
// once the caller's loops are unrolled).  Inside a row of 16 lanes the move
// is a DPP operand (no LDS traffic): xor 1 and 2 are quad permutations, xor
// 4 a mirror of each 8 lanes followed by a reversal of each 4
// (i ^ 7 ^ 3 = i ^ 4), xor 8 a rotation of the row by 8; xor 16 is a
// swizzle in bitmask mode (and 31, xor 16) and xor 32 a permute.
__device__ __forceinline__ uint32_t xor_lane32(uint32_t v, int j) {
    const int x = (int)v;
    switch (j) {
        case 1: return (uint32_t)__builtin_amdgcn_update_dpp(0, x, 0xB1, 0xf, 0xf, true);  // quad_perm 1,0,3,2
        case 2: return (uint32_t)__builtin_amdgcn_update_dpp(0, x, 0x4E, 0xf, 0xf, true);  // quad_perm 2,3,0,1
        case 4: {
            const int t = __builtin_amdgcn_update_dpp(0, x, 0x141, 0xf, 0xf, true);        // row_half_mirror
            return (uint32_t)__builtin_amdgcn_update_dpp(0, t, 0x1B, 0xf, 0xf, true);      // quad_perm 3,2,1,0
        }
        case 8: return (uint32_t)__builtin_amdgcn_update_dpp(0, x, 0x128, 0xf, 0xf, true);  // row_ror:8
        case 16: return (uint32_t)__builtin_amdgcn_ds_swizzle(x, 0x401F);
        default: return (uint32_t)__shfl_xor(x, j);
    }
}

__device__ __forceinline__ uint64_t xor_lane64(uint64_t v, int j) {
    return ((uint64_t)xor_lane32((uint32_t)(v >> 32), j) << 32) | xor_lane32((uint32_t)v, j);
}

// Sorts R independent sets of the wave's 64*KS keys ascending with a
// bitonic network, stage by stage for all R (independent work in flight
// while each cross-lane move completes): lane i holds elements
// KS*i .. KS*i + KS-1 of set r in v[r][0..KS-1], so a compare-exchange whose
// partner distance j is below KS pairs two registers of one lane and only
// the 21 stages with j >= KS read another lane (lane i ^ j/KS, the same
// register).  Afterwards element e of each set is its e-th smallest key.
template <int KS, int R>
__device__ __forceinline__ void wave_bitonic(uint64_t (&v)[R][KS], int lane) {
#pragma unroll
    for (int kk = 2; kk <= 64 * KS; kk <<= 1) {
#pragma unroll
        for (int j = kk >> 1; j > 0; j >>= 1) {
            if (j < KS) {
#pragma unroll
                for (int r = 0; r < R; ++r)
#pragma unroll
                    for (int k = 0; k < KS; ++k) {
                        const int l = k ^ j;
                        if (l > k) {
                            const bool asc = (((lane * KS) | k) & kk) == 0;
                            const uint64_t a = v[r][k], c = v[r][l];
                            const bool sw = asc ? (c < a) : (a < c);
                            v[r][k] = sw ? c : a;
                            v[r][l] = sw ? a : c;
                        }
                    }
            } else {
                const int jl = j / KS;
                // kk > j >= KS: the direction bit is in the lane number
                const bool asc = ((lane * KS) & kk) == 0;
                const bool lower = (lane & jl) == 0;
                // the lower element of an ascending pair keeps the minimum
                const bool take_min = lower == asc;
#pragma unroll
                for (int r = 0; r < R; ++r)
#pragma unroll
                    for (int k = 0; k < KS; ++k) {
                        const uint64_t p = xor_lane64(v[r][k], jl);
                        const bool less = p < v[r][k];
                        v[r][k] = (less == take_min) ? p : v[r][k];
                    }
            }
        }
    }
}

// Sorts the n <= 64*KS keys h[0..n) of one row (slots past n hold all-ones
// keys, which compare above every key of a row and stay at the end) and
// writes the first keep in order, coalesced.
template <int KS>
__device__ __forceinline__ void sort_and_write(const uint64_t *h, uint32_t n, uint32_t keep, int32_t *idx,
                                               float *d2, int lane) {
    uint64_t v[1][KS];
#pragma unroll
    for (int k = 0; k < KS; ++k) {
        const uint32_t e = (uint32_t)(lane * KS + k);
        v[0][k] = e < n ? h[e] : ~0ull;
    }
    wave_bitonic<KS, 1>(v, lane);
#pragma unroll
    for (int k = 0; k < KS; ++k) {
        const uint32_t e = (uint32_t)(lane * KS + k);
        if (e < keep) {
            idx[e] = (int32_t)(uint32_t)v[0][k];
            if (d2) d2[e] = __uint_as_float((uint32_t)(v[0][k] >> 32));
        }
    }
}

// Position of candidate v (0 <= v < L) among the group's concatenated runs.
__device__ __forceinline__ uint32_t locate(const WaveLds &s, int nruns, uint32_t v) {
    int lo = 0, hi = nruns - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (s.run_pref[mid] <= v)
            lo = mid;
        else
            hi = mid - 1;
    }
    return s.run_base[lo] + (v - s.run_pref[lo]);
}

// True when the run's output fits the output's capacities (every block of
// a fill kernel reads the same counters, so a block leaves whole).
__device__ __forceinline__ bool out_fits(const Bufs &b) {
    return (int64_t)b.ctr->nnz <= b.out->cap_pairs && (int64_t)b.ctr->long_total <= b.out->cap_long;
}

// Work assignment.  The sorted queries of each event are cut into windows
// of kn.window (<= 64) consecutive slots (each chunk of kChunkRows slots
// holds kChunkRows / window of them).  A wave evaluates one window at a time.
// Workgroups are dispatched to the 8 XCDs round robin, so the windows are
// remapped to give every XCD one contiguous range (neighbouring windows
// read the same points, which then stay in that XCD's L2).
//   plain:      one window per wave, grid covers all windows
//   persistent: resident waves drain 8 per-XCD queues of windows, then
//               help the other XCDs' queues
//
// Inside a window, one lane per query loads its cell key, original index and
// (fill pass) row length and scratch offset, and the query rows go to LDS,
// all in one round of parallel loads; the window's cell-block groups are the
// runs of equal block keys (a ballot).  For each group the wave lists the
// neighbour key runs (the next group's runs are fetched while this group is
// evaluated) and evaluates every query of the group against each chunk of 64
// candidates, one per lane.  The fill pass takes only the windows the count
// pass listed, and sorts each long row of a group as soon as the group is done.
// rows of fewer floats than this load the next candidate chunk while the
// current one is evaluated
constexpr int kPrefetchBelow = 8;
// rows of at least this many floats run the window bookkeeping and the
// per-query loop on scalar registers
constexpr int kScalarWaveFrom = 12;

// The query rows of each wave's window (window x DP floats per wave), in the
// launch's dynamic LDS, so that the block's LDS follows the window size.
extern __shared__ float4 q_rows_lds[];

template <int DT, bool EXACT_D, bool FILL, bool PERS, bool EXCL>
__device__ __forceinline__ void query_body(Bufs &b, Knobs &kn) {
    constexpr int DP = (DT + 3) & ~3;
    __shared__ WaveLds slds[kWavesPerBlock];
    __shared__ unsigned long long s_cand[kWavesPerBlock];
    __shared__ uint32_t s_groups[kWavesPerBlock];
    const int lane = lane_id();
    // the wave's index; read through a scalar register, everything derived
    // from it (window, chunk, group bounds, the query loop) is scalar
    const int w = DT >= kScalarWaveFrom ? (int)uniform(threadIdx.x >> 6) : (int)(threadIdx.x >> 6);
    WaveLds &L = slds[w];
    if (lane_id() == 0) L.starts = 0;
    wave_lds_sync();
    const BatchDesc &bd = *b.bd;
    const int D = EXACT_D ? DT : bd.D;
    const int Dp = EXACT_D ? DP : bd.Dp;
    const float r2 = kn.r2;
    const uint32_t SC = (uint32_t)kn.stash_cap;
    const uint32_t *cells = b.cells;
    const uint32_t *sqkey = kn.self_query ? b.skey : b.sqkey;
    const float *qs = kn.self_query ? b.xs : b.qs;
    const int32_t *qperm = kn.self_query ? b.perm : b.qperm;
    uint64_t *long_keys = FILL ? b.out->long_keys : nullptr;
    const int Wn = kn.window;
    float4 *const sq = q_rows_lds + (int64_t)w * Wn * (DP / 4);  // this wave's rows
    const uint32_t wpc = kChunkRows / Wn;
    const uint32_t nwin = (uint32_t)bd.n_qchunks * wpc;
    uint64_t my_cand = 0;
    uint32_t my_groups = 0;
    uint32_t win_fill = 0;  // count pass: the window's fill work (long queries x candidates)
    bool more = false;  // count pass: the window holds a row longer than the stash

    auto process_window = [&](uint32_t wid) {
        const uint32_t c = wid / wpc, sub = wid % wpc;
        if (c >= (uint32_t)bd.n_qchunks) return;
        const Chunk ch = b.qchunks[c];
        const int64_t p0 = ch.r0 + (int64_t)sub * Wn;
        const int64_t pend = min(ch.r1, p0 + Wn);
        if (p0 >= pend) return;
        const int nwq = (int)(pend - p0);
        const int e = ch.ev;
        const GridDesc &g = b.grid[e];
        const int G = g.G, m = g.m, runs = g.runs;
        // the per-axis cell counts, read once per window into scalar
        // registers (all loads together): read through the reference inside
        // the group loop, the compiler reloads them after every store, one
        // dependent round trip per axis and probe
        int gn[kGMax];
#pragma unroll
        for (int a = 0; a < kGMax; ++a) gn[a] = (int)uniform((uint32_t)g.n[a]);
        const int n0 = G > 0 ? gn[0] : 1;
        const int R = kn.cells_per_item;
        const int64_t coff = b.cell_off[e];
        const int64_t q_off = b.ev[e].q_off;
        const RunEntry *rtab = b.runs + (int64_t)e * kRunsMax;
        // one lane per query of the window
        const bool inw = lane < nwq;
        const uint32_t wkey = inw ? sqkey[p0 + lane] : 0u;
        const int32_t wperm = inw ? qperm[p0 + lane] : 0;
        // one run-table entry per lane, loaded once per window (tables with
        // more than 64 runs, and rows of more than 8 floats, are read per
        // group instead: there it was measured faster)
        RunEntry wre{};
        if (DT <= 8 && lane < runs) wre = rtab[lane];
        const uint32_t wdeg = (FILL && inw) ? b.deg[q_off + wperm] : 0u;
        const int64_t wrow = (FILL && inw) ? b.lofs[q_off + wperm] : 0;  // scratch row (fill pass)
        // its address (fill pass)
        const int64_t wrp = FILL ? (int64_t)(uintptr_t)(long_keys + wrow) : 0;
        const int64_t woffs = (FILL && inw) ? b.offs[q_off + wperm] : 0;  // output row (fill pass)
        // stash row address (count pass)
        const int64_t wst = (!FILL && inw) ? (int64_t)(uintptr_t)(b.stash + (q_off + wperm) * (int64_t)SC) : 0;
        uint64_t need = ballot(inw);
        if (FILL) {
            need = ballot(inw && wdeg > SC);  // rows the stash did not hold
            if (!need) return;
        }
        {
            const float4 *src = reinterpret_cast<const float4 *>(qs + p0 * Dp);
            float4 *dst = sq;
            for (int i = lane; i < nwq * (Dp / 4); i += 64) dst[i] = src[i];
        }
        // grid coordinates of each lane's query cell, decoded once per window
        // (coordinate 0 stays in a register; the others go to LDS and are read
        // back per group, which keeps them out of the registers of the loop)
        int cw0 = 0;
        {
            uint32_t rem = wkey;
#pragma unroll
            for (int a = 0; a < kGMax; ++a) {
                int ca = 0;
                if (a < G) {
                    ca = (int)(rem % (uint32_t)gn[a]);
                    rem /= (uint32_t)gn[a];
                }
                if (a == 0)
                    cw0 = ca;
                else
                    L.cw[a - 1][lane] = ca;
            }
        }
        const uint32_t c0 = (uint32_t)cw0;
        const uint32_t bkey = wkey - c0 + (c0 / R) * R;  // key of the cell block's first cell
        const uint32_t prev = (uint32_t)__shfl_up((int)bkey, 1);
        const uint64_t starts = ballot(inw && (lane == 0 || bkey != prev));
        // groups with work: those holding a needed query
        uint64_t todo = 0;
        for (uint64_t sm = starts; sm;) {
            const int gb = __ffsll((unsigned long long)sm) - 1;
            sm &= sm - 1;
            const int ge = sm ? __ffsll((unsigned long long)sm) - 1 : nwq;
            const uint64_t range = (ge >= 64 ? ~0ull : ((1ull << ge) - 1)) & ~((1ull << gb) - 1);
            if (need & range) todo |= 1ull << gb;
        }
        wave_lds_sync();

        // every load of the window's setup is complete here: the group loop
        // then waits only for its own loads (the compiler cannot count loads
        // issued before a loop, and would wait for all of them at the first
        // use of one)
        __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
        // neighbour runs of the group whose first query is window lane gb:
        // lane s < runs probes run s
        // (start, end) of the run in the sorted points; the subtraction is
        // left to commit, so a probe made ahead is not waited for until then
        auto probe = [&](int gb, int s, uint32_t &start, uint32_t &end) {
            start = 0;
            end = 0;
            if (s >= runs) return;
            const uint32_t key = (uint32_t)__builtin_amdgcn_readlane((int)wkey, gb);
            int cc[kGMax];
#pragma unroll
            for (int a = 0; a < kGMax; ++a)
                cc[a] = a == 0 ? __builtin_amdgcn_readlane(cw0, gb) : (int)uniform((uint32_t)L.cw[a - 1][gb]);
            int lo0 = 0, hi0 = 0;
            uint32_t kbase = key;
            if (G > 0) {
                const int b0 = (cc[0] / R) * R;
                const int b1 = min(b0 + R - 1, n0 - 1);
                kbase = key - (uint32_t)cc[0];
                lo0 = max(b0 - m, 0);
                hi0 = min(b1 + m, n0 - 1);
            }
            const RunEntry re = (DT <= 8 && runs <= 64) ? wre : rtab[s];
            bool ok = true;
#pragma unroll
            for (int a = 1; a < kGMax; ++a) {
                if (a < G) {
                    const int ca = cc[a] + re.o[a];
                    ok = ok & (ca >= 0) & (ca < gn[a]);  // no short circuit: no branch per axis
                }
            }
            if (ok) {
                const int64_t k0 = coff + (int64_t)kbase + re.koff;
                start = cells[k0 + lo0];
                end = cells[k0 + hi0 + 1];
            }
        };
        // compacts probed runs into the LDS table from entry tb; returns the
        // candidates so far
        auto commit = [&](int tb, uint32_t start, uint32_t end, uint32_t &total, int &nruns) {
            const uint32_t len = end - start;
            const uint64_t nz = ballot(len > 0);
            const uint32_t inc = wave_incl_scan(len);
            if (len > 0) {
                const int at = tb + nruns + (int)lanes_below(nz);
                L.run_base[at] = start;
                L.run_pref[at] = total + inc - len;
            }
            total += (uint32_t)__builtin_amdgcn_readlane((int)inc, 63);
            nruns += __popcll(nz);
        };

        // With at most 64 runs the run table has two halves: the next
        // group's runs are probed and committed into one while the current
        // group's, in the other, are read.
        const bool one_batch = runs <= 64;
        constexpr int kHalf = kRunsMax / 2;
        int t_next = 0;  // half holding the next group's runs
        uint32_t tot_next = 0;
        int nr_next = 0;
        auto commit_next = [&](int tb, uint32_t st0, uint32_t en0) {
            t_next = tb;
            tot_next = 0;
            nr_next = 0;
            commit(tb, st0, en0, tot_next, nr_next);
            if (lane == 0) L.run_pref[tb + nr_next] = tot_next;
        };
        if (one_batch && todo) {
            uint32_t st0, en0;
            probe(__ffsll((unsigned long long)todo) - 1, lane, st0, en0);
            commit_next(0, st0, en0);
        }
        while (todo) {
            const int gb = __ffsll((unsigned long long)todo) - 1;
            todo &= todo - 1;
            const uint64_t later = starts & ~((2ull << gb) - 1);
            const int ge = later ? __ffsll((unsigned long long)later) - 1 : nwq;
            ++my_groups;
            uint32_t total = 0;
            int nruns = 0, tb0 = 0;
            if (one_batch) {
                total = tot_next;
                nruns = nr_next;
                tb0 = t_next;
            } else {
                for (int s0 = 0; s0 < runs; s0 += 64) {
                    uint32_t st0, en0;
                    probe(gb, s0 + lane, st0, en0);
                    commit(0, st0, en0, total, nruns);
                }
                if (lane == 0) L.run_pref[nruns] = total;
            }
            wave_lds_sync();
            {
                // candidates in chunks of 64 (one per lane), every query of the
                // group against each chunk while the next chunk loads; lane t
                // keeps the running count of window query t.  The count pass
                // keeps each query's first SC hit keys in its stash row; the
                // fill pass evaluates only the queries with longer rows and
                // writes all their hit keys to their scratch rows, whose
                // lengths are the counts
                uint32_t cntv = 0;
                uint32_t pn = 0, jn = 0;
                CandRow<DT> xn;
                // with at most 64 runs, lane s holds run s's first candidate
                // number; a candidate's run is the number of runs starting at
                // or before it, minus one (runs are non-empty, so their
                // starts are distinct), counted with one 64-bit word of run
                // starts per chunk
                const bool few = nruns <= 64;
                const uint32_t rp = (few && lane < nruns) ? L.run_pref[tb0 + lane] : 0xffffffffu;
                auto fetch = [&](uint32_t v0) {
                    const uint32_t v = v0 + lane;
                    if (few) {
                        if (rp >= v0 && rp - v0 < 64u) atomicOr(&L.starts, 1ull << (rp - v0));
                        wave_lds_sync();
                        const uint64_t sm = L.starts;
                        wave_lds_sync();
                        if (lane == 0) L.starts = 0;
                        const uint32_t before = (uint32_t)__popcll(ballot(rp < v0));
                        const uint32_t kr = before + lanes_below(sm) + (uint32_t)((sm >> lane) & 1ull) - 1u;
                        pn = v < total ? L.run_base[tb0 + kr] + (v - L.run_pref[tb0 + kr]) : 0u;
                    } else {
                        pn = v < total ? locate(L, nruns, v) : 0u;  // (one table: tb0 == 0)
                    }
                    // the index before the row: waiting for the row (always
                    // used) then covers the index (used only by hits)
                    jn = (uint32_t)b.perm[pn];
                    load_row<DT, EXACT_D>(xn, b.xs + (int64_t)pn * Dp, D);
                };
                // the next group's probe is issued first and this group's first
                // chunk second, so their round trips overlap, and committing
                // the probe (a wait for its loads) leaves the chunk's loads in
                // flight (loads complete in issue order)
                // (the first chunk is fetched even when the group has no
                // candidate, lanes past the end reading row 0, so that the
                // loads in flight at the commit are the same on every path)
                const bool ahead = one_batch && todo;
                uint32_t pst = 0, pen = 0;
                if (ahead) probe(__ffsll((unsigned long long)todo) - 1, lane, pst, pen);
                fetch(0);
                if (ahead) commit_next(tb0 ^ kHalf, pst, pen);
                // one query of the group against one chunk; self-exclusion is
                // decided once per launch (two copies of the loop)
                auto eval_chunk = [&](auto excl, uint32_t pos, uint32_t j, const CandRow<DT> &x, float thr) {
                    // the group's query range through scalar registers: the
                    // loop index is then scalar
                    const int tb = (int)uniform((uint32_t)gb), te = (int)uniform((uint32_t)ge);
                    // a group holds at least one query (tb < te): the first
                    // pass always reads the chunk, so the compiler knows its
                    // loads are complete afterwards and does not wait for the
                    // stores made meanwhile before the next chunk's loads
                    int t = tb;
                    do {
                        if constexpr (FILL)
                            if ((uint32_t)__builtin_amdgcn_readlane((int)wdeg, t) <= SC) continue;
                        QueryRow<DT> qr;
#pragma unroll
                        for (int d4 = 0; d4 < DP; d4 += 4) {
                            if (EXACT_D || d4 < Dp) {
                                const float4 v = sq[t * (Dp / 4) + d4 / 4];
                                qr.q[d4] = v.x;
                                if (d4 + 1 < DT) qr.q[d4 + 1] = v.y;
                                if (d4 + 2 < DT) qr.q[d4 + 2] = v.z;
                                if (d4 + 3 < DT) qr.q[d4 + 3] = v.w;
                            }
                        }
                        const float s = dist2<DT, EXACT_D>(qr, x, D);
                        // thr < 0 on lanes past the group's candidates; with
                        // self-exclusion the mask comes from two ballots of
                        // plain compares and each lane tests its own bit
                        const bool in = s <= thr;
                        uint64_t hm = ballot(in);
                        if constexpr (decltype(excl)::value) hm &= ~ballot(pos == (uint32_t)(p0 + t));
                        const bool hit = decltype(excl)::value ? ((hm >> lane) & 1ull) != 0 : in;
                        if (hm) {
                            const uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)cntv, t);
                            if constexpr (FILL) {
                                const uint32_t slot = c + lanes_below(hm);
                                if (hit && slot < (uint32_t)__builtin_amdgcn_readlane((int)wdeg, t))
                                    *(FRNN_GLOBAL uint64_t *)((FRNN_GLOBAL char *)(uintptr_t)readlane64(wrp, t) +
                                                         (uint32_t)(slot * 8u)) =
                                        ((uint64_t)__float_as_uint(s) << 32) | j;
                            } else if (c < SC) {
                                // the first SC hit keys of each query go to its stash row
                                const uint32_t slot = c + lanes_below(hm);
                                if (hit && slot < SC) {
                                    // row address in scalar registers, the slot's byte
                                    // offset in a 32-bit vector register (one add in the
                                    // store's addressing instead of 64-bit arithmetic)
                                    *(FRNN_GLOBAL uint64_t *)((FRNN_GLOBAL char *)(uintptr_t)readlane64(wst, t) +
                                                         (uint32_t)(slot * 8u)) =
                                        ((uint64_t)__float_as_uint(s) << 32) | j;
                                }
                            }
                            // query t's count lives in lane t (t is scalar; every
                            // lane is active here), updated by a single lane write
                            cntv = (uint32_t)frnn_writelane_i32((int)(c + (uint32_t)__popcll(hm)), t, (int)cntv);
                        }
                    } while (++t < te);
                };
                if constexpr (DT >= kPrefetchBelow) {
                    // rows of 8 floats or more: no next-chunk prefetch (one
                    // candidate row live instead of two; measured faster at
                    // D = 8 and D = 12, where the extra resident waves hide
                    // the load instead).  The first chunk (fetched above; a
                    // group without candidates evaluates it with every lane
                    // past the end) is evaluated before the loop, so every
                    // path into the loop has its loads complete
                    eval_chunk(std::integral_constant<bool, EXCL>{}, pn, jn, xn, lane < total ? r2 : -1.0f);
                    for (uint32_t v0 = 64; v0 < total; v0 += 64) {
                        fetch(v0);
                        eval_chunk(std::integral_constant<bool, EXCL>{}, pn, jn, xn, v0 + lane < total ? r2 : -1.0f);
                    }
                } else {
                    for (uint32_t v0 = 0; v0 < total; v0 += 64) {
                        const uint32_t pos = pn, j = jn;
                        const CandRow<DT> x = xn;
                        const float thr = v0 + lane < total ? r2 : -1.0f;
                        if (v0 + 64 < total) fetch(v0 + 64);
                        eval_chunk(std::integral_constant<bool, EXCL>{}, pos, j, x, thr);
                    }
                }
                const bool mine = lane >= gb && lane < ge;
                if constexpr (FILL) {
                    // each long row received exactly its counted hits; the
                    // rows are listed for the row sort (one atomic per group)
                    const bool lst = mine && wdeg > SC;
                    if (ballot(lst && cntv != wdeg) && lane == 0) atomicOr(&b.ctr->status, kStatusInternal);
                    const uint64_t lm = ballot(lst);
                    uint32_t base = 0;
                    if (lane == 0) base = atomicAdd(&b.ctr->n_long, (uint32_t)__popcll(lm));
                    base = uniform((uint32_t)__shfl((int)base, 0));
                    if (lst) {
                        const uint32_t li = base + lanes_below(lm);
                        b.long_rows[li] = wdeg;
                        *reinterpret_cast<longlong2 *>(b.long_at + 2 * (int64_t)li) = make_longlong2(wrow, woffs);
                    }
                } else {
                    if (mine) b.deg[q_off + wperm] = cntv;
                    const uint32_t nlong = (uint32_t)__popcll(ballot(mine && cntv > SC));
                    more = more || nlong != 0;
                    win_fill += nlong * total;
                    my_cand += (uint64_t)total * (uint64_t)(ge - gb);
                }
            }
            wave_lds_sync();
        }
        if (!FILL && more) {
            // the costlier windows from the front of the list, so that the
            // fill pass starts them first (longest processing time first)
            if (lane == 0) {
                if (win_fill >= kFillHeavy)
                    b.fill_list[atomicAdd(&b.ctr->n_fill, 1u)] = wid;
                else
                    b.fill_list[kn.fill_cap - 1u - atomicAdd(&b.ctr->n_fill_light, 1u)] = wid;
            }
            more = false;
        }
        win_fill = 0;
    };

    if constexpr (FILL) {
        // the listed windows: the heavier ones (front of the list) first,
        // then the lighter ones (back of the list)
        const uint32_t nh = b.ctr->n_fill, n = nh + b.ctr->n_fill_light;
        auto listed = [&](uint32_t i) { return b.fill_list[i < nh ? i : kn.fill_cap - 1u - (i - nh)]; };
        if constexpr (PERS) {
            // persistent: the resident waves take the list round robin
            // (heaviest first), without atomics
            const uint32_t nw = gridDim.x * kWavesPerBlock;
            for (uint32_t i = uniform(blockIdx.x * kWavesPerBlock + (uint32_t)w); i < n; i += nw)
                process_window(listed(i));
        } else {
            const uint32_t nw = gridDim.x * kWavesPerBlock;
            for (uint32_t i = blockIdx.x * kWavesPerBlock + w; i < n; i += nw) process_window(listed(i));
        }
    } else if constexpr (PERS) {
        // persistent: the resident waves of each XCD take its queue (built
        // by k_lpt: costliest events first) round robin.  The queue is dealt
        // statically: a shared counter per queue costs a device-scope atomic
        // per window, and those on one address were measured to serialise
        // at a few hundred nanoseconds each, slower than the whole pass
        const BatchDesc &bdr = *b.bd;
        const uint32_t E = (uint32_t)bdr.E;
        const uint32_t x = blockIdx.x & 7;
        const uint32_t wx = uniform((blockIdx.x >> 3) * kWavesPerBlock + (uint32_t)w);
        const uint32_t Wx = (gridDim.x >> 3) * kWavesPerBlock;  // grid is a multiple of 8 blocks
        const uint32_t *order = b.lpt, *chunk0 = b.lpt + E, *nwe = b.lpt + 2 * E;
        const uint32_t *pre = b.lpt + 3 * E + x * (E + 1);
        const uint32_t nx = pre[E];
        uint32_t k = 0, kend = pre[1];
        for (uint32_t v = wx; v < nx; v += Wx) {
            while (kend <= v) kend = pre[++k + 1];
            const uint32_t e = order[k];
            const uint32_t we = (uint32_t)((uint64_t)nwe[e] * x / 8) + (v - pre[k]);
            process_window(chunk0[e] * wpc + we);
        }
    } else {
        const uint32_t nb = gridDim.x, per = nb / 8;  // grid is a multiple of 8 blocks
        const uint32_t vb = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
        const uint32_t wid = vb * kWavesPerBlock + w;
        if (wid < nwin) process_window(wid);
    }
    // one atomic per workgroup for the work counters
    if (!FILL) {
        if (lane == 0) {
            s_cand[w] = my_cand;
            s_groups[w] = my_groups;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long cs = 0;
            uint32_t gsum = 0;
            for (int i = 0; i < kWavesPerBlock; ++i) {
                cs += s_cand[i];
                gsum += s_groups[i];
            }
            if (cs) atomicAdd((unsigned long long *)&b.ctr->candidates, cs);
            if (gsum) atomicAdd(&b.ctr->n_groups, gsum);
        }
    }
}

// Two entry points with the same body: the second asks the compiler for at
// least 5 resident waves per SIMD (at most 96 registers), used for the
// count pass at D = 8 and D = 12 and the D = 12 fill without self-exclusion,
// each of which fits that bound without spilling.
// PERS selects the persistent scheduling at compile time, so each kernel
// holds one copy of the window body.
template <int DT, bool EXACT_D, bool FILL, bool PERS, bool EXCL>
__global__ void __launch_bounds__(256) k_query(Bufs b, Knobs kn) {
    if constexpr (FILL)
        if (!out_fits(b)) return;
    query_body<DT, EXACT_D, FILL, PERS, EXCL>(b, kn);
}


template <int DT, bool EXACT_D, bool FILL, bool PERS, bool EXCL>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) k_query_o5(Bufs b, Knobs kn) {
    if constexpr (FILL)
        if (!out_fits(b)) return;
    query_body<DT, EXACT_D, FILL, PERS, EXCL>(b, kn);
}

// ------------------------------------------------------------ short rows
// Ascending bitonic network over N keys held in registers (compile-time
// indices: no cross-lane traffic).
template <int N>
__device__ __forceinline__ void sort_regs(uint64_t (&v)[N]) {
#pragma unroll
    for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const int l = i ^ j;
                if (l > i) {
                    const uint64_t a = v[i], c = v[l];
                    const bool sw = ((i & k) == 0) ? (a > c) : (a < c);
                    v[i] = sw ? c : a;
                    v[l] = sw ? a : c;
                }
            }
        }
    }
}

// Every row's per-event offset, and the rows the count pass kept whole
// (0 < length <= SC): one lane per query row, in output order, sorts the
// row's keys in registers (rows of up to 16 keys); rows of 17..SC keys (the
// 32-, 64-, 128- and 256-key stashes) are sorted by the whole wave with the
// bitonic network of the long-row sort.  The query chunks partition
// each event's rows, so
// chunk c covers global rows r0..r1-1 of one event and its output is the
// contiguous range offs[r0]..offs[r1]; one block per chunk.  When that range
// fits in LDS the rows are assembled there and written out coalesced; the
// places of longer rows receive filler that the fill pass, which runs later
// on the same stream, overwrites.
// Staged output pairs per block: with the mid-row list the block stays
// within 32 KB of LDS (five blocks per CU).
constexpr int short_stage(int sc) {
    return sc > 128 ? kChunkRows * 13 : sc > 64 ? kChunkRows * 27 / 2 : kChunkRows * 29 / 2;
}

template <int N>
__device__ __forceinline__ void place_row(uint64_t (&v)[N], uint32_t keep, bool staged, int64_t rel,
                                          uint32_t *sidx, float *sd2, int32_t *oi, float *od) {
    sort_regs<N>(v);
#pragma unroll
    for (int i = 0; i < N; ++i) {
        if ((uint32_t)i < keep) {
            const uint32_t j = (uint32_t)v[i];
            const float d = __uint_as_float((uint32_t)(v[i] >> 32));
            if (staged) {
                sidx[rel + i] = j;
                sd2[rel + i] = d;
            } else {
                oi[i] = (int32_t)j;
                if (od) od[i] = d;
            }
        }
    }
}

__device__ __forceinline__ void publish_block(const Publish &p);

template <int SC>
__global__ void __launch_bounds__(kChunkRows) __attribute__((amdgpu_waves_per_eu(5))) k_short_rows(Bufs b, Knobs kn,
                                                                                                   Publish pub) {
    // rows of up to LM keys: one lane per row; longer stash rows (up to SC):
    // one wave per row, ranked
    constexpr int LM = SC < 16 ? SC : 16;
    constexpr int kShortStage = short_stage(SC);
    __shared__ uint32_t sidx[SC > 0 ? kShortStage : 1];
    __shared__ float sd2[SC > 0 ? kShortStage : 1];
    __shared__ uint16_t s_mid[SC > LM ? kChunkRows : 1];  // rows of LM+1..min(SC, 128) keys
    __shared__ uint16_t s_huge[SC > 128 ? kChunkRows : 1];  // rows of 129..SC keys
    __shared__ uint32_t s_nmid, s_nbig, s_nhuge;
    // the read-back of the counts when this launch follows the count pass
    // directly (the host needs them whether or not the output fits)
    if (pub.flag && blockIdx.x == 0) publish_block(pub);
    if (!out_fits(b)) return;
    if (blockIdx.x == 0)  // each event's leading offset, the one entry no row writes
        for (int e = threadIdx.x; e < b.bd->E; e += blockDim.x) b.out->offsets[b.ev[e].q_off + e] = 0;
    if (blockIdx.x >= (unsigned)b.bd->n_qchunks) return;
    const Chunk ch = b.qchunks[blockIdx.x];
    const int64_t qid = ch.r0 + (int64_t)threadIdx.x;
    const bool row = qid < ch.r1;
    const int e = ch.ev;
    const int64_t off = row ? b.offs[qid] : 0;
    if (row) b.out->offsets[qid + e + 1] = b.offs[qid + 1] - b.bases[e];
    if constexpr (SC > 0) {
        const int64_t base = b.offs[ch.r0];
        const int64_t len = b.offs[ch.r1] - base;
        const bool staged = len <= kShortStage;
        int32_t *oi = b.out->indices + off;
        float *od = b.out->dist2 ? b.out->dist2 + off : nullptr;
        // the first LM/2 keys of the stash row are read before the row
        // length arrives (one memory round trip less; most rows are that
        // short), the next LM/2 only for longer rows; entries past the
        // length are masked afterwards
        const uint64_t *st = b.stash + qid * SC;
        uint64_t v[LM];
#pragma unroll
        for (int i = 0; i < LM; i += 2) {
            ulonglong2 t = make_ulonglong2(~0ull, ~0ull);
            if (row && i < LM / 2) t = *reinterpret_cast<const ulonglong2 *>(st + i);
            v[i] = t.x;
            v[i + 1] = t.y;
        }
        const uint32_t dq = row ? b.deg[qid] : 0u;
        const bool mine = dq > 0 && dq <= (uint32_t)LM;
        const bool full = ballot(mine && dq > (uint32_t)(LM / 2)) != 0;  // network size, per wave
        if (mine) {
            const uint32_t keep = (kn.K > 0 && dq > (uint32_t)kn.K) ? (uint32_t)kn.K : dq;
            if (dq > (uint32_t)(LM / 2)) {
#pragma unroll
                for (int i = LM / 2; i < LM; i += 2) {
                    const ulonglong2 t = *reinterpret_cast<const ulonglong2 *>(st + i);
                    v[i] = t.x;
                    v[i + 1] = t.y;
                }
            }
#pragma unroll
            for (int i = 0; i < LM; ++i)
                if ((uint32_t)i >= dq) v[i] = ~0ull;
            if (full) {
                place_row<LM>(v, keep, staged, off - base, sidx, sd2, oi, od);
            } else {
                uint64_t h[LM / 2];
#pragma unroll
                for (int i = 0; i < LM / 2; ++i) h[i] = v[i];
                place_row<LM / 2>(h, keep, staged, off - base, sidx, sd2, oi, od);
            }
        }
        if constexpr (SC > LM) {
            // stash rows of LM+1..SC keys: the block lists them in LDS (rows
            // of up to 64 keys from the front of one list, 65..128 keys from
            // its back, longer ones in a second list) and its waves take them
            // in turn, RB at a time (a block of dense rows keeps all four
            // busy); lane i holds keys KS*i .. KS*i + KS-1 of each row (KS =
            // 1 up to 64 keys, 2 up to 128, else 4; slots past a row's length
            // read as all ones) and the wave sorts the RB rows together with
            // the wave-wide bitonic network (rows past the list are all ones
            // and are not written)
            const int lane = lane_id(), wv = threadIdx.x >> 6;
            if (threadIdx.x == 0) {
                s_nmid = 0;
                s_nbig = 0;
                s_nhuge = 0;
            }
            __syncthreads();
            const bool midr = row && dq > (uint32_t)LM && dq <= (uint32_t)SC;
            const bool huge = midr && dq > 128u;
            const bool big = midr && dq > 64u && !huge;
            const uint64_t mm = ballot(midr && dq <= 64u), mb = ballot(big);
            if (mm) {
                uint32_t at = 0;
                if (lane == 0) at = atomicAdd(&s_nmid, (uint32_t)__popcll(mm));
                at = uniform((uint32_t)__shfl((int)at, 0));
                if (midr && dq <= 64u) s_mid[at + lanes_below(mm)] = (uint16_t)threadIdx.x;
            }
            if (mb) {
                uint32_t at = 0;
                if (lane == 0) at = atomicAdd(&s_nbig, (uint32_t)__popcll(mb));
                at = uniform((uint32_t)__shfl((int)at, 0));
                if (big) s_mid[kChunkRows - 1 - (at + lanes_below(mb))] = (uint16_t)threadIdx.x;
            }
            if constexpr (SC > 128) {
                const uint64_t mh = ballot(huge);
                if (mh) {
                    uint32_t at = 0;
                    if (lane == 0) at = atomicAdd(&s_nhuge, (uint32_t)__popcll(mh));
                    at = uniform((uint32_t)__shfl((int)at, 0));
                    if (huge) s_huge[at + lanes_below(mh)] = (uint16_t)threadIdx.x;
                }
            }
            __syncthreads();
            auto sort_rows = [&](auto ks, uint32_t nlist, const uint16_t *list, bool from_back) {
                // RB rows per round, their lengths, offsets and keys loaded
                // together (the stash row has SC >= 64*KS slots)
                constexpr int KS = decltype(ks)::value;
                constexpr int RB = KS == 1 ? 4 : 2;
                constexpr uint32_t NW = kChunkRows / 64;
                for (uint32_t m0 = wv; m0 < nlist; m0 += RB * NW) {
                    uint32_t n[RB];
                    int64_t ot[RB];
                    uint64_t v[RB][KS];
#pragma unroll
                    for (int k = 0; k < RB; ++k) {
                        const uint32_t m = m0 + k * NW;
                        n[k] = 0;
                        ot[k] = 0;
#pragma unroll
                        for (int p = 0; p < KS; ++p) v[k][p] = ~0ull;
                        if (m < nlist) {
                            const uint32_t slot = from_back ? kChunkRows - 1 - m : m;
                            const int64_t qr = ch.r0 + (int64_t)uniform((uint32_t)list[slot]);
                            n[k] = b.deg[qr];
                            ot[k] = b.offs[qr];
                            const uint64_t *sr = b.stash + qr * SC + lane * KS;
                            if constexpr (KS >= 2) {
#pragma unroll
                                for (int p = 0; p < KS; p += 2) {
                                    const ulonglong2 t = *reinterpret_cast<const ulonglong2 *>(sr + p);
                                    v[k][p] = t.x;
                                    v[k][p + 1] = t.y;
                                }
                            } else {
                                v[k][0] = sr[0];
                            }
                        }
                    }
#pragma unroll
                    for (int k = 0; k < RB; ++k)
#pragma unroll
                        for (int p = 0; p < KS; ++p)
                            if ((uint32_t)(lane * KS + p) >= n[k]) v[k][p] = ~0ull;
                    wave_bitonic<KS, RB>(v, lane);
#pragma unroll
                    for (int k = 0; k < RB; ++k) {
                        const uint32_t keep = (kn.K > 0 && n[k] > (uint32_t)kn.K) ? (uint32_t)kn.K : n[k];
#pragma unroll
                        for (int p = 0; p < KS; ++p) {
                            const uint32_t e = (uint32_t)(lane * KS + p);
                            if (e < keep) {
                                const uint32_t jj = (uint32_t)v[k][p];
                                const float d = __uint_as_float((uint32_t)(v[k][p] >> 32));
                                if (staged) {
                                    sidx[ot[k] - base + e] = jj;
                                    sd2[ot[k] - base + e] = d;
                                } else {
                                    b.out->indices[ot[k] + e] = (int32_t)jj;
                                    if (b.out->dist2) b.out->dist2[ot[k] + e] = d;
                                }
                            }
                        }
                    }
                }
            };
            sort_rows(std::integral_constant<int, 1>{}, s_nmid, s_mid, false);
            if constexpr (SC > 64) sort_rows(std::integral_constant<int, 2>{}, s_nbig, s_mid, true);
            if constexpr (SC > 128) sort_rows(std::integral_constant<int, 4>{}, s_nhuge, s_huge, false);
        }
        if (staged) {
            __syncthreads();
            int32_t *gi = b.out->indices + base;
            float *gd = b.out->dist2 ? b.out->dist2 + base : nullptr;
            for (int i = threadIdx.x; i < (int)len; i += kChunkRows) {
                gi[i] = (int32_t)sidx[i];
                if (gd) gd[i] = sd2[i];
            }
        }
    }
}

// ------------------------------------------------------------ long rows
// Rows longer than the stash, listed by the fill pass with their keys in
// their scratch rows, one wave per row: up to the on-chip limit (at most 512
// keys) sorted in registers by a wave-wide bitonic network, longer rows
// sorted in place in global memory with the all-ascending bitonic network
// (absent elements past n act as +infinity and never move).  Either way the
// first min(n, K) are written.
__global__ void __launch_bounds__(256) k_long_sort(Bufs b, Knobs kn) {
    if (!out_fits(b)) return;
    // the fill pass, which ran before this launch on the same stream, flags
    // a row whose recount differs; the output carries the flag to the host
    if (blockIdx.x == 0 && threadIdx.x == 0 && b.out->status) *b.out->status = b.ctr->status & kStatusInternal;
    const uint32_t n_long = b.ctr->n_long;
    const int lane = lane_id();
    const int w = threadIdx.x >> 6;
    const uint32_t nw = gridDim.x * kWavesPerBlock;
    for (uint32_t li = blockIdx.x * kWavesPerBlock + w; li < n_long; li += nw) {
        const uint64_t n = b.long_rows[li];
        const longlong2 at = *reinterpret_cast<const longlong2 *>(b.long_at + 2 * (int64_t)li);
        uint64_t *a = b.out->long_keys + at.x;
        const uint64_t keep = (kn.K > 0 && n > (uint64_t)kn.K) ? (uint64_t)kn.K : n;
        const int64_t off = at.y;
        int32_t *oi = b.out->indices + off;
        float *od = b.out->dist2 ? b.out->dist2 + off : nullptr;
        if (n <= (uint64_t)kn.long_cap) {
            const uint32_t n32 = (uint32_t)n, k32 = (uint32_t)keep;
            if (n <= 64)
                sort_and_write<1>(a, n32, k32, oi, od, lane);
            else if (n <= 128)
                sort_and_write<2>(a, n32, k32, oi, od, lane);
            else if (n <= 256)
                sort_and_write<4>(a, n32, k32, oi, od, lane);
            else
                sort_and_write<8>(a, n32, k32, oi, od, lane);
            continue;
        }
        uint64_t P = 1;
        while (P < n) P <<= 1;
        for (uint64_t k = 2; k <= P; k <<= 1) {
            const uint64_t half = k >> 1;
            for (uint64_t t = lane; t < P / 2; t += 64) {
                const uint64_t lo = ((t & ~(half - 1)) << 1) | (t & (half - 1));  // half: a power of two
                const uint64_t hi = lo ^ (k - 1);
                if (hi < n) {
                    uint64_t x = a[lo], y = a[hi];
                    if (y < x) {
                        a[lo] = y;
                        a[hi] = x;
                    }
                }
            }
            // the wave's stores are read back by its other lanes
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            for (uint64_t j = k >> 2; j >= 1; j >>= 1) {
                for (uint64_t t = lane; t < P / 2; t += 64) {
                    const uint64_t lo = ((t & ~(j - 1)) << 1) | (t & (j - 1));  // j: a power of two
                    const uint64_t hi = lo + j;
                    if (hi < n) {
                        uint64_t x = a[lo], y = a[hi];
                        if (y < x) {
                            a[lo] = y;
                            a[hi] = x;
                        }
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            }
        }
        for (uint64_t e = lane; e < keep; e += 64) {
            oi[e] = (int32_t)(uint32_t)a[e];
            if (od) od[e] = __uint_as_float((uint32_t)(a[e] >> 32));
        }
    }
}

// The read-back (one block): copies n16 16-byte words of counters and event
// bases (the query counters first) into device-mapped host memory, then,
// after a system-scope fence, stores the counters' run number into *flag,
// which the host polls: once it reads this run's number the block is whole.
__device__ __forceinline__ void publish_block(const Publish &p) {
    const uint4 *src = static_cast<const uint4 *>(p.src);
    uint4 *dst = static_cast<uint4 *>(p.dst);
    for (int64_t i = threadIdx.x; i < p.n16; i += blockDim.x) dst[i] = src[i];
    __threadfence_system();
    __syncthreads();
    if (threadIdx.x == 0)
        __hip_atomic_store(p.flag, static_cast<const Counters *>(p.src)->run_id, __ATOMIC_RELEASE,
                           __HIP_MEMORY_SCOPE_SYSTEM);
}

__global__ void __launch_bounds__(256) k_publish(Publish p) { publish_block(p); }

// Writes the output descriptor from kernel arguments (so the values are
// captured at launch time, unlike a copy from host memory).
__global__ void k_set_out(Bufs b, OutDesc v) { *b.out = v; }

// --------------------------------------------------------------- launches
#define FRNN_CHECK_LAUNCH() \
    do {                    \
        hipError_t e_ = hipGetLastError(); \
        if (e_ != hipSuccess) return e_;   \
    } while (0)

static thread_local GraphRecorder *t_rec = nullptr;

void set_recorder(GraphRecorder *r) { t_rec = r; }

// One kernel launch on stream s, or, while this thread records, one kernel
// node after the recorder's last (the argument values are copied into the
// node; the stream is not used).
template <class... P, class... A>
static void emit(void (*kern)(P...), dim3 grid, dim3 block, size_t lds, hipStream_t s, A... args) {
    GraphRecorder *r = t_rec;
    if (!r) {
        hipLaunchKernelGGL(kern, grid, block, lds, s, args...);
        return;
    }
    if (r->err != hipSuccess) return;
    std::tuple<std::decay_t<P>...> vals(args...);  // converted to the parameter types
    void *params[sizeof...(P) + 1] = {};
    std::apply([&](auto &...v) {
        int i = 0;
        ((params[i++] = (void *)&v), ...);
    }, vals);
    hipKernelNodeParams kp{};
    kp.func = (void *)kern;
    kp.gridDim = grid;
    kp.blockDim = block;
    kp.sharedMemBytes = (unsigned)lds;
    kp.kernelParams = params;
    kp.extra = nullptr;
    hipGraphNode_t node = nullptr;
    const hipError_t e = hipGraphAddKernelNode(&node, r->graph, r->last ? &r->last : nullptr, r->last ? 1 : 0, &kp);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        r->err = e;
        return;
    }
    r->last = node;
}

hipError_t launch_init(const Bufs &b, hipStream_t s, Counters *also, const void *src, void *dst, int64_t bytes) {
    static_assert(sizeof(Counters) / 4 <= 256, "one block clears the counters");
    const int64_t n16 = src ? (bytes + 15) / 16 : 0;
    const int64_t per = 256 * kFetchUnroll;
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(256, (n16 + per - 1) / per));
    emit(k_init, dim3(blocks), dim3(256), 0, s, b, also, reinterpret_cast<const uint4 *>(src),
                       reinterpret_cast<uint4 *>(dst), n16);
    FRNN_CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_extent(const Bufs &b, int nchunks, int E_cap, bool queries, int64_t zero_n, hipStream_t s) {
    // units: sum over events of ceil(n / kExtentRows) <= nchunks / 4 + E
    static_assert(kExtentRows == 4 * kChunkRows, "unit bound");
    const int units = (nchunks + 3) / 4 + E_cap;
    const int blocks = std::max(1, std::max(units, (int)std::min<int64_t>((zero_n + 4095) / 4096, 4096)));
    emit(k_extent, dim3(blocks), dim3(256), 0, s, b, (int32_t)queries, zero_n);
    FRNN_CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_plan(const Bufs &b, int E_cap, hipStream_t s, const Knobs *lpt) {
    emit(k_plan, dim3(std::max(1, E_cap)), dim3(256), 0, s, b, lpt ? *lpt : Knobs{}, (int32_t)(lpt != nullptr));
    FRNN_CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_keys(const Bufs &b, int nchunks, bool queries, hipStream_t s) {
    if (nchunks <= 0) return hipSuccess;
    emit(k_keys, dim3(std::min(nchunks, 8192)), dim3(256), 0, s, b, (int32_t)queries);
    FRNN_CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_scatter(const Bufs &b, int nchunks, bool queries, hipStream_t s) {
    if (nchunks <= 0) return hipSuccess;
    emit(k_scatter, dim3(std::min(nchunks, 8192)), dim3(256), 0, s, b, (int32_t)queries);
    FRNN_CHECK_LAUNCH();
    return hipSuccess;
}

static int scan_blocks(int64_t n_cap) {
    int64_t nb = (n_cap + kScanThreads * kScanItems - 1) / (kScanThreads * kScanItems);
    return (int)std::max<int64_t>(1, std::min<int64_t>(nb, kScanBlocks));
}

template <int MODE>
static hipError_t launch_scan_mode(const Bufs &b, const Knobs &kn, int64_t n_cap, hipStream_t s) {
    const int nb = scan_blocks(n_cap);
    emit(k_scan_reduce<MODE>, dim3(nb), dim3(kScanThreads), 0, s, b, kn);
    FRNN_CHECK_LAUNCH();
    emit(k_scan_apply<MODE>, dim3(nb), dim3(kScanThreads), 0, s, b, kn);
    FRNN_CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_scan_cells(const Bufs &b, int64_t cells_cap, bool queries, hipStream_t s) {
    Knobs kn{};
    return queries ? launch_scan_mode<kScanQCells>(b, kn, cells_cap + 1, s)
                   : launch_scan_mode<kScanCells>(b, kn, cells_cap + 1, s);
}

hipError_t launch_scan_rows(const Bufs &b, const Knobs &kn, int64_t total_q, hipStream_t s) {
    return launch_scan_mode<kScanRows>(b, kn, total_q + 1, s);
}

// Resident blocks per CU of a kernel at its launch configuration (cached:
// the query does not enqueue work, and is asked once per kernel and size).
static int resident_blocks(const void *fn, size_t lds) {
    static std::mutex mu;
    static std::map<std::pair<const void *, size_t>, int> *cache = new std::map<std::pair<const void *, size_t>, int>();
    std::lock_guard<std::mutex> g(mu);
    auto it = cache->find({fn, lds});
    if (it != cache->end()) return it->second;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, 64 * kWavesPerBlock, lds) != hipSuccess) {
        (void)hipGetLastError();
        n = 1;
    }
    n = std::max(1, n);
    (*cache)[{fn, lds}] = n;
    return n;
}

static int device_cus() {
    static int cus = [] {
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
            (void)hipGetLastError();
            n = 256;
        }
        return std::max(8, n);
    }();
    return cus;
}

template <bool FILL>
static hipError_t launch_query_t(const Bufs &b, const Knobs &kn, int D, int blocks, hipStream_t s) {
    blocks = (blocks + 7) / 8 * 8;  // whole XCD rounds (see the window remap)
    dim3 grid(blocks), block(64 * kWavesPerBlock);
    // self-exclusion and persistent scheduling are compile-time choices, so
    // each kernel holds one copy of the evaluation loop
    // dynamic LDS: the query rows of a window per wave (rows padded to a
    // multiple of 4 floats)
    auto lds = [&](int dt) { return (size_t)kWavesPerBlock * kn.window * ((dt + 3) & ~3) * sizeof(float); };
    // a persistent grid is at most what stays resident (the count pass
    // assigns its queue statically, so a block started late would finish
    // late): blocks (a multiple of 256 CUs) capped at the kernel's occupancy
    auto launch = [&](auto kern, int dt, bool pers) {
        const size_t l = lds(dt);
        dim3 g = grid;
        if (pers) {
            const int cus = device_cus();
            const int res = resident_blocks((const void *)kern, l);
            const int per_cu = std::min(std::max(1, FILL ? res : blocks / cus), res);
            g = dim3((unsigned)(per_cu * cus / 8 * 8));
        }
        emit(kern, g, block, l, s, b, kn);
    };
    auto go = [&](auto pers, auto excl) {
        constexpr bool P = decltype(pers)::value, X = decltype(excl)::value;
        if constexpr (FILL) {
            switch (D) {
            case 3: launch(k_query<3, true, true, P, X>, 3, P); break;
            case 8: launch(k_query<8, true, true, P, X>, 8, P); break;
            case 12:  // the launch bound of 5 waves per SIMD, only without self-exclusion
                if constexpr (X)
                    launch(k_query<12, true, true, P, X>, 12, P);
                else
                    launch(k_query_o5<12, true, true, P, X>, 12, P);
                break;
            default:
                if (D <= 4)
                    launch(k_query<4, false, true, P, X>, 4, P);
                else if (D <= 16)
                    launch(k_query<16, false, true, P, X>, 16, P);
                else
                    launch(k_query<32, false, true, P, X>, 32, P);
            }
        } else {
            switch (D) {
            case 3: launch(k_query<3, true, false, P, X>, 3, P); break;
            case 8: launch(k_query_o5<8, true, false, P, X>, 8, P); break;
            case 12: launch(k_query_o5<12, true, false, P, X>, 12, P); break;
            default:
                if (D <= 4)
                    launch(k_query<4, false, false, P, X>, 4, P);
                else if (D <= 16)
                    launch(k_query<16, false, false, P, X>, 16, P);
                else
                    launch(k_query<32, false, false, P, X>, 32, P);
            }
        }
    };
    auto go_x = [&](auto pers) {
        if (kn.exclude_self)
            go(pers, std::true_type{});
        else
            go(pers, std::false_type{});
    };
    if (kn.persistent)
        go_x(std::true_type{});
    else
        go_x(std::false_type{});
    FRNN_CHECK_LAUNCH();
    return hipSuccess;
}

int count_resident_blocks(const Knobs &kn, int D) {
    // the count kernel of this D at its launch configuration, persistent
    // flavour (the same registers as the plain one within a few)
    const size_t l = (size_t)kWavesPerBlock * kn.window * ((std::min(D, 32) + 3) & ~3) * sizeof(float);
    const void *fn;
    switch (D) {
    case 3: fn = (const void *)k_query<3, true, false, true, false>; break;
    case 8: fn = (const void *)k_query_o5<8, true, false, true, false>; break;
    case 12: fn = (const void *)k_query_o5<12, true, false, true, false>; break;
    default:
        fn = D <= 4 ? (const void *)k_query<4, false, false, true, false>
                    : D <= 16 ? (const void *)k_query<16, false, false, true, false>
                              : (const void *)k_query<32, false, false, true, false>;
    }
    return resident_blocks(fn, l) * device_cus();
}

hipError_t launch_count(const Bufs &b, const Knobs &kn, int D, int blocks, hipStream_t s) {
    return launch_query_t<false>(b, kn, D, blocks, s);
}

hipError_t launch_fill(const Bufs &b, const Knobs &kn, int D, int blocks, hipStream_t s) {
    return launch_query_t<true>(b, kn, D, blocks, s);
}

hipError_t launch_short_rows(const Bufs &b, const Knobs &kn, int nqchunks, hipStream_t s, const Publish *pub) {
    static_assert(kChunkRows == 256, "one block per chunk");
    dim3 grid(std::max(1, nqchunks)), block(kChunkRows);
    const Publish p = pub ? *pub : Publish{};
    switch (kn.stash_cap) {
    case 0: emit(k_short_rows<0>, grid, block, 0, s, b, kn, p); break;
    case 8: emit(k_short_rows<8>, grid, block, 0, s, b, kn, p); break;
    case 16: emit(k_short_rows<16>, grid, block, 0, s, b, kn, p); break;
    case 32: emit(k_short_rows<32>, grid, block, 0, s, b, kn, p); break;
    case 64: emit(k_short_rows<64>, grid, block, 0, s, b, kn, p); break;
    case 128: emit(k_short_rows<128>, grid, block, 0, s, b, kn, p); break;
    case 256: emit(k_short_rows<256>, grid, block, 0, s, b, kn, p); break;
    default: return hipErrorInvalidValue;
    }
    FRNN_CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_long_sort(const Bufs &b, const Knobs &kn, int blocks, hipStream_t s) {
    emit(k_long_sort, dim3(std::max(1, blocks)), dim3(256), 0, s, b, kn);
    FRNN_CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_lpt(const Bufs &b, const Knobs &kn, hipStream_t s) {
    emit(k_lpt, dim3(1), dim3(256), 0, s, b, kn);
    FRNN_CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_publish(const Publish &p, hipStream_t s) {
    emit(k_publish, dim3(1), dim3(256), 0, s, p);
    FRNN_CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_set_out(const Bufs &b, const OutDesc &v, hipStream_t s) {
    emit(k_set_out, dim3(1), dim3(1), 0, s, b, v);
    FRNN_CHECK_LAUNCH();
    return hipSuccess;
}


}  // namespace frnn
