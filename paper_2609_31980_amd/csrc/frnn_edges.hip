// Edge export from a self-query CSR (see frnn_csr_edges in include/frnn.h):
// a per-row count, the library's row scan, then a fill.  One thread per row;
// rows are short (at most K, or the degree), so the reverse-direction test of
// the symmetrised mode is a linear scan of the other row.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "frnn_edges.h"

namespace frnn {

namespace {

// Does row i export its entry j?  Sets *bad for an index outside 0..M-1.
__device__ __forceinline__ bool exported(const int64_t *off, const int32_t *idx, int64_t M, int64_t i,
                                         int32_t j, int mode, bool *bad) {
    if (j < 0 || (int64_t)j >= M) {
        *bad = true;
        return false;
    }
    if ((int64_t)j == i) return false;
    if ((int64_t)j > i) return true;
    if (mode == kEdgesUpper) return false;
    // j < i: exported from here only when row j does not hold i
    for (int64_t p = off[j]; p < off[j + 1]; ++p)
        if ((int64_t)idx[p] == i) return false;
    return true;
}

__global__ void k_edge_count(EdgeArgs a) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.M;
         i += (int64_t)gridDim.x * blockDim.x) {
        bool bad = false;
        uint32_t c = 0;
        for (int64_t p = a.off[i]; p < a.off[i + 1]; ++p) c += exported(a.off, a.idx, a.M, i, a.idx[p], a.mode, &bad);
        a.deg[i] = c;
        if (bad) atomicOr(a.status, 1u);
    }
}

__global__ void k_edge_fill(EdgeArgs a) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.M;
         i += (int64_t)gridDim.x * blockDim.x) {
        bool bad = false;
        int64_t o = a.eoff[i];
        for (int64_t p = a.off[i]; p < a.off[i + 1]; ++p) {
            const int32_t j = a.idx[p];
            if (exported(a.off, a.idx, a.M, i, j, a.mode, &bad)) {
                a.src[o] = (int32_t)min((int64_t)j, i);
                a.dst[o] = (int32_t)max((int64_t)j, i);
                ++o;
            }
        }
    }
}

int grid_for(int64_t M) { return (int)std::max<int64_t>(1, std::min<int64_t>((M + 255) / 256, 4096)); }

}  // namespace

hipError_t launch_edge_count(const EdgeArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_edge_count, dim3(grid_for(a.M)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_edge_fill(const EdgeArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_edge_fill, dim3(grid_for(a.M)), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace frnn
