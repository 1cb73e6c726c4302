// Device side of the edge export (frnn_edges.hip).
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace frnn {

constexpr int kEdgesUpper = 0;
constexpr int kEdgesSymmetrized = 1;

struct EdgeArgs {
    const int64_t *off;   // CSR offsets [M+1]
    const int32_t *idx;   // CSR indices
    int64_t M;
    int32_t mode;
    uint32_t *deg;        // [M] exported entries per row (count pass)
    const int64_t *eoff;  // [M+1] exclusive scan of deg (fill pass)
    int32_t *src, *dst;   // [n] output
    uint32_t *status;     // bit 0: an index outside 0..M-1
};

hipError_t launch_edge_count(const EdgeArgs &a, hipStream_t s);
hipError_t launch_edge_fill(const EdgeArgs &a, hipStream_t s);

}  // namespace frnn
