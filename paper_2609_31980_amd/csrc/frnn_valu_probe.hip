// Measured rate of the distance evaluation's operation mix on this GPU: the
// same chain of float32 subtract, multiply and add, each rounded on its own
// (no fused multiply-add: -ffp-contract=off and the pragma below; no packed
// FP32: the library is built without it), run by every resident wave with
// enough independent chains per lane to keep the vector ALU busy.  This is
// the denominator the distance kernels' roofline fraction is quoted against,
// beside the rate derived from the unit counts and the clock.
#include <hip/hip_runtime.h>

#include "../../include/frnn.h"
#include "frnn_runtime.h"

#pragma clang fp contract(off)

namespace frnn {
namespace {

constexpr int kChains = 8;       // independent accumulators per lane
constexpr int kPerStep = 8;      // subtract / multiply / add triples per chain per step

__global__ void __launch_bounds__(256) k_valu_chain(float *out, int steps, float seed) {
    const float base = seed + 1e-3f * (float)(threadIdx.x & 63);
    float q[kPerStep], s[kChains];
#pragma unroll
    for (int d = 0; d < kPerStep; ++d) q[d] = base + 0.125f * (float)d;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s[c] = 0.0f;
    float x = base * 0.5f;
    for (int i = 0; i < steps; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
#pragma unroll
            for (int d = 0; d < kPerStep; ++d) {
                float t = q[d] - x;  // the candidate coordinate differs per chain and step
                float u = t * t;
                s[c] = s[c] + u;
            }
            x = x + 1e-7f;
        }
    }
    float r = 0.0f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) r = r + s[c];
    if (r == -1.0f) out[blockIdx.x * blockDim.x + threadIdx.x] = r;  // keeps the chain alive
}

}  // namespace
}  // namespace frnn

using namespace frnn;

extern "C" frnn_status frnn_measure_valu_rate(void *stream, double *ops_per_s) {
    if (!ops_per_s) return fail(FRNN_ERR_INVALID_ARG, "null output");
    *ops_per_s = 0.0;
    try {
        hipStream_t s = (hipStream_t)stream;
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return fail(FRNN_ERR_HIP, "device query failed");
        // 8 blocks of 4 waves per CU: 8 waves per SIMD
        const int blocks = cus * 8, steps = 2048;
        DevBuf out((size_t)blocks * 256 * sizeof(float), s);
        hipEvent_t a, b;
        FRNN_HIP(hipEventCreate(&a));
        FRNN_HIP(hipEventCreate(&b));
        hipLaunchKernelGGL(k_valu_chain, dim3(blocks), dim3(256), 0, s, out.as<float>(), 64, 0.5f);  // warm-up
        FRNN_HIP(hipEventRecord(a, s));
        hipLaunchKernelGGL(k_valu_chain, dim3(blocks), dim3(256), 0, s, out.as<float>(), steps, 0.5f);
        FRNN_HIP(hipGetLastError());
        FRNN_HIP(hipEventRecord(b, s));
        FRNN_HIP(hipEventSynchronize(b));
        float ms = 0.f;
        FRNN_HIP(hipEventElapsedTime(&ms, a, b));
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        // per chain and step: kPerStep (subtract, multiply, add) triples and
        // the add that moves x, per lane
        const double ops = (3.0 * kPerStep + 1.0) * kChains * (double)steps * (double)blocks * 256.0;
        *ops_per_s = ops / (ms * 1e-3);
        return FRNN_OK;
    } catch (const Fail &f) {
        return fail(f.st, f.msg);
    } catch (...) {
        return fail(FRNN_ERR_INTERNAL, "unknown internal error");
    }
}
