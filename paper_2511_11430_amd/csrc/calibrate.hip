// Calibration kernel for hardware counters: a known number of FP32 fused multiply-adds, so
// that the instruction counts rocprofv3 reports for the particle kernels can be scaled to
// per-wavefront instructions and FLOPs (counters on this GPU are aggregated per shader engine).
//
// Each lane runs kChains independent chains of `fmas` dependent a = a * b + c steps (runtime
// b and c, so nothing folds), then adds its chains and stores one float.  Per wavefront that is
// exactly kChains * fmas FP32 FMA instructions (the compiler emits one v_fma/v_fmac per step;
// the final sum is kChains - 1 FP32 adds).
#include <hip/hip_runtime.h>

#include "vpm_internal.h"

namespace vpm {

namespace {

constexpr int kChains = 8;

__global__ __launch_bounds__(256) void k_fma_chain(int64_t n, int fmas, float b, float c, float* out) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    float a[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) a[k] = float(int(threadIdx.x) + k);
    for (int s = 0; s < fmas; s += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int k = 0; k < kChains; ++k) a[k] = fmaf(a[k], b, c);
    }
    float t = a[0];
#pragma unroll
    for (int k = 1; k < kChains; ++k) t += a[k];
    if (i < n) out[i] = t;
}

}  // namespace

int fma_chain_count() { return kChains; }

hipError_t launch_fma_chain(int64_t n, int fmas, float* out, hipStream_t st) {
    const unsigned nb = unsigned((n + 255) / 256);
    hipLaunchKernelGGL(k_fma_chain, dim3(nb), dim3(256), 0, st, n, fmas, 0.999f, 1e-3f, out);
    return hipGetLastError();
}

}  // namespace vpm
