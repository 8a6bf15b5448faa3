// Calibration kernel for hardware counters and for the FP32 FMA rate of this GPU: a known
// number of FP32 fused multiply-adds, so that the instruction counts rocprofv3 reports for the
// particle kernels can be scaled to per-wavefront instructions and FLOPs (counters on this GPU
// are aggregated per shader engine), and so that the VALU rate the pair kernels compete with
// is measured rather than assumed.
//
// Each lane runs kChains independent chains of `fmas` dependent steps, then adds its chains and
// stores one float.  Per wavefront that is exactly kChains * fmas FP32 FMA instructions (the
// final sum is kChains - 1 FP32 adds).  Two operand forms:
//  - form 0: a = b * d + a with b, d per-lane registers, the accumulating VOP2 form
//    (v_fmac_f32 with VGPR operands) that the pair kernels' sums use;
//  - form 1: a = a * s + t with s, t kernel arguments, one of them read from a scalar
//    register (v_fma_f32 with an SGPR operand);
//  - form 2: a = a * b + d, the three-operand VOP3 encoding (v_fma_f32) with register operands;
//  - form 3: FP32 matrix FMAs instead, four independent v_mfma_f32_16x16x4f32 chains per
//    wavefront (one 16x16x4 step is 1024 FMAs, 16 wavefront FMA instructions' worth);
//  - form 4: forms 0 and 3 interleaved in every wavefront (independent registers), to see
//    whether the matrix cores and the VALU run concurrently.
// On gfx950 form 1 issues at about half the rate of form 0, form 2 in between, and form 4
// takes as long as forms 0 and 3 one after the other.
#include <hip/hip_runtime.h>

#include "vpm_internal.h"

namespace vpm {

namespace {

constexpr int kChains = 8;

typedef float MfmaAcc __attribute__((ext_vector_type(4)));

template <int FORM>
__global__ __launch_bounds__(256) void k_fma_chain(int64_t n, int fmas, float s, float t, float* out) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    // per-lane factors (not foldable, not uniform, and formed without an FMA): b is s moved
    // by a few ulps, d small
    const float b = __int_as_float(__float_as_int(s) + int(threadIdx.x & 7));
    const float d = t * float(1 + (threadIdx.x & 3));
    float a[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) a[k] = float(int(threadIdx.x) + k);
    for (int r = 0; r < fmas; r += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int k = 0; k < kChains; ++k)
                a[k] = FORM == 0 ? fmaf(b, d, a[k]) : (FORM == 1 ? fmaf(a[k], s, t) : fmaf(a[k], b, d));
    }
    float acc = a[0];
#pragma unroll
    for (int k = 1; k < kChains; ++k) acc += a[k];
    if (i < n) out[i] = acc;
}

// Forms 3 and 4: per step of four, four 16x16x4 matrix FMAs on independent accumulators
// (fmas steps in all per wavefront), and for form 4 also the 32 FMAs of form 0's step.
template <bool VALU_TOO>
__global__ __launch_bounds__(256) void k_mfma_chain(int64_t n, int fmas, float s, float t, float* out) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const float b = __int_as_float(__float_as_int(s) + int(threadIdx.x & 7));
    const float d = t * float(1 + (threadIdx.x & 3));
    MfmaAcc c[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) c[k] = MfmaAcc{0.0f, 0.0f, 0.0f, 0.0f};
    float a[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) a[k] = float(int(threadIdx.x) + k);
    for (int r = 0; r < fmas; r += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            c[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(b, d, c[u], 0, 0, 0);
            if (VALU_TOO) {
#pragma unroll
                for (int k = 0; k < kChains; ++k) a[k] = fmaf(b, d, a[k]);
            }
        }
    }
    float acc = c[0][0] + c[1][1] + c[2][2] + c[3][3];
    if (VALU_TOO) {
#pragma unroll
        for (int k = 0; k < kChains; ++k) acc += a[k];
    }
    if (i < n) out[i] = acc;
}

}  // namespace

int fma_chain_count() { return kChains; }

hipError_t launch_fma_chain(int64_t n, int fmas, int form, float* out, hipStream_t st) {
    const unsigned nb = unsigned((n + 255) / 256);
    if (form == 0)
        hipLaunchKernelGGL(k_fma_chain<0>, dim3(nb), dim3(256), 0, st, n, fmas, 0.999f, 1e-3f, out);
    else if (form == 1)
        hipLaunchKernelGGL(k_fma_chain<1>, dim3(nb), dim3(256), 0, st, n, fmas, 0.999f, 1e-3f, out);
    else if (form == 2)
        hipLaunchKernelGGL(k_fma_chain<2>, dim3(nb), dim3(256), 0, st, n, fmas, 0.999f, 1e-3f, out);
    else if (form == 3)
        hipLaunchKernelGGL(k_mfma_chain<false>, dim3(nb), dim3(256), 0, st, n, fmas, 0.999f, 1e-3f, out);
    else
        hipLaunchKernelGGL(k_mfma_chain<true>, dim3(nb), dim3(256), 0, st, n, fmas, 0.999f, 1e-3f, out);
    return hipGetLastError();
}

}  // namespace vpm
