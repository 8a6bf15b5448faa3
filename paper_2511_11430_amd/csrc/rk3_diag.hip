// Memory-bound helpers: one stage of the low-storage third-order Runge-Kutta scheme used to
// advance particle positions and strengths (Fu & Laurendeau, Sec. II.B; Williamson's
// 2N-storage form) and its adjoint, and FP64 invariant diagnostics of an evaluation
// (total vorticity and linear impulse, the conserved quantities of Eq. 1).
#include <hip/hip_runtime.h>

#include "vpm_internal.h"

namespace vpm {

namespace {

// 2N-storage coefficients: Q <- A_k Q + dt F; Y <- Y + B_k Q.
__constant__ double kRkA[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
__constant__ double kRkB[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};

// The six component arrays (x, Gamma) are processed as one flat index space of 6 n items.
// S: type of the state and register (x, Gamma, Q); T: type of F = (u, dGamma/dt) and of the
// optional copies (xe, ge) of the updated state used by the next evaluation.
template <typename S, typename T>
__global__ __launch_bounds__(256) void k_rk3_stage(int stage, int64_t n, S dt, S* x, S* g, S* qx, S* qg,
                                                   const T* u, const T* dg, int64_t ld, T* xe, T* ge) {
    const S A = S(kRkA[stage]);
    const S B = S(kRkB[stage]);
    const int64_t total = 6 * n;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
         i += int64_t(gridDim.x) * blockDim.x) {
        const int64_t c = i / n;
        const int64_t e = i - c * n;
        const int64_t off = (c % 3) * ld + e;
        S* y = c < 3 ? x : g;
        S* q = c < 3 ? qx : qg;
        const T* f = c < 3 ? u : dg;
        const S qn = A * q[off] + dt * S(f[off]);
        q[off] = qn;
        const S yn = y[off] + B * qn;
        y[off] = yn;
        if (xe) (c < 3 ? xe : ge)[off] = T(yn);
    }
}

// Stage k for points carried by the flow in a free stream (wake-line points, particles of the
// closed step): Qx <- A_k Qx + dt (u + v_inf), x <- x + B_k Qx and, when g is given,
// Qg <- A_k Qg + dt dg, g <- g + B_k Qg.  State and register are stored in T, the arithmetic
// is FP64; stage 0 does not read the registers.  One thread per point, all three components.
template <typename T>
__global__ __launch_bounds__(256) void k_rk3_advect(int stage, int64_t n, double dt, T* x, T* qx, const T* u,
                                                    T* g, T* qg, const T* dg, int64_t ld, double v0, double v1,
                                                    double v2) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double A = kRkA[stage], B = kRkB[stage];
    const double v[3] = {v0, v1, v2};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int64_t o = c * ld + i;
        const double q = (stage ? A * double(qx[o]) : 0.0) + dt * (double(u[o]) + v[c]);
        qx[o] = T(q);
        x[o] = T(double(x[o]) + B * double(T(q)));
        if (g) {
            const double p = (stage ? A * double(qg[o]) : 0.0) + dt * double(dg[o]);
            qg[o] = T(p);
            g[o] = T(double(g[o]) + B * double(T(p)));
        }
    }
}

// Adjoint: qtot = Qbar + B_k Ybar;  seed = dt qtot;  Qbar <- A_k qtot.
template <typename S, typename T>
__global__ __launch_bounds__(256) void k_rk3_stage_bwd(int stage, int64_t n, S dt, const S* xb,
                                                       const S* gb, S* qxb, S* qgb, T* us, T* ds,
                                                       int64_t ld) {
    const S A = S(kRkA[stage]);
    const S B = S(kRkB[stage]);
    const int64_t total = 6 * n;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
         i += int64_t(gridDim.x) * blockDim.x) {
        const int64_t c = i / n;
        const int64_t e = i - c * n;
        const int64_t off = (c % 3) * ld + e;
        const S* yb = c < 3 ? xb : gb;
        S* qb = c < 3 ? qxb : qgb;
        T* sd = c < 3 ? us : ds;
        const S qt = qb[off] + B * yb[off];
        sd[off] = T(dt * qt);
        qb[off] = A * qt;
    }
}

// dst = src or dst += src over [3][ld] arrays, converting the element type.
template <typename SRC, typename DST>
__global__ __launch_bounds__(256) void k_convert(int64_t n, const SRC* src, int64_t lds, DST* dst, int64_t ldd,
                                                 int add) {
    const int64_t total = 3 * n;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
         i += int64_t(gridDim.x) * blockDim.x) {
        const int64_t c = i / n;
        const int64_t e = i - c * n;
        const DST v = DST(src[c * lds + e]);
        DST* d = dst + c * ldd + e;
        *d = add ? DST(*d + v) : v;
    }
}

// Per-block FP64 partial sums (each lane sums its strided items, then a tree over the block),
// written to partials[block][kDiagSlots].
template <typename T>
__global__ __launch_bounds__(256) void k_diag_partial(int64_t n, const T* x, const T* g, const T* u,
                                                      const T* dg, int64_t ld, double* partials) {
    double s[13];
#pragma unroll
    for (int c = 0; c < 13; ++c) s[c] = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x) {
        const double x0 = x[i], x1 = x[ld + i], x2 = x[2 * ld + i];
        const double g0 = g[i], g1 = g[ld + i], g2 = g[2 * ld + i];
        const double u0 = u[i], u1 = u[ld + i], u2 = u[2 * ld + i];
        const double d0 = dg[i], d1 = dg[ld + i], d2 = dg[2 * ld + i];
        s[0] += g0;
        s[1] += g1;
        s[2] += g2;
        s[3] += d0;
        s[4] += d1;
        s[5] += d2;
        s[6] += 0.5 * (x1 * g2 - x2 * g1);
        s[7] += 0.5 * (x2 * g0 - x0 * g2);
        s[8] += 0.5 * (x0 * g1 - x1 * g0);
        s[9] += 0.5 * ((u1 * g2 - u2 * g1) + (x1 * d2 - x2 * d1));
        s[10] += 0.5 * ((u2 * g0 - u0 * g2) + (x2 * d0 - x0 * d2));
        s[11] += 0.5 * ((u0 * g1 - u1 * g0) + (x0 * d1 - x1 * d0));
        const double vals[12] = {x0, x1, x2, g0, g1, g2, u0, u1, u2, d0, d1, d2};
        int bad = 0;
#pragma unroll
        for (int c = 0; c < 12; ++c) bad += isfinite(vals[c]) ? 0 : 1;
        s[12] += double(bad);
    }
    __shared__ double red[256][13];
#pragma unroll
    for (int c = 0; c < 13; ++c) red[threadIdx.x][c] = s[c];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w) {
#pragma unroll
            for (int c = 0; c < 13; ++c) red[threadIdx.x][c] += red[threadIdx.x + w][c];
        }
        __syncthreads();
    }
    if (threadIdx.x < 13) partials[int64_t(blockIdx.x) * kDiagSlots + threadIdx.x] = red[0][threadIdx.x];
}

__global__ __launch_bounds__(256) void k_diag_final(int nblocks, const double* partials, double* out) {
    __shared__ double red[256];
    for (int c = 0; c < 13; ++c) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += blockDim.x) s += partials[int64_t(b) * kDiagSlots + c];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[c] = red[0];
        __syncthreads();
    }
}

// L = sum_c u_z(c)^2 in FP64 (one workgroup) and the seed u_bar = 2 loss_bar (0, 0, u_z).
template <typename T>
__global__ __launch_bounds__(256) void k_axial_loss(int64_t m, const T* u, int64_t ld, double* loss,
                                                    T* ubar, const double* loss_bar) {
    __shared__ double red[256];
    const double lb = loss_bar ? *loss_bar : 1.0;
    double s = 0.0;
    for (int64_t c = threadIdx.x; c < m; c += blockDim.x) {
        const double uz = double(u[2 * ld + c]);
        s += uz * uz;
        if (ubar) {
            ubar[c] = T(0);
            ubar[ld + c] = T(0);
            ubar[2 * ld + c] = T(2.0 * lb * uz);
        }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && loss) *loss = red[0];
}

// Input check: per block, the number of particles with sigma <= 0 or non-finite sigma, and
// the number of non-finite entries among x and Gamma (FP64 counts, summed by k_diag_final).
template <typename T>
__global__ __launch_bounds__(256) void k_validate_partial(int64_t n, const T* x, const T* g, const T* sg,
                                                          int64_t ld, double* partials) {
    double bad_sigma = 0.0, bad_vals = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x) {
        const double s = sg[i];
        bad_sigma += (isfinite(s) && s > 0.0) ? 0.0 : 1.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            bad_vals += isfinite(double(x[c * ld + i])) ? 0.0 : 1.0;
            bad_vals += isfinite(double(g[c * ld + i])) ? 0.0 : 1.0;
        }
    }
    __shared__ double red[256][2];
    red[threadIdx.x][0] = bad_sigma;
    red[threadIdx.x][1] = bad_vals;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w) {
            red[threadIdx.x][0] += red[threadIdx.x + w][0];
            red[threadIdx.x][1] += red[threadIdx.x + w][1];
        }
        __syncthreads();
    }
    if (threadIdx.x < kDiagSlots) {
        const double v = threadIdx.x < 2 ? red[0][threadIdx.x] : 0.0;
        partials[int64_t(blockIdx.x) * kDiagSlots + threadIdx.x] = v;
    }
}

int grid_for(int64_t items) {
    int64_t g = (items + 255) / 256;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    return int(g);
}

}  // namespace

hipError_t launch_rk3_stage(int dtype, int state_dtype, int stage, int64_t n, double dt, void* x, void* g,
                            void* qx, void* qg, const void* u, const void* dg, int64_t ld, void* xe, void* ge,
                            hipStream_t st) {
    if (n == 0) return hipSuccess;
    const int grid = grid_for(6 * n);
    if (state_dtype == kDtypeF64 && dtype == kDtypeF64)
        hipLaunchKernelGGL((k_rk3_stage<double, double>), dim3(grid), dim3(256), 0, st, stage, n, dt,
                           (double*)x, (double*)g, (double*)qx, (double*)qg, (const double*)u,
                           (const double*)dg, ld, (double*)xe, (double*)ge);
    else if (state_dtype == kDtypeF64)
        hipLaunchKernelGGL((k_rk3_stage<double, float>), dim3(grid), dim3(256), 0, st, stage, n, dt,
                           (double*)x, (double*)g, (double*)qx, (double*)qg, (const float*)u,
                           (const float*)dg, ld, (float*)xe, (float*)ge);
    else
        hipLaunchKernelGGL((k_rk3_stage<float, float>), dim3(grid), dim3(256), 0, st, stage, n, float(dt),
                           (float*)x, (float*)g, (float*)qx, (float*)qg, (const float*)u,
                           (const float*)dg, ld, (float*)xe, (float*)ge);
    return hipGetLastError();
}

hipError_t launch_rk3_advect(int dtype, int stage, int64_t n, double dt, void* x, void* qx, const void* u, void* g,
                            void* qg, const void* dg, int64_t ld, const double* vinf, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const unsigned nb = unsigned((n + 255) / 256);
    if (dtype == kDtypeF64)
        hipLaunchKernelGGL(k_rk3_advect<double>, dim3(nb), dim3(256), 0, st, stage, n, dt, (double*)x, (double*)qx,
                           (const double*)u, (double*)g, (double*)qg, (const double*)dg, ld, vinf[0], vinf[1],
                           vinf[2]);
    else
        hipLaunchKernelGGL(k_rk3_advect<float>, dim3(nb), dim3(256), 0, st, stage, n, dt, (float*)x, (float*)qx,
                           (const float*)u, (float*)g, (float*)qg, (const float*)dg, ld, vinf[0], vinf[1],
                           vinf[2]);
    return hipGetLastError();
}

hipError_t launch_rk3_stage_bwd(int dtype, int state_dtype, int stage, int64_t n, double dt, const void* xb,
                                const void* gb, void* qxb, void* qgb, void* us, void* ds, int64_t ld,
                                hipStream_t st) {
    if (n == 0) return hipSuccess;
    const int grid = grid_for(6 * n);
    if (state_dtype == kDtypeF64 && dtype == kDtypeF64)
        hipLaunchKernelGGL((k_rk3_stage_bwd<double, double>), dim3(grid), dim3(256), 0, st, stage, n, dt,
                           (const double*)xb, (const double*)gb, (double*)qxb, (double*)qgb,
                           (double*)us, (double*)ds, ld);
    else if (state_dtype == kDtypeF64)
        hipLaunchKernelGGL((k_rk3_stage_bwd<double, float>), dim3(grid), dim3(256), 0, st, stage, n, dt,
                           (const double*)xb, (const double*)gb, (double*)qxb, (double*)qgb,
                           (float*)us, (float*)ds, ld);
    else
        hipLaunchKernelGGL((k_rk3_stage_bwd<float, float>), dim3(grid), dim3(256), 0, st, stage, n,
                           float(dt), (const float*)xb, (const float*)gb, (float*)qxb,
                           (float*)qgb, (float*)us, (float*)ds, ld);
    return hipGetLastError();
}

hipError_t launch_convert(int src_dtype, int dst_dtype, int64_t n, const void* src, int64_t lds, void* dst,
                          int64_t ldd, int add, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const int grid = grid_for(3 * n);
    if (src_dtype == kDtypeF64 && dst_dtype == kDtypeF64)
        hipLaunchKernelGGL((k_convert<double, double>), dim3(grid), dim3(256), 0, st, n, (const double*)src, lds,
                           (double*)dst, ldd, add);
    else if (src_dtype == kDtypeF64)
        hipLaunchKernelGGL((k_convert<double, float>), dim3(grid), dim3(256), 0, st, n, (const double*)src, lds,
                           (float*)dst, ldd, add);
    else if (dst_dtype == kDtypeF64)
        hipLaunchKernelGGL((k_convert<float, double>), dim3(grid), dim3(256), 0, st, n, (const float*)src, lds,
                           (double*)dst, ldd, add);
    else
        hipLaunchKernelGGL((k_convert<float, float>), dim3(grid), dim3(256), 0, st, n, (const float*)src, lds,
                           (float*)dst, ldd, add);
    return hipGetLastError();
}

hipError_t launch_validate(int dtype, int64_t n, const void* x, const void* g, const void* sg, int64_t ld,
                           double* out, double* partials, hipStream_t st) {
    int nb = int((n + 255) / 256);
    if (nb > kDiagBlocks) nb = kDiagBlocks;
    if (nb < 1) nb = 1;
    if (dtype == kDtypeF64)
        hipLaunchKernelGGL(k_validate_partial<double>, dim3(nb), dim3(256), 0, st, n, (const double*)x,
                           (const double*)g, (const double*)sg, ld, partials);
    else
        hipLaunchKernelGGL(k_validate_partial<float>, dim3(nb), dim3(256), 0, st, n, (const float*)x,
                           (const float*)g, (const float*)sg, ld, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(256), 0, st, nb, partials, out);
    return hipGetLastError();
}

hipError_t launch_diagnostics(int dtype, int64_t n, const void* x, const void* g, const void* u,
                              const void* dg, int64_t ld, double* out, double* partials,
                              hipStream_t st) {
    int nb = int((n + 255) / 256);
    if (nb > kDiagBlocks) nb = kDiagBlocks;
    if (nb < 1) nb = 1;
    if (dtype == kDtypeF64)
        hipLaunchKernelGGL(k_diag_partial<double>, dim3(nb), dim3(256), 0, st, n, (const double*)x,
                           (const double*)g, (const double*)u, (const double*)dg, ld, partials);
    else
        hipLaunchKernelGGL(k_diag_partial<float>, dim3(nb), dim3(256), 0, st, n, (const float*)x,
                           (const float*)g, (const float*)u, (const float*)dg, ld, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(256), 0, st, nb, partials, out);
    return hipGetLastError();
}

}  // namespace vpm

namespace vpm {

hipError_t launch_axial_loss(int dtype, int64_t m, const void* u, int64_t ld, double* loss, void* ubar,
                             const double* loss_bar, hipStream_t st) {
    if (dtype == kDtypeF64)
        hipLaunchKernelGGL(k_axial_loss<double>, dim3(1), dim3(256), 0, st, m, (const double*)u, ld, loss,
                           (double*)ubar, loss_bar);
    else
        hipLaunchKernelGGL(k_axial_loss<float>, dim3(1), dim3(256), 0, st, m, (const float*)u, ld, loss,
                           (float*)ubar, loss_bar);
    return hipGetLastError();
}

}  // namespace vpm
