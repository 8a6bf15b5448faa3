// Velocity induced by straight vortex segments with a Vatistas core (Fu & Laurendeau,
// Sec. II.A: vortex-ring edges of the blade lattice and straight wake lines, Biot-Savart law
// with the Vatistas smoothing kernel).
//
// For a point P and a segment a->b of circulation Gamma (r1 = P - a, r2 = P - b, r0 = b - a):
//   u = Gamma/(4 pi) (r1 x r2) [r0 . (r1/|r1| - r2/|r2|)] / (|r0|^2 (d^2n + rc^2n)^(1/n))
// where d^2 = |r1 x r2|^2 / |r0|^2 is the squared distance to the segment's line; with
// rc = 0 the denominator is |r1 x r2|^2 (the singular finite-segment formula).
// Identities used per pair: r1 x r2 = r0 x r1 and r0 . r2 = r0 . r1 - |r0|^2.
//
// Schedule: like the particle kernel, K targets per lane, segment tiles staged in LDS with
// per-segment constants (Gamma / (4 pi |r0|^2), r0, |r0|^2, the degeneracy threshold), and
// FP32 tile partials folded into two-sum pairs (VPM_F32C) or plain FP64 sums (VPM_F64).
#include <hip/hip_runtime.h>

#include "device_math.h"
#include "vpm_internal.h"

namespace vpm {

namespace {

template <typename T>
using V4 = typename std::conditional<std::is_same<T, float>::value, float4, double4>::type;

// VN: 0 = no core (rc == 0), 1, 2 = Vatistas exponent, 3 = general exponent n.
template <typename T, int VN>
__device__ __forceinline__ T core_factor(T d2, T rc2n, T inv_n, T n_f) {
    if constexpr (VN == 1) {
        return T(1) / (d2 + rc2n);
    } else if constexpr (VN == 2) {
        return rsqrt_fast(d2 * d2 + rc2n);
    } else {
        // (d^2n + rc^2n)^(-1/n)
        const T d2n = pow(d2, n_f);
        return pow(d2n + rc2n, -inv_n);
    }
}

template <typename T, int K, int WG, int VN>
__global__ __launch_bounds__(WG) void k_segments(SegArgs a) {
    constexpr bool kComp = std::is_same<T, float>::value;
    __shared__ V4<T> l0[WG];  // (ax, ay, az, coef)   coef = Gamma / (4 pi |r0|^2)  (rc == 0: Gamma/(4 pi))
    __shared__ V4<T> l1[WG];  // (r0x, r0y, r0z, |r0|^2)
    __shared__ T l2[WG];      // eps^2 for the arms
    const T* __restrict__ A = static_cast<const T*>(a.a);
    const T* __restrict__ B = static_cast<const T*>(a.b);
    const T* __restrict__ Gs = static_cast<const T*>(a.gam);
    const T* __restrict__ X = static_cast<const T*>(a.xt);
    const int tid = threadIdx.x;
    const int64_t t0 = int64_t(blockIdx.x) * (WG * K);
    const T rc2 = T(a.rc * a.rc);
    const T n_f = T(a.vn);
    const T inv_n = T(1.0 / a.vn);
    T rc2n;
    if constexpr (VN == 0) rc2n = T(0);
    else if constexpr (VN == 1) rc2n = rc2;
    else if constexpr (VN == 2) rc2n = rc2 * rc2;
    else rc2n = T(pow(double(rc2), double(a.vn)));

    T P[K][3];
    bool valid[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t t = t0 + tid + int64_t(k) * WG;
        valid[k] = t < a.n_tgt;
        const int64_t tt = valid[k] ? t : 0;
        P[k][0] = X[tt];
        P[k][1] = X[a.ldt + tt];
        P[k][2] = X[2 * a.ldt + tt];
    }
    T acc[K][3], hi[K][3], lo[K][3];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[k][c] = hi[k][c] = lo[k][c] = T(0);

    for (int64_t j0 = 0; j0 < a.n_seg; j0 += WG) {
        const int cnt = int((a.n_seg - j0) < WG ? (a.n_seg - j0) : WG);
        __syncthreads();
        if (tid < cnt) {
            const int64_t j = j0 + tid;
            const T ax = A[j], ay = A[a.ld_seg + j], az = A[2 * a.ld_seg + j];
            const T r0x = B[j] - ax, r0y = B[a.ld_seg + j] - ay, r0z = B[2 * a.ld_seg + j] - az;
            const T L02 = r0x * r0x + r0y * r0y + r0z * r0z;
            const T L0 = dsqrt(L02);
            const T eps = T(1e-12) * (L0 > T(1) ? L0 : T(1));
            const bool dead = L0 < eps;
            T coef = T(kInv4PiD) * Gs[j];
            if (VN != 0) coef = coef / L02;
            if (dead) coef = T(0);
            V4<T> p, q;
            p.x = ax; p.y = ay; p.z = az; p.w = coef;
            q.x = r0x; q.y = r0y; q.z = r0z; q.w = dead ? T(1) : L02;
            l0[tid] = p;
            l1[tid] = q;
            l2[tid] = eps * eps;
        }
        __syncthreads();
#pragma unroll 2
        for (int jj = 0; jj < cnt; ++jj) {
            const V4<T> p = l0[jj];
            const V4<T> q = l1[jj];
            const T eps2 = l2[jj];
            const T inv_l02 = T(1) / q.w;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const T r1x = P[k][0] - p.x, r1y = P[k][1] - p.y, r1z = P[k][2] - p.z;
                const T r2x = r1x - q.x, r2y = r1y - q.y, r2z = r1z - q.z;
                // r1 x r2 = r0 x r1
                const T cx = q.y * r1z - q.z * r1y;
                const T cy = q.z * r1x - q.x * r1z;
                const T cz = q.x * r1y - q.y * r1x;
                const T c2 = cx * cx + cy * cy + cz * cz;
                const T l1s = r1x * r1x + r1y * r1y + r1z * r1z;
                const T l2s = r2x * r2x + r2y * r2y + r2z * r2z;
                const T d1 = q.x * r1x + q.y * r1y + q.z * r1z;
                const T d2 = d1 - q.w;
                const T D = d1 * rsqrt_fast(l1s) - d2 * rsqrt_fast(l2s);
                T f;
                if constexpr (VN == 0) {
                    f = (c2 > T(0)) ? p.w * D / c2 : T(0);
                } else {
                    f = p.w * D * core_factor<T, VN>(c2 * inv_l02, rc2n, inv_n, n_f);
                }
                f = (l1s < eps2 || l2s < eps2) ? T(0) : f;
                acc[k][0] += f * cx;
                acc[k][1] += f * cy;
                acc[k][2] += f * cz;
            }
        }
        if constexpr (kComp) {
#pragma unroll
            for (int k = 0; k < K; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    T s, e;
                    two_sum(hi[k][c], acc[k][c], s, e);
                    hi[k][c] = s;
                    lo[k][c] += e;
                    acc[k][c] = T(0);
                }
        }
    }
    T* __restrict__ U = static_cast<T*>(a.u);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (!valid[k]) continue;
        const int64_t t = t0 + tid + int64_t(k) * WG;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double v = kComp ? double(hi[k][c]) + double(lo[k][c]) : double(acc[k][c]);
            T* dst = U + c * a.ldo + t;
            *dst = a.accumulate ? T(double(*dst) + v) : T(v);
        }
    }
}

// Gradient form: velocity and its gradient J = du/dP at the targets, and from J the
// stretching of target particles of strength gamma_t.  With u = f c, c = r0 x r1,
// f = coef D K(d^2), D = r0 . (r1/|r1| - r2/|r2|), d^2 = |c|^2 / |r0|^2:
//   J = f [r0]x + c (grad f)^T,
//   grad D   = r0 (1/|r1| - 1/|r2|) - r1 (r0.r1)/|r1|^3 + r2 (r0.r2)/|r2|^3,
//   grad d^2 = 2 (c x r0) / |r0|^2,
//   grad f   = coef (K grad D + D K'(d^2) grad d^2),
// with K' = -K^2 (n = 1), -d^2 K^3 (n = 2), -d^(2(n-1)) K / (d^2n + rc^2n) (general n).
// Without a core (rc = 0): f = Gamma/(4 pi) D / |c|^2 and grad f = Gamma/(4 pi)
// (grad D - 2 D (c x r0) / |c|^2) / |c|^2.  Pairs that the velocity form drops (short arms,
// zero denominator) contribute nothing here either.
template <typename T, int K, int WG, int VN>
__global__ __launch_bounds__(WG) void k_segments_grad(SegArgs a) {
    constexpr bool kComp = std::is_same<T, float>::value;
    constexpr int NA = 12;  // u (3), J row-major (9)
    __shared__ V4<T> l0[WG];
    __shared__ V4<T> l1[WG];
    __shared__ T l2[WG];
    const T* __restrict__ A = static_cast<const T*>(a.a);
    const T* __restrict__ B = static_cast<const T*>(a.b);
    const T* __restrict__ Gs = static_cast<const T*>(a.gam);
    const T* __restrict__ X = static_cast<const T*>(a.xt);
    const int tid = threadIdx.x;
    const int64_t t0 = int64_t(blockIdx.x) * (WG * K);
    const T rc2 = T(a.rc * a.rc);
    const T n_f = T(a.vn);
    const T inv_n = T(1.0 / a.vn);
    T rc2n;
    if constexpr (VN == 0) rc2n = T(0);
    else if constexpr (VN == 1) rc2n = rc2;
    else if constexpr (VN == 2) rc2n = rc2 * rc2;
    else rc2n = T(pow(double(rc2), double(a.vn)));

    T P[K][3];
    bool valid[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t t = t0 + tid + int64_t(k) * WG;
        valid[k] = t < a.n_tgt;
        const int64_t tt = valid[k] ? t : 0;
        P[k][0] = X[tt];
        P[k][1] = X[a.ldt + tt];
        P[k][2] = X[2 * a.ldt + tt];
    }
    T acc[K][NA], hi[K][NA], lo[K][NA];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int c = 0; c < NA; ++c) acc[k][c] = hi[k][c] = lo[k][c] = T(0);

    for (int64_t j0 = 0; j0 < a.n_seg; j0 += WG) {
        const int cnt = int((a.n_seg - j0) < WG ? (a.n_seg - j0) : WG);
        __syncthreads();
        if (tid < cnt) {
            const int64_t j = j0 + tid;
            const T ax = A[j], ay = A[a.ld_seg + j], az = A[2 * a.ld_seg + j];
            const T r0x = B[j] - ax, r0y = B[a.ld_seg + j] - ay, r0z = B[2 * a.ld_seg + j] - az;
            const T L02 = r0x * r0x + r0y * r0y + r0z * r0z;
            const T L0 = dsqrt(L02);
            const T eps = T(1e-12) * (L0 > T(1) ? L0 : T(1));
            const bool dead = L0 < eps;
            T coef = T(kInv4PiD) * Gs[j];
            if (VN != 0) coef = coef / L02;
            if (dead) coef = T(0);
            V4<T> p, q;
            p.x = ax; p.y = ay; p.z = az; p.w = coef;
            q.x = r0x; q.y = r0y; q.z = r0z; q.w = dead ? T(1) : L02;
            l0[tid] = p;
            l1[tid] = q;
            l2[tid] = eps * eps;
        }
        __syncthreads();
        for (int jj = 0; jj < cnt; ++jj) {
            const V4<T> p = l0[jj];
            const V4<T> q = l1[jj];
            const T eps2 = l2[jj];
            const T inv_l02 = T(1) / q.w;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const T r1x = P[k][0] - p.x, r1y = P[k][1] - p.y, r1z = P[k][2] - p.z;
                const T r2x = r1x - q.x, r2y = r1y - q.y, r2z = r1z - q.z;
                const T cx = q.y * r1z - q.z * r1y;
                const T cy = q.z * r1x - q.x * r1z;
                const T cz = q.x * r1y - q.y * r1x;
                const T c2 = cx * cx + cy * cy + cz * cz;
                const T l1s = r1x * r1x + r1y * r1y + r1z * r1z;
                const T l2s = r2x * r2x + r2y * r2y + r2z * r2z;
                const T d1 = q.x * r1x + q.y * r1y + q.z * r1z;
                const T d2 = d1 - q.w;
                const T i1 = rsqrt_fast(l1s), i2 = rsqrt_fast(l2s);
                const T D = d1 * i1 - d2 * i2;
                const T e1 = d1 * i1 * i1 * i1, e2 = d2 * i2 * i2 * i2;
                const T gDx = q.x * (i1 - i2) - r1x * e1 + r2x * e2;
                const T gDy = q.y * (i1 - i2) - r1y * e1 + r2y * e2;
                const T gDz = q.z * (i1 - i2) - r1z * e1 + r2z * e2;
                // c x r0
                const T wx = cy * q.z - cz * q.y;
                const T wy = cz * q.x - cx * q.z;
                const T wz = cx * q.y - cy * q.x;
                T f, ga, gb;  // grad f = ga grad D + gb (c x r0)
                if constexpr (VN == 0) {
                    const T ic2 = c2 > T(0) ? T(1) / c2 : T(0);
                    f = p.w * D * ic2;
                    ga = p.w * ic2;
                    gb = T(-2) * f * ic2;
                } else {
                    const T d2l = c2 * inv_l02;
                    T Kc, Kp;
                    if constexpr (VN == 1) {
                        Kc = T(1) / (d2l + rc2n);
                        Kp = -Kc * Kc;
                    } else if constexpr (VN == 2) {
                        Kc = rsqrt_fast(d2l * d2l + rc2n);
                        Kp = -d2l * Kc * Kc * Kc;
                    } else {
                        const T sden = pow(d2l, n_f) + rc2n;
                        Kc = pow(sden, -inv_n);
                        Kp = -pow(d2l, n_f - T(1)) * Kc / sden;
                    }
                    f = p.w * D * Kc;
                    ga = p.w * Kc;
                    gb = T(2) * p.w * D * Kp * inv_l02;
                }
                // selected after the products: an arm of zero length makes grad D non-finite
                const bool off = l1s < eps2 || l2s < eps2;
                f = off ? T(0) : f;
                const T gx = off ? T(0) : ga * gDx + gb * wx;
                const T gy = off ? T(0) : ga * gDy + gb * wy;
                const T gz = off ? T(0) : ga * gDz + gb * wz;
                T* ac = acc[k];
                ac[0] += f * cx;
                ac[1] += f * cy;
                ac[2] += f * cz;
                // f [r0]x + c g^T
                ac[3] += cx * gx;
                ac[4] += cx * gy - f * q.z;
                ac[5] += cx * gz + f * q.y;
                ac[6] += cy * gx + f * q.z;
                ac[7] += cy * gy;
                ac[8] += cy * gz - f * q.x;
                ac[9] += cz * gx - f * q.y;
                ac[10] += cz * gy + f * q.x;
                ac[11] += cz * gz;
            }
        }
        if constexpr (kComp) {
#pragma unroll
            for (int k = 0; k < K; ++k)
#pragma unroll
                for (int c = 0; c < NA; ++c) {
                    T s, e;
                    two_sum(hi[k][c], acc[k][c], s, e);
                    hi[k][c] = s;
                    lo[k][c] += e;
                    acc[k][c] = T(0);
                }
        }
    }
    T* __restrict__ U = static_cast<T*>(a.u);
    T* __restrict__ Jo = static_cast<T*>(a.grad);
    T* __restrict__ Do = static_cast<T*>(a.dg);
    const T* __restrict__ Gt = static_cast<const T*>(a.gt);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (!valid[k]) continue;
        const int64_t t = t0 + tid + int64_t(k) * WG;
        double v[NA];
#pragma unroll
        for (int c = 0; c < NA; ++c) v[c] = kComp ? double(hi[k][c]) + double(lo[k][c]) : double(acc[k][c]);
        if (U) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                T* dst = U + c * a.ldo + t;
                *dst = a.accumulate ? T(double(*dst) + v[c]) : T(v[c]);
            }
        }
        if (Jo) {
#pragma unroll
            for (int c = 0; c < 9; ++c) {
                T* dst = Jo + c * a.ldo + t;
                *dst = a.accumulate ? T(double(*dst) + v[3 + c]) : T(v[3 + c]);
            }
        }
        if (Do) {
            const double g[3] = {double(Gt[t]), double(Gt[a.ldt + t]), double(Gt[2 * a.ldt + t])};
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                // transposed: sum_b J[b][c] g_b; classical: sum_b J[c][b] g_b
                double s = 0.0;
#pragma unroll
                for (int b = 0; b < 3; ++b) s += (a.classical ? v[3 + 3 * c + b] : v[3 + 3 * b + c]) * g[b];
                T* dst = Do + c * a.ldo + t;
                *dst = a.accumulate ? T(double(*dst) + s) : T(s);
            }
        }
    }
}

template <typename T, int K, int WG>
hipError_t launch_t(const SegArgs& a, hipStream_t st) {
    const int grid = int((a.n_tgt + WG * K - 1) / (WG * K));
    if (a.rc == 0.0)
        hipLaunchKernelGGL((k_segments<T, K, WG, 0>), dim3(grid), dim3(WG), 0, st, a);
    else if (a.vn == 1)
        hipLaunchKernelGGL((k_segments<T, K, WG, 1>), dim3(grid), dim3(WG), 0, st, a);
    else if (a.vn == 2)
        hipLaunchKernelGGL((k_segments<T, K, WG, 2>), dim3(grid), dim3(WG), 0, st, a);
    else
        hipLaunchKernelGGL((k_segments<T, K, WG, 3>), dim3(grid), dim3(WG), 0, st, a);
    return hipGetLastError();
}

template <typename T, int K, int WG>
hipError_t launch_grad_t(const SegArgs& a, hipStream_t st) {
    const int grid = int((a.n_tgt + WG * K - 1) / (WG * K));
    if (a.rc == 0.0)
        hipLaunchKernelGGL((k_segments_grad<T, K, WG, 0>), dim3(grid), dim3(WG), 0, st, a);
    else if (a.vn == 1)
        hipLaunchKernelGGL((k_segments_grad<T, K, WG, 1>), dim3(grid), dim3(WG), 0, st, a);
    else if (a.vn == 2)
        hipLaunchKernelGGL((k_segments_grad<T, K, WG, 2>), dim3(grid), dim3(WG), 0, st, a);
    else
        hipLaunchKernelGGL((k_segments_grad<T, K, WG, 3>), dim3(grid), dim3(WG), 0, st, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_segments_gradient(int dtype, const SegArgs& a, hipStream_t st) {
    if (a.n_tgt == 0) return hipSuccess;
    if (dtype == kDtypeF64) return launch_grad_t<double, 1, 256>(a, st);
    return launch_grad_t<float, 1, 256>(a, st);
}

hipError_t launch_segments(int dtype, const SegArgs& a, hipStream_t st) {
    if (a.n_tgt == 0) return hipSuccess;
    if (dtype == kDtypeF64) return launch_t<double, 1, 256>(a, st);
    return launch_t<float, 2, 256>(a, st);
}

}  // namespace vpm
