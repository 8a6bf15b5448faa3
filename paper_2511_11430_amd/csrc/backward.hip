// Adjoint (vector-Jacobian product) of the particle sums of Eqs. 2-5 (Fu & Laurendeau,
// Sec. II.B), transposed stretching scheme, written out by hand.
//
// One pair (target i, source j, r = x_i - x_j) contributes, for seeds (ub_i, Sb_i) on
// (u_i, dGamma_i/dt), with v = Gamma_j x r, w = Gamma_i x Gamma_j, a = ub_i.v, b = Sb_i.w,
// tau = Gamma_i.v, c = Sb_i.r and weights g, h = g'/s, k = h'/s:
//   dphi/dr        = [(a + b) h + tau c k] r + g ub_i x Gamma_j + h c w + h tau Sb_i
//   xbar_i        += dphi/dr,         xbar_j -= dphi/dr
//   Gammabar_i    += g Gamma_j x Sb_i + h c v
//   Gammabar_j    += g (r x ub_i + Sb_i x Gamma_i) + h c (r x Gamma_i)
//
// Gather form, no atomics: each lane owns one particle p of the "lane set" and loops over the
// "loop set" q, collecting the terms where p is the target (role A, uses p's seeds) and where
// p is the source (role B, uses q's seeds).  Written with r = x_p - x_q in both roles:
//   role A: xbar_p += [(a+b) h + tau c k] r + g ub_p x Gamma_q + h c w + h tau Sb_p
//           Gbar_p += g Gamma_q x Sb_p + h c v
//   role B: a' = -ub_q.(Gamma_p x r), b' = -Sb_q.w, c' = -Sb_q.r  (tau is the same)
//           xbar_p += [(a'+b') h' + tau c' k'] r - g' ub_q x Gamma_p + h' c' w - h' tau Sb_q
//           Gbar_p += g' (Sb_q x Gamma_q - r x ub_q) + h' c' v
// with v = Gamma_q x r, w = Gamma_p x Gamma_q.  Self evaluation uses both roles over the one
// set and skips q == p; control-point targets use role B only (sources' gradients) or role A
// only (targets' gradients).  Weights follow the core-size rule of the forward pass: role A
// uses sigma_q (source rule), role B sigma_p; outside both cores they coincide.
// The kernel carries 4 pi g, 4 pi h and 4 pi k and scales by 1/(4 pi) at the end.
#include <hip/hip_runtime.h>

#include "device_math.h"
#include "vpm_internal.h"

namespace vpm {

namespace {

template <typename T>
using V4 = typename std::conditional<std::is_same<T, float>::value, float4, double4>::type;

// 4 pi (g, h, k) for one pair from the far-field powers and, inside the core, the series/closed form.
// SYM: the pair core is sigma_ij with 1/sigma_ij^2 = RHO_FAR^2 / cut; otherwise isig = 1/sigma.
template <typename T, bool SYM>
__device__ __forceinline__ void weights3(T s2, T isig, T cut, T Gf, T Hf, T Kf, T& g, T& h, T& k) {
    T G = Gf, Hn = Hf, Kn = Kf;
    if (s2 < cut) {
        T is = isig, is2;
        if (SYM) {
            is2 = T(Prec<T>::kFarRho2) * rcp_fast(cut);
            is = sqrt_fast(is2);
        } else {
            is2 = is * is;
        }
        core_weights3<T>(s2, is, is2, Gf, Hf, Kf, G, Hn, Kn);
    }
    g = G;
    h = T(-3) * Hn;
    k = T(15) * Kn;
}

template <typename T, int WG, bool RA, bool RB, bool STR, bool SYM>
__global__ __launch_bounds__(WG) void k_backward(BwdArgs a) {
    constexpr bool kComp = std::is_same<T, float>::value;
    __shared__ V4<T> l0[WG];  // (x, y, z, 1/sigma)
    __shared__ V4<T> l1[WG];  // (Gamma, cut)
    __shared__ V4<T> l2[RB ? WG : 1];  // ub_q
    __shared__ V4<T> l3[(RB && STR) ? WG : 1];  // Sb_q
    __shared__ V4<T> l4[(RB && STR) ? WG : 1];  // Sb_q x Gamma_q
    const T* __restrict__ xl = static_cast<const T*>(a.xl);
    const T* __restrict__ gl = static_cast<const T*>(a.gl);
    const T* __restrict__ sl = static_cast<const T*>(a.sl);
    const T* __restrict__ ubl = static_cast<const T*>(a.ubl);
    const T* __restrict__ sbl = static_cast<const T*>(a.sbl);
    const T* __restrict__ xo = static_cast<const T*>(a.xo);
    const T* __restrict__ go = static_cast<const T*>(a.go);
    const T* __restrict__ so = static_cast<const T*>(a.so);
    const T* __restrict__ ubo = static_cast<const T*>(a.ubo);
    const T* __restrict__ sbo = static_cast<const T*>(a.sbo);
    const T far2 = T(Prec<T>::kFarRho2);
    const int tid = threadIdx.x;
    const int64_t p = int64_t(blockIdx.x) * WG + tid;
    const bool valid = p < a.nl;
    const int64_t pp = valid ? p : 0;

    const T xp0 = xl[pp], xp1 = xl[a.ldl + pp], xp2 = xl[2 * a.ldl + pp];
    T gp0 = T(0), gp1 = T(0), gp2 = T(0);
    if (RB || STR) {
        gp0 = gl[pp];
        gp1 = gl[a.ldl + pp];
        gp2 = gl[2 * a.ldl + pp];
    }
    T sp = T(1);
    if (RB || SYM) sp = sl[pp];
    const T isig_p = T(1) / sp;
    const T cut_p = SYM ? T(0.5) * far2 * sp * sp : far2 * sp * sp;
    T up0 = T(0), up1 = T(0), up2 = T(0), sb0 = T(0), sb1 = T(0), sb2 = T(0);
    if (RA) {
        up0 = ubl[pp];
        up1 = ubl[a.ldl + pp];
        up2 = ubl[2 * a.ldl + pp];
        if (STR) {
            sb0 = sbl[pp];
            sb1 = sbl[a.ldl + pp];
            sb2 = sbl[2 * a.ldl + pp];
        }
    }

    T acc[6], hi[6], lo[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) acc[c] = hi[c] = lo[c] = T(0);

    for (int64_t j0 = 0; j0 < a.no; j0 += WG) {
        const int cnt = int((a.no - j0) < WG ? (a.no - j0) : WG);
        __syncthreads();
        if (tid < cnt) {
            const int64_t j = j0 + tid;
            // sigma_q is needed when q acts as a source (role A) or for the symmetric rule;
            // Gamma_q when q is a source or carries stretching seeds.
            const T sq = (RA || SYM) ? so[j] : T(1);
            V4<T> v0, v1;
            v0.x = xo[j]; v0.y = xo[a.ldo + j]; v0.z = xo[2 * a.ldo + j]; v0.w = T(1) / sq;
            if (RA || STR) {
                v1.x = go[j]; v1.y = go[a.ldo + j]; v1.z = go[2 * a.ldo + j];
            } else {
                v1.x = v1.y = v1.z = T(0);
            }
            v1.w = SYM ? T(0.5) * far2 * sq * sq : far2 * sq * sq;
            l0[tid] = v0;
            l1[tid] = v1;
            if (RB) {
                V4<T> v2;
                v2.x = ubo[j]; v2.y = ubo[a.ldo + j]; v2.z = ubo[2 * a.ldo + j]; v2.w = T(0);
                l2[tid] = v2;
                if (STR) {
                    V4<T> v3, v4;
                    v3.x = sbo[j]; v3.y = sbo[a.ldo + j]; v3.z = sbo[2 * a.ldo + j]; v3.w = T(0);
                    v4.x = v3.y * v1.z - v3.z * v1.y;
                    v4.y = v3.z * v1.x - v3.x * v1.z;
                    v4.z = v3.x * v1.y - v3.y * v1.x;
                    v4.w = T(0);
                    l3[tid] = v3;
                    l4[tid] = v4;
                }
            }
        }
        const int64_t pb0 = int64_t(blockIdx.x) * WG;
        const bool diag = a.self && (j0 < pb0 + WG) && (pb0 < j0 + cnt);
        __syncthreads();
        for (int jj = 0; jj < cnt; ++jj) {
            const V4<T> q0 = l0[jj];
            const V4<T> q1 = l1[jj];
            const T rx = xp0 - q0.x, ry = xp1 - q0.y, rz = xp2 - q0.z;
            const T s2 = rx * rx + ry * ry + rz * rz;
            const T rinv = rsqrt_fast(s2);
            const T rinv2 = rinv * rinv;
            const T Gf = rinv2 * rinv;
            const T Hf = Gf * rinv2;
            const T Kf = Hf * rinv2;
            const bool skip = diag && (j0 + jj == p);
            // v = Gamma_q x r
            const T vx = q1.y * rz - q1.z * ry;
            const T vy = q1.z * rx - q1.x * rz;
            const T vz = q1.x * ry - q1.y * rx;
            T wx = T(0), wy = T(0), wz = T(0), tau = T(0);
            if (STR) {
                wx = gp1 * q1.z - gp2 * q1.y;
                wy = gp2 * q1.x - gp0 * q1.z;
                wz = gp0 * q1.y - gp1 * q1.x;
                tau = gp0 * vx + gp1 * vy + gp2 * vz;
            }
            if (RA) {
                // sigma_q (source rule) or sigma_pq
                const T cut = SYM ? q1.w + cut_p : q1.w;
                T g, h, k;
                weights3<T, SYM>(s2, q0.w, cut, Gf, Hf, Kf, g, h, k);
                if (skip) g = h = k = T(0);
                const T av = up0 * vx + up1 * vy + up2 * vz;
                // g ub_p x Gamma_q
                const T ux = up1 * q1.z - up2 * q1.y;
                const T uy = up2 * q1.x - up0 * q1.z;
                const T uz = up0 * q1.y - up1 * q1.x;
                if (STR) {
                    const T b = sb0 * wx + sb1 * wy + sb2 * wz;
                    const T c = sb0 * rx + sb1 * ry + sb2 * rz;
                    const T sr = (av + b) * h + tau * c * k;
                    const T hc = h * c;
                    const T ht = h * tau;
                    acc[0] += sr * rx + g * ux + hc * wx + ht * sb0;
                    acc[1] += sr * ry + g * uy + hc * wy + ht * sb1;
                    acc[2] += sr * rz + g * uz + hc * wz + ht * sb2;
                    // g Gamma_q x Sb_p + h c v
                    acc[3] += g * (q1.y * sb2 - q1.z * sb1) + hc * vx;
                    acc[4] += g * (q1.z * sb0 - q1.x * sb2) + hc * vy;
                    acc[5] += g * (q1.x * sb1 - q1.y * sb0) + hc * vz;
                } else {
                    const T sr = av * h;
                    acc[0] += sr * rx + g * ux;
                    acc[1] += sr * ry + g * uy;
                    acc[2] += sr * rz + g * uz;
                }
            }
            if (RB) {
                const V4<T> q2 = l2[jj];
                // sigma_p (source rule) or sigma_pq
                const T cut = SYM ? q1.w + cut_p : cut_p;
                T g, h, k;
                weights3<T, SYM>(s2, isig_p, cut, Gf, Hf, Kf, g, h, k);
                if (skip) g = h = k = T(0);
                // Gamma_p x r
                const T v2x = gp1 * rz - gp2 * ry;
                const T v2y = gp2 * rx - gp0 * rz;
                const T v2z = gp0 * ry - gp1 * rx;
                const T ap = -(q2.x * v2x + q2.y * v2y + q2.z * v2z);
                // ub_q x Gamma_p
                const T ux = q2.y * gp2 - q2.z * gp1;
                const T uy = q2.z * gp0 - q2.x * gp2;
                const T uz = q2.x * gp1 - q2.y * gp0;
                // r x ub_q
                const T rux = ry * q2.z - rz * q2.y;
                const T ruy = rz * q2.x - rx * q2.z;
                const T ruz = rx * q2.y - ry * q2.x;
                if (STR) {
                    const V4<T> q3 = l3[jj];
                    const V4<T> q4 = l4[jj];
                    const T bp = -(q3.x * wx + q3.y * wy + q3.z * wz);
                    const T cp = -(q3.x * rx + q3.y * ry + q3.z * rz);
                    const T sr = (ap + bp) * h + tau * cp * k;
                    const T hc = h * cp;
                    const T ht = h * tau;
                    acc[0] += sr * rx - g * ux + hc * wx - ht * q3.x;
                    acc[1] += sr * ry - g * uy + hc * wy - ht * q3.y;
                    acc[2] += sr * rz - g * uz + hc * wz - ht * q3.z;
                    acc[3] += g * (q4.x - rux) + hc * vx;
                    acc[4] += g * (q4.y - ruy) + hc * vy;
                    acc[5] += g * (q4.z - ruz) + hc * vz;
                } else {
                    const T sr = ap * h;
                    acc[0] += sr * rx - g * ux;
                    acc[1] += sr * ry - g * uy;
                    acc[2] += sr * rz - g * uz;
                    acc[3] -= g * rux;
                    acc[4] -= g * ruy;
                    acc[5] -= g * ruz;
                }
            }
        }
        if constexpr (kComp) {
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                T s, e;
                two_sum(hi[c], acc[c], s, e);
                hi[c] = s;
                lo[c] += e;
                acc[c] = T(0);
            }
        }
    }
    if (!valid) return;
    T* __restrict__ xb = static_cast<T*>(a.xbar);
    T* __restrict__ gb = static_cast<T*>(a.gbar);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        const double v = kInv4PiD * (kComp ? double(hi[c]) + double(lo[c]) : double(acc[c]));
        if (c >= 3 && !(RB || STR)) continue;  // velocity-only target gradients touch x only
        T* dst = (c < 3 ? xb : gb) + (c % 3) * a.ldg + p;
        *dst = T(double(*dst) + v);
    }
}

template <typename T, int WG, bool RA, bool RB>
hipError_t launch_rs(bool stretch, bool sym, const BwdArgs& a, hipStream_t st) {
    const int grid = int((a.nl + WG - 1) / WG);
    if (stretch) {
        if (sym) hipLaunchKernelGGL((k_backward<T, WG, RA, RB, true, true>), dim3(grid), dim3(WG), 0, st, a);
        else hipLaunchKernelGGL((k_backward<T, WG, RA, RB, true, false>), dim3(grid), dim3(WG), 0, st, a);
    } else {
        if (sym) hipLaunchKernelGGL((k_backward<T, WG, RA, RB, false, true>), dim3(grid), dim3(WG), 0, st, a);
        else hipLaunchKernelGGL((k_backward<T, WG, RA, RB, false, false>), dim3(grid), dim3(WG), 0, st, a);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_t(bool ra, bool rb, bool stretch, bool sym, const BwdArgs& a, hipStream_t st) {
    if (ra && rb) return launch_rs<T, 256, true, true>(stretch, sym, a, st);
    if (ra) return launch_rs<T, 256, true, false>(stretch, sym, a, st);
    return launch_rs<T, 256, false, true>(stretch, sym, a, st);
}

}  // namespace

hipError_t launch_backward(int dtype, bool role_a, bool role_b, bool stretch, bool sym,
                           const BwdArgs& a, hipStream_t st) {
    if (a.nl == 0) return hipSuccess;
    if (!role_a && !role_b) return hipErrorInvalidValue;
    if (dtype == kDtypeF64) return launch_t<double>(role_a, role_b, stretch, sym, a, st);
    return launch_t<float>(role_a, role_b, stretch, sym, a, st);
}

}  // namespace vpm
