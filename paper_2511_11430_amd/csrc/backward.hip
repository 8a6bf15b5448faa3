// Adjoint (vector-Jacobian product) of the particle sums of Eqs. 2-5 (Fu & Laurendeau,
// Sec. II.B), transposed stretching scheme, written out by hand.  (The classical scheme's
// adjoint is composed from this kernel and the forward kernel on the host side: its pair
// term S.(J Gamma_i) equals the transposed term Gamma_i.(J^T S) with the target strength and
// the stretching seed exchanged.)
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
// "loop set" q, collecting the terms where p is the target (role A: weights gA, hA, kA from the
// source core sigma_q, p's seeds) and where p is the source (role B: gB, hB, kB from sigma_p,
// q's seeds).  With r = x_p - x_q, v = Gamma_q x r, R = r x ub_q, E_p = Sb_p x Gamma_p and
// Z_q = Sb_q x Gamma_q:
//   a = ub_p.v, a' = -Gamma_p.R, b = Gamma_q.E_p, b' = Gamma_p.Z_q, tau = Gamma_p.v,
//   c = Sb_p.r, c' = -Sb_q.r, hcs = hA c + hB c'
//   xbar_p += sum [(a+b) hA + tau c kA + (a'+b') hB + tau c' kB] r        (accumulator SR)
//           + ub_p x sum gA Gamma_q                                         (A)
//           + Gamma_p x sum (gB ub_q + hcs Gamma_q)                          (UW)
//           + (sum hA tau) Sb_p - sum hB tau Sb_q                           (T, V)
//   Gbar_p += (sum gA Gamma_q) x Sb_p + sum (gB (Z_q - R) + hcs v)           (A, Q)
// Terms that are a per-particle vector times a sum over q are summed first and finished once
// per particle, which is what keeps the pair cost near three forward pairs.  Outside every
// core (decided per tile from bounding boxes) the two roles share one set of point-vortex
// weights; inside, each role takes its own core.  The kernel carries 4 pi (g, h, k) and
// scales by 1/(4 pi) at the end.  Per-particle sums are FP32 tile partials folded into two-sum
// pairs (VPM_F32C) or plain FP64 (VPM_F64).
#include <hip/hip_runtime.h>

#include "device_math.h"

// The FP64 kernels call their in-core weights (a convergent call), and clang then reports the
// unroll requests of the loops around that call as not honoured.
#pragma clang diagnostic ignored "-Wpass-failed"
#include "vpm_internal.h"

namespace vpm {

namespace {

template <typename T>
using V4 = typename std::conditional<std::is_same<T, float>::value, float4, double4>::type;

// Keeps a value opaque to the optimiser so that work derived from it inside the rare core
// branch is not hoisted into the hot path (emits no instruction).
__device__ __forceinline__ float opaque_b(float v) {
    asm volatile("" : "+v"(v));
    return v;
}
__device__ __forceinline__ double opaque_b(double v) {
    asm volatile("" : "+v"(v));
    return v;
}

// 4 pi (g, h, k) inside the core (s2 < cut); SYM: 1/sigma^2 = RHO_FAR^2 / cut.
template <typename T, bool SYM>
__device__ __forceinline__ void core3(T s2, T isig, T cut, T Gf, T Hf, T Kf, T& g, T& h, T& k) {
    T is, is2;
    if (SYM) {
        is2 = T(Prec<T>::kFarRho2) * rcp_fast(opaque_b(cut));
        is = sqrt_fast(is2);
    } else {
        is = opaque_b(isig);
        is2 = is * is;
    }
    T G, Hn, Kn;
    core_weights3_call(s2, is, is2, Gf, Hf, Kf, G, Hn, Kn);
    g = G;
    h = T(-3) * Hn;
    k = T(15) * Kn;
}

// Accumulator slots: 0-2 SR r, 3-5 A, 6-8 UW, 9-11 Q, and with stretching seeds 12-14 V, 15 T.
template <typename T, int WG, bool RA, bool RB, bool STR, bool SYM>
struct Bwd {
    static constexpr bool kComp = std::is_same<T, float>::value;
    static constexpr int kN = STR ? 16 : 12;

    // Both roles with one set of weights (g, h, k): q1 = (Gamma_q, .), q2 = ub_q, q3 = Sb_q,
    // q4 = Sb_q x Gamma_q (q3, q4 unused without stretching seeds).
    static __device__ __forceinline__ void far_pair(const V4<T>& q1, const V4<T>& q2, const V4<T>& q3,
                                                    const V4<T>& q4, T rx, T ry, T rz, T g, T h, T k,
                                                    const T (&gp)[3], const T (&up)[3], const T (&sp)[3],
                                                    const T (&ep)[3], T (&acc)[kN]) {
        // v = Gamma_q x r,  R = r x ub_q
        const T vx = q1.y * rz - q1.z * ry;
        const T vy = q1.z * rx - q1.x * rz;
        const T vz = q1.x * ry - q1.y * rx;
        const T Rx = ry * q2.z - rz * q2.y;
        const T Ry = rz * q2.x - rx * q2.z;
        const T Rz = rx * q2.y - ry * q2.x;
        acc[3] += g * q1.x;
        acc[4] += g * q1.y;
        acc[5] += g * q1.z;
        acc[6] += g * q2.x;
        acc[7] += g * q2.y;
        acc[8] += g * q2.z;
        T sr;
        if (STR) {
            // D = Z_q - R, so a' + b' = Gamma_p . D and the Q term is g D + hcc v
            const T Dx = q4.x - Rx, Dy = q4.y - Ry, Dz = q4.z - Rz;
            // s_ab = a + b + a' + b' = ub_p.v + Gamma_q.E_p + Gamma_p.D, one FMA chain
            T s_ab = up[0] * vx;
            s_ab = fma(up[1], vy, s_ab);
            s_ab = fma(up[2], vz, s_ab);
            s_ab = fma(q1.x, ep[0], s_ab);
            s_ab = fma(q1.y, ep[1], s_ab);
            s_ab = fma(q1.z, ep[2], s_ab);
            s_ab = fma(gp[0], Dx, s_ab);
            s_ab = fma(gp[1], Dy, s_ab);
            s_ab = fma(gp[2], Dz, s_ab);
            // c + c' = (Sb_p - Sb_q) . r
            T cc = (sp[0] - q3.x) * rx;
            cc = fma(sp[1] - q3.y, ry, cc);
            cc = fma(sp[2] - q3.z, rz, cc);
            T tau = gp[0] * vx;
            tau = fma(gp[1], vy, tau);
            tau = fma(gp[2], vz, tau);
            sr = fma(k * tau, cc, h * s_ab);
            const T hcc = h * cc;
            const T ht = h * tau;
            acc[15] += ht;
            acc[12] += ht * q3.x;
            acc[13] += ht * q3.y;
            acc[14] += ht * q3.z;
            acc[6] += hcc * q1.x;
            acc[7] += hcc * q1.y;
            acc[8] += hcc * q1.z;
            acc[9] += g * Dx;
            acc[10] += g * Dy;
            acc[11] += g * Dz;
            acc[9] += hcc * vx;
            acc[10] += hcc * vy;
            acc[11] += hcc * vz;
        } else {
            T s_ab = up[0] * vx;
            s_ab = fma(up[1], vy, s_ab);
            s_ab = fma(up[2], vz, s_ab);
            s_ab = fma(-gp[0], Rx, s_ab);
            s_ab = fma(-gp[1], Ry, s_ab);
            s_ab = fma(-gp[2], Rz, s_ab);
            sr = h * s_ab;
            acc[9] -= g * Rx;
            acc[10] -= g * Ry;
            acc[11] -= g * Rz;
        }
        acc[0] += sr * rx;
        acc[1] += sr * ry;
        acc[2] += sr * rz;
    }

    template <bool CHECK, bool NEAR>
    static __device__ __forceinline__ void tile(const V4<T>* l0, const V4<T>* l1, const V4<T>* l2, const V4<T>* l3,
                                                const V4<T>* l4, int cnt, int64_t j0, int64_t p, const T (&xp)[3],
                                                const T (&gp)[3], const T (&up)[3], const T (&sp)[3],
                                                const T (&ep)[3], T isig_p, T cut_p, T (&acc)[kN]) {
#pragma unroll 2
        for (int jj = 0; jj < cnt; ++jj) {
            const V4<T> q0 = l0[jj];  // x_q, 1/sigma_q
            const V4<T> q1 = l1[jj];  // Gamma_q, cut_q
            const T rx = xp[0] - q0.x, ry = xp[1] - q0.y, rz = xp[2] - q0.z;
            const T s2 = rx * rx + ry * ry + rz * rz;
            const T rinv = rsqrt_fast(s2);
            const T rinv2 = rinv * rinv;
            const T Gf = rinv2 * rinv;
            const T Hf = Gf * rinv2;
            const T Kf = Hf * rinv2;
            T gA = Gf, hA = T(-3) * Hf, kA = T(15) * Kf;
            T gB = gA, hB = hA, kB = kA;
            if (NEAR) {
                const T cutA = SYM ? q1.w + cut_p : q1.w;
                const T cutB = SYM ? cutA : cut_p;
                if (RA && s2 < cutA) core3<T, SYM>(s2, q0.w, cutA, Gf, Hf, Kf, gA, hA, kA);
                if (RB && s2 < cutB) {
                    if (SYM && RA) {  // one symmetric core for both roles
                        gB = gA;
                        hB = hA;
                        kB = kA;
                    } else {
                        core3<T, SYM>(s2, isig_p, cutB, Gf, Hf, Kf, gB, hB, kB);
                    }
                }
            }
            if (CHECK && j0 + jj == p) gA = hA = kA = gB = hB = kB = T(0);
            if constexpr (!NEAR && !CHECK && RA && RB) {
                // Outside every core both roles share (g, h, k): add the roles' terms before
                // multiplying by the weights.
                far_pair(q1, l2[jj], STR ? l3[jj] : q1, STR ? l4[jj] : q1, rx, ry, rz, gA, hA, kA, gp, up, sp, ep,
                         acc);
            } else {
                pair_general(q1, jj, l2, l3, l4, rx, ry, rz, gA, hA, kA, gB, hB, kB, gp, up, sp, ep, acc);
            }
        }
    }

    // Both roles with their own weights (cores, excluded pairs, single-role launches).
    static __device__ __forceinline__ void pair_general(const V4<T>& q1, int jj, const V4<T>* l2, const V4<T>* l3,
                                                        const V4<T>* l4, T rx, T ry, T rz, T gA, T hA, T kA, T gB,
                                                        T hB, T kB, const T (&gp)[3], const T (&up)[3],
                                                        const T (&sp)[3], const T (&ep)[3], T (&acc)[kN]) {
        {
            // v = Gamma_q x r
            const T vx = q1.y * rz - q1.z * ry;
            const T vy = q1.z * rx - q1.x * rz;
            const T vz = q1.x * ry - q1.y * rx;
            T sr = T(0);
            if (RA) {
                const T a = up[0] * vx + up[1] * vy + up[2] * vz;
                sr = a * hA;
                acc[3] += gA * q1.x;
                acc[4] += gA * q1.y;
                acc[5] += gA * q1.z;
            }
            if (RB) {
                const V4<T> q2 = l2[jj];  // ub_q
                // R = r x ub_q
                const T Rx = ry * q2.z - rz * q2.y;
                const T Ry = rz * q2.x - rx * q2.z;
                const T Rz = rx * q2.y - ry * q2.x;
                const T ap = -(gp[0] * Rx + gp[1] * Ry + gp[2] * Rz);
                sr += ap * hB;
                acc[6] += gB * q2.x;
                acc[7] += gB * q2.y;
                acc[8] += gB * q2.z;
                acc[9] -= gB * Rx;
                acc[10] -= gB * Ry;
                acc[11] -= gB * Rz;
            }
            if (STR) {
                const T tau = gp[0] * vx + gp[1] * vy + gp[2] * vz;
                T hcs = T(0);
                if (RA) {
                    const T b = q1.x * ep[0] + q1.y * ep[1] + q1.z * ep[2];
                    const T c = sp[0] * rx + sp[1] * ry + sp[2] * rz;
                    sr += b * hA + tau * c * kA;
                    hcs = hA * c;
                    acc[15] += hA * tau;
                }
                if (RB) {
                    const V4<T> q3 = l3[jj];  // Sb_q
                    const V4<T> q4 = l4[jj];  // Z_q = Sb_q x Gamma_q
                    const T bp = gp[0] * q4.x + gp[1] * q4.y + gp[2] * q4.z;
                    const T cp = -(q3.x * rx + q3.y * ry + q3.z * rz);
                    sr += bp * hB + tau * cp * kB;
                    hcs += hB * cp;
                    const T ht = hB * tau;
                    acc[12] += ht * q3.x;
                    acc[13] += ht * q3.y;
                    acc[14] += ht * q3.z;
                    acc[9] += gB * q4.x;
                    acc[10] += gB * q4.y;
                    acc[11] += gB * q4.z;
                }
                acc[6] += hcs * q1.x;
                acc[7] += hcs * q1.y;
                acc[8] += hcs * q1.z;
                acc[9] += hcs * vx;
                acc[10] += hcs * vy;
                acc[11] += hcs * vz;
            }
            acc[0] += sr * rx;
            acc[1] += sr * ry;
            acc[2] += sr * rz;
        }
    }
};

// Workgroup bounding box (v[0..2] min, v[3..5] max) and largest cut (v[6]): a shuffle
// reduction per wavefront, then LDS.  Ends with a barrier; every thread gets the result.
template <typename T>
__device__ __forceinline__ void box_reduce(T (&v)[7], T* scratch) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int c = 0; c < 7; ++c) {
            const T o = __shfl_xor(v[c], off, 64);
            v[c] = c < 3 ? fmin(v[c], o) : fmax(v[c], o);
        }
    }
    const int wave = threadIdx.x >> 6;
    const int nwave = (blockDim.x + 63) >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int c = 0; c < 7; ++c) scratch[wave * 7 + c] = v[c];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 7; ++c) v[c] = scratch[c];
    for (int w = 1; w < nwave; ++w) {
#pragma unroll
        for (int c = 0; c < 7; ++c) v[c] = c < 3 ? fmin(v[c], scratch[w * 7 + c]) : fmax(v[c], scratch[w * 7 + c]);
    }
}

// One workgroup's lane block blk of a lane set [lb, lb + nl) against the loop set
// [ob, ob + no) (indices into the arrays of a; with a.self both sets are the same range).
template <typename T, int WG, bool RA, bool RB, bool STR, bool SYM>
__device__ __forceinline__ void backward_body(const BwdArgs& a, int64_t blk, int64_t lb, int64_t nl, int64_t ob,
                                              int64_t no) {
    using B = Bwd<T, WG, RA, RB, STR, SYM>;
    constexpr int kN = B::kN;
    constexpr bool kComp = B::kComp;
    __shared__ V4<T> l0[WG];                    // (x, y, z, 1/sigma)
    __shared__ V4<T> l1[WG];                    // (Gamma, cut)
    __shared__ V4<T> l2[RB ? WG : 1];           // ub_q
    __shared__ V4<T> l3[(RB && STR) ? WG : 1];  // Sb_q
    __shared__ V4<T> l4[(RB && STR) ? WG : 1];  // Sb_q x Gamma_q
    __shared__ T box[7 * (WG / 64)];
    // the set bases are folded into the pointers (null pointers stay null)
    auto at = [](const void* q, int64_t base) { return q ? static_cast<const T*>(q) + base : nullptr; };
    const T* __restrict__ xl = at(a.xl, lb);
    const T* __restrict__ gl = at(a.gl, lb);
    const T* __restrict__ sl = at(a.sl, lb);
    const T* __restrict__ ubl = at(a.ubl, lb);
    const T* __restrict__ sbl = at(a.sbl, lb);
    const T* __restrict__ xo = at(a.xo, ob);
    const T* __restrict__ go = at(a.go, ob);
    const T* __restrict__ so = at(a.so, ob);
    const T* __restrict__ ubo = at(a.ubo, ob);
    const T* __restrict__ sbo = at(a.sbo, ob);
    const T far2 = T(Prec<T>::kFarRho2);
    const int tid = threadIdx.x;
    const int64_t pb0 = blk * WG;
    const int64_t p = pb0 + tid;
    const bool valid = p < nl;
    const int64_t pp = valid ? p : pb0;

    T xp[3] = {xl[pp], xl[a.ldl + pp], xl[2 * a.ldl + pp]};
    T gp[3] = {T(0), T(0), T(0)};
    if (RB || STR) {
        gp[0] = gl[pp];
        gp[1] = gl[a.ldl + pp];
        gp[2] = gl[2 * a.ldl + pp];
    }
    T sgp = T(1);
    if (RB || SYM) sgp = sl[pp];
    const T isig_p = T(1) / sgp;
    // this particle's role-B core cut (source rule) or its half of the symmetric cut
    const T cut_p = SYM ? T(0.5) * far2 * sgp * sgp : (RB ? far2 * sgp * sgp : T(0));
    T up[3] = {T(0), T(0), T(0)}, sp[3] = {T(0), T(0), T(0)}, ep[3] = {T(0), T(0), T(0)};
    if (RA) {
        up[0] = ubl[pp];
        up[1] = ubl[a.ldl + pp];
        up[2] = ubl[2 * a.ldl + pp];
        if (STR) {
            sp[0] = sbl[pp];
            sp[1] = sbl[a.ldl + pp];
            sp[2] = sbl[2 * a.ldl + pp];
            ep[0] = sp[1] * gp[2] - sp[2] * gp[1];
            ep[1] = sp[2] * gp[0] - sp[0] * gp[2];
            ep[2] = sp[0] * gp[1] - sp[1] * gp[0];
        }
    }
    // bounding box of this workgroup's lane particles and their largest cut
    T bb[7] = {xp[0], xp[1], xp[2], xp[0], xp[1], xp[2], valid ? cut_p : T(0)};
    box_reduce(bb, box);

    T acc[kN], hi[kN], lo[kN];
#pragma unroll
    for (int c = 0; c < kN; ++c) acc[c] = hi[c] = lo[c] = T(0);

    for (int64_t j0 = 0; j0 < no; j0 += WG) {
        const int cnt = int((no - j0) < WG ? (no - j0) : WG);
        __syncthreads();
        // idle slots (tid >= cnt) read the tile's first particle, which keeps the box exact
        const int64_t jl = j0 + (tid < cnt ? tid : 0);
        // sigma_q is needed when q acts as a source (role A) or for the symmetric rule;
        // Gamma_q when q is a source or carries stretching seeds.
        const T sq = (RA || SYM) ? so[jl] : T(1);
        V4<T> v0, v1;
        v0.x = xo[jl]; v0.y = xo[a.ldo + jl]; v0.z = xo[2 * a.ldo + jl]; v0.w = T(1) / sq;
        if (RA || STR) {
            v1.x = go[jl]; v1.y = go[a.ldo + jl]; v1.z = go[2 * a.ldo + jl];
        } else {
            v1.x = v1.y = v1.z = T(0);
        }
        v1.w = SYM ? T(0.5) * far2 * sq * sq : (RA ? far2 * sq * sq : T(0));
        if (tid < cnt) {
            l0[tid] = v0;
            l1[tid] = v1;
            if (RB) {
                V4<T> v2;
                v2.x = ubo[jl]; v2.y = ubo[a.ldo + jl]; v2.z = ubo[2 * a.ldo + jl]; v2.w = T(0);
                l2[tid] = v2;
                if (STR) {
                    V4<T> v3, v4;
                    v3.x = sbo[jl]; v3.y = sbo[a.ldo + jl]; v3.z = sbo[2 * a.ldo + jl]; v3.w = T(0);
                    v4.x = v3.y * v1.z - v3.z * v1.y;
                    v4.y = v3.z * v1.x - v3.x * v1.z;
                    v4.z = v3.x * v1.y - v3.y * v1.x;
                    v4.w = T(0);
                    l3[tid] = v3;
                    l4[tid] = v4;
                }
            }
        }
        // tile box and its largest role-A cut; the reduction's barriers also publish the tile
        T tb[7] = {v0.x, v0.y, v0.z, v0.x, v0.y, v0.z, tid < cnt ? v1.w : T(0)};
        box_reduce(tb, box);
        T d2 = T(0);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const T gap = fmax(fmax(tb[c] - bb[3 + c], bb[c] - tb[3 + c]), T(0));
            d2 += gap * gap;
        }
        const T reach = SYM ? tb[6] + bb[6] : fmax(tb[6], bb[6]);
        const bool near = d2 < reach;
        const bool diag = a.self && (j0 < pb0 + WG) && (pb0 < j0 + cnt);
        if (diag) {
            if (near) B::template tile<true, true>(l0, l1, l2, l3, l4, cnt, j0, p, xp, gp, up, sp, ep, isig_p, cut_p, acc);
            else B::template tile<true, false>(l0, l1, l2, l3, l4, cnt, j0, p, xp, gp, up, sp, ep, isig_p, cut_p, acc);
        } else {
            if (near) B::template tile<false, true>(l0, l1, l2, l3, l4, cnt, j0, p, xp, gp, up, sp, ep, isig_p, cut_p, acc);
            else B::template tile<false, false>(l0, l1, l2, l3, l4, cnt, j0, p, xp, gp, up, sp, ep, isig_p, cut_p, acc);
        }
        if constexpr (kComp) {
#pragma unroll
            for (int c = 0; c < kN; ++c) {
                T s, e;
                two_sum(hi[c], acc[c], s, e);
                hi[c] = s;
                lo[c] += e;
                acc[c] = T(0);
            }
        }
    }
    if (!valid) return;  // (nothing follows in a caller's loop that this lane must reach)
    double t[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) t[c] = 0.0;
#pragma unroll
    for (int c = 0; c < kN; ++c) t[c] = kComp ? double(hi[c]) + double(lo[c]) : double(acc[c]);
    const double u0 = up[0], u1 = up[1], u2 = up[2];
    const double g0 = gp[0], g1 = gp[1], g2 = gp[2];
    const double s0 = sp[0], s1 = sp[1], s2 = sp[2];
    // xbar = SR + ub_p x A + Gamma_p x UW + T Sb_p - V
    double xb[3] = {t[0], t[1], t[2]};
    xb[0] += u1 * t[5] - u2 * t[4] + g1 * t[8] - g2 * t[7];
    xb[1] += u2 * t[3] - u0 * t[5] + g2 * t[6] - g0 * t[8];
    xb[2] += u0 * t[4] - u1 * t[3] + g0 * t[7] - g1 * t[6];
    // Gbar = A x Sb_p + Q
    double gb[3] = {t[9], t[10], t[11]};
    if (STR) {
        xb[0] += t[15] * s0 - t[12];
        xb[1] += t[15] * s1 - t[13];
        xb[2] += t[15] * s2 - t[14];
        gb[0] += t[4] * s2 - t[5] * s1;
        gb[1] += t[5] * s0 - t[3] * s2;
        gb[2] += t[3] * s1 - t[4] * s0;
    }
    T* __restrict__ xo_bar = static_cast<T*>(a.xbar) + lb;
    T* __restrict__ go_bar = a.gbar ? static_cast<T*>(a.gbar) + lb : nullptr;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        T* d = xo_bar + c * a.ldg + p;
        *d = T(double(*d) + kInv4PiD * xb[c]);
    }
    // velocity-only target gradients touch x only; a null gbar drops the strength gradient
    // (the classical scheme's composition discards the target-role part it recomputes)
    if ((RB || STR) && go_bar) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            T* d = go_bar + c * a.ldg + p;
            *d = T(double(*d) + kInv4PiD * gb[c]);
        }
    }
}

// FP32: ask for 4 wavefronts per SIMD (<= 128 VGPRs; no spills at these shapes).  FP64 keeps
// the compiler's choice: its accumulators need twice the registers.
template <typename T, int WG, bool RA, bool RB, bool STR, bool SYM>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(4))) void k_backward_f32(BwdArgs a) {
    backward_body<T, WG, RA, RB, STR, SYM>(a, blockIdx.x, 0, a.nl, 0, a.no);
}
template <typename T, int WG, bool RA, bool RB, bool STR, bool SYM>
__global__ __launch_bounds__(WG) void k_backward_f64(BwdArgs a) {
    backward_body<T, WG, RA, RB, STR, SYM>(a, blockIdx.x, 0, a.nl, 0, a.no);
}

// Many independent sets in one launch: persistent workgroups pop (set, lane block) items,
// ordered by decreasing cost, from the queue's counter; the lane set of item set b is
// [src_off[b], src_off[b+1]) and the loop set [tgt_off[b], tgt_off[b+1]) (exchanged when
// lane_is_tgt).  Every workgroup leaves once the counter passes the item count.
template <typename T, int WG, bool RA, bool RB, bool STR, bool SYM>
__device__ __forceinline__ void backward_queue(const BwdArgs& a, const BatchQueue& q, int lane_is_tgt) {
    __shared__ int item_s;
    for (;;) {
        if (threadIdx.x == 0) item_s = atomicAdd(q.counter, 1);
        __syncthreads();
        const int item = item_s;
        __syncthreads();
        if (item >= q.n_items) break;
        const int2 it = q.items[item];
        const int64_t* lo = lane_is_tgt ? q.tgt_off : q.src_off;
        const int64_t* oo = lane_is_tgt ? q.src_off : q.tgt_off;
        const int64_t lb = lo[it.x], ob = oo[it.x];
        backward_body<T, WG, RA, RB, STR, SYM>(a, it.y, lb, lo[it.x + 1] - lb, ob, oo[it.x + 1] - ob);
    }
}
template <typename T, int WG, bool RA, bool RB, bool STR, bool SYM>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(4))) void k_backward_batched_f32(
    BwdArgs a, BatchQueue q, int lane_is_tgt) {
    backward_queue<T, WG, RA, RB, STR, SYM>(a, q, lane_is_tgt);
}
template <typename T, int WG, bool RA, bool RB, bool STR, bool SYM>
__global__ __launch_bounds__(WG) void k_backward_batched_f64(BwdArgs a, BatchQueue q, int lane_is_tgt) {
    backward_queue<T, WG, RA, RB, STR, SYM>(a, q, lane_is_tgt);
}

template <typename T, int WG, bool RA, bool RB, bool STR, bool SYM>
void launch_k(int grid, const BwdArgs& a, hipStream_t st) {
    if constexpr (std::is_same<T, float>::value)
        hipLaunchKernelGGL((k_backward_f32<T, WG, RA, RB, STR, SYM>), dim3(grid), dim3(WG), 0, st, a);
    else
        hipLaunchKernelGGL((k_backward_f64<T, WG, RA, RB, STR, SYM>), dim3(grid), dim3(WG), 0, st, a);
}

// Persistent launch over a queue (grid <= 0: only report the kernel's resident workgroups
// per CU through *occ).
template <typename T, int WG, bool RA, bool RB, bool STR, bool SYM>
hipError_t launch_kq(int grid, const BwdArgs& a, const BatchQueue& q, int lane_is_tgt, int* occ, hipStream_t st) {
    if (grid <= 0) {
        if constexpr (std::is_same<T, float>::value)
            return hipOccupancyMaxActiveBlocksPerMultiprocessor(
                occ, reinterpret_cast<const void*>(k_backward_batched_f32<T, WG, RA, RB, STR, SYM>), WG, 0);
        else
            return hipOccupancyMaxActiveBlocksPerMultiprocessor(
                occ, reinterpret_cast<const void*>(k_backward_batched_f64<T, WG, RA, RB, STR, SYM>), WG, 0);
    }
    if constexpr (std::is_same<T, float>::value)
        hipLaunchKernelGGL((k_backward_batched_f32<T, WG, RA, RB, STR, SYM>), dim3(grid), dim3(WG), 0, st, a, q,
                           lane_is_tgt);
    else
        hipLaunchKernelGGL((k_backward_batched_f64<T, WG, RA, RB, STR, SYM>), dim3(grid), dim3(WG), 0, st, a, q,
                           lane_is_tgt);
    return hipGetLastError();
}

template <typename T, int WG, bool RA, bool RB>
hipError_t launch_rs(bool stretch, bool sym, const BwdArgs& a, const BatchQueue* q, int grid, int lane_is_tgt,
                     int* occ, hipStream_t st) {
    if (q) {
        if (stretch) {
            if (sym) return launch_kq<T, WG, RA, RB, true, true>(grid, a, *q, lane_is_tgt, occ, st);
            return launch_kq<T, WG, RA, RB, true, false>(grid, a, *q, lane_is_tgt, occ, st);
        }
        if (sym) return launch_kq<T, WG, RA, RB, false, true>(grid, a, *q, lane_is_tgt, occ, st);
        return launch_kq<T, WG, RA, RB, false, false>(grid, a, *q, lane_is_tgt, occ, st);
    }
    grid = int((a.nl + WG - 1) / WG);
    if (stretch) {
        if (sym) launch_k<T, WG, RA, RB, true, true>(grid, a, st);
        else launch_k<T, WG, RA, RB, true, false>(grid, a, st);
    } else {
        if (sym) launch_k<T, WG, RA, RB, false, true>(grid, a, st);
        else launch_k<T, WG, RA, RB, false, false>(grid, a, st);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_t(bool ra, bool rb, bool stretch, bool sym, const BwdArgs& a, const BatchQueue* q, int grid,
                    int lane_is_tgt, int* occ, hipStream_t st) {
    if (ra && rb) return launch_rs<T, kBwdWG, true, true>(stretch, sym, a, q, grid, lane_is_tgt, occ, st);
    if (ra) return launch_rs<T, kBwdWG, true, false>(stretch, sym, a, q, grid, lane_is_tgt, occ, st);
    return launch_rs<T, kBwdWG, false, true>(stretch, sym, a, q, grid, lane_is_tgt, occ, st);
}

}  // namespace

hipError_t launch_backward(int dtype, bool role_a, bool role_b, bool stretch, bool sym,
                           const BwdArgs& a, hipStream_t st) {
    if (a.nl == 0) return hipSuccess;
    if (!role_a && !role_b) return hipErrorInvalidValue;
    if (dtype == kDtypeF64) return launch_t<double>(role_a, role_b, stretch, sym, a, nullptr, 0, 0, nullptr, st);
    return launch_t<float>(role_a, role_b, stretch, sym, a, nullptr, 0, 0, nullptr, st);
}

hipError_t launch_backward_batched(int dtype, bool role_a, bool role_b, bool stretch, bool sym, const BwdArgs& a,
                                   const BatchQueue& q, int grid, int lane_is_tgt, hipStream_t st) {
    if (!role_a && !role_b) return hipErrorInvalidValue;
    if (dtype == kDtypeF64) return launch_t<double>(role_a, role_b, stretch, sym, a, &q, grid, lane_is_tgt, nullptr, st);
    return launch_t<float>(role_a, role_b, stretch, sym, a, &q, grid, lane_is_tgt, nullptr, st);
}

int backward_occupancy(int dtype, bool role_a, bool role_b, bool stretch, bool sym) {
    int occ = 0;
    BwdArgs a{};
    BatchQueue q{};
    hipError_t e = dtype == kDtypeF64 ? launch_t<double>(role_a, role_b, stretch, sym, a, &q, 0, 0, &occ, nullptr)
                                      : launch_t<float>(role_a, role_b, stretch, sym, a, &q, 0, 0, &occ, nullptr);
    return e == hipSuccess ? occ : 0;
}

}  // namespace vpm
