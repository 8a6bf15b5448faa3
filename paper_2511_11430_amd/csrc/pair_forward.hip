// Particle-to-particle velocity and stretching by direct summation (Fu & Laurendeau,
// Sec. II.B, Eqs. 2-5), for one MI355X (gfx950).
//
// Layout and schedule
//  - Each workgroup owns WG*K consecutive targets of one particle set; lane l holds targets
//    l, l+WG, ..., l+(K-1)WG (coalesced loads and stores for every k).
//  - Sources stream through LDS in tiles of WG particles.  Each lane stages one source and
//    precomputes what every pair needs (x, Gamma, -Gamma_z and the far-field cut; 1/sigma in
//    an array of its own that only in-core pairs read), so the inner loop reads a source with
//    two LDS loads that all lanes share (broadcast), and uses it for K register-resident
//    targets.
//  - Sign-folded cross product: a cross-product component is a difference of two products,
//    which as one multiply-add needs a negated operand (the longer three-operand encoding,
//    which issues slower).  The pair holds r' = (r_x, -r_y, r_z), v' = (v_x, -v_y, -v_z) and
//    the staged -Gamma_z instead, with which each component is a multiply and an
//    accumulating multiply-add; the sums then hold some components negated, and the
//    epilogue restores their signs (an exact operation).
//  - A pair takes the point-vortex weights (s^-3, s^-5) unless it lies inside RHO_FAR cores,
//    where the in-core weights replace them (series or erf/exp; core_weights).  The branch is
//    skipped by a whole wavefront when none of its lanes is in a core, which is the common case
//    for spatially ordered wakes.
//  - FP32 (VPM_F32C): each target's 9 partial sums (u, A = sum G Gamma_j, B) are plain FP32
//    within chunks of 256 sources and folded into compensated (hi, lo) pairs after every
//    chunk (Dekker's FastTwoSum, its error carried into the next chunk as in Kahan's
//    summation), so the error does not grow with N.  The per-target epilogue runs in FP64.
//  - FP64 (VPM_F64): the same schedule with K = 1 and plain FP64 sums.
//  - Gradient mode adds the velocity gradient du/dx (nine more FP32 sums per target) for the
//    sub-grid model; the stretching then comes from the same sums.
//  - Stretching is assembled per target from A and B:
//      transposed: dGamma_i/dt = (Gamma_i x A - 3 B)/(4 pi),  B = sum Hn (Gamma_i . (Gamma_j x r)) r
//      classical:  dGamma_i/dt = (-Gamma_i x A - 3 B)/(4 pi), B = sum Hn (r . Gamma_i) (Gamma_j x r)
//    with A = sum G Gamma_j, G = 4 pi g, Hn = -(4 pi/3) h.
//  - The self pair (and a caller-chosen source per target) is skipped by index; only tiles that
//    contain such a source run the checked inner loop.
//  - Many independent sets run in one persistent launch: each workgroup pops (set, target
//    block) items from a queue ordered by decreasing cost (longest-processing-time first).
#include <hip/hip_runtime.h>

#include "device_math.h"
#include "vpm_internal.h"

// The FP64 kernels call their in-core weights (a convergent call), and clang then reports the
// unroll request of their source loop, which is 1, as not honoured.
#pragma clang diagnostic ignored "-Wpass-failed"

namespace vpm {

template <typename T>
struct SrcTile {
    // p = (x, y, z, -Gamma_z), q = (Gamma_x, Gamma_y, Gamma_z, cut) with cut = RHO_FAR^2
    // sigma^2 for the source rule and RHO_FAR^2 sigma^2 / 2 for the symmetric rule; 1/sigma
    // is staged apart.
    using V4 = typename std::conditional<std::is_same<T, float>::value, float4, double4>::type;
};

// Signs that the held partial sums carry relative to the sums they stand for (the
// sign-folded cross product): u' = (u_x, -u_y, -u_z); transposed B' = (B_x, -B_y, B_z)
// (B = sum w r); classical B' = (B_x, -B_y, -B_z) (B = sum w v); gradient H'_ab = s_a t_b H_ab
// with s = (+, -, -) from v and t = (+, -, +) from r.
__host__ __device__ constexpr double held_sign(int mode, int c) {
    return c == 1 || c == 2 ? -1.0
         : c < 6 ? 1.0
         : mode == kModeTransposed ? (c == 7 ? -1.0 : 1.0)
         : mode == kModeClassical ? (c == 7 || c == 8 ? -1.0 : 1.0)
         : mode == kModeGradient && c < 15
             ? ((c - 6) / 3 == 0 ? 1.0 : -1.0) * ((c - 6) % 3 == 1 ? -1.0 : 1.0)
             : 1.0;
}

// One pair: accumulate into the tile partials of one target.
// Keeps a value opaque to the optimiser so that what is computed from it inside a rarely
// taken branch is not hoisted to the hot path (emits no instruction).
__device__ __forceinline__ float opaque(float v) {
    asm volatile("" : "+v"(v));
    return v;
}
__device__ __forceinline__ double opaque(double v) {
    asm volatile("" : "+v"(v));
    return v;
}

// One pair: accumulate into the partial sums p[] of one target.  Layout of p (held signs as
// held_sign gives them):
//   velocity:               u' = p[0..2]
//   transposed / classical: u' = p[0..2], A = p[3..5], B' = p[6..8]
//   gradient:               u' = p[0..2], A = p[3..5] (pairs outside the cores),
//                           H' = p[6..14] = sum Hn v' r'^T (row-major, v = Gamma_j x r),
//                           A_core = p[15..17], C = p[18..20] = sum over in-core pairs of G Gamma_i x Gamma_j
// (px, py, pz, nqz) = (x_j, -Gamma_j,z), (qx, qy, qz, qw) = (Gamma_j, cut_j); ngi1 = -Gamma_i,y,
// ngi2 = -Gamma_i,z; isig_j = 1/sigma_j, read only for in-core pairs under the source rule.
// The point-vortex parts of A and B (transposed and classical) go to pab[3..8], which is p or
// a second set of sums (the odd sources of tiles near the targets).
template <typename T, int MODE, bool SYM, bool CHECK, bool NEAR>
__device__ __forceinline__ void pair_fwd(const T px, const T py, const T pz, const T nqz, const T qx,
                                         const T qy, const T qz, const T qw, const T* isig_j,
                                         const T xi0, const T xi1, const T xi2, const T gi0,
                                         const T gi1, const T gi2, const T ngi1, const T ngi2,
                                         const T cut_i, const int64_t jglob, const int64_t ex, T* p,
                                         T* pab) {
    const T rx = xi0 - px;
    const T ryn = py - xi1;  // -r_y
    const T rz = xi2 - pz;
    const T s2 = rx * rx + ryn * ryn + rz * rz;
    const T rinv = rsqrt_fast(s2);
    const T rinv2 = rinv * rinv;
    T G = rinv2 * rinv;
    T Hn = G * rinv2;
    T Ga = G;  // weight of Gamma_j in A
    const T cut = SYM ? (qw + cut_i) : qw;
    // NEAR is false for source tiles that lie entirely outside every core of this block.
    if (NEAR && s2 < cut) {
        // source rule: 1/sigma_j; symmetric rule: 1/sigma_ij^2 = RHO_FAR^2 / cut
        T isig, isig2;
        if (SYM) {
            isig2 = T(Prec<T>::kFarRho2) * rcp_fast(opaque(cut));
            isig = sqrt_fast(isig2);
        } else {
            isig = *isig_j;
            isig2 = isig * isig;
        }
        core_weights_call(s2, isig, isig2, G, Hn);
        if (CHECK && jglob == ex) {  // the self pair: r = 0, always in the core
            G = T(0);
            Hn = T(0);
        }
        if (MODE != kModeVelocity) {
            // In-core pairs dominate A and along a filament their strengths are nearly
            // parallel to Gamma_i, where Gamma_i x (sum) would cancel in FP32.  Their term
            // G Gamma_i x Gamma_j is formed per pair instead: added to the stretching sum
            // through B (dGamma = (Gamma_i x A - 3B)/4pi; classical: -Gamma_i x A - 3B), or
            // kept in C (gradient mode, which also needs their A for the gradient).
            const T cx = gi1 * qz - gi2 * qy;
            const T cy = gi2 * qx - gi0 * qz;
            const T cz = gi0 * qy - gi1 * qx;
            if (MODE == kModeGradient) {
                p[15] += G * qx;
                p[16] += G * qy;
                p[17] += G * qz;
                p[18] += G * cx;
                p[19] += G * cy;
                p[20] += G * cz;
            } else {
                const T f = (MODE == kModeTransposed ? T(-1.0 / 3.0) : T(1.0 / 3.0)) * G;
                p[6] += f * cx;
                p[7] -= f * cy;
                if (MODE == kModeTransposed) p[8] += f * cz;
                else p[8] -= f * cz;
            }
            Ga = T(0);
        } else {
            Ga = G;
        }
    } else if (CHECK) {
        if (jglob == ex) {
            G = T(0);
            Hn = T(0);
            Ga = T(0);
        }
    }
    // v' = (v_x, -v_y, -v_z), each a multiply and an accumulating multiply-add
    const T vx = qy * rz + qz * ryn;
    const T vyn = nqz * rx + qx * rz;
    const T vzn = qx * ryn + qy * rx;
    p[0] += G * vx;
    p[1] += G * vyn;
    p[2] += G * vzn;
    if (MODE != kModeVelocity) {
        if (MODE == kModeGradient) pab = p;
        pab[3] += Ga * qx;
        pab[4] += Ga * qy;
        pab[5] += Ga * qz;
        if (MODE == kModeTransposed) {
            const T tau = gi0 * vx + ngi1 * vyn + ngi2 * vzn;
            const T w = Hn * tau;
            pab[6] += w * rx;
            pab[7] += w * ryn;
            pab[8] += w * rz;
        } else if (MODE == kModeClassical) {
            const T rg = rx * gi0 + ryn * ngi1 + rz * gi2;
            const T w = Hn * rg;
            pab[6] += w * vx;
            pab[7] += w * vyn;
            pab[8] += w * vzn;
        } else {
            const T hx = Hn * vx, hy = Hn * vyn, hz = Hn * vzn;
            p[6] += hx * rx;
            p[7] += hx * ryn;
            p[8] += hx * rz;
            p[9] += hy * rx;
            p[10] += hy * ryn;
            p[11] += hy * rz;
            p[12] += hz * rx;
            p[13] += hz * ryn;
            p[14] += hz * rz;
        }
    }
}

// Per-target epilogue in FP64: u = U/(4 pi) and the stretching from A and B (tot holds U, A, B).
// Gradient mode (tot holds U, A, H, A_core, C):
//   J = du/dx = ([A + A_core]_x - 3 H) / (4 pi)          ([w]_x y = w x y)
//   transposed stretching J^T Gamma_i = (Gamma_i x A + C - 3 H^T Gamma_i) / (4 pi)
//   classical stretching  J Gamma_i   = (A x Gamma_i - C - 3 H Gamma_i) / (4 pi)
template <typename T, int MODE>
__device__ __forceinline__ void store_target(const FwdArgs& a, int64_t t, double g0, double g1, double g2,
                                             const double* tot) {
    // No contraction here, so every kernel that ends in this epilogue rounds the same way.
#pragma clang fp contract(off)
    double res[6];
#pragma unroll
    for (int c = 0; c < 3; ++c) res[c] = kInv4PiD * tot[c];
    if (MODE == kModeTransposed || MODE == kModeClassical) {
        const double A0 = tot[3], A1 = tot[4], A2 = tot[5];
        double c0 = g1 * A2 - g2 * A1;
        double c1 = g2 * A0 - g0 * A2;
        double c2 = g0 * A1 - g1 * A0;
        if (MODE == kModeClassical) {
            c0 = -c0;
            c1 = -c1;
            c2 = -c2;
        }
        res[3] = kInv4PiD * (c0 - 3.0 * tot[6]);
        res[4] = kInv4PiD * (c1 - 3.0 * tot[7]);
        res[5] = kInv4PiD * (c2 - 3.0 * tot[8]);
    }
    if (MODE == kModeGradient) {
        const double* H = tot + 6;
        const double gi[3] = {g0, g1, g2};
        const double A0 = tot[3], A1 = tot[4], A2 = tot[5];
        double c0 = g1 * A2 - g2 * A1;  // Gamma_i x A
        double c1 = g2 * A0 - g0 * A2;
        double c2 = g0 * A1 - g1 * A0;
        const double sgn = a.classical ? -1.0 : 1.0;
        double hg[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            hg[r] = a.classical ? H[3 * r] * gi[0] + H[3 * r + 1] * gi[1] + H[3 * r + 2] * gi[2]
                                : H[r] * gi[0] + H[3 + r] * gi[1] + H[6 + r] * gi[2];
        }
        res[3] = kInv4PiD * (sgn * (c0 + tot[18]) - 3.0 * hg[0]);
        res[4] = kInv4PiD * (sgn * (c1 + tot[19]) - 3.0 * hg[1]);
        res[5] = kInv4PiD * (sgn * (c2 + tot[20]) - 3.0 * hg[2]);
        const double At0 = tot[3] + tot[15], At1 = tot[4] + tot[16], At2 = tot[5] + tot[17];
        const double X[9] = {0.0, -At2, At1, At2, 0.0, -At0, -At1, At0, 0.0};
        T* __restrict__ jo = static_cast<T*>(a.grad);
#pragma unroll
        for (int c = 0; c < 9; ++c) {
            const double v = kInv4PiD * (X[c] - 3.0 * H[c]);
            T* dst = jo + c * a.ldo + t;
            *dst = a.accumulate ? T(double(*dst) + v) : T(v);
        }
    }
    // (the library's own stretching-only use passes no velocity output)
    T* __restrict__ uo = static_cast<T*>(a.u);
    if (uo) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            T* dst = uo + c * a.ldo + t;
            *dst = a.accumulate ? T(double(*dst) + res[c]) : T(res[c]);
        }
    }
    if (MODE != kModeVelocity) {
        T* __restrict__ dgo = static_cast<T*>(a.dg);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            T* dst = dgo + c * a.ldo + t;
            *dst = a.accumulate ? T(double(*dst) + res[3 + c]) : T(res[3 + c]);
        }
    }
}

template <typename T, int K, int WG, int MODE, bool SYM, int U>
struct FwdBlock {
    static constexpr bool kComp = std::is_same<T, float>::value;
    static constexpr int kNacc = nacc_of(MODE);
    using V4 = typename SrcTile<T>::V4;

    // Process targets [t0, t1) (at most WG*K of them) against sources [s0, s1) of one set.
    // self_shift: with self evaluation, target t is source t + self_shift (else ignored).
    static __device__ void run(const FwdArgs& a, int64_t s0, int64_t s1, int64_t t0, int64_t t1,
                               int64_t self_shift, V4* lp, V4* lq, T* ls, T* box_scratch, int chunk_id) {
        const T* __restrict__ xs = static_cast<const T*>(a.xs);
        const T* __restrict__ gs = static_cast<const T*>(a.gs);
        const T* __restrict__ ss = static_cast<const T*>(a.ss);
        const T* __restrict__ xt = static_cast<const T*>(a.xt);
        const T* __restrict__ gt = static_cast<const T*>(a.gt);
        const T* __restrict__ st = static_cast<const T*>(a.st);
        const int tid = threadIdx.x;
        const T far2 = T(Prec<T>::kFarRho2);

        T xi[K][3], gi[K][3], ngi[K][2], cut_i[K];
        int64_t ex[K];
        bool valid[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int64_t t = t0 + tid + int64_t(k) * WG;
            valid[k] = t < t1;
            const int64_t tt = valid[k] ? t : t0;
            xi[k][0] = xt[tt];
            xi[k][1] = xt[a.ldt + tt];
            xi[k][2] = xt[2 * a.ldt + tt];
            if (MODE != kModeVelocity) {
                gi[k][0] = gt[tt];
                gi[k][1] = gt[a.ldt + tt];
                gi[k][2] = gt[2 * a.ldt + tt];
            } else {
                gi[k][0] = gi[k][1] = gi[k][2] = T(0);
            }
            // (kept opaque so that the products stay plain multiplies by a register)
            ngi[k][0] = opaque(-gi[k][1]);
            ngi[k][1] = opaque(-gi[k][2]);
            if (SYM) {
                const T sg = st[tt];
                cut_i[k] = T(0.5) * far2 * sg * sg;
            } else {
                cut_i[k] = T(0);
            }
            if (a.self) ex[k] = valid[k] ? t + self_shift : -2;
            else if (a.excl) ex[k] = valid[k] ? int64_t(a.excl[tt]) : -2;
            else ex[k] = -2;
        }

        // Bounding box of this workgroup's targets and their largest core cut (symmetric rule).
        T blo[3], bhi[3], bcut;
        {
            T lo3[3], hi3[3], mc = T(0);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                lo3[c] = xi[0][c];
                hi3[c] = xi[0][c];
            }
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (!valid[k]) continue;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    lo3[c] = fmin(lo3[c], xi[k][c]);
                    hi3[c] = fmax(hi3[c], xi[k][c]);
                }
                mc = fmax(mc, cut_i[k]);
            }
            block_box(lo3, hi3, mc, blo, bhi, bcut, box_scratch);
        }

        T acc[K][kNacc];   // tile partials
        T acc2[K][kNacc];  // A and B of the odd sources of near tiles (kDual)
        T hi[K][kNacc];    // compensated totals (FP32 path)
        T lo[K][kNacc];
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int c = 0; c < kNacc; ++c) {
                acc[k][c] = T(0);
                acc2[k][c] = T(0);
                hi[k][c] = T(0);
                lo[k][c] = T(0);
            }

        for (int64_t j0 = s0; j0 < s1; j0 += WG) {
            const int cnt = int((s1 - j0) < WG ? (s1 - j0) : WG);
            __syncthreads();
            T slo[3], shi[3], scut = T(0);
            if (tid < cnt) {
                const int64_t j = j0 + tid;
                const T sg = ss[j];
                V4 p, q;
                p.x = xs[j];
                p.y = xs[a.lds + j];
                p.z = xs[2 * a.lds + j];
                q.x = gs[j];
                q.y = gs[a.lds + j];
                q.z = gs[2 * a.lds + j];
                q.w = SYM ? T(0.5) * far2 * sg * sg : far2 * sg * sg;
                p.w = -q.z;
                lp[tid] = p;
                lq[tid] = q;
                ls[tid] = T(1) / sg;
                slo[0] = shi[0] = p.x;
                slo[1] = shi[1] = p.y;
                slo[2] = shi[2] = p.z;
                scut = q.w;
            } else {
                // an empty slot: take the first source's position, which is already in the box
                const T p0 = xs[j0], p1 = xs[a.lds + j0], p2 = xs[2 * a.lds + j0];
                slo[0] = shi[0] = p0;
                slo[1] = shi[1] = p1;
                slo[2] = shi[2] = p2;
            }
            T tlo[3], thi[3], tcut;
            block_box(slo, shi, scut, tlo, thi, tcut, box_scratch);
            // Does any of this workgroup's targets skip a source in this tile?
            bool mine = false;
#pragma unroll
            for (int k = 0; k < K; ++k) mine |= (ex[k] >= j0 && ex[k] < j0 + cnt);
            const bool check = __syncthreads_or(mine);
            // Is some pair of this block and tile inside a core?  Box-to-box distance vs the
            // largest cut.
            T d2 = T(0);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const T gap = fmax(fmax(tlo[c] - bhi[c], blo[c] - thi[c]), T(0));
                d2 += gap * gap;
            }
            const bool near = d2 < (SYM ? tcut + bcut : tcut);
            if (check) {
                if (near) tile<true, true>(lp, lq, ls, cnt, j0, xi, gi, ngi, cut_i, ex, acc, acc2, hi, lo);
                else tile<true, false>(lp, lq, ls, cnt, j0, xi, gi, ngi, cut_i, ex, acc, acc2, hi, lo);
            } else {
                if (near) tile<false, true>(lp, lq, ls, cnt, j0, xi, gi, ngi, cut_i, ex, acc, acc2, hi, lo);
                else tile<false, false>(lp, lq, ls, cnt, j0, xi, gi, ngi, cut_i, ex, acc, acc2, hi, lo);
            }
        }

        // Epilogue in FP64 (or FP64 partials of one source chunk).
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (!valid[k]) continue;
            const int64_t t = t0 + tid + int64_t(k) * WG;
            double tot[kNacc];
#pragma unroll
            for (int c = 0; c < kNacc; ++c)
                tot[c] = held_sign(MODE, c) * (kComp ? double(hi[k][c]) + double(lo[k][c]) : double(acc[k][c]));
            if (chunk_id >= 0) {
#pragma unroll
                for (int c = 0; c < kNacc; ++c) a.part[(int64_t(chunk_id) * kNacc + c) * a.tgt_end + t] = tot[c];
            } else {
                store_target<T, MODE>(a, t, gi[k][0], gi[k][1], gi[k][2], tot);
            }
        }
    }

    // FP32 partials are folded into the (hi, lo) pairs every kFold sources: the in-chunk FP32
    // sum error grows with the chunk length and is amplified in Gamma_i x A when neighbouring
    // strengths are nearly parallel (vortex filaments).  A chunk of 256 is one whole tile of
    // the 256-lane shapes, whose pair loop then needs no chunk loop around it (91 instead of
    // 109 VGPRs, five wavefronts per SIMD instead of four).  In tiles near the targets, where
    // the large terms are, the odd sources add their A and B into a second set of sums, so
    // that each FP32 sum there runs over 128 terms (one target per lane, outside the gradient
    // mode: the register budget of the other shapes has no room for it).
    static constexpr int kFold = 256;
    static constexpr bool kDual = kComp && K == 1 && MODE != kModeGradient && MODE != kModeVelocity;

    // One fold: y = acc + lo (the chunk and the error carried from the previous fold); the
    // FastTwoSum of (hi, y) gives hi + y = t + e exactly whenever |hi| >= |y| (and when hi = 0),
    // and e becomes the new lo.  A chunk that outweighs the sum so far loses at most the
    // rounding of that one addition, as a plain FP32 sum would.  Five instructions per sum
    // against eight for the branch-free TwoSum.
    static __device__ __forceinline__ void fold(T (&acc)[K][kNacc], T (&acc2)[K][kNacc], T (&hi)[K][kNacc],
                                                T (&lo)[K][kNacc]) {
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int c = 0; c < kNacc; ++c) {
                const bool two = kDual && c >= 3 && c < 9;
                const T y = (two ? acc[k][c] + acc2[k][c] : acc[k][c]) + lo[k][c];
                const T t = hi[k][c] + y;
                lo[k][c] = y - (t - hi[k][c]);
                hi[k][c] = t;
                acc[k][c] = T(0);
                if (two) acc2[k][c] = T(0);
            }
    }

    template <bool CHECK, bool NEAR>
    static __device__ __forceinline__ void tile(const V4* lp, const V4* lq, const T* ls, int cnt, int64_t j0,
                                                T (&xi)[K][3], T (&gi)[K][3], T (&ngi)[K][2], T (&cut_i)[K],
                                                int64_t (&ex)[K], T (&acc)[K][kNacc], T (&acc2)[K][kNacc],
                                                T (&hi)[K][kNacc], T (&lo)[K][kNacc]) {
        for (int c0 = 0; c0 < cnt; c0 += kFold) {
            const int c1 = (cnt - c0) < kFold ? cnt : c0 + kFold;
            int jj = c0;
            if constexpr (kDual && NEAR) {
                // sources in pairs: the even one into acc, the odd one's A and B into acc2
#pragma unroll U / 2
                for (; jj + 1 < c1; jj += 2) {
                    const V4 p = lp[jj], q = lq[jj];
                    const V4 p2 = lp[jj + 1], q2 = lq[jj + 1];
                    pair_fwd<T, MODE, SYM, CHECK, NEAR>(p.x, p.y, p.z, p.w, q.x, q.y, q.z, q.w, ls + jj,
                                                        xi[0][0], xi[0][1], xi[0][2], gi[0][0], gi[0][1],
                                                        gi[0][2], ngi[0][0], ngi[0][1], cut_i[0], j0 + jj,
                                                        ex[0], &acc[0][0], &acc[0][0]);
                    pair_fwd<T, MODE, SYM, CHECK, NEAR>(p2.x, p2.y, p2.z, p2.w, q2.x, q2.y, q2.z, q2.w,
                                                        ls + jj + 1, xi[0][0], xi[0][1], xi[0][2], gi[0][0],
                                                        gi[0][1], gi[0][2], ngi[0][0], ngi[0][1], cut_i[0],
                                                        j0 + jj + 1, ex[0], &acc[0][0], &acc2[0][0]);
                }
            }
#pragma unroll U
            for (; jj < c1; ++jj) {
                const V4 p = lp[jj];
                const V4 q = lq[jj];
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    pair_fwd<T, MODE, SYM, CHECK, NEAR>(p.x, p.y, p.z, p.w, q.x, q.y, q.z, q.w, ls + jj,
                                                        xi[k][0], xi[k][1], xi[k][2], gi[k][0], gi[k][1],
                                                        gi[k][2], ngi[k][0], ngi[k][1], cut_i[k], j0 + jj,
                                                        ex[k], &acc[k][0], &acc[k][0]);
                }
            }
            if constexpr (kComp) fold(acc, acc2, hi, lo);
        }
    }
};

// One workgroup per target block of a single particle set.
template <typename T, int K, int WG, int MODE, bool SYM, int U>
__global__ __launch_bounds__(WG) void k_pair_fwd(FwdArgs a) {
    using B = FwdBlock<T, K, WG, MODE, SYM, U>;
    __shared__ typename B::V4 lp[WG];
    __shared__ typename B::V4 lq[WG];
    __shared__ T ls[WG];
    __shared__ T box[7 * (WG / 64)];
    const int64_t t0 = a.tgt_begin + int64_t(blockIdx.x) * (WG * K);
    int64_t t1 = t0 + WG * K;
    if (t1 > a.tgt_end) t1 = a.tgt_end;
    int64_t s0 = a.src_begin, s1 = a.src_end;
    int chunk_id = -1;
    if (a.nchunk > 1) {
        chunk_id = int(blockIdx.y);
        s0 = a.src_begin + int64_t(blockIdx.y) * a.chunk;
        s1 = s0 + a.chunk < a.src_end ? s0 + a.chunk : a.src_end;
    }
    B::run(a, s0, s1, t0, t1, a.src_begin - a.tgt_begin, lp, lq, ls, box, chunk_id);
}

// Adds the per-chunk FP64 partials of every target in chunk order and stores the result.
template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_pair_fwd_finish(FwdArgs a) {
    constexpr int kNacc = nacc_of(MODE);
    const int64_t t = a.tgt_begin + int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (t >= a.tgt_end) return;
    double tot[kNacc];
#pragma unroll
    for (int c = 0; c < kNacc; ++c) tot[c] = 0.0;
    for (int ch = 0; ch < a.nchunk; ++ch)
#pragma unroll
        for (int c = 0; c < kNacc; ++c) tot[c] += a.part[(int64_t(ch) * kNacc + c) * a.tgt_end + t];
    double g0 = 0.0, g1 = 0.0, g2 = 0.0;
    if (MODE != kModeVelocity) {
        const T* gt = static_cast<const T*>(a.gt);
        g0 = double(gt[t]);
        g1 = double(gt[a.ldt + t]);
        g2 = double(gt[2 * a.ldt + t]);
    }
    store_target<T, MODE>(a, t, g0, g1, g2, tot);
}

// Persistent workgroups over a queue of (set, target block) items in decreasing cost order.
// Every workgroup leaves the loop once the shared counter passes the item count.
template <typename T, int K, int WG, int MODE, bool SYM, int U>
__global__ __launch_bounds__(WG) void k_pair_fwd_batched(FwdArgs a, BatchQueue bq) {
    using B = FwdBlock<T, K, WG, MODE, SYM, U>;
    __shared__ typename B::V4 lp[WG];
    __shared__ typename B::V4 lq[WG];
    __shared__ T ls[WG];
    __shared__ T box[7 * (WG / 64)];
    __shared__ int item_s;
    for (;;) {
        if (threadIdx.x == 0) item_s = atomicAdd(bq.counter, 1);
        __syncthreads();
        const int item = item_s;
        __syncthreads();
        if (item >= bq.n_items) break;
        const int2 it = bq.items[item];
        const int b = it.x;
        const int64_t s0 = bq.src_off[b], s1 = bq.src_off[b + 1];
        const int64_t tb0 = bq.tgt_off[b], tb1 = bq.tgt_off[b + 1];
        const int64_t t0 = tb0 + int64_t(it.y) * (WG * K);
        int64_t t1 = t0 + WG * K;
        if (t1 > tb1) t1 = tb1;
        B::run(a, s0, s1, t0, t1, s0 - tb0, lp, lq, ls, box, -1);
    }
}

// ------------------------------------------------------------------ host-side launchers
namespace {

template <typename T, int K, int WG, int MODE, bool SYM, int U>
hipError_t launch_one(const FwdArgs& a, const BatchQueue* bq, int grid, hipStream_t st) {
    if (bq) {
        hipLaunchKernelGGL((k_pair_fwd_batched<T, K, WG, MODE, SYM, U>), dim3(grid), dim3(WG), 0, st, a, *bq);
        return hipGetLastError();
    }
    const int ny = a.nchunk > 1 ? a.nchunk : 1;
    hipLaunchKernelGGL((k_pair_fwd<T, K, WG, MODE, SYM, U>), dim3(grid, ny), dim3(WG), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || ny == 1) return e;
    const int64_t nt = a.tgt_end - a.tgt_begin;
    hipLaunchKernelGGL((k_pair_fwd_finish<T, MODE>), dim3(int((nt + 255) / 256)), dim3(256), 0, st, a);
    return hipGetLastError();
}

template <typename T, int K, int WG, int MODE, bool SYM, int U>
int occupancy_one(bool batched) {
    int nb = 0;
    hipError_t e;
    if (batched)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_pair_fwd_batched<T, K, WG, MODE, SYM, U>, WG, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_pair_fwd<T, K, WG, MODE, SYM, U>, WG, 0);
    return e == hipSuccess ? nb : 0;
}

template <typename T, int K, int WG, int U>
hipError_t dispatch_mode(int mode, bool sym, const FwdArgs& a, const BatchQueue* bq, int grid,
                         hipStream_t st) {
    if (mode == kModeTransposed)
        return sym ? launch_one<T, K, WG, kModeTransposed, true, U>(a, bq, grid, st)
                   : launch_one<T, K, WG, kModeTransposed, false, U>(a, bq, grid, st);
    if (mode == kModeClassical)
        return sym ? launch_one<T, K, WG, kModeClassical, true, U>(a, bq, grid, st)
                   : launch_one<T, K, WG, kModeClassical, false, U>(a, bq, grid, st);
    return sym ? launch_one<T, K, WG, kModeVelocity, true, U>(a, bq, grid, st)
               : launch_one<T, K, WG, kModeVelocity, false, U>(a, bq, grid, st);
}

template <typename T, int K, int WG, int U>
int occupancy_mode(int mode, bool sym, bool batched) {
    if (mode == kModeTransposed)
        return sym ? occupancy_one<T, K, WG, kModeTransposed, true, U>(batched)
                   : occupancy_one<T, K, WG, kModeTransposed, false, U>(batched);
    if (mode == kModeClassical)
        return sym ? occupancy_one<T, K, WG, kModeClassical, true, U>(batched)
                   : occupancy_one<T, K, WG, kModeClassical, false, U>(batched);
    return sym ? occupancy_one<T, K, WG, kModeVelocity, true, U>(batched)
               : occupancy_one<T, K, WG, kModeVelocity, false, U>(batched);
}

}  // namespace

// FP32C variants: (targets per lane, workgroup size, source unroll).  Index 0 is variant 1.
const FwdVariant kF32Variants[kNumF32Variants] = {
    {2, 256, 2}, {1, 256, 2}, {1, 256, 4}, {2, 128, 2}, {2, 256, 4}, {1, 128, 2}, {1, 128, 4}, {1, 512, 2},
};

#define VPM_F32_VARIANTS(X) \
    X(0, 2, 256, 2) X(1, 1, 256, 2) X(2, 1, 256, 4) X(3, 2, 128, 2) X(4, 2, 256, 4) X(5, 1, 128, 2) X(6, 1, 128, 4) X(7, 1, 512, 2)

hipError_t launch_pair_fwd(int dtype, int variant, int mode, bool sym, const FwdArgs& a,
                           const BatchQueue* bq, int grid, hipStream_t st) {
    if (mode == kModeGradient) {
        if (dtype == kDtypeF64)
            return sym ? launch_one<double, 1, 256, kModeGradient, true, 1>(a, bq, grid, st)
                       : launch_one<double, 1, 256, kModeGradient, false, 1>(a, bq, grid, st);
        if (variant != kGradientVariant) return hipErrorInvalidValue;
        return sym ? launch_one<float, 1, 256, kModeGradient, true, 2>(a, bq, grid, st)
                   : launch_one<float, 1, 256, kModeGradient, false, 2>(a, bq, grid, st);
    }
    if (dtype == kDtypeF64) return dispatch_mode<double, 1, 256, 1>(mode, sym, a, bq, grid, st);
    switch (variant) {
#define X(i, k, wg, u) case i: return dispatch_mode<float, k, wg, u>(mode, sym, a, bq, grid, st);
        VPM_F32_VARIANTS(X)
#undef X
        default: return hipErrorInvalidValue;
    }
}

int pair_fwd_occupancy(int dtype, int variant, int mode, bool sym, bool batched) {
    if (mode == kModeGradient) {
        if (dtype == kDtypeF64)
            return sym ? occupancy_one<double, 1, 256, kModeGradient, true, 1>(batched)
                       : occupancy_one<double, 1, 256, kModeGradient, false, 1>(batched);
        if (variant != kGradientVariant) return 0;
        return sym ? occupancy_one<float, 1, 256, kModeGradient, true, 2>(batched)
                   : occupancy_one<float, 1, 256, kModeGradient, false, 2>(batched);
    }
    if (dtype == kDtypeF64) return occupancy_mode<double, 1, 256, 1>(mode, sym, batched);
    switch (variant) {
#define X(i, k, wg, u) case i: return occupancy_mode<float, k, wg, u>(mode, sym, batched);
        VPM_F32_VARIANTS(X)
#undef X
        default: return 0;
    }
}

}  // namespace vpm
