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
// per-segment constants (Gamma / (4 pi |r0|^2), r0, |r0|^2, 1/|r0|^2, -r0_y, -r0_z, the
// degeneracy threshold), and FP32 tile partials folded into two-sum pairs (VPM_F32C) or plain
// FP64 sums (VPM_F64).  As in the particle kernel, the cross product is sign-folded: with
// r1' = (r1_x, -r1_y, r1_z) and the staged -r0_y, -r0_z every component of
// c' = (c_x, -c_y, -c_z) and the dot product r0 . r1 are multiplies and accumulating
// multiply-adds, and the sums hold u_y and u_z negated until the epilogue.
#include <hip/hip_runtime.h>

#include "device_math.h"
#include "vpm_internal.h"

namespace vpm {

namespace {

template <typename T>
using V4 = typename std::conditional<std::is_same<T, float>::value, float4, double4>::type;
template <typename T>
using V2 = typename std::conditional<std::is_same<T, float>::value, float2, double2>::type;

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
    __shared__ V4<T> l2[WG];  // (eps^2 for the arms, 1/|r0|^2, -r0y, -r0z)
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
            V4<T> e;
            e.x = eps * eps;
            e.y = T(1) / q.w;
            e.z = -r0y;
            e.w = -r0z;
            l2[tid] = e;
        }
        __syncthreads();
#pragma unroll 2
        for (int jj = 0; jj < cnt; ++jj) {
            const V4<T> p = l0[jj];
            const V4<T> q = l1[jj];
            const V4<T> e = l2[jj];
            const T eps2 = e.x;
            const T inv_l02 = e.y;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                // r1' = (r1_x, -r1_y, r1_z), r2' likewise
                const T r1x = P[k][0] - p.x, r1yn = p.y - P[k][1], r1z = P[k][2] - p.z;
                const T r2x = r1x - q.x, r2yn = r1yn + q.y, r2z = r1z - q.z;
                // r1 x r2 = r0 x r1, held as c' = (c_x, -c_y, -c_z)
                const T cx = q.y * r1z + q.z * r1yn;
                const T cyn = q.x * r1z + e.w * r1x;
                const T czn = q.y * r1x + q.x * r1yn;
                const T c2 = cx * cx + cyn * cyn + czn * czn;
                const T l1s = r1x * r1x + r1yn * r1yn + r1z * r1z;
                const T l2s = r2x * r2x + r2yn * r2yn + r2z * r2z;
                const T d1 = q.x * r1x + e.z * r1yn + q.z * r1z;
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
                acc[k][1] += f * cyn;
                acc[k][2] += f * czn;
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
            // (the sums hold u_y and u_z negated)
            const double v = (c == 0 ? 1.0 : -1.0) * (kComp ? double(hi[k][c]) + double(lo[k][c]) : double(acc[k][c]));
            T* dst = U + c * a.ldo + t;
            *dst = a.accumulate ? T(double(*dst) + v) : T(v);
        }
    }
}

// Few targets (collocation and lattice points): one wavefront per target, its lanes take the
// segments in turn (segment j in lane j mod 64, read straight from memory), each lane sums in
// FP64, and the lanes' sums are added by a fixed butterfly.  The per-pair arithmetic is that of
// k_segments; the segment set-up is repeated per target, which costs nothing at these sizes but
// fills the GPU where k_segments would run a handful of workgroups.
constexpr int64_t kSegSmallTargets = 8192;

template <typename T, int VN>
__global__ __launch_bounds__(256) void k_segments_few(SegArgs a) {
    const T* __restrict__ A = static_cast<const T*>(a.a);
    const T* __restrict__ B = static_cast<const T*>(a.b);
    const T* __restrict__ Gs = static_cast<const T*>(a.gam);
    const T* __restrict__ X = static_cast<const T*>(a.xt);
    const int lane = threadIdx.x & 63;
    const int64_t t = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (t >= a.n_tgt) return;  // whole wavefronts
    const T rc2 = T(a.rc * a.rc);
    const T n_f = T(a.vn);
    const T inv_n = T(1.0 / a.vn);
    T rc2n;
    if constexpr (VN == 0) rc2n = T(0);
    else if constexpr (VN == 1) rc2n = rc2;
    else if constexpr (VN == 2) rc2n = rc2 * rc2;
    else rc2n = T(pow(double(rc2), double(a.vn)));
    const T P0 = X[t], P1 = X[a.ldt + t], P2 = X[2 * a.ldt + t];
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t j = lane; j < a.n_seg; j += 64) {
        const T ax = A[j], ay = A[a.ld_seg + j], az = A[2 * a.ld_seg + j];
        const T r0x = B[j] - ax, r0y = B[a.ld_seg + j] - ay, r0z = B[2 * a.ld_seg + j] - az;
        const T L02 = r0x * r0x + r0y * r0y + r0z * r0z;
        const T L0 = dsqrt(L02);
        const T eps = T(1e-12) * (L0 > T(1) ? L0 : T(1));
        const bool dead = L0 < eps;
        T coef = T(kInv4PiD) * Gs[j];
        if (VN != 0) coef = coef / L02;
        if (dead) coef = T(0);
        const T qw = dead ? T(1) : L02;
        const T eps2 = eps * eps;
        const T inv_l02 = T(1) / qw;
        const T r1x = P0 - ax, r1y = P1 - ay, r1z = P2 - az;
        const T r2x = r1x - r0x, r2y = r1y - r0y, r2z = r1z - r0z;
        const T cx = r0y * r1z - r0z * r1y;
        const T cy = r0z * r1x - r0x * r1z;
        const T cz = r0x * r1y - r0y * r1x;
        const T c2 = cx * cx + cy * cy + cz * cz;
        const T l1s = r1x * r1x + r1y * r1y + r1z * r1z;
        const T l2s = r2x * r2x + r2y * r2y + r2z * r2z;
        const T d1 = r0x * r1x + r0y * r1y + r0z * r1z;
        const T d2 = d1 - qw;
        const T D = d1 * rsqrt_fast(l1s) - d2 * rsqrt_fast(l2s);
        T f;
        if constexpr (VN == 0) {
            f = (c2 > T(0)) ? coef * D / c2 : T(0);
        } else {
            f = coef * D * core_factor<T, VN>(c2 * inv_l02, rc2n, inv_n, n_f);
        }
        f = (l1s < eps2 || l2s < eps2) ? T(0) : f;
        acc[0] += double(f * cx);
        acc[1] += double(f * cy);
        acc[2] += double(f * cz);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
        for (int off = 32; off > 0; off >>= 1) acc[c] += __shfl_xor(acc[c], off, 64);
    if (lane == 0) {
        T* __restrict__ U = static_cast<T*>(a.u);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            T* dst = U + c * a.ldo + t;
            *dst = a.accumulate ? T(double(*dst) + acc[c]) : T(acc[c]);
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
//
// The same arithmetic runs on plain numbers (gradient kernel) and on dual numbers (value,
// derivative along one direction) for the vector-Jacobian product, which needs the
// derivative of J along a seed direction.

template <typename T>
struct Dl {
    T v, d;
    __device__ Dl() : v(T(0)), d(T(0)) {}
    __device__ Dl(T x) : v(x), d(T(0)) {}
    __device__ Dl(T x, T dx) : v(x), d(dx) {}
};
template <typename T> __device__ __forceinline__ Dl<T> operator+(Dl<T> a, Dl<T> b) { return {a.v + b.v, a.d + b.d}; }
template <typename T> __device__ __forceinline__ Dl<T> operator-(Dl<T> a, Dl<T> b) { return {a.v - b.v, a.d - b.d}; }
template <typename T> __device__ __forceinline__ Dl<T> operator-(Dl<T> a) { return {-a.v, -a.d}; }
template <typename T> __device__ __forceinline__ Dl<T> operator*(Dl<T> a, Dl<T> b) {
    return {a.v * b.v, a.d * b.v + a.v * b.d};
}
template <typename T> __device__ __forceinline__ Dl<T> operator-(Dl<T> a, T b) { return {a.v - b, a.d}; }
template <typename T> __device__ __forceinline__ Dl<T> operator+(Dl<T> a, T b) { return {a.v + b, a.d}; }
template <typename T> __device__ __forceinline__ Dl<T> operator*(Dl<T> a, T b) { return {a.v * b, a.d * b}; }
template <typename T> __device__ __forceinline__ Dl<T> operator*(T a, Dl<T> b) { return {a * b.v, a * b.d}; }

__device__ __forceinline__ float val(float x) { return x; }
__device__ __forceinline__ double val(double x) { return x; }
template <typename T> __device__ __forceinline__ T val(Dl<T> x) { return x.v; }
__device__ __forceinline__ float recip(float x) { return 1.0f / x; }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }
template <typename T> __device__ __forceinline__ Dl<T> recip(Dl<T> x) {
    const T r = T(1) / x.v;
    return {r, -r * r * x.d};
}
using vpm::rsqrt_fast;
template <typename T> __device__ __forceinline__ Dl<T> rsqrt_fast(Dl<T> x) {
    const T y = rsqrt_fast(x.v);
    return {y, T(-0.5) * y * y * y * x.d};
}
__device__ __forceinline__ float powr(float x, float p) { return pow(x, p); }
__device__ __forceinline__ double powr(double x, double p) { return pow(x, p); }
template <typename T> __device__ __forceinline__ Dl<T> powr(Dl<T> x, T p) {  // x > 0, or p >= 1
    const T r = pow(x.v, p);
    return {r, p * pow(x.v, p - T(1)) * x.d};
}

// One segment (tile constants p = (a, coef), q = (r0, |r0|^2 or 1 when dead), eps2) at
// point P: f, c = r0 x r1 (u = f c) and g = grad f.
template <typename S, typename T, int VN>
__device__ __forceinline__ void seg_pair(const S (&P)[3], const V4<T>& p, const V4<T>& q, T eps2, T inv_l02,
                                         T rc2n, T inv_n, T n_f, S& f, S (&c)[3], S (&g)[3]) {
    const S r1x = P[0] - p.x, r1y = P[1] - p.y, r1z = P[2] - p.z;
    const S r2x = r1x - q.x, r2y = r1y - q.y, r2z = r1z - q.z;
    c[0] = q.y * r1z - q.z * r1y;
    c[1] = q.z * r1x - q.x * r1z;
    c[2] = q.x * r1y - q.y * r1x;
    const S c2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
    const S l1s = r1x * r1x + r1y * r1y + r1z * r1z;
    const S l2s = r2x * r2x + r2y * r2y + r2z * r2z;
    const S d1 = q.x * r1x + q.y * r1y + q.z * r1z;
    const S d2 = d1 - q.w;
    const S i1 = rsqrt_fast(l1s), i2 = rsqrt_fast(l2s);
    const S D = d1 * i1 - d2 * i2;
    const S e1 = d1 * i1 * i1 * i1, e2 = d2 * i2 * i2 * i2;
    const S di = i1 - i2;
    const S gDx = q.x * di - r1x * e1 + r2x * e2;
    const S gDy = q.y * di - r1y * e1 + r2y * e2;
    const S gDz = q.z * di - r1z * e1 + r2z * e2;
    // c x r0
    const S wx = c[1] * q.z - c[2] * q.y;
    const S wy = c[2] * q.x - c[0] * q.z;
    const S wz = c[0] * q.y - c[1] * q.x;
    S ga, gb;  // grad f = ga grad D + gb (c x r0)
    if constexpr (VN == 0) {
        const S ic2 = val(c2) > T(0) ? recip(c2) : S(T(0));
        f = p.w * D * ic2;
        ga = p.w * ic2;
        gb = T(-2) * f * ic2;
    } else {
        const S d2l = c2 * inv_l02;
        S Kc, Kp;
        if constexpr (VN == 1) {
            Kc = recip(d2l + rc2n);
            Kp = -(Kc * Kc);
        } else if constexpr (VN == 2) {
            Kc = rsqrt_fast(d2l * d2l + rc2n);
            Kp = -(d2l * Kc * Kc * Kc);
        } else {
            const S sden = powr(d2l, n_f) + rc2n;
            Kc = powr(sden, -inv_n);
            Kp = -(powr(d2l, n_f - T(1)) * Kc * recip(sden));
        }
        f = p.w * D * Kc;
        ga = p.w * Kc;
        gb = (T(2) * p.w) * D * Kp * inv_l02;
    }
    // selected after the products: an arm of zero length makes grad D non-finite
    const bool off = val(l1s) < eps2 || val(l2s) < eps2;
    const S zero(T(0));
    f = off ? zero : f;
    g[0] = off ? zero : ga * gDx + gb * wx;
    g[1] = off ? zero : ga * gDy + gb * wy;
    g[2] = off ? zero : ga * gDz + gb * wz;
}

// Stages one tile of segments in LDS (shared by the gradient and adjoint kernels).
template <typename T, int WG, int VN>
__device__ __forceinline__ void stage_segments(const SegArgs& a, int64_t j0, int cnt, V4<T>* l0, V4<T>* l1,
                                               V2<T>* l2) {
    const int tid = threadIdx.x;
    if (tid < cnt) {
        const T* __restrict__ A = static_cast<const T*>(a.a);
        const T* __restrict__ B = static_cast<const T*>(a.b);
        const T* __restrict__ Gs = static_cast<const T*>(a.gam);
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
        V2<T> e;
        e.x = eps * eps;
        e.y = T(1) / q.w;
        l2[tid] = e;
    }
}

template <typename T>
__device__ __forceinline__ T core_power(const SegArgs& a, int vn_kind) {
    const T rc2 = T(a.rc * a.rc);
    if (vn_kind == 0) return T(0);
    if (vn_kind == 1) return rc2;
    if (vn_kind == 2) return rc2 * rc2;
    return T(pow(double(rc2), double(a.vn)));
}

template <typename T, int NA>
__device__ __forceinline__ void fold_tile(T (&acc)[NA], T (&hi)[NA], T (&lo)[NA]) {
#pragma unroll
    for (int c = 0; c < NA; ++c) {
        T s, e;
        two_sum(hi[c], acc[c], s, e);
        hi[c] = s;
        lo[c] += e;
        acc[c] = T(0);
    }
}

// LPT lanes per target (neighbouring lanes of one wavefront) split each staged tile of segments
// between them, lane q taking the segments q, q + LPT, ...; their sums are added in FP64 by a
// butterfly before the write, so a launch with few targets still has several wavefronts per SIMD.
template <typename T, int K, int WG, int VN, int LPT>
__global__ __launch_bounds__(WG) void k_segments_grad(SegArgs a) {
    static_assert(LPT == 1 || K == 1, "lanes per target only with one target per lane group");
    static_assert((LPT & (LPT - 1)) == 0 && LPT <= 64, "a power of two within a wavefront");
    constexpr bool kComp = std::is_same<T, float>::value;
    constexpr int NA = 12;  // u (3), J row-major (9)
    constexpr int kSlots = WG / LPT;  // targets per workgroup and K
    __shared__ V4<T> l0[WG];
    __shared__ V4<T> l1[WG];
    __shared__ V2<T> l2[WG];  // (eps^2 for the arms, 1/|r0|^2)
    const T* __restrict__ X = static_cast<const T*>(a.xt);
    const int tid = threadIdx.x / LPT, q = threadIdx.x % LPT;
    const int64_t t0 = int64_t(blockIdx.x) * (kSlots * K);
    const T n_f = T(a.vn);
    const T inv_n = T(1.0 / a.vn);
    const T rc2n = core_power<T>(a, VN);

    T P[K][3];
    bool valid[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t t = t0 + tid + int64_t(k) * kSlots;
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
        stage_segments<T, WG, VN>(a, j0, cnt, l0, l1, l2);
        __syncthreads();
        for (int jj = q; jj < cnt; jj += LPT) {
            const V4<T> p = l0[jj];
            const V4<T> q = l1[jj];
            const T eps2 = l2[jj].x;
            const T inv_l02 = l2[jj].y;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                T f, c[3], g[3];
                seg_pair<T, T, VN>(P[k], p, q, eps2, inv_l02, rc2n, inv_n, n_f, f, c, g);
                T* ac = acc[k];
                ac[0] += f * c[0];
                ac[1] += f * c[1];
                ac[2] += f * c[2];
                // f [r0]x + c g^T
                ac[3] += c[0] * g[0];
                ac[4] += c[0] * g[1] - f * q.z;
                ac[5] += c[0] * g[2] + f * q.y;
                ac[6] += c[1] * g[0] + f * q.z;
                ac[7] += c[1] * g[1];
                ac[8] += c[1] * g[2] - f * q.x;
                ac[9] += c[2] * g[0] - f * q.y;
                ac[10] += c[2] * g[1] + f * q.x;
                ac[11] += c[2] * g[2];
            }
        }
        if constexpr (kComp) {
#pragma unroll
            for (int k = 0; k < K; ++k) fold_tile<T, NA>(acc[k], hi[k], lo[k]);
        }
    }
    T* __restrict__ U = static_cast<T*>(a.u);
    T* __restrict__ Jo = static_cast<T*>(a.grad);
    T* __restrict__ Do = static_cast<T*>(a.dg);
    const T* __restrict__ Gt = static_cast<const T*>(a.gt);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double v[NA];
#pragma unroll
        for (int c = 0; c < NA; ++c) v[c] = kComp ? double(hi[k][c]) + double(lo[k][c]) : double(acc[k][c]);
        if constexpr (LPT > 1) {  // every lane takes part; each ends with the same sums
#pragma unroll
            for (int m = 1; m < LPT; m <<= 1)
#pragma unroll
                for (int c = 0; c < NA; ++c) v[c] += __shfl_xor(v[c], m, 64);
        }
        if (!valid[k] || q != 0) continue;
        const int64_t t = t0 + tid + int64_t(k) * kSlots;
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

// Vector-Jacobian product at the targets: with seeds ubar, dbar and the stretching
// s = J^T G (transposed) or J G (classical),
//   xbar += J^T ubar + d/dx [w2 . (J w1)] ,   (w1, w2) = (dbar, G) transposed, (G, dbar) classical,
//   Gbar += J dbar (transposed) or J^T dbar (classical).
// The second term is the derivative of J along w1 contracted with w2: the pair arithmetic
// runs on dual numbers with the point's tangent w1, so the tangent of J_ab is
// d/dw1 J_ab and term_b = sum_a w2_a (d/dw1 J)_ab = f' (w2 x r0)_b + (w2 . c') g_b +
// (w2 . c) g'_b (primes: tangents), with J = f [r0]x + c g^T.
template <typename T, int WG, int VN>
__global__ __launch_bounds__(WG) void k_segments_vjp(SegArgs a) {
    constexpr bool kComp = std::is_same<T, float>::value;
    constexpr int NA = 12;  // J row-major (9), term (3)
    using S = Dl<T>;
    __shared__ V4<T> l0[WG];
    __shared__ V4<T> l1[WG];
    __shared__ V2<T> l2[WG];  // (eps^2 for the arms, 1/|r0|^2)
    const T* __restrict__ X = static_cast<const T*>(a.xt);
    const T* __restrict__ Gt = static_cast<const T*>(a.gt);
    const T* __restrict__ Ub = static_cast<const T*>(a.ub);
    const T* __restrict__ Db = static_cast<const T*>(a.db);
    const int tid = threadIdx.x;
    const int64_t t = int64_t(blockIdx.x) * WG + tid;
    const bool valid = t < a.n_tgt;
    const int64_t tt = valid ? t : 0;
    const T n_f = T(a.vn);
    const T inv_n = T(1.0 / a.vn);
    const T rc2n = core_power<T>(a, VN);

    T gam[3] = {T(0), T(0), T(0)}, db[3] = {T(0), T(0), T(0)};
    if (Db) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            gam[c] = Gt[c * a.ldt + tt];
            db[c] = Db[c * a.ldb + tt];
        }
    }
    const T* w1 = a.classical ? gam : db;
    const T* w2 = a.classical ? db : gam;
    S P[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) P[c] = S(X[c * a.ldt + tt], w1[c]);
    T acc[NA], hi[NA], lo[NA];
#pragma unroll
    for (int c = 0; c < NA; ++c) acc[c] = hi[c] = lo[c] = T(0);

    for (int64_t j0 = 0; j0 < a.n_seg; j0 += WG) {
        const int cnt = int((a.n_seg - j0) < WG ? (a.n_seg - j0) : WG);
        __syncthreads();
        stage_segments<T, WG, VN>(a, j0, cnt, l0, l1, l2);
        __syncthreads();
        for (int jj = 0; jj < cnt; ++jj) {
            const V4<T> p = l0[jj];
            const V4<T> q = l1[jj];
            const T eps2 = l2[jj].x;
            const T inv_l02 = l2[jj].y;
            S f, c[3], g[3];
            seg_pair<S, T, VN>(P, p, q, eps2, inv_l02, rc2n, inv_n, n_f, f, c, g);
            acc[0] += c[0].v * g[0].v;
            acc[1] += c[0].v * g[1].v - f.v * q.z;
            acc[2] += c[0].v * g[2].v + f.v * q.y;
            acc[3] += c[1].v * g[0].v + f.v * q.z;
            acc[4] += c[1].v * g[1].v;
            acc[5] += c[1].v * g[2].v - f.v * q.x;
            acc[6] += c[2].v * g[0].v - f.v * q.y;
            acc[7] += c[2].v * g[1].v + f.v * q.x;
            acc[8] += c[2].v * g[2].v;
            const T wc = w2[0] * c[0].v + w2[1] * c[1].v + w2[2] * c[2].v;
            const T wcd = w2[0] * c[0].d + w2[1] * c[1].d + w2[2] * c[2].d;
            // w2 x r0
            const T xr0 = w2[1] * q.z - w2[2] * q.y;
            const T xr1 = w2[2] * q.x - w2[0] * q.z;
            const T xr2 = w2[0] * q.y - w2[1] * q.x;
            acc[9] += f.d * xr0 + wcd * g[0].v + wc * g[0].d;
            acc[10] += f.d * xr1 + wcd * g[1].v + wc * g[1].d;
            acc[11] += f.d * xr2 + wcd * g[2].v + wc * g[2].d;
        }
        if constexpr (kComp) fold_tile<T, NA>(acc, hi, lo);
    }
    if (!valid) return;
    double v[NA];
#pragma unroll
    for (int c = 0; c < NA; ++c) v[c] = kComp ? double(hi[c]) + double(lo[c]) : double(acc[c]);
    T* __restrict__ Xb = static_cast<T*>(a.xb);
    T* __restrict__ Gb = static_cast<T*>(a.gb);
    double ub[3] = {0.0, 0.0, 0.0};
    if (Ub) {
#pragma unroll
        for (int c = 0; c < 3; ++c) ub[c] = double(Ub[c * a.ldb + t]);
    }
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        double s = v[9 + b];
#pragma unroll
        for (int aa = 0; aa < 3; ++aa) s += v[3 * aa + b] * ub[aa];
        T* dst = Xb + b * a.ldo + t;
        *dst = T(double(*dst) + s);
    }
    if (Db) {
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            // transposed: sum_c J[b][c] dbar_c; classical: sum_c J[c][b] dbar_c
            double s = 0.0;
#pragma unroll
            for (int c = 0; c < 3; ++c) s += (a.classical ? v[3 * c + b] : v[3 * b + c]) * double(db[c]);
            T* dst = Gb + b * a.ldo + t;
            *dst = T(double(*dst) + s);
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

template <typename T, int K, int WG, int LPT>
hipError_t launch_grad_t(const SegArgs& a, hipStream_t st) {
    const int64_t per = int64_t(WG / LPT) * K;
    const int grid = int((a.n_tgt + per - 1) / per);
    if (a.rc == 0.0)
        hipLaunchKernelGGL((k_segments_grad<T, K, WG, 0, LPT>), dim3(grid), dim3(WG), 0, st, a);
    else if (a.vn == 1)
        hipLaunchKernelGGL((k_segments_grad<T, K, WG, 1, LPT>), dim3(grid), dim3(WG), 0, st, a);
    else if (a.vn == 2)
        hipLaunchKernelGGL((k_segments_grad<T, K, WG, 2, LPT>), dim3(grid), dim3(WG), 0, st, a);
    else
        hipLaunchKernelGGL((k_segments_grad<T, K, WG, 3, LPT>), dim3(grid), dim3(WG), 0, st, a);
    return hipGetLastError();
}

// Lanes per target for the gradient kernel: one above kSegGradSplit1 targets (four or more
// wavefronts per SIMD on 256 compute units), four above kSegGradSplit4, sixteen below.
constexpr int64_t kSegGradSplit1 = 196608;
constexpr int64_t kSegGradSplit4 = 16384;

template <typename T>
hipError_t launch_grad_split(const SegArgs& a, hipStream_t st) {
    if (a.n_tgt > kSegGradSplit1) return launch_grad_t<T, 1, 256, 1>(a, st);
    if (a.n_tgt > kSegGradSplit4) return launch_grad_t<T, 1, 256, 4>(a, st);
    return launch_grad_t<T, 1, 256, 16>(a, st);
}

template <typename T, int WG>
hipError_t launch_vjp_t(const SegArgs& a, hipStream_t st) {
    const int grid = int((a.n_tgt + WG - 1) / WG);
    if (a.rc == 0.0)
        hipLaunchKernelGGL((k_segments_vjp<T, WG, 0>), dim3(grid), dim3(WG), 0, st, a);
    else if (a.vn == 1)
        hipLaunchKernelGGL((k_segments_vjp<T, WG, 1>), dim3(grid), dim3(WG), 0, st, a);
    else if (a.vn == 2)
        hipLaunchKernelGGL((k_segments_vjp<T, WG, 2>), dim3(grid), dim3(WG), 0, st, a);
    else
        hipLaunchKernelGGL((k_segments_vjp<T, WG, 3>), dim3(grid), dim3(WG), 0, st, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_segments_gradient(int dtype, const SegArgs& a, hipStream_t st) {
    if (a.n_tgt == 0) return hipSuccess;
    if (dtype == kDtypeF64) return launch_grad_split<double>(a, st);
    return launch_grad_split<float>(a, st);
}

hipError_t launch_segments_vjp(int dtype, const SegArgs& a, hipStream_t st) {
    if (a.n_tgt == 0) return hipSuccess;
    if (dtype == kDtypeF64) return launch_vjp_t<double, 256>(a, st);
    return launch_vjp_t<float, 256>(a, st);
}

template <typename T>
hipError_t launch_few_t(const SegArgs& a, hipStream_t st) {
    const int grid = int((a.n_tgt + 3) / 4);
    if (a.rc == 0.0)
        hipLaunchKernelGGL((k_segments_few<T, 0>), dim3(grid), dim3(256), 0, st, a);
    else if (a.vn == 1)
        hipLaunchKernelGGL((k_segments_few<T, 1>), dim3(grid), dim3(256), 0, st, a);
    else if (a.vn == 2)
        hipLaunchKernelGGL((k_segments_few<T, 2>), dim3(grid), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((k_segments_few<T, 3>), dim3(grid), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_segments(int dtype, const SegArgs& a, hipStream_t st) {
    if (a.n_tgt == 0) return hipSuccess;
    if (a.n_tgt <= kSegSmallTargets)
        return dtype == kDtypeF64 ? launch_few_t<double>(a, st) : launch_few_t<float>(a, st);
    if (dtype == kDtypeF64) return launch_t<double, 1, 256>(a, st);
    return launch_t<float, 2, 256>(a, st);
}

}  // namespace vpm
