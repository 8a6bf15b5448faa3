// Device-side arithmetic shared by the libvpm kernels (gfx950 only).
//
// Kernel weights of the Gaussian blob (Fu & Laurendeau, Sec. II.B, Eq. 3).  With
// rho = s/sigma and q(rho) = erf(rho/sqrt2) - c0 rho exp(-rho^2/2), c0 = sqrt(2/pi):
//   g(s) = q / (4 pi s^3)                      velocity weight
//   h(s) = g'(s)/s = (rho q' - 3 q)/(4 pi s^5)  gradient weight (stretching)
//   k(s) = h'(s)/s = (rho^2 q'' - 7 rho q' + 15 q)/(4 pi s^7)   (adjoint only)
// The kernels carry 4 pi g, -(4 pi/3) h and (4 pi/15) k, which are exactly s^-3, s^-5, s^-7
// outside the core (rho >= RHO_FAR, where the blob is a point vortex to working precision),
// and apply 1/(4 pi) and the integer factors once per target.
//
// Inside the core:
//   rho < 1:  Taylor series in t = rho^2 (the closed form cancels there).  From
//             q = c0 sum_n (-1)^n rho^(2n+3) / ((2n+3) 2^n n!):
//               q/rho^3              = c0 sum_{n>=0} a_n t^n,          a_n = (-1)^n/((2n+3) 2^n n!)
//               (rho q'-3q)/rho^5    = c0 sum_{n>=1} 2n a_n t^(n-1)
//               (rho^2 q''-7 rho q'+15 q)/rho^7 = c0 sum_{n>=2} 4n(n-1) a_n t^(n-2)
//   rho >= 1: closed form (cancellation at most ~10x there): erf and exp in FP64; in FP32
//             q = 1 - E (F + c0 rho) with E = exp(-rho^2/2) and F = erfcx(rho/sqrt2) fitted
//             (closed_q below).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vpm {

constexpr double kPiD = 3.14159265358979323846264338327950288;
constexpr double kC0D = 0.79788456080286535587989211986876373;      // sqrt(2/pi)
constexpr double kInvSqrt2D = 0.70710678118654752440084436210484903;
constexpr double kInv4PiD = 1.0 / (4.0 * kPiD);

// a_n = (-1)^n / ((2n+3) 2^n n!)
constexpr double series_a(int n) {
    double a = 1.0;
    for (int k = 1; k <= n; ++k) a /= (2.0 * k);
    return ((n & 1) ? -a : a) / (2 * n + 3);
}

// Horner evaluation of sum_{n=N0}^{NMAX} w(n) a_n t^(n-N0), coefficients folded at compile time.
// W selects the weight: 0 -> 1, 1 -> 2n, 2 -> 4n(n-1).
template <int W>
constexpr double series_w(int n) {
    return W == 0 ? series_a(n) : (W == 1 ? 2.0 * n * series_a(n) : 4.0 * n * (n - 1) * series_a(n));
}
template <typename T, int W, int N, int NMAX>
struct Horner {
    static __device__ __forceinline__ T eval(T t) {
        constexpr double c = series_w<W>(N);
        if constexpr (N == NMAX) {
            return T(c);
        } else {
            return Horner<T, W, N + 1, NMAX>::eval(t) * t + T(c);
        }
    }
};

// Precision-dependent constants.
template <typename T> struct Prec;
template <> struct Prec<float> {
    // Beyond rho = 7 the dropped terms of g and h are below 2.1e-9 relative (< FP32 half ulp).
    static constexpr float kFarRho2 = 49.0f;
    static constexpr int kTermsG = 9;   // n = 0..8: truncation < 2.5e-8 relative at rho = 1
    static constexpr int kTermsH = 10;  // n = 1..9
    static constexpr int kTermsK = 11;  // n = 2..10
};
template <> struct Prec<double> {
    // Beyond rho = 9.5 the dropped terms are below 1e-16 relative.
    static constexpr double kFarRho2 = 90.25;
    static constexpr int kTermsG = 17;  // n = 0..16
    static constexpr int kTermsH = 18;
    static constexpr int kTermsK = 19;
};

// Hardware reciprocal square root / square root / reciprocal (about 1 ulp) for FP32; the
// library's correctly rounded square root and division for FP64.
__device__ __forceinline__ float rsqrt_fast(float x) { return __builtin_amdgcn_rsqf(x); }
// FP64 1/sqrt(x) for finite x > 0 (callers never use the result at x = 0): the hardware
// estimate y (about 23 good bits) times the first terms of the binomial series
// (1 - e)^(-1/2) = 1 + e/2 + 3e^2/8 + ..., e = 1 - x y^2, which leaves a relative error of
// order e^3 plus a few roundings.
__device__ __forceinline__ double rsqrt_fast(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}
__device__ __forceinline__ float sqrt_fast(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double sqrt_fast(double x) { return sqrt(x); }
__device__ __forceinline__ float rcp_fast(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_fast(double x) { return 1.0 / x; }
__device__ __forceinline__ float dsqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double dsqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float dexp(float x) { return expf(x); }
__device__ __forceinline__ double dexp(double x) { return exp(x); }
__device__ __forceinline__ float derf(float x) { return erff(x); }
__device__ __forceinline__ double derf(double x) { return erf(x); }

// Closed form for 1 <= t < rho_far^2: rho = sqrt(t), e = exp(-t/2) and q(rho).
__device__ __forceinline__ void closed_q(double t, double& rho, double& q, double& e) {
    rho = sqrt_fast(t);
    e = dexp(-0.5 * t);
    q = derf(rho * kInvSqrt2D) - kC0D * rho * e;
}
// FP32: erf(x) = 1 - exp(-x^2) erfcx(x) turns q into 1 - E (F + c0 rho), E = exp(-t/2),
// F = erfcx(rho/sqrt2), so that one exponential serves q and the gradient weight.  F is a
// degree-7 polynomial in w = 1/(1 + p rho) (the variable of Hastings' rational approximations
// of erfc), fitted for minimax relative error on 1 <= rho <= 7: below 1e-8 with the FP32
// coefficients (gen_core_fit.py prints them).  E comes from the hardware base-2 exponential
// (t <= 49 keeps it a normal number).  Against erf and exp of the math library this saves an
// exponential and erf's two-branch split at rho = sqrt2, with the same FP32 cancellation at
// rho ~ 1 (1 - E (F + c0 rho) ~ 0.2 there).
constexpr float kErfcxP = 0.26f;
constexpr float kErfcxC[8] = {0.00024324792f, 0.20333688f, 0.23765302f, 0.06786008f,
                              0.487162f,      -0.38822648f, 0.565143f,  -0.17319544f};
__device__ __forceinline__ void closed_q(float t, float& rho, float& q, float& e) {
    rho = sqrt_fast(t);
    e = __builtin_amdgcn_exp2f(t * -0.72134752044448170368f);  // exp(-t/2) = 2^(-t log2(e)/2)
    const float w = rcp_fast(fmaf(kErfcxP, rho, 1.0f));
    float f = kErfcxC[7];
#pragma unroll
    for (int k = 6; k >= 0; --k) f = fmaf(f, w, kErfcxC[k]);
    q = fmaf(-e, fmaf(float(kC0D), rho, f), 1.0f);
}

// In-core weights.  Inputs: s2 = |r|^2, isig = 1/sigma, isig2 = 1/sigma^2, Gf = s^-3 and
// Hf = s^-5 (valid when s > 0).  Outputs G = 4 pi g and Hn = -(4 pi/3) h.
template <typename T>
__device__ __forceinline__ void core_weights(T s2, T isig, T isig2, T Gf, T Hf, T& G, T& Hn) {
    const T t = s2 * isig2;
    if (t < T(1)) {
        const T isig3 = isig * isig2;
        const T isig5 = isig3 * isig2;
        const T gw = Horner<T, 0, 0, Prec<T>::kTermsG - 1>::eval(t);
        const T hw = Horner<T, 1, 1, Prec<T>::kTermsH>::eval(t);
        G = T(kC0D) * gw * isig3;
        Hn = T(-kC0D / 3.0) * hw * isig5;
    } else {
        T rho, q, e;
        closed_q(t, rho, q, e);
        G = q * Gf;
        Hn = (q - T(kC0D / 3.0) * rho * t * e) * Hf;
    }
}

// Same, also returning Kn = (4 pi/15) k (adjoint); Kf = s^-7.
template <typename T>
__device__ __forceinline__ void core_weights3(T s2, T isig, T isig2, T Gf, T Hf, T Kf, T& G, T& Hn,
                                              T& Kn) {
    const T t = s2 * isig2;
    if (t < T(1)) {
        const T isig3 = isig * isig2;
        const T isig5 = isig3 * isig2;
        const T isig7 = isig5 * isig2;
        const T gw = Horner<T, 0, 0, Prec<T>::kTermsG - 1>::eval(t);
        const T hw = Horner<T, 1, 1, Prec<T>::kTermsH>::eval(t);
        const T kw = Horner<T, 2, 2, Prec<T>::kTermsK>::eval(t);
        G = T(kC0D) * gw * isig3;
        Hn = T(-kC0D / 3.0) * hw * isig5;
        Kn = T(kC0D / 15.0) * kw * isig7;
    } else {
        T rho, q, e;
        closed_q(t, rho, q, e);
        const T r3e = rho * t * e;  // rho^3 e
        G = q * Gf;
        Hn = (q - T(kC0D / 3.0) * r3e) * Hf;
        // 15 q - c0 e (5 rho^3 + rho^5)
        Kn = (q - T(kC0D / 15.0) * r3e * (T(5) + t)) * Kf;
    }
}

// Wavefront-wide bounding box and maximum cut (shuffle reduction only; every lane receives
// the result).
template <typename T>
__device__ __forceinline__ void wave_box(const T (&lo)[3], const T (&hi)[3], T cut, T (&olo)[3], T (&ohi)[3],
                                         T& ocut) {
    T v[7] = {lo[0], lo[1], lo[2], hi[0], hi[1], hi[2], cut};
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int c = 0; c < 7; ++c) {
            const T o = __shfl_xor(v[c], off, 64);
            v[c] = c < 3 ? fmin(v[c], o) : fmax(v[c], o);
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        olo[c] = v[c];
        ohi[c] = v[3 + c];
    }
    ocut = v[6];
}

// A value known to be equal in every lane, moved to a scalar register.
__device__ __forceinline__ float uniform(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ double uniform(double v) {
    const unsigned long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane(int(b & 0xffffffffull));
    const int hi = __builtin_amdgcn_readfirstlane(int(b >> 32));
    return __longlong_as_double((static_cast<unsigned long long>(unsigned(hi)) << 32) | unsigned(lo));
}

// Workgroup-wide bounding box (lo, hi per component) and maximum cut: a shuffle reduction in
// each wavefront, then the wavefront results through LDS (scratch: 7 values per wavefront).
// Ends with a barrier; every thread receives the result.
template <typename T>
__device__ __forceinline__ void block_box(const T (&lo)[3], const T (&hi)[3], T cut, T (&olo)[3], T (&ohi)[3],
                                          T& ocut, T* scratch) {
    T v[7] = {lo[0], lo[1], lo[2], hi[0], hi[1], hi[2], cut};
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
    __syncthreads();  // previous readers of scratch are done
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
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        olo[c] = v[c];
        ohi[c] = v[3 + c];
    }
    ocut = v[6];
}

// Knuth's TwoSum: s + e == a + b exactly.
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// The kernels call these.  The FP64 versions are calls, not inlined: their series and erf hold
// many FP64 constants (no FP64 literal operands), which inlined would raise the register count
// of the whole pair loop that contains this rarely taken branch (FP64 transposed pair kernel:
// 249 -> 124 VGPRs, two -> four wavefronts per SIMD).
__device__ __forceinline__ void core_weights_call(float s2, float isig, float isig2, float& G, float& Hn) {
    core_weights<float>(s2, isig, isig2, G, Hn, G, Hn);
}
static __device__ __attribute__((noinline, unused)) void core_weights_call(double s2, double isig, double isig2, double& G,
                                                                   double& Hn) {
    core_weights<double>(s2, isig, isig2, G, Hn, G, Hn);
}
__device__ __forceinline__ void core_weights3_call(float s2, float is, float is2, float Gf, float Hf, float Kf,
                                                   float& G, float& Hn, float& Kn) {
    core_weights3<float>(s2, is, is2, Gf, Hf, Kf, G, Hn, Kn);
}
static __device__ __attribute__((noinline, unused)) void core_weights3_call(double s2, double is, double is2, double Gf,
                                                                    double Hf, double Kf, double& G, double& Hn,
                                                                    double& Kn) {
    core_weights3<double>(s2, is, is2, Gf, Hf, Kf, G, Hn, Kn);
}

}  // namespace vpm
