// Viscous part of the particle right-hand side (Fu & Laurendeau, Sec. II.B): the diffusion term
// nu lap(Gamma_i) of Eq. 5 by particle strength exchange (PSE) with the Gaussian of Eq. 3 as the
// exchange kernel, and Vreman's sub-grid eddy viscosity (the paper's C_V = 0.07) that enters it.
//
// PSE, for the particles of one set, with omega = Gamma / V (V = particle volume):
//   dGamma_i/dt = V_i sum_j (2 nu_ij / sigma_ij^2) V_j (omega_j - omega_i) zeta_{sigma_ij}(|x_i - x_j|)
//   zeta_s(r) = (2 pi s^2)^(-3/2) exp(-r^2 / (2 s^2)),  sigma_ij^2 = (sigma_i^2 + sigma_j^2)/2,
//   nu_ij = nu + (nu_t,i + nu_t,j)/2.
// (V_i V_j (omega_j - omega_i) is the usual V_i Gamma_j - V_j Gamma_i; the omega form keeps the
// per-pair difference small when the field is smooth.)  The Gaussian is below 2e-11 of its peak
// beyond rho_ij^2 = 49 (FP32) and 9e-21 beyond 90.25 (FP64), so pairs farther apart than the
// far-field cut of the velocity kernels contribute nothing and whole source tiles are skipped
// by a box test: the work is proportional to the number of near pairs.
//
// Layout and schedule
//  - k_tile_box: one workgroup per tile of kTile sources writes the tile's bounding box and its
//    largest sigma^2/2 (8 values) to the workspace.
//  - k_pse: one workgroup per kTile targets; it reads each tile's box (all lanes the same
//    address), skips tiles out of reach of every target of the block, and stages the others
//    through LDS (x, sigma^2/2 | omega, V | (nu + nu_t)/2) for a broadcast inner loop, where
//    sigma_i^2/2 + sigma_j^2/2 = sigma_ij^2 and (nu + nu_t,i)/2 + (nu + nu_t,j)/2 = nu_ij.  Pairs
//    outside the cut take no transcendental.  FP32 sums are folded into two-sum pairs every
//    128 sources; the epilogue runs in FP64.
//  - k_vreman: one lane per particle, FP64 arithmetic.
#include <hip/hip_runtime.h>

#include "device_math.h"
#include "vpm_internal.h"

namespace vpm {

namespace {

constexpr int kTile = 256;
constexpr int kFold = 128;

template <typename T>
using V4 = typename std::conditional<std::is_same<T, float>::value, float4, double4>::type;

template <typename T>
__global__ __launch_bounds__(kTile) void k_tile_box(const T* __restrict__ x, const T* __restrict__ sg, int64_t ld,
                                                    int64_t begin, int64_t end, T* __restrict__ boxes) {
    __shared__ T scratch[7 * (kTile / 64)];
    const int64_t j0 = begin + int64_t(blockIdx.x) * kTile;
    const int64_t j = j0 + threadIdx.x;
    const int64_t jj = j < end ? j : j0;  // empty slots repeat the first source of the tile
    T lo[3], hi[3];
    lo[0] = hi[0] = x[jj];
    lo[1] = hi[1] = x[ld + jj];
    lo[2] = hi[2] = x[2 * ld + jj];
    const T s = sg[jj];
    T olo[3], ohi[3], ocut;
    block_box(lo, hi, T(0.5) * s * s, olo, ohi, ocut, scratch);
    if (threadIdx.x == 0) {
        T* b = boxes + 8 * int64_t(blockIdx.x);
        b[0] = olo[0];
        b[1] = olo[1];
        b[2] = olo[2];
        b[3] = ohi[0];
        b[4] = ohi[1];
        b[5] = ohi[2];
        b[6] = ocut;  // largest sigma^2/2 of the tile
        b[7] = T(0);
    }
}

struct PseArgs {
    const void* x;
    const void* g;
    const void* sg;
    const void* vol;
    const void* nut;  // may be nullptr
    int64_t ld;
    double nu;
    void* dg;
    int64_t ldo;
    int64_t begin, end;
    const void* boxes;  // tile boxes of this set, 8 values each
    int32_t accumulate;
};

template <typename T>
__global__ __launch_bounds__(kTile) void k_pse(PseArgs a) {
    constexpr bool kComp = std::is_same<T, float>::value;
    __shared__ V4<T> lp[kTile];  // x, y, z, sigma^2/2
    __shared__ V4<T> lq[kTile];  // omega, V
    __shared__ T lnu[kTile];     // (nu + nu_t)/2
    __shared__ T scratch[7 * (kTile / 64)];
    const T* __restrict__ x = static_cast<const T*>(a.x);
    const T* __restrict__ g = static_cast<const T*>(a.g);
    const T* __restrict__ sg = static_cast<const T*>(a.sg);
    const T* __restrict__ vol = static_cast<const T*>(a.vol);
    const T* __restrict__ nut = static_cast<const T*>(a.nut);
    const T* __restrict__ boxes = static_cast<const T*>(a.boxes);
    const T far2 = T(Prec<T>::kFarRho2);
    const T nuh = T(0.5 * a.nu);

    const int tid = threadIdx.x;
    const int64_t i = a.begin + int64_t(blockIdx.x) * kTile + tid;
    const bool valid = i < a.end;
    const int64_t ii = valid ? i : a.begin + int64_t(blockIdx.x) * kTile;
    const T xi0 = x[ii], xi1 = x[a.ld + ii], xi2 = x[2 * a.ld + ii];
    const T vi = vol[ii];
    const T ivi = T(1) / vi;
    const T wi0 = g[ii] * ivi, wi1 = g[a.ld + ii] * ivi, wi2 = g[2 * a.ld + ii] * ivi;
    const T si = sg[ii];
    const T hi_sig = T(0.5) * si * si;
    const T nui = nuh + (nut ? T(0.5) * nut[ii] : T(0));

    T blo[3], bhi[3], bh;
    {
        const T lo3[3] = {xi0, xi1, xi2};
        block_box(lo3, lo3, hi_sig, blo, bhi, bh, scratch);
    }

    T acc[3] = {T(0), T(0), T(0)}, shi[3] = {T(0), T(0), T(0)}, slo[3] = {T(0), T(0), T(0)};
    const int64_t ntiles = (a.end - a.begin + kTile - 1) / kTile;
    for (int64_t tt = 0; tt < ntiles; ++tt) {
        const T* b = boxes + 8 * tt;
        T d2 = T(0);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const T gap = fmax(fmax(b[c] - bhi[c], blo[c] - b[3 + c]), T(0));
            d2 += gap * gap;
        }
        // uniform over the workgroup: every lane read the same box and holds the same block box
        if (!(d2 < far2 * (b[6] + bh))) continue;
        const int64_t j0 = a.begin + tt * kTile;
        const int cnt = int((a.end - j0) < kTile ? (a.end - j0) : kTile);
        __syncthreads();  // the previous tile's readers are done
        if (tid < cnt) {
            const int64_t j = j0 + tid;
            const T sj = sg[j];
            const T vj = vol[j];
            const T ivj = T(1) / vj;
            V4<T> p, q;
            p.x = x[j];
            p.y = x[a.ld + j];
            p.z = x[2 * a.ld + j];
            p.w = T(0.5) * sj * sj;
            q.x = g[j] * ivj;
            q.y = g[a.ld + j] * ivj;
            q.z = g[2 * a.ld + j] * ivj;
            q.w = vj;
            lp[tid] = p;
            lq[tid] = q;
            lnu[tid] = nuh + (nut ? T(0.5) * nut[j] : T(0));
        }
        __syncthreads();
        for (int c0 = 0; c0 < cnt; c0 += kFold) {
            const int c1 = (cnt - c0) < kFold ? cnt : c0 + kFold;
            for (int jj = c0; jj < c1; ++jj) {
                const V4<T> p = lp[jj];
                const T rx = xi0 - p.x, ry = xi1 - p.y, rz = xi2 - p.z;
                const T s2 = rx * rx + ry * ry + rz * rz;
                const T sij2 = hi_sig + p.w;  // sigma_ij^2
                if (s2 < far2 * sij2) {
                    const V4<T> q = lq[jj];
                    const T inv = rcp_fast(sij2);          // 1 / sigma_ij^2
                    const T e = dexp(T(-0.5) * s2 * inv);  // exp(-s^2 / (2 sigma_ij^2))
                    const T w = (nui + lnu[jj]) * inv * inv * sqrt_fast(inv) * e * q.w;
                    acc[0] += w * (q.x - wi0);
                    acc[1] += w * (q.y - wi1);
                    acc[2] += w * (q.z - wi2);
                }
            }
            if constexpr (kComp) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    T s, e;
                    two_sum(shi[c], acc[c], s, e);
                    shi[c] = s;
                    slo[c] += e;
                    acc[c] = T(0);
                }
            }
        }
    }
    if (!valid) return;
    {
        // With inv = 1 / sigma_ij^2 the pair weight (2 nu_ij / sigma_ij^2) zeta_{sigma_ij} equals
        // nu_ij inv^(5/2) exp(-s^2 inv / 2) 2 (2 pi)^(-3/2); the sums above hold everything but
        // the constant and V_i.
#pragma clang fp contract(off)
        constexpr double kPseScale = 0.1269872718684819395715266098692720;  // 2 (2 pi)^(-3/2)
        double tot[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) tot[c] = kComp ? double(shi[c]) + double(slo[c]) : double(acc[c]);
        T* __restrict__ out = static_cast<T*>(a.dg);
        const double f = kPseScale * double(vi);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            T* dst = out + c * a.ldo + i;
            const double v = f * tot[c];
            *dst = a.accumulate ? T(double(*dst) + v) : T(v);
        }
    }
}

// Vreman: alpha_ab = du_b/dx_a = J[b][a]; beta = sigma^2 alpha^T alpha, i.e.
// beta_ab = sigma^2 sum_m J[a][m] J[b][m]; B_beta = sum of the principal 2x2 minors of beta.
template <typename T>
__global__ __launch_bounds__(256) void k_vreman(int64_t n, const T* __restrict__ J, int64_t ld,
                                                const T* __restrict__ sg, double cv, T* __restrict__ nut) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double j[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) j[c] = double(J[c * ld + i]);
    double m[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) m[a][b] = j[3 * a] * j[3 * b] + j[3 * a + 1] * j[3 * b + 1] + j[3 * a + 2] * j[3 * b + 2];
    const double aa = m[0][0] + m[1][1] + m[2][2];
    double r = 0.0;
    if (aa > 0.0) {
        const double d2 = double(sg[i]) * double(sg[i]);
        const double bb = d2 * d2 * (m[0][0] * m[1][1] - m[0][1] * m[0][1] + m[0][0] * m[2][2] - m[0][2] * m[0][2] +
                                     m[1][1] * m[2][2] - m[1][2] * m[1][2]);
        r = bb > 0.0 ? cv * sqrt(bb / aa) : 0.0;
    }
    nut[i] = T(r);
}

}  // namespace

hipError_t launch_pse(int dtype, int64_t begin, int64_t end, const void* x, const void* g, const void* sg,
                      const void* vol, const void* nut, int64_t ld, double nu, void* dg, int64_t ldo,
                      int accumulate, void* boxes, hipStream_t st) {
    const int64_t n = end - begin;
    if (n <= 0) return hipSuccess;
    const int nt = int((n + kTile - 1) / kTile);
    PseArgs a;
    a.x = x;
    a.g = g;
    a.sg = sg;
    a.vol = vol;
    a.nut = nut;
    a.ld = ld;
    a.nu = nu;
    a.dg = dg;
    a.ldo = ldo;
    a.begin = begin;
    a.end = end;
    a.boxes = boxes;
    a.accumulate = accumulate;
    if (dtype == kDtypeF64) {
        hipLaunchKernelGGL(k_tile_box<double>, dim3(nt), dim3(kTile), 0, st, (const double*)x, (const double*)sg, ld,
                           begin, end, (double*)boxes);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_pse<double>, dim3(nt), dim3(kTile), 0, st, a);
    } else {
        hipLaunchKernelGGL(k_tile_box<float>, dim3(nt), dim3(kTile), 0, st, (const float*)x, (const float*)sg, ld,
                           begin, end, (float*)boxes);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_pse<float>, dim3(nt), dim3(kTile), 0, st, a);
    }
    return hipGetLastError();
}

int64_t pse_tiles(int64_t n) { return (n + kTile - 1) / kTile; }

hipError_t launch_vreman(int dtype, int64_t n, const void* J, int64_t ld, const void* sg, double cv, void* nut,
                         hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int nb = int((n + 255) / 256);
    if (dtype == kDtypeF64)
        hipLaunchKernelGGL(k_vreman<double>, dim3(nb), dim3(256), 0, st, n, (const double*)J, ld, (const double*)sg,
                           cv, (double*)nut);
    else
        hipLaunchKernelGGL(k_vreman<float>, dim3(nb), dim3(256), 0, st, n, (const float*)J, ld, (const float*)sg, cv,
                           (float*)nut);
    return hipGetLastError();
}

}  // namespace vpm
