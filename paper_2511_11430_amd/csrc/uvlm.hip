// Blade solve and wake management of one NL-UVLM-VPM step (Fu & Laurendeau, Sec. II.A and the
// adaptive wake conversion of Sec. II.C, Eqs. 6-8), for one MI355X (gfx950).
//
//  - k_aic: influence matrix of the blade vortex-ring lattice, FP64, one lane per (collocation
//    point, ring) entry (a row of the matrix is contiguous, so stores coalesce).  A ring is the
//    closed path c00 -> c01 -> c11 -> c10 with unit circulation; each edge is the finite
//    straight segment law (r1 x r2) r0 . (r1/|r1| - r2/|r2|) / (4 pi |r0|^2 (d^2n + rc^2n)^(1/n))
//    with the Vatistas core, d^2 = |r1 x r2|^2 / |r0|^2.  Entry = n_i . u_ring_j(c_i).
//  - k_lu_panel / k_lu_swap_trsm / k_lu_gemm: dense LU with partial pivoting, blocked
//    in panels of 16 columns for n <= 1024 (a panel in one workgroup with a row per lane, the
//    rest on many workgroups); k_lu_factor: the same column by column in one workgroup for
//    larger n; k_lu_solve_blocked / k_lu_solve: the two triangular solves in one workgroup (in
//    blocks of 64 rows for n <= 1024).  Pivot = largest |entry|
//    of the column, the first such row on ties.
//  - k_wake_shed: Kutta condition and the strengths of the newest wake row's lines (Eq. 7):
//    trailed line at span station c: Gamma_te(c-1) - Gamma_te(c) (0 outside the blade), shed
//    line of strip c: Gamma_te,prev(c) - Gamma_te(c); the previous values are then replaced.
//  - k_conv_count / k_conv_scan / k_conv_emit: panel-line to particle conversion.  Counts
//    n = ceil(ds / ds_t * n_t) (Eq. 8; FP64, evaluated as written, no contraction) for trailed
//    lines, 1 for shed lines; an exclusive scan in one workgroup gives each line its first
//    particle; each line then writes its n particles (midpoints of n equal sub-segments,
//    strength dGamma (b - a) / n, Eq. 6).
#include <hip/hip_runtime.h>

#include "device_math.h"
#include "vpm_internal.h"

namespace vpm {

namespace {

// Velocity of a straight segment a -> b of unit circulation at p (FP64), Vatistas core.
// Zero for a vanishing arm or length (below 1e-12 max(|r0|, 1)) or a vanishing denominator.
__device__ __forceinline__ void segment_unit(const double p[3], const double a[3], const double b[3], double rc2n,
                                             double inv_n, int vn, double u[3]) {
    const double r1[3] = {p[0] - a[0], p[1] - a[1], p[2] - a[2]};
    const double r2[3] = {p[0] - b[0], p[1] - b[1], p[2] - b[2]};
    const double r0[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    const double c[3] = {r1[1] * r2[2] - r1[2] * r2[1], r1[2] * r2[0] - r1[0] * r2[2], r1[0] * r2[1] - r1[1] * r2[0]};
    const double l1 = sqrt(r1[0] * r1[0] + r1[1] * r1[1] + r1[2] * r1[2]);
    const double l2 = sqrt(r2[0] * r2[0] + r2[1] * r2[1] + r2[2] * r2[2]);
    const double l02 = r0[0] * r0[0] + r0[1] * r0[1] + r0[2] * r0[2];
    const double l0 = sqrt(l02);
    const double eps = 1e-12 * fmax(l0, 1.0);
    u[0] = u[1] = u[2] = 0.0;
    if (l1 < eps || l2 < eps || l0 < eps) return;
    const double c2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
    const double d2 = c2 / l02;
    double den;
    if (vn == 1) den = d2 + rc2n;
    else if (vn == 2) den = sqrt(d2 * d2 + rc2n);
    else den = pow(pow(d2, 1.0 / inv_n) + rc2n, inv_n);
    den *= l02;
    if (!(den > 0.0)) return;
    const double D = (r0[0] * r1[0] + r0[1] * r1[1] + r0[2] * r1[2]) / l1 -
                     (r0[0] * r2[0] + r0[1] * r2[1] + r0[2] * r2[2]) / l2;
    const double f = kInv4PiD * D / den;
    u[0] = f * c[0];
    u[1] = f * c[1];
    u[2] = f * c[2];
}

struct AicArgs {
    int64_t n;
    const double* c00;
    const double* c01;
    const double* c11;
    const double* c10;
    int64_t ldr;
    const double* col;
    const double* nrm;
    int64_t ldc;
    double rc2n, inv_n;
    int vn;
    double* A;
    int64_t lda;
};

__global__ __launch_bounds__(256) void k_aic(AicArgs a) {
    const int64_t i = blockIdx.y;
    const int64_t j = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i >= a.n || j >= a.n) return;
    const double p[3] = {a.col[i], a.col[a.ldc + i], a.col[2 * a.ldc + i]};
    const double nn[3] = {a.nrm[i], a.nrm[a.ldc + i], a.nrm[2 * a.ldc + i]};
    const double* cs[4] = {a.c00, a.c01, a.c11, a.c10};
    double q[4][3];
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int c = 0; c < 3; ++c) q[e][c] = cs[e][c * a.ldr + j];
    double s = 0.0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        double u[3];
        segment_unit(p, q[e], q[(e + 1) & 3], a.rc2n, a.inv_n, a.vn, u);
        s += nn[0] * u[0] + nn[1] * u[1] + nn[2] * u[2];
    }
    a.A[i * a.lda + j] = s;
}

constexpr int kLuThreads = 1024;

// Largest |x| with its index over the workgroup (first index on ties).
__device__ __forceinline__ void block_argmax(double& v, int64_t& idx, double* sv, int64_t* si) {
    for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(v, off, 64);
        const int64_t oi = __shfl_xor(idx, off, 64);
        if (ov > v || (ov == v && oi < idx)) {
            v = ov;
            idx = oi;
        }
    }
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        sv[w] = v;
        si[w] = idx;
    }
    __syncthreads();
    v = sv[0];
    idx = si[0];
    const int nw = int(blockDim.x) >> 6;
    for (int k = 1; k < nw; ++k) {
        if (sv[k] > v || (sv[k] == v && si[k] < idx)) {
            v = sv[k];
            idx = si[k];
        }
    }
}

__global__ __launch_bounds__(kLuThreads) void k_lu_factor(int64_t n, double* A, int64_t lda, int32_t* ipiv,
                                                          int32_t* info) {
    __shared__ double sv[kLuThreads / 64];
    __shared__ int64_t si[kLuThreads / 64];
    const int t = threadIdx.x;
    int32_t first_zero = 0;
    for (int64_t k = 0; k < n; ++k) {
        double v = -1.0;
        int64_t idx = k;
        for (int64_t r = k + t; r < n; r += kLuThreads) {
            const double x = fabs(A[r * lda + k]);
            if (x > v) {
                v = x;
                idx = r;
            }
        }
        block_argmax(v, idx, sv, si);
        if (t == 0) ipiv[k] = int32_t(idx);
        if (v == 0.0) {  // singular column: record the first one, leave the column as is
            if (first_zero == 0) first_zero = int32_t(k + 1);
            __syncthreads();
            continue;
        }
        if (idx != k) {
            for (int64_t c = t; c < n; c += kLuThreads) {
                const double x = A[k * lda + c];
                A[k * lda + c] = A[idx * lda + c];
                A[idx * lda + c] = x;
            }
        }
        __syncthreads();
        const double piv = A[k * lda + k];
        for (int64_t r = k + 1 + t; r < n; r += kLuThreads) A[r * lda + k] /= piv;
        __syncthreads();
        const int64_t m = n - k - 1;
        for (int64_t e = t; e < m * m; e += kLuThreads) {
            const int64_t r = k + 1 + e / m;
            const int64_t c = k + 1 + e % m;
            A[r * lda + c] -= A[r * lda + k] * A[k * lda + c];
        }
        __syncthreads();
    }
    if (t == 0) *info = first_zero;
}

// ---- blocked LU for n <= kLuThreads: panels of kPanel columns.  Each panel is factored in one
// workgroup with its rows in registers (one row per lane); the row exchanges are then applied
// to the other columns, the panel's block row of U is solved, and the trailing matrix takes the
// panel's rank-kPanel update on many workgroups.  Every entry receives the same operations in
// the same order as in the unblocked factorisation above (a_rc -= l_rk u_kc for k = 0, 1, ...,
// a_rk /= u_kk), and the pivots are chosen the same way, so the factors agree with the
// unblocked ones up to how each update is contracted into an FMA.
constexpr int kPanel = 16;

// Panel [j0, j0 + nb): rows [j0, n), row j0 + t in lane t (the workgroup has as many
// wavefronts as the rows need).
// Unsigned maximum over lanes 0 .. 16 * kRows - 1 of a full wavefront, returned in every lane:
// row shifts by 1, 2, 4 and 8 leave each 16-lane row's maximum in its last lane; for a whole
// wavefront the two row broadcasts then carry row 0 into row 1, row 2 into row 3 and lane 31
// into rows 2 and 3, so lane 63 holds the maximum.  Lanes a DPP move does not write read 0, the
// identity.  Every lane of the wavefront must be active.
template <int kRows>
__device__ __forceinline__ uint32_t lanes_umax(uint32_t k) {
    static_assert(kRows == 1 || kRows == 4, "one row or the whole wavefront");
    k = max(k, uint32_t(__builtin_amdgcn_update_dpp(0, int(k), 0x111, 0xf, 0xf, false)));  // row_shr:1
    k = max(k, uint32_t(__builtin_amdgcn_update_dpp(0, int(k), 0x112, 0xf, 0xf, false)));  // row_shr:2
    k = max(k, uint32_t(__builtin_amdgcn_update_dpp(0, int(k), 0x114, 0xf, 0xf, false)));  // row_shr:4
    k = max(k, uint32_t(__builtin_amdgcn_update_dpp(0, int(k), 0x118, 0xf, 0xf, false)));  // row_shr:8
    if constexpr (kRows == 4) {
        k = max(k, uint32_t(__builtin_amdgcn_update_dpp(0, int(k), 0x142, 0xa, 0xf, false)));  // row_bcast:15
        k = max(k, uint32_t(__builtin_amdgcn_update_dpp(0, int(k), 0x143, 0xc, 0xf, false)));  // row_bcast:31
    }
    return uint32_t(__builtin_amdgcn_readlane(int(k), kRows * 16 - 1));
}

// The first lane (lowest lane index) holding the largest 64-bit key among lanes 0 .. 16 * kRows
// - 1 (lanes beyond hold 0): maximum of the high words, then of the low words among the lanes
// that hold the high maximum, then a ballot.  Returns the lane and the maximum.
template <int kRows>
__device__ __forceinline__ int first_umax(uint64_t key, uint64_t& kmax) {
    const uint32_t hi = uint32_t(key >> 32), lo = uint32_t(key);
    const uint32_t hmax = lanes_umax<kRows>(hi);
    const uint32_t lmax = lanes_umax<kRows>(hi == hmax ? lo : 0u);
    kmax = (uint64_t(hmax) << 32) | lmax;
    return __ffsll((unsigned long long)__ballot(hi == hmax && lo == lmax)) - 1;
}

// One panel of kPanel columns in one workgroup, a row per lane held in registers (rows j0 ..
// n-1; the launch has whole wavefronts).  Pivot search on the key bits(|a|) + 1 (0 for rows
// above the diagonal or past n): for non-negative doubles the bit patterns order as the
// values, so the largest key is the largest magnitude, and the first lane holding it is the
// first row on ties.  Each wavefront posts its candidate row (key, row index and the row's
// kPanel entries) and lane cc posts row cc, in buffers alternating by column; one barrier, then
// every wavefront reduces the posted keys the same way (the first wavefront on ties) and reads
// the pivot row.  A buffer written at column cc is next written at column cc + 2, after the
// barrier of column cc + 1 that every lane reaches only when done reading it.  A column without
// a nonzero pivot has every candidate at key 1, so its pivot is row cc itself and nothing moves.
__global__ __launch_bounds__(kLuThreads) void k_lu_panel(int64_t n, double* A, int64_t lda, int64_t j0, int nb,
                                                         int32_t* ipiv, int32_t* info) {
    constexpr int kWaves = kLuThreads / 64;
    static_assert(kWaves <= 16, "the posted keys are reduced within one 16-lane row");
    __shared__ double srow[2][kPanel][kWaves + 1];  // [buffer][column][wavefront candidates, then row cc]
    __shared__ uint64_t skey[2][kWaves];
    __shared__ int sidx[2][kWaves];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, nw = int(blockDim.x) >> 6;
    const int64_t r = j0 + t;
    const bool has = r < n;
    int32_t piv = 0;          // lane cc: the pivot row of column j0 + cc
    int first_singular = -1;  // uniform
    double p[kPanel];
#pragma unroll
    for (int j = 0; j < kPanel; ++j) p[j] = (has && j < nb) ? A[r * lda + j0 + j] : 0.0;
#pragma unroll
    for (int cc = 0; cc < kPanel; ++cc) {
        if (cc < nb) {  // uniform
            const int b = cc & 1;
            const uint64_t key = (has && t >= cc) ? uint64_t(__double_as_longlong(fabs(p[cc]))) + 1 : 0;
            uint64_t wmax;
            const int lead = first_umax<4>(key, wmax);
            if (lane == lead) {
                skey[b][w] = wmax;
                sidx[b][w] = t;
#pragma unroll
                for (int j = 0; j < kPanel; ++j) srow[b][j][w] = p[j];
            }
            if (t == cc) {
#pragma unroll
                for (int j = 0; j < kPanel; ++j) srow[b][j][kWaves] = p[j];
            }
            __syncthreads();
            uint64_t gmax;
            const int ww = first_umax<1>(lane < nw ? skey[b][lane] : 0, gmax);
            const int idx = sidx[b][ww];
            const bool singular = gmax == 1;
            if (t == cc) piv = int32_t(j0 + idx);
            if (singular && first_singular < 0) first_singular = cc;
            // rows cc and idx trade places
            if (idx != cc && (t == cc || t == idx)) {
                const int from = t == cc ? ww : kWaves;
#pragma unroll
                for (int j = 0; j < kPanel; ++j) p[j] = srow[b][j][from];
            }
            if (has && t > cc && !singular) {
                p[cc] /= srow[b][cc][ww];
#pragma unroll
                for (int j = cc + 1; j < kPanel; ++j)
                    if (j < nb) p[j] -= p[cc] * srow[b][j][ww];
            }
        }
    }
    if (has) {
#pragma unroll
        for (int j = 0; j < kPanel; ++j)
            if (j < nb) A[r * lda + j0 + j] = p[j];
    }
    // The pivots and the status are written once at the end: a global store pending at a
    // barrier holds every wavefront there until the store completes.
    if (t < nb) ipiv[j0 + t] = piv;
    if (t == 0) {
        if (j0 == 0) *info = 0;
        if (first_singular >= 0 && *info == 0) *info = int32_t(j0 + first_singular + 1);  // the first such column
    }
}

// One lane per column outside the panel: the panel's row exchanges, in order, and for the
// columns right of the panel the block row of U by forward substitution with the panel's unit
// lower block (staged in LDS).
__global__ __launch_bounds__(256) void k_lu_swap_trsm(int64_t n, double* A, int64_t lda, int64_t j0, int nb,
                                                      const int32_t* ipiv) {
    __shared__ double sl[kPanel][kPanel];
    for (int e = threadIdx.x; e < nb * nb; e += 256) sl[e / nb][e % nb] = A[(j0 + e / nb) * lda + j0 + e % nb];
    __syncthreads();
    const int64_t c = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (c >= n || (c >= j0 && c < j0 + nb)) return;
    for (int cc = 0; cc < nb; ++cc) {
        const int64_t k = j0 + cc, q = ipiv[k];
        if (q != k) {
            const double x = A[k * lda + c];
            A[k * lda + c] = A[q * lda + c];
            A[q * lda + c] = x;
        }
    }
    if (c < j0) return;
    double x[kPanel];
#pragma unroll
    for (int i = 0; i < kPanel; ++i) x[i] = i < nb ? A[(j0 + i) * lda + c] : 0.0;
#pragma unroll
    for (int i = 1; i < kPanel; ++i) {
        if (i < nb) {
#pragma unroll
            for (int k = 0; k < i; ++k) x[i] -= sl[i][k] * x[k];
        }
    }
#pragma unroll
    for (int i = 1; i < kPanel; ++i)
        if (i < nb) A[(j0 + i) * lda + c] = x[i];
}

// Trailing update a_rc -= sum_k l_rk u_kc (k over the panel, in order), r, c >= j0 + nb:
// 64 x 64 tiles, 4 x 4 entries per lane, the panel's L and U parts staged in LDS.
__global__ __launch_bounds__(256) void k_lu_gemm(int64_t n, double* A, int64_t lda, int64_t j0, int nb) {
    __shared__ double sL[64][kPanel + 1];
    __shared__ double sU[kPanel][64];
    const int64_t b0 = j0 + nb;
    const int64_t r0 = b0 + int64_t(blockIdx.y) * 64, c0 = b0 + int64_t(blockIdx.x) * 64;
    for (int e = threadIdx.x; e < 64 * kPanel; e += 256) {
        const int i = e / kPanel, k = e % kPanel;
        const int64_t r = r0 + i;
        sL[i][k] = (r < n && k < nb) ? A[r * lda + j0 + k] : 0.0;
        const int kk = e / 64, j = e % 64;
        const int64_t c = c0 + j;
        sU[kk][j] = (c < n && kk < nb) ? A[(j0 + kk) * lda + c] : 0.0;
    }
    __syncthreads();
    const int ty = threadIdx.x / 16, tx = threadIdx.x % 16;
    double acc[4][4];
    bool ok[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int64_t r = r0 + ty + 16 * a, c = c0 + tx + 16 * b;
            ok[a][b] = r < n && c < n;
            acc[a][b] = ok[a][b] ? A[r * lda + c] : 0.0;
        }
    for (int k = 0; k < nb; ++k)
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] -= sL[ty + 16 * a][k] * sU[k][tx + 16 * b];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
            if (ok[a][b]) A[(r0 + ty + 16 * a) * lda + c0 + tx + 16 * b] = acc[a][b];
}

__global__ __launch_bounds__(kLuThreads) void k_lu_solve(int64_t n, const double* LU, int64_t lda,
                                                         const int32_t* ipiv, double* b) {
    const int t = threadIdx.x;
    if (t == 0) {
        for (int64_t k = 0; k < n; ++k) {
            const int64_t p = ipiv[k];
            if (p != k && p >= 0 && p < n) {
                const double x = b[k];
                b[k] = b[p];
                b[p] = x;
            }
        }
    }
    __syncthreads();
    for (int64_t k = 0; k < n; ++k) {  // L y = P b, unit diagonal
        const double bk = b[k];
        for (int64_t r = k + 1 + t; r < n; r += kLuThreads) b[r] -= LU[r * lda + k] * bk;
        __syncthreads();
    }
    for (int64_t k = n - 1; k >= 0; --k) {  // U x = y
        if (t == 0) b[k] /= LU[k * lda + k];
        __syncthreads();
        const double xk = b[k];
        for (int64_t r = t; r < k; r += kLuThreads) b[r] -= LU[r * lda + k] * xk;
        __syncthreads();
    }
}

// The two triangular solves for n <= kLuThreads, b in LDS, in blocks of 64 rows: one
// wavefront solves a diagonal block (staged in LDS) in the order of k_lu_solve, then the lanes
// update the remaining rows with that block's columns (lu_solve_rows: the block's 64 products
// of a row summed as eight partial sums and a butterfly, so the rounding differs from
// k_lu_solve's sequential sums).

// A uniform lane's double, read into scalar registers.
__device__ __forceinline__ double lane_value(double v, int k) {
    const int64_t b = __double_as_longlong(v);
    const uint32_t lo = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(b)), k));
    const uint32_t hi = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(uint64_t(b) >> 32)), k));
    return __longlong_as_double(int64_t((uint64_t(hi) << 32) | lo));
}

// sb[r] -= sum_k LU[r][kb + k] sb[kb + k] (k < nbk <= 64) for rows r0 <= r < r1: eight lanes
// per row, lane s taking the columns s, s + 8, ..., so that one load instruction of a wavefront
// reads eight rows' consecutive 64-byte runs; the eight partial sums are added by a butterfly.
__device__ __forceinline__ void lu_solve_rows(const double* LU, int64_t lda, double* sb, int64_t kb, int nbk,
                                              int64_t r0, int64_t r1) {
    const int g = threadIdx.x >> 3, sub = threadIdx.x & 7;
    for (int64_t rb = r0; rb < r1; rb += kLuThreads / 8) {
        const int64_t r = rb + g;  // uniform per eight lanes; the shuffles below run on all lanes
        double v = 0.0;
        if (r < r1) {
            const double* row = LU + r * lda + kb;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int k = sub + 8 * i;
                if (k < nbk) v += row[k] * sb[kb + k];
            }
        }
        v += __shfl_xor(v, 1, 64);
        v += __shfl_xor(v, 2, 64);
        v += __shfl_xor(v, 4, 64);
        if (r < r1 && sub == 0) sb[r] -= v;
    }
}

__global__ __launch_bounds__(kLuThreads) void k_lu_solve_blocked(int64_t n, const double* LU, int64_t lda,
                                                                 const int32_t* ipiv, double* b) {
    __shared__ double sb[kLuThreads];
    __shared__ double sd[64][65];
    const int t = threadIdx.x, lane = t & 63;
    if (t < n) sb[t] = b[t];
    __syncthreads();
    if (t == 0)
        for (int64_t k = 0; k < n; ++k) {
            const int64_t p = ipiv[k];
            if (p != k && p >= 0 && p < n) {
                const double x = sb[k];
                sb[k] = sb[p];
                sb[p] = x;
            }
        }
    __syncthreads();
    // L y = P b, unit diagonal, in blocks of 64 rows: one wavefront solves the diagonal block
    // (the solved entry broadcast from its lane), then all lanes update the rows below.
    for (int64_t kb = 0; kb < n; kb += 64) {
        const int nbk = int(n - kb < 64 ? n - kb : 64);
        for (int e = t; e < nbk * nbk; e += kLuThreads) sd[e / nbk][e % nbk] = LU[(kb + e / nbk) * lda + kb + e % nbk];
        __syncthreads();
        if (t < 64) {
            double y = lane < nbk ? sb[kb + lane] : 0.0;
            for (int k = 0; k < nbk; ++k) {
                const double yk = lane_value(y, k);
                if (lane > k && lane < nbk) y -= sd[lane][k] * yk;
            }
            if (lane < nbk) sb[kb + lane] = y;
        }
        __syncthreads();
        lu_solve_rows(LU, lda, sb, kb, nbk, kb + nbk, n);
        __syncthreads();
    }
    // U x = y, the blocks from the last: the diagonal block, then the rows above
    const int64_t nblk = (n + 63) / 64;
    for (int64_t bi = nblk - 1; bi >= 0; --bi) {
        const int64_t kb = bi * 64;
        const int nbk = int(n - kb < 64 ? n - kb : 64);
        for (int e = t; e < nbk * nbk; e += kLuThreads) sd[e / nbk][e % nbk] = LU[(kb + e / nbk) * lda + kb + e % nbk];
        __syncthreads();
        if (t < 64) {
            double y = lane < nbk ? sb[kb + lane] : 0.0;
            for (int k = nbk - 1; k >= 0; --k) {
                if (lane == k) y /= sd[k][k];
                const double xk = lane_value(y, k);
                if (lane < k) y -= sd[lane][k] * xk;
            }
            if (lane < nbk) sb[kb + lane] = y;
        }
        __syncthreads();
        lu_solve_rows(LU, lda, sb, kb, nbk, 0, kb);
        __syncthreads();
    }
    if (t < n) b[t] = sb[t];
}

template <typename T>
__global__ __launch_bounds__(256) void k_wake_shed(int n_blades, int n_span, const T* gb, const int32_t* te,
                                                   T* prev, T* trailed, T* shed) {
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    const int per = 2 * n_span + 1;
    if (id >= n_blades * per) return;
    const int b = id / per;
    const int k = id % per;
    if (k <= n_span) {  // trailed line at station k
        const double left = k > 0 ? double(gb[te[b * n_span + k - 1]]) : 0.0;
        const double right = k < n_span ? double(gb[te[b * n_span + k]]) : 0.0;
        trailed[b * (n_span + 1) + k] = T(left - right);
    } else {  // shed line of strip c
        const int c = k - n_span - 1;
        shed[b * n_span + c] = T(double(prev[b * n_span + c]) - double(gb[te[b * n_span + c]]));
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_wake_keep(int n, const T* gb, const int32_t* te, T* prev) {
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id < n) prev[id] = gb[te[id]];
}

template <typename T>
__global__ __launch_bounds__(256) void k_conv_count(int64_t n, const T* a, const T* b, int64_t ld,
                                                    const int32_t* tip, int n_tip, int n_max, int32_t* cnt) {
#pragma clang fp contract(off)
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t t = tip[i];
    int32_t c = 1;
    if (t >= 0 && t < n) {
        const double dx = double(b[i]) - double(a[i]), dy = double(b[ld + i]) - double(a[ld + i]),
                     dz = double(b[2 * ld + i]) - double(a[2 * ld + i]);
        const double tx = double(b[t]) - double(a[t]), ty = double(b[ld + t]) - double(a[ld + t]),
                     tz = double(b[2 * ld + t]) - double(a[2 * ld + t]);
        const double ds = sqrt(dx * dx + dy * dy + dz * dz);
        const double dt = sqrt(tx * tx + ty * ty + tz * tz);
        if (dt > 0.0) {
            const double q = ceil(ds / dt * double(n_tip));
            c = q > double(n_max) ? n_max : int32_t(q);
        }
    }
    cnt[i] = c;
}

// Exclusive scan of n counts in one workgroup of 1024 lanes: lane l owns a contiguous chunk.
__global__ __launch_bounds__(1024) void k_conv_scan(int64_t n, const int32_t* cnt, int64_t* first, int64_t* total) {
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int64_t chunk = (n + 1023) / 1024;
    const int64_t lo = t * chunk < n ? t * chunk : n;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    int64_t s = 0;
    for (int64_t i = lo; i < hi; ++i) s += cnt[i];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t run = t > 0 ? part[t - 1] : 0;
    for (int64_t i = lo; i < hi; ++i) {
        first[i] = run;
        run += cnt[i];
    }
    if (t == 1023) *total = part[1023];
}

template <typename T>
__global__ __launch_bounds__(256) void k_conv_emit(int64_t n, const T* a, const T* b, int64_t ld, const T* dg,
                                                   const int32_t* cnt, const int64_t* first, double sigma,
                                                   int64_t capacity, T* xo, T* go, T* so, int64_t ldo) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t m = cnt[i];
    const int64_t f = first[i];
    if (m <= 0 || f + m > capacity) return;  // a line that does not fit is left out whole
    const double A[3] = {double(a[i]), double(a[ld + i]), double(a[2 * ld + i])};
    const double dl[3] = {double(b[i]) - A[0], double(b[ld + i]) - A[1], double(b[2 * ld + i]) - A[2]};
    const double w = double(dg[i]) / double(m);
    for (int32_t k = 0; k < m; ++k) {
        const double s = (double(k) + 0.5) / double(m);
        const int64_t o = f + k;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            xo[c * ldo + o] = T(A[c] + s * dl[c]);
            go[c * ldo + o] = T(w * dl[c]);
        }
        so[o] = T(sigma);
    }
}

// AIC of one time step: out = base plus, in the columns that ring_of_col maps to an extra ring q,
// the influence of ring q (the wake row at the trailing edge carries the unknown circulation
// of the trailing-edge panel it hangs from).
struct AicUpdArgs {
    int64_t n;
    const double* base;
    double* out;
    int64_t ldb, ldo;
    const double* col;
    const double* nrm;
    int64_t ldc;
    const double* r00;
    const double* r01;
    const double* r11;
    const double* r10;
    int64_t ldr;
    const int32_t* ring_of_col;
    int64_t m;
    double rc2n, inv_n;
    int vn;
};

__global__ __launch_bounds__(256) void k_aic_update(AicUpdArgs a) {
    const int64_t i = blockIdx.y;
    const int64_t j = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i >= a.n || j >= a.n) return;
    double v = a.base[i * a.ldb + j];
    const int64_t q = a.ring_of_col[j];
    if (q >= 0 && q < a.m) {
        const double p[3] = {a.col[i], a.col[a.ldc + i], a.col[2 * a.ldc + i]};
        const double nn[3] = {a.nrm[i], a.nrm[a.ldc + i], a.nrm[2 * a.ldc + i]};
        const double* cs[4] = {a.r00, a.r01, a.r11, a.r10};
        double c[4][3];
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int d = 0; d < 3; ++d) c[e][d] = cs[e][d * a.ldr + q];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            double u[3];
            segment_unit(p, c[e], c[(e + 1) & 3], a.rc2n, a.inv_n, a.vn, u);
            v += nn[0] * u[0] + nn[1] * u[1] + nn[2] * u[2];
        }
    }
    a.out[i * a.ldo + j] = v;
}

// Neumann right-hand side: rhs_i = -((v_inf - omega x c_i + u_i) . n_i).
template <typename T>
__global__ __launch_bounds__(256) void k_neumann_rhs(int64_t n, const double* col, const double* nrm, int64_t ldc,
                                                     const T* u, int64_t ldu, double v0, double v1, double v2,
                                                     double w0, double w1, double w2, double* rhs) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double c0 = col[i], c1 = col[ldc + i], c2 = col[2 * ldc + i];
    const double r0 = v0 - (w1 * c2 - w2 * c1) + double(u[i]);
    const double r1 = v1 - (w2 * c0 - w0 * c2) + double(u[ldu + i]);
    const double r2 = v2 - (w0 * c1 - w1 * c0) + double(u[2 * ldu + i]);
    rhs[i] = -(r0 * nrm[i] + r1 * nrm[ldc + i] + r2 * nrm[2 * ldc + i]);
}

// Explicit Euler move of points: x += dt (u + v_inf); optionally g += dt dg.
}  // namespace

hipError_t launch_aic(int64_t n, const double* c00, const double* c01, const double* c11, const double* c10,
                      int64_t ldr, const double* col, const double* nrm, int64_t ldc, double rc, int vn, double* A,
                      int64_t lda, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    AicArgs a;
    a.n = n;
    a.c00 = c00;
    a.c01 = c01;
    a.c11 = c11;
    a.c10 = c10;
    a.ldr = ldr;
    a.col = col;
    a.nrm = nrm;
    a.ldc = ldc;
    a.vn = vn;
    a.inv_n = 1.0 / double(vn);
    a.rc2n = rc > 0.0 ? pow(rc * rc, double(vn)) : 0.0;
    a.A = A;
    a.lda = lda;
    hipLaunchKernelGGL(k_aic, dim3(unsigned((n + 255) / 256), unsigned(n)), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_lu_factor(int64_t n, double* A, int64_t lda, int32_t* ipiv, int32_t* info, hipStream_t st) {
    if (n > kLuThreads) {  // one workgroup, column by column
        hipLaunchKernelGGL(k_lu_factor, dim3(1), dim3(kLuThreads), 0, st, n, A, lda, ipiv, info);
        return hipGetLastError();
    }
    hipError_t e;
    for (int64_t j0 = 0; j0 < n; j0 += kPanel) {
        const int nb = int(n - j0 < kPanel ? n - j0 : kPanel);
        const unsigned lanes = unsigned((n - j0 + 63) / 64 * 64);
        hipLaunchKernelGGL(k_lu_panel, dim3(1), dim3(lanes), 0, st, n, A, lda, j0, nb, ipiv, info);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (n > nb) {
            hipLaunchKernelGGL(k_lu_swap_trsm, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, n, A, lda, j0, nb,
                               ipiv);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        const int64_t m = n - j0 - nb;
        if (m > 0) {
            const unsigned tiles = unsigned((m + 63) / 64);
            hipLaunchKernelGGL(k_lu_gemm, dim3(tiles, tiles), dim3(256), 0, st, n, A, lda, j0, nb);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

hipError_t launch_lu_solve(int64_t n, const double* LU, int64_t lda, const int32_t* ipiv, double* b,
                           hipStream_t st) {
    if (n <= kLuThreads)
        hipLaunchKernelGGL(k_lu_solve_blocked, dim3(1), dim3(kLuThreads), 0, st, n, LU, lda, ipiv, b);
    else
        hipLaunchKernelGGL(k_lu_solve, dim3(1), dim3(kLuThreads), 0, st, n, LU, lda, ipiv, b);
    return hipGetLastError();
}

hipError_t launch_wake_shed(int dtype, int n_blades, int n_span, const void* gb, const int32_t* te, void* prev,
                            void* trailed, void* shed, hipStream_t st) {
    const int total = n_blades * (2 * n_span + 1);
    const int nb = (total + 255) / 256;
    const int nk = (n_blades * n_span + 255) / 256;
    if (dtype == kDtypeF64) {
        hipLaunchKernelGGL(k_wake_shed<double>, dim3(nb), dim3(256), 0, st, n_blades, n_span, (const double*)gb, te,
                           (double*)prev, (double*)trailed, (double*)shed);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_wake_keep<double>, dim3(nk), dim3(256), 0, st, n_blades * n_span, (const double*)gb, te,
                           (double*)prev);
    } else {
        hipLaunchKernelGGL(k_wake_shed<float>, dim3(nb), dim3(256), 0, st, n_blades, n_span, (const float*)gb, te,
                           (float*)prev, (float*)trailed, (float*)shed);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_wake_keep<float>, dim3(nk), dim3(256), 0, st, n_blades * n_span, (const float*)gb, te,
                           (float*)prev);
    }
    return hipGetLastError();
}

size_t conv_workspace(int64_t n) { return ((size_t(n) * 4 + 255) / 256) * 256 + size_t(n + 1) * 8; }

hipError_t launch_wake_convert(int dtype, int64_t n, const void* a, const void* b, int64_t ld, const void* dg,
                               const int32_t* tip, int n_tip, int n_max, double sigma, int64_t capacity, void* xo,
                               void* go, void* so, int64_t ldo, int64_t* count, void* ws, hipStream_t st) {
    unsigned char* w = static_cast<unsigned char*>(ws);
    int32_t* cnt = reinterpret_cast<int32_t*>(w);
    int64_t* first = reinterpret_cast<int64_t*>(w + ((size_t(n) * 4 + 255) / 256) * 256);
    const unsigned nb = unsigned((n + 255) / 256);
    hipError_t e;
    if (n == 0) {  // no lines: only the zero total is written
        hipLaunchKernelGGL(k_conv_scan, dim3(1), dim3(1024), 0, st, n, cnt, first, count);
        return hipGetLastError();
    }
    if (dtype == kDtypeF64)
        hipLaunchKernelGGL(k_conv_count<double>, dim3(nb), dim3(256), 0, st, n, (const double*)a, (const double*)b, ld,
                           tip, n_tip, n_max, cnt);
    else
        hipLaunchKernelGGL(k_conv_count<float>, dim3(nb), dim3(256), 0, st, n, (const float*)a, (const float*)b, ld,
                           tip, n_tip, n_max, cnt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_conv_scan, dim3(1), dim3(1024), 0, st, n, cnt, first, count);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (dtype == kDtypeF64)
        hipLaunchKernelGGL(k_conv_emit<double>, dim3(nb), dim3(256), 0, st, n, (const double*)a, (const double*)b, ld,
                           (const double*)dg, cnt, first, sigma, capacity, (double*)xo, (double*)go, (double*)so, ldo);
    else
        hipLaunchKernelGGL(k_conv_emit<float>, dim3(nb), dim3(256), 0, st, n, (const float*)a, (const float*)b, ld,
                           (const float*)dg, cnt, first, sigma, capacity, (float*)xo, (float*)go, (float*)so, ldo);
    return hipGetLastError();
}

}  // namespace vpm

namespace vpm {

hipError_t launch_aic_update(int64_t n, const double* base, int64_t ldb, double* out, int64_t ldo, const double* col,
                             const double* nrm, int64_t ldc, int64_t m, const double* r00, const double* r01,
                             const double* r11, const double* r10, int64_t ldr, const int32_t* ring_of_col,
                             double rc, int vn, hipStream_t st) {
    AicUpdArgs a;
    a.n = n;
    a.base = base;
    a.out = out;
    a.ldb = ldb;
    a.ldo = ldo;
    a.col = col;
    a.nrm = nrm;
    a.ldc = ldc;
    a.r00 = r00;
    a.r01 = r01;
    a.r11 = r11;
    a.r10 = r10;
    a.ldr = ldr;
    a.ring_of_col = ring_of_col;
    a.m = m;
    a.vn = vn;
    a.inv_n = 1.0 / double(vn);
    a.rc2n = rc > 0.0 ? pow(rc * rc, double(vn)) : 0.0;
    hipLaunchKernelGGL(k_aic_update, dim3(unsigned((n + 255) / 256), unsigned(n)), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_neumann_rhs(int dtype, int64_t n, const double* col, const double* nrm, int64_t ldc, const void* u,
                              int64_t ldu, const double* vinf, const double* omega, double* rhs, hipStream_t st) {
    const unsigned nb = unsigned((n + 255) / 256);
    if (dtype == kDtypeF64)
        hipLaunchKernelGGL(k_neumann_rhs<double>, dim3(nb), dim3(256), 0, st, n, col, nrm, ldc, (const double*)u, ldu,
                           vinf[0], vinf[1], vinf[2], omega[0], omega[1], omega[2], rhs);
    else
        hipLaunchKernelGGL(k_neumann_rhs<float>, dim3(nb), dim3(256), 0, st, n, col, nrm, ldc, (const float*)u, ldu,
                           vinf[0], vinf[1], vinf[2], omega[0], omega[1], omega[2], rhs);
    return hipGetLastError();
}

}  // namespace vpm
