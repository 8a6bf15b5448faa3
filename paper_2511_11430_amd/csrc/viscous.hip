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
// Layout and schedule (PSE)
//  The work is proportional to the number of pairs whose boxes are near, so it depends on how
//  compact each group of consecutive particles is.  Callers may hand particles in any order
//  (shedding order interleaves far-apart particles), so every set is first put in Morton order
//  inside the workspace:
//   1. k_tile_box + k_bbox: bounding box of the set;
//   2. k_morton: 30-bit Morton code of each position on cubic cells of that box,
//      key = code << 32 | index;
//   3. bitonic sort of the keys (deterministic: the index breaks ties);
//   4. k_pack: one 12-value record per particle in sorted order
//      (x, y, z, sigma^2/2 | omega = Gamma/V, V | (nu + nu_t)/2, 0, 0, 0);
//   5. k_sub_box: bounding box and largest sigma^2/2 of every 64 records (and of every 256);
//   6. k_pse: one wavefront per 64 sorted targets, independent of the other wavefronts (no
//      workgroup barrier).  It skips 256-record tiles and then 64-record subtiles that are out of
//      reach of its own box (boxes read with scalar loads, the next tile's ahead of its test),
//      stages each remaining subtile into its own LDS slot with one coalesced load, and reads the
//      records from there by broadcast.  Pairs outside the cut take no transcendental.  FP32
//      sums are folded into two-sum pairs after every subtile; the epilogue runs in FP64 and
//      writes each result to the particle's original index.
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

// Bounding box of a set from its tile boxes (one workgroup).
template <typename T>
__global__ __launch_bounds__(256) void k_bbox(const T* __restrict__ tiles, int64_t ntiles, T* __restrict__ bb) {
    __shared__ T scratch[7 * 4];
    T lo[3], hi[3];
    for (int c = 0; c < 3; ++c) {
        lo[c] = tiles[c];
        hi[c] = tiles[3 + c];
    }
    for (int64_t t = threadIdx.x; t < ntiles; t += blockDim.x) {
        for (int c = 0; c < 3; ++c) {
            lo[c] = fmin(lo[c], tiles[8 * t + c]);
            hi[c] = fmax(hi[c], tiles[8 * t + 3 + c]);
        }
    }
    T olo[3], ohi[3], ocut;
    block_box(lo, hi, T(0), olo, ohi, ocut, scratch);
    if (threadIdx.x == 0) {
        for (int c = 0; c < 3; ++c) {
            bb[c] = olo[c];
            bb[3 + c] = ohi[c];
        }
    }
}

// Spread the low 10 bits of v to every third bit.
__device__ __forceinline__ uint32_t spread3(uint32_t v) {
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

template <typename T>
__global__ __launch_bounds__(256) void k_morton(const T* __restrict__ x, int64_t ld, int64_t begin, int64_t n,
                                                const T* __restrict__ bb, uint64_t* __restrict__ keys, int64_t P) {
    const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= P) return;
    if (p >= n) {
        keys[p] = ~0ull;  // padding sorts last
        return;
    }
    // cubic cells (one edge length for the three axes), so that the curve's locality holds in space
    double ext = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) ext = fmax(ext, double(bb[3 + c]) - double(bb[c]));
    uint32_t code = 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double q = ext > 0.0 ? (double(x[c * ld + begin + p]) - double(bb[c])) / ext * 1024.0 : 0.0;
        q = q < 0.0 ? 0.0 : (q > 1023.0 ? 1023.0 : q);
        code |= spread3(uint32_t(q)) << c;
    }
    keys[p] = (uint64_t(code) << 32) | uint64_t(p);
}

// Bitonic sort of P (a power of two, >= 1024) keys, ascending.  Global step: pairs (i, i + j)
// for j >= 1024; local steps: one workgroup sorts networks inside 1024 consecutive keys in LDS.
__global__ __launch_bounds__(256) void k_bitonic_global(uint64_t* __restrict__ a, int64_t P, int64_t j, int64_t k) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= P / 2) return;
    const int64_t i = 2 * j * (t / j) + (t % j);
    const int64_t l = i + j;
    const bool up = (i & k) == 0;
    const uint64_t ai = a[i], al = a[l];
    if ((ai > al) == up) {
        a[i] = al;
        a[l] = ai;
    }
}

__global__ __launch_bounds__(512) void k_bitonic_local(uint64_t* __restrict__ a, int64_t k_lo, int64_t k_hi,
                                                       int64_t j_first) {
    __shared__ uint64_t s[1024];
    const int64_t base = int64_t(blockIdx.x) * 1024;
    const int t = threadIdx.x;
    s[t] = a[base + t];
    s[t + 512] = a[base + t + 512];
    for (int64_t k = k_lo; k <= k_hi; k <<= 1) {
        for (int64_t j = (k == k_lo ? j_first : k >> 1); j > 0; j >>= 1) {
            __syncthreads();
            const int i = int(2 * j * (t / j) + (t % j));
            const int l = i + int(j);
            const bool up = ((base + i) & k) == 0;
            const uint64_t ai = s[i], al = s[l];
            if ((ai > al) == up) {
                s[i] = al;
                s[l] = ai;
            }
        }
    }
    __syncthreads();
    a[base + t] = s[t];
    a[base + t + 512] = s[t + 512];
}

template <typename T>
struct alignas(16) PseRec {
    T x, y, z, h;      // position, sigma^2 / 2
    T wx, wy, wz, v;   // omega = Gamma / V, V
    T nu, p0, p1, p2;  // (nu + nu_t) / 2
};

template <typename T>
__global__ __launch_bounds__(256) void k_pack(const T* __restrict__ x, const T* __restrict__ g,
                                              const T* __restrict__ sg, const T* __restrict__ vol,
                                              const T* __restrict__ nut, int64_t ld, int64_t begin, int64_t n,
                                              double nu, const uint64_t* __restrict__ keys,
                                              PseRec<T>* __restrict__ rec) {
    const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= n) return;
    uint64_t li = keys[p] & 0xffffffffull;
    if (li >= uint64_t(n)) li = 0;  // never taken after a correct sort; keeps every read in bounds
    const int64_t j = begin + int64_t(li);
    const T vj = vol[j];
    const T ivj = T(1) / vj;
    const T sj = sg[j];
    PseRec<T> r;
    r.x = x[j];
    r.y = x[ld + j];
    r.z = x[2 * ld + j];
    r.h = T(0.5) * sj * sj;
    r.wx = g[j] * ivj;
    r.wy = g[ld + j] * ivj;
    r.wz = g[2 * ld + j] * ivj;
    r.v = vj;
    r.nu = T(0.5 * nu) + (nut ? T(0.5) * nut[j] : T(0));
    r.p0 = r.p1 = r.p2 = T(0);
    rec[p] = r;
}

// Boxes of every 64 records (subtile) and every 256 records (tile) of the sorted set.
template <typename T>
__global__ __launch_bounds__(256) void k_sub_box(const PseRec<T>* __restrict__ rec, int64_t n, T* __restrict__ sub,
                                                 T* __restrict__ tile) {
    __shared__ T scratch[7 * 4];
    const int64_t p0 = int64_t(blockIdx.x) * 256;
    const int64_t ps = p0 + (threadIdx.x & ~63);  // first record of this lane's subtile
    const int64_t p = p0 + threadIdx.x;
    const int64_t pp = p < n ? p : (ps < n ? ps : p0);
    const PseRec<T> r = rec[pp];
    const T lo[3] = {r.x, r.y, r.z};
    T wl[3], wh[3], wc;
    wave_box(lo, lo, r.h, wl, wh, wc);
    const int64_t st = p0 / 64 + (threadIdx.x >> 6);
    if ((threadIdx.x & 63) == 0 && ps < n) {
        T* b = sub + 8 * st;
        for (int c = 0; c < 3; ++c) {
            b[c] = wl[c];
            b[3 + c] = wh[c];
        }
        b[6] = wc;
        b[7] = T(0);
    }
    T tl[3], th[3], tc;
    block_box(wl, wh, wc, tl, th, tc, scratch);
    if (threadIdx.x == 0) {
        T* b = tile + 8 * int64_t(blockIdx.x);
        for (int c = 0; c < 3; ++c) {
            b[c] = tl[c];
            b[3 + c] = th[c];
        }
        b[6] = tc;
        b[7] = T(0);
    }
}

struct PseArgs {
    const void* rec;
    const void* sub;
    const void* tile;
    const uint64_t* keys;
    int64_t begin, n;
    void* dg;
    int64_t ldo;
    int32_t accumulate;
};

template <typename T>
__device__ __forceinline__ bool box_near(const T* b, const T (&lo)[3], const T (&hi)[3], T h, T far2) {
    T d2 = T(0);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const T gap = fmax(fmax(b[c] - hi[c], lo[c] - b[3 + c]), T(0));
        d2 += gap * gap;
    }
    return d2 < far2 * (b[6] + h);
}

template <typename T>
__global__ __launch_bounds__(256) void k_pse(PseArgs a) {
    using CT = __attribute__((address_space(4))) const T*;
    constexpr bool kComp = std::is_same<T, float>::value;
    using V4 = typename std::conditional<kComp, float4, double4>::type;
    // each wavefront stages the 64 records of one near subtile at a time in its own slot
    __shared__ V4 lrec[4][64][3];
    const T far2 = T(Prec<T>::kFarRho2);
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const int64_t p0 = (int64_t(blockIdx.x) * 4 + wave) * 64;
    if (p0 >= a.n) return;  // the whole wavefront
    const int lane = threadIdx.x & 63;
    const int64_t p = p0 + lane;
    const bool valid = p < a.n;
    const V4* grec = static_cast<const V4*>(a.rec);  // record r = grec[3r .. 3r+2]
    const int64_t pm = valid ? p : p0;
    const V4 m0 = grec[3 * pm], m1 = grec[3 * pm + 1], m2 = grec[3 * pm + 2];
    const T xi = m0.x, yi = m0.y, zi = m0.z, hi_ = m0.w;
    const T wxi = m1.x, wyi = m1.y, wzi = m1.z, vi = m1.w, nui = m2.x;
    const CT csub = (CT)(static_cast<const T*>(a.sub));
    const CT ctile = (CT)(static_cast<const T*>(a.tile));
    V4(*buf)[3] = lrec[wave];

    T blo[3], bhi[3], bh;
    {
        const T lo3[3] = {xi, yi, zi};
        wave_box(lo3, lo3, hi_, blo, bhi, bh);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            blo[c] = uniform(blo[c]);
            bhi[c] = uniform(bhi[c]);
        }
        bh = uniform(bh);
    }
    T acc[3] = {T(0), T(0), T(0)}, shi[3] = {T(0), T(0), T(0)}, slo[3] = {T(0), T(0), T(0)};
    const int64_t ntiles = (a.n + 255) / 256;
    const int64_t nsub = (a.n + 63) / 64;
    T tb[7];
#pragma unroll
    for (int c = 0; c < 7; ++c) tb[c] = ctile[c];
    for (int64_t tt = 0; tt < ntiles; ++tt) {
        // the next tile's box is read before this one is tested
        const int64_t tn = tt + 1 < ntiles ? tt + 1 : tt;
        T nb[7];
#pragma unroll
        for (int c = 0; c < 7; ++c) nb[c] = ctile[8 * tn + c];
        if (box_near(tb, blo, bhi, bh, far2)) {
            const int64_t s1 = (4 * tt + 4) < nsub ? (4 * tt + 4) : nsub;
            for (int64_t st = 4 * tt; st < s1; ++st) {
                T sb[7];
#pragma unroll
                for (int c = 0; c < 7; ++c) sb[c] = csub[8 * st + c];
                if (!box_near(sb, blo, bhi, bh, far2)) continue;
                const int64_t j0 = st * 64;
                const int cnt = int(a.n - j0 < 64 ? a.n - j0 : 64);
                // stage: lane l brings record j0 + l (coalesced), then the wavefront reads them all
                if (lane < cnt) {
                    const V4* r = grec + 3 * (j0 + lane);
                    buf[lane][0] = r[0];
                    buf[lane][1] = r[1];
                    buf[lane][2] = r[2];
                }
                __builtin_amdgcn_wave_barrier();
                for (int jj = 0; jj < cnt; ++jj) {
                    const V4 q0 = buf[jj][0];
                    const T rx = xi - q0.x, ry = yi - q0.y, rz = zi - q0.z;
                    const T s2 = rx * rx + ry * ry + rz * rz;
                    const T sij2 = hi_ + q0.w;  // sigma_ij^2
                    if (s2 < far2 * sij2) {
                        const V4 q1 = buf[jj][1];
                        const T nuj = buf[jj][2].x;
                        const T inv = rcp_fast(sij2);          // 1 / sigma_ij^2
                        const T e = dexp(T(-0.5) * s2 * inv);  // exp(-s^2 / (2 sigma_ij^2))
                        const T w = (nui + nuj) * inv * inv * sqrt_fast(inv) * e * q1.w;
                        acc[0] += w * (q1.x - wxi);
                        acc[1] += w * (q1.y - wyi);
                        acc[2] += w * (q1.z - wzi);
                    }
                }
                __builtin_amdgcn_wave_barrier();  // every lane is done with the slot before it is refilled
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
#pragma unroll
        for (int c = 0; c < 7; ++c) tb[c] = nb[c];
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
        uint64_t li = a.keys[p] & 0xffffffffull;
        if (li >= uint64_t(a.n)) return;  // never taken after a correct sort
        const int64_t i = a.begin + int64_t(li);
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

// Workspace of one set of n particles (sets reuse it one after the other):
// [keys: P x 8 B][records: n x 12 T][subtile boxes: ceil(n/64) x 8 T][tile boxes: ceil(n/256) x 8 T][bbox: 8 T]
namespace {

size_t al256(size_t v) { return (v + 255) / 256 * 256; }
struct PseLayout {
    size_t keys, rec, sub, tile, bb, total;
};
PseLayout pse_layout(int64_t n, size_t es) {
    PseLayout L;
    L.keys = 0;
    L.rec = al256(size_t(sort_len(n)) * 8);
    L.sub = L.rec + al256(size_t(n) * 12 * es);
    L.tile = L.sub + al256(size_t((n + 63) / 64) * 8 * es);
    L.bb = L.tile + al256(size_t((n + 255) / 256) * 8 * es);
    L.total = L.bb + al256(8 * es);
    return L;
}

template <typename T>
hipError_t pse_set(int64_t begin, int64_t end, const T* x, const T* g, const T* sg, const T* vol, const T* nut,
                   int64_t ld, double nu, T* dg, int64_t ldo, int accumulate, unsigned char* ws, hipStream_t st) {
    const int64_t n = end - begin;
    const PseLayout L = pse_layout(n, sizeof(T));
    uint64_t* keys = reinterpret_cast<uint64_t*>(ws + L.keys);
    PseRec<T>* rec = reinterpret_cast<PseRec<T>*>(ws + L.rec);
    T* sub = reinterpret_cast<T*>(ws + L.sub);
    T* tile = reinterpret_cast<T*>(ws + L.tile);
    T* bb = reinterpret_cast<T*>(ws + L.bb);
    const int64_t ntiles = (n + 255) / 256;
    const int64_t P = sort_len(n);
    hipLaunchKernelGGL(k_tile_box<T>, dim3(unsigned(ntiles)), dim3(kTile), 0, st, x, sg, ld, begin, end, tile);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bbox<T>, dim3(1), dim3(256), 0, st, tile, ntiles, bb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_morton<T>, dim3(unsigned(P / 256)), dim3(256), 0, st, x, ld, begin, n, bb, keys, P);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = sort_keys(keys, P, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_pack<T>, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, x, g, sg, vol, nut, ld, begin, n,
                       nu, keys, rec);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_sub_box<T>, dim3(unsigned(ntiles)), dim3(256), 0, st, rec, n, sub, tile);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    PseArgs a;
    a.rec = rec;
    a.sub = sub;
    a.tile = tile;
    a.keys = keys;
    a.begin = begin;
    a.n = n;
    a.dg = dg;
    a.ldo = ldo;
    a.accumulate = accumulate;
    hipLaunchKernelGGL(k_pse<T>, dim3(unsigned(ntiles)), dim3(256), 0, st, a);
    return hipGetLastError();
}
}  // namespace

int64_t sort_len(int64_t n) {
    int64_t P = 1024;
    while (P < n) P <<= 1;
    return P;
}

hipError_t sort_keys(uint64_t* keys, int64_t P, hipStream_t st) {
    hipLaunchKernelGGL(k_bitonic_local, dim3(unsigned(P / 1024)), dim3(512), 0, st, keys, int64_t(2), int64_t(1024),
                       int64_t(1));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    for (int64_t k = 2048; k <= P; k <<= 1) {
        for (int64_t j = k >> 1; j >= 1024; j >>= 1) {
            hipLaunchKernelGGL(k_bitonic_global, dim3(unsigned(P / 2 / 256)), dim3(256), 0, st, keys, P, j, k);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        hipLaunchKernelGGL(k_bitonic_local, dim3(unsigned(P / 1024)), dim3(512), 0, st, keys, k, k, int64_t(512));
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

size_t pse_workspace(int64_t n, int dtype) {
    return pse_layout(n, dtype == kDtypeF64 ? sizeof(double) : sizeof(float)).total;
}

hipError_t launch_pse(int dtype, int64_t begin, int64_t end, const void* x, const void* g, const void* sg,
                      const void* vol, const void* nut, int64_t ld, double nu, void* dg, int64_t ldo,
                      int accumulate, void* ws, hipStream_t st) {
    if (end <= begin) return hipSuccess;
    unsigned char* w = static_cast<unsigned char*>(ws);
    if (dtype == kDtypeF64)
        return pse_set<double>(begin, end, (const double*)x, (const double*)g, (const double*)sg, (const double*)vol,
                               (const double*)nut, ld, nu, (double*)dg, ldo, accumulate, w, st);
    return pse_set<float>(begin, end, (const float*)x, (const float*)g, (const float*)sg, (const float*)vol,
                          (const float*)nut, ld, nu, (float*)dg, ldo, accumulate, w, st);
}

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
