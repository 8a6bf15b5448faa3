// Cartesian fast multipole evaluation of the particle right-hand side (Fu & Laurendeau,
// Sec. II.B: a Cartesian FMM accelerates the velocity and its gradient for the particles).
//
// Far field.  Beyond about seven core radii the Gaussian blob acts as a point vortex (the
// weights differ by less than 2e-9), so well-separated cells interact through the vector
// potential of the singular kernel,
//   psi(y) = sum_j Gamma_j G(y - x_j),  G(r) = 1/(4 pi |r|),
//   u = curl psi,   J_ae = du_a/dy_e = eps_abc d_e d_b psi_c,
// stretching J^T Gamma_i (transposed) or J Gamma_i (classical).  Each cell carries Taylor
// moments of total order p about its centre c,
//   M_k = sum_j Gamma_j (x_j - c)^k / k!,
// shifted to the parent by M_k(c') = sum_{m<=k} M_m(c) (c - c')^(k-m)/(k-m)!, converted to
// local coefficients of a well-separated target cell t,
//   L_n = sum_{|k| <= p - |n|} (-1)^|k| d^(n+k) G (c_t - c_s) M_k,
// shifted down by L_n(c') = sum_{m >= n} L_m(c) (c' - c)^(m-n)/(m-n)!, and evaluated at a
// particle as d_b psi = sum_n L_(n+e_b) a^n/n!, d_e d_b psi = sum_n L_(n+e_b+e_e) a^n/n!.
//
// Tree.  A uniform octree of depth `level` over the particles' bounding cube (centre of the
// box, half of its largest extent): every particle goes to the leaf floor((x - corner)/w),
// clamped to the grid.  Leaves interact directly with their 27 neighbours through the exact
// Gaussian kernel (the pair arithmetic of the direct kernel, self pair excluded); from level
// 2 down every cell receives the moments of the children of its parent's neighbours that
// are not its own neighbours.  Only occupied cells exist: particles are sorted by the Morton
// code of their leaf, and each level's cells are the distinct code prefixes, found by
// segmented scans on the device; neighbours are found by binary search in the sorted codes.
//
// Derivatives of 1/r.  With phi = 1/|R|, r^2 d_i phi + R_i phi = 0; applying d^(n - e_i)
// and Leibniz's rule gives, for any i with n_i >= 1,
//   r^2 D_n = -[(2 n_i - 1) R_i D_(n-e_i) + sum_(j != i) 2 n_j R_j D_(n-e_j)
//               + (n_i - 1)^2 D_(n-2e_i) + sum_(j != i) n_j (n_j - 1) D_(n-2e_j)],
// computed degree by degree.  D of the offset Delta w equals w^(-1-|n|) D of Delta, so one
// table for unit spacing (offsets in [-3, 3]^3) serves every level; M2L scales the source
// moments by (-1/w)^|k| and the result by w^(-1-|n|)/(4 pi).
//
// Precision: expansions and the far field in FP64; the near field in the caller's type
// (FP32 with per-tile two-sum folding, or FP64), summed in FP64 at the end.
#include <hip/hip_runtime.h>

#include "device_math.h"

// The FP64 kernels call their in-core weights (a convergent call), and clang then reports the
// unroll requests of the loops around that call as not honoured.
#pragma clang diagnostic ignored "-Wpass-failed"
#include "vpm_internal.h"

namespace vpm {

namespace {

constexpr int kMaxOrder = 20;
constexpr int kMaxTerms = (kMaxOrder + 1) * (kMaxOrder + 2) * (kMaxOrder + 3) / 6;  // 1771
// terms per lane in the kernels whose 256 lanes own the terms t = lane + 256 j
constexpr int kSlots = (kMaxTerms + 255) / 256;  // 7
constexpr int kMaxLevel = 10;
// how far the M2L's batches of eight scalar loads can read past a cell's last moment
constexpr int kM2lOverrun = 8;
constexpr int kNearTile = 256;
constexpr int kOffsets = 343;  // [-3, 3]^3
constexpr double kInv4Pi = 0.0795774715459476678844418816862571810;
// 1/k for the monomial recurrences a^k/k! = (a^(k-1)/(k-1)!) a (1/k) (a multiply, not an FP64
// division, in the per-particle loops)
__constant__ double kInvInt[kMaxOrder + 2] = {0.0,      1.0,      1.0 / 2,  1.0 / 3,  1.0 / 4,  1.0 / 5,
                                              1.0 / 6,  1.0 / 7,  1.0 / 8,  1.0 / 9,  1.0 / 10, 1.0 / 11,
                                              1.0 / 12, 1.0 / 13, 1.0 / 14, 1.0 / 15, 1.0 / 16, 1.0 / 17,
                                              1.0 / 18, 1.0 / 19, 1.0 / 20, 1.0 / 21};

__host__ __device__ constexpr int nterms(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }

// Position of the multi-index (a, b, c): by total degree d, then decreasing a, then
// decreasing b.  Terms of degree < d: d(d+1)(d+2)/6; with e = d - a, the terms of degree d
// before a: e(e+1)/2; within a: e - b.
__device__ __forceinline__ int mpos(int a, int b, int c) {
    const int d = a + b + c;
    const int e = d - a;
    return d * (d + 1) * (d + 2) / 6 + e * (e + 1) / 2 + (e - b);
}

__device__ __forceinline__ uint32_t spread_bits(uint32_t v) {
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}
__device__ __forceinline__ uint32_t gather_bits(uint32_t v) {
    v &= 0x09249249u;
    v = (v | (v >> 2)) & 0x030c30c3u;
    v = (v | (v >> 4)) & 0x0300f00fu;
    v = (v | (v >> 8)) & 0x030000ffu;
    v = (v | (v >> 16)) & 0x3ffu;
    return v;
}
// x in the highest of each bit triple, z in the lowest: the parent's code is code >> 3.
__device__ __forceinline__ uint32_t cell_code(int ix, int iy, int iz) {
    return (spread_bits(uint32_t(ix)) << 2) | (spread_bits(uint32_t(iy)) << 1) | spread_bits(uint32_t(iz));
}
__device__ __forceinline__ void cell_coords(uint32_t code, int* i) {
    i[0] = int(gather_bits(code >> 2));
    i[1] = int(gather_bits(code >> 1));
    i[2] = int(gather_bits(code));
}

// box: corner[3], H, leaf width.  Centre of cell i at level l: corner + (i + 1/2) w_l, each
// operation rounded on its own.
__device__ __forceinline__ double cell_centre(const double* box, int d, int i, int l) {
    const double w = ldexp(2.0 * box[3], -l);
    return __dadd_rn(box[d], __dmul_rn(double(i) + 0.5, w));
}

// Index of `key` in the ascending codes[0, n), or -1.
__device__ __forceinline__ int find_code(const uint32_t* codes, int n, uint32_t key) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (codes[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return (lo < n && codes[lo] == key) ? lo : -1;
}

struct FmmLevel {
    uint32_t* code;    // [cap]
    int32_t* first;    // [cap + 1]: first particle (leaves) or first child (inner levels)
    int32_t* pstart;   // [cap + 1]: first particle of the cell
    int32_t* parent;   // [cap]: parent index (levels >= 1)
    double* M;         // [cap][3][nt]
    double* L;         // [cap][3][nt]
    int64_t cap;
};

// ---------------------------------------------------------------- tree
constexpr int kBoxParts = 1024;   // most workgroups of the bounding-box reduction
constexpr int kScanChunk = 4096;  // leaf codes per workgroup of the leaf enumeration

// min and max of one value per lane over a workgroup of 256 (result valid in thread 0)
__device__ __forceinline__ void block_minmax6(double (&v)[6], double (*red)[4]) {
    for (int off = 32; off > 0; off >>= 1)
        for (int d = 0; d < 3; ++d) {
            v[d] = fmin(v[d], __shfl_xor(v[d], off));
            v[3 + d] = fmax(v[3 + d], __shfl_xor(v[3 + d], off));
        }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int c = 0; c < 6; ++c) red[c][wv] = v[c];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int w = 1; w < 4; ++w)
            for (int d = 0; d < 3; ++d) {
                v[d] = fmin(v[d], red[d][w]);
                v[3 + d] = fmax(v[3 + d], red[3 + d][w]);
            }
}

// Bounding box, first pass: each workgroup reduces a grid-strided share of the particles to
// part[c][blockIdx.x] (c = min x, y, z, max x, y, z).
template <typename T>
__global__ __launch_bounds__(256) void k_fmm_box_part(const T* __restrict__ x, int64_t ld, int64_t n,
                                                      double* __restrict__ part) {
    __shared__ double red[6][4];
    double v[6];
    for (int d = 0; d < 3; ++d) {
        v[d] = INFINITY;
        v[3 + d] = -INFINITY;
    }
    const int64_t stride = int64_t(gridDim.x) * 256;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += stride)
        for (int d = 0; d < 3; ++d) {
            const double xv = double(x[d * ld + i]);
            v[d] = fmin(v[d], xv);
            v[3 + d] = fmax(v[3 + d], xv);
        }
    block_minmax6(v, red);
    if (threadIdx.x == 0)
        for (int c = 0; c < 6; ++c) part[c * gridDim.x + blockIdx.x] = v[c];
}

// Second pass (one workgroup): the cube around the box, box = (corner[3], H, leaf width).
__global__ __launch_bounds__(256) void k_fmm_box(const double* __restrict__ part, int nparts, int level,
                                                 double* __restrict__ box) {
    __shared__ double red[6][4];
    double v[6];
    for (int d = 0; d < 3; ++d) {
        v[d] = INFINITY;
        v[3 + d] = -INFINITY;
    }
    for (int b = threadIdx.x; b < nparts; b += 256)
        for (int d = 0; d < 3; ++d) {
            v[d] = fmin(v[d], part[d * nparts + b]);
            v[3 + d] = fmax(v[3 + d], part[(3 + d) * nparts + b]);
        }
    block_minmax6(v, red);
    if (threadIdx.x == 0) {
        double H = 0.0, c[3];
        for (int d = 0; d < 3; ++d) {
            c[d] = 0.5 * (v[d] + v[3 + d]);
            H = fmax(H, 0.5 * (v[3 + d] - v[d]));
        }
        if (!(H > 0.0)) H = 1.0;
        for (int d = 0; d < 3; ++d) box[d] = c[d] - H;
        box[3] = H;
        box[4] = ldexp(2.0 * H, -level);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_fmm_keys(const T* __restrict__ x, int64_t ld, int64_t n, int level,
                                                  const double* __restrict__ box, uint64_t* __restrict__ keys,
                                                  int64_t P) {
    const int64_t p = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (p >= P) return;
    if (p >= n) {
        keys[p] = ~0ull;
        return;
    }
    // cells of the finest grid (1024 per axis): w_10 = w_level 2^-(10 - level) exactly, so
    // the quotient is the level's quotient times a power of two and its floor, shifted, is the
    // level's cell; sorting by the full code keeps the particles of a leaf in space order too
    const double w = ldexp(box[4], level - kMaxLevel);
    int ic[3];
    for (int d = 0; d < 3; ++d) {
        const double q = floor((double(x[d * ld + p]) - box[d]) / w);
        ic[d] = q < 0.0 ? 0 : (q >= 1024.0 ? 1023 : int(q));
    }
    keys[p] = (uint64_t(cell_code(ic[0], ic[1], ic[2])) << 32) | uint64_t(p);
}

template <typename T>
__global__ __launch_bounds__(256) void k_fmm_gather(const T* __restrict__ x, const T* __restrict__ g,
                                                    const T* __restrict__ sg, int64_t ld, int64_t n,
                                                    const uint64_t* __restrict__ keys, T* __restrict__ xs,
                                                    T* __restrict__ gs, T* __restrict__ ss, int32_t* __restrict__ perm,
                                                    uint32_t* __restrict__ lcode, int level) {
    const int64_t q = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (q >= n) return;
    const uint64_t k = keys[q];
    const int64_t i = int64_t(k & 0xffffffffull);
    for (int d = 0; d < 3; ++d) {
        xs[d * n + q] = x[d * ld + i];
        gs[d * n + q] = g[d * ld + i];
    }
    ss[q] = sg[i];
    perm[q] = int32_t(i);
    lcode[q] = uint32_t(k >> 32) >> (3 * (kMaxLevel - level));
}

// Distinct leaf codes of the sorted particles in three passes over workgroups of kScanChunk
// codes (the single-workgroup k_fmm_unique below serves the short inner levels).
// Pass 1: the number of segment starts (i = 0 or in[i] != in[i - 1]) in each chunk.
__global__ __launch_bounds__(256) void k_fmm_leaf_count(const uint32_t* __restrict__ in, int64_t n,
                                                        int32_t* __restrict__ bsum) {
    __shared__ int32_t red[4];
    const int64_t b0 = int64_t(blockIdx.x) * kScanChunk;
    int32_t cnt = 0;
    for (int k = 0; k < kScanChunk / 256; ++k) {
        const int64_t i = b0 + k * 256 + threadIdx.x;
        if (i < n && (i == 0 || in[i] != in[i - 1])) ++cnt;
    }
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) bsum[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// Pass 2 (one workgroup): exclusive scan of the chunk counts in place; the leaf count and
// first_out[count] = n.
__global__ __launch_bounds__(1024) void k_fmm_leaf_scan(int32_t* __restrict__ bsum, int64_t nb, int64_t n,
                                                        int32_t* __restrict__ first_out,
                                                        int32_t* __restrict__ count_out) {
    __shared__ int32_t part[1024];
    const int tid = threadIdx.x;
    int32_t carry = 0;
    for (int64_t base = 0; base < nb; base += 1024) {
        const int32_t v = base + tid < nb ? bsum[base + tid] : 0;
        part[tid] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int32_t w = tid >= off ? part[tid - off] : 0;
            __syncthreads();
            part[tid] += w;
            __syncthreads();
        }
        if (base + tid < nb) bsum[base + tid] = carry + part[tid] - v;
        carry += part[1023];
        __syncthreads();
    }
    if (tid == 0) {
        *count_out = carry;
        first_out[carry] = int32_t(n);
    }
}

// Pass 3: each chunk writes its segment starts at its scanned offset: code_out[seg] = code,
// first_out[seg] = first particle.  Thread t takes 16 consecutive codes of the chunk (staged
// in LDS with the code before the chunk).
__global__ __launch_bounds__(256) void k_fmm_leaf_scatter(const uint32_t* __restrict__ in, int64_t n,
                                                          const int32_t* __restrict__ boff,
                                                          uint32_t* __restrict__ code_out,
                                                          int32_t* __restrict__ first_out) {
    constexpr int kPer = kScanChunk / 256;
    __shared__ uint32_t sc[kScanChunk + 1];
    __shared__ int32_t wsum[4];
    const int64_t b0 = int64_t(blockIdx.x) * kScanChunk;
    const int tid = threadIdx.x;
    for (int k = 0; k < kPer; ++k) {
        const int64_t i = b0 + k * 256 + tid;
        sc[1 + k * 256 + tid] = i < n ? in[i] : 0u;
    }
    if (tid == 0) sc[0] = b0 > 0 ? in[b0 - 1] : ~in[0];  // code 0 always starts a segment
    __syncthreads();
    int32_t cnt = 0;
    for (int k = 0; k < kPer; ++k) {
        const int j = tid * kPer + k;
        if (b0 + j < n && sc[1 + j] != sc[j]) ++cnt;
    }
    // exclusive prefix of cnt over the workgroup
    int32_t incl = cnt;
    const int lane = tid & 63;
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t w = __shfl_up(incl, off);
        if (lane >= off) incl += w;
    }
    if (lane == 63) wsum[tid >> 6] = incl;
    __syncthreads();
    int32_t seg = boff[blockIdx.x] + incl - cnt;
    for (int w = 0; w < (tid >> 6); ++w) seg += wsum[w];
    for (int k = 0; k < kPer; ++k) {
        const int j = tid * kPer + k;
        if (b0 + j < n && sc[1 + j] != sc[j]) {
            code_out[seg] = sc[1 + j];
            first_out[seg] = int32_t(b0 + j);
            ++seg;
        }
    }
}

// Distinct values of in[i] >> shift over a sorted input (one workgroup): code_out, the first
// input index of each (first_out, with first_out[count] = n_in), each input's segment
// (seg_of, optional), the count, and the first particle of each (pstart_out, optional:
// pstart_child of the first member, pstart_out[count] = n_particles).
__global__ __launch_bounds__(1024) void k_fmm_unique(const uint32_t* __restrict__ in, const int32_t* __restrict__ n_dev,
                                                     int64_t n_host, int shift, uint32_t* __restrict__ code_out,
                                                     int32_t* __restrict__ first_out, int32_t* __restrict__ seg_of,
                                                     int32_t* __restrict__ count_out,
                                                     const int32_t* __restrict__ pstart_child,
                                                     int32_t* __restrict__ pstart_out, int32_t n_particles) {
    __shared__ int32_t part[1024];
    const int64_t n_in = n_dev ? int64_t(*n_dev) : n_host;
    const int tid = threadIdx.x;
    const int64_t chunk = (n_in + 1023) / 1024;
    const int64_t b = int64_t(tid) * chunk;
    const int64_t e = b + chunk < n_in ? b + chunk : n_in;
    int32_t cnt = 0;
    for (int64_t i = b; i < e; ++i)
        if (i == 0 || (in[i] >> shift) != (in[i - 1] >> shift)) ++cnt;
    part[tid] = cnt;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int32_t v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int32_t seg = part[tid] - cnt - 1;
    for (int64_t i = b; i < e; ++i) {
        if (i == 0 || (in[i] >> shift) != (in[i - 1] >> shift)) {
            ++seg;
            code_out[seg] = in[i] >> shift;
            first_out[seg] = int32_t(i);
            if (pstart_out) pstart_out[seg] = pstart_child ? pstart_child[i] : int32_t(i);
        }
        if (seg_of) seg_of[i] = seg;
    }
    if (tid == 1023) {
        const int32_t total = part[1023];
        *count_out = total;
        first_out[total] = int32_t(n_in);
        if (pstart_out) pstart_out[total] = n_particles;
    }
}

// Multi-index table: terms[t] = a | b << 8 | c << 16 for |n| <= p, and at terms[kMaxTerms + t]
// the index of term t on the (p + 1)^3 grid, (a Q + b) Q + c with Q = p + 1 (the grid index
// of n + k is the sum of those of n and k).
__global__ __launch_bounds__(64) void k_fmm_terms(int p, uint32_t* __restrict__ terms) {
    const int d = threadIdx.x;
    if (d > p) return;
    const int Q = p + 1;
    for (int a = d; a >= 0; --a)
        for (int b = d - a; b >= 0; --b) {
            const int c = d - a - b;
            terms[mpos(a, b, c)] = uint32_t(a) | (uint32_t(b) << 8) | (uint32_t(c) << 16);
            terms[kMaxTerms + mpos(a, b, c)] = uint32_t((a * Q + b) * Q + c);
        }
}

// D_n(Delta) of 1/|R| for unit spacing, |n| <= p, for the offsets in [-3, 3]^3 that are not
// neighbours (one workgroup per offset, one degree at a time).
__global__ __launch_bounds__(256) void k_fmm_dtab(int p, const uint32_t* __restrict__ terms, double* __restrict__ dtab) {
    const int o = blockIdx.x;
    const int R[3] = {o / 49 - 3, (o / 7) % 7 - 3, o % 7 - 3};
    if (abs(R[0]) <= 1 && abs(R[1]) <= 1 && abs(R[2]) <= 1) return;
    const int nt = nterms(p);
    double* D = dtab + int64_t(o) * nt;
    const double r2 = double(R[0] * R[0] + R[1] * R[1] + R[2] * R[2]);
    const double ir2 = 1.0 / r2;
    if (threadIdx.x == 0) D[0] = 1.0 / sqrt(r2);
    for (int d = 1; d <= p; ++d) {
        __syncthreads();
        const int t0 = d * (d + 1) * (d + 2) / 6;
        const int nd = (d + 1) * (d + 2) / 2;
        for (int t = t0 + int(threadIdx.x); t < t0 + nd; t += 256) {
            const uint32_t m = terms[t];
            const int n[3] = {int(m & 0xff), int((m >> 8) & 0xff), int(m >> 16)};
            const int i = n[0] > 0 ? 0 : (n[1] > 0 ? 1 : 2);
            double s = 0.0;
            for (int j = 0; j < 3; ++j) {
                if (n[j] == 0) continue;
                int q1[3] = {n[0], n[1], n[2]};
                q1[j] -= 1;
                const double c1 = (j == i) ? double(2 * n[i] - 1) : double(2 * n[j]);
                s += c1 * double(R[j]) * D[mpos(q1[0], q1[1], q1[2])];
                if (n[j] >= 2) {
                    int q2[3] = {n[0], n[1], n[2]};
                    q2[j] -= 2;
                    const double c2 = (j == i) ? double((n[i] - 1) * (n[i] - 1)) : double(n[j] * (n[j] - 1));
                    s += c2 * D[mpos(q2[0], q2[1], q2[2])];
                }
            }
            D[t] = -s * ir2;
        }
    }
}

// ---------------------------------------------------------------- upward pass
template <typename T>
__global__ __launch_bounds__(256) void k_fmm_p2m(const T* __restrict__ xs, const T* __restrict__ gs, int64_t n,
                                                 FmmLevel lv, const int32_t* __restrict__ count,
                                                 const double* __restrict__ box, int level, int p,
                                                 const uint32_t* __restrict__ terms) {
    const int cell = blockIdx.x;
    if (cell >= *count) return;
    const int nt = nterms(p);
    __shared__ double pw[64][3][kMaxOrder + 1];
    __shared__ double gg[64][3];
    int ic[3];
    cell_coords(lv.code[cell], ic);
    double c[3];
    for (int d = 0; d < 3; ++d) c[d] = cell_centre(box, d, ic[d], level);
    double acc[kSlots][3];
    for (int j = 0; j < kSlots; ++j)
        for (int d = 0; d < 3; ++d) acc[j][d] = 0.0;
    const int b0 = lv.pstart[cell], b1 = lv.pstart[cell + 1];
    for (int base = b0; base < b1; base += 64) {
        const int m = b1 - base < 64 ? b1 - base : 64;
        __syncthreads();
        if (int(threadIdx.x) < 3 * m) {
            const int q = threadIdx.x / 3, d = threadIdx.x % 3;
            const double a = double(xs[d * n + base + q]) - c[d];
            double v = 1.0;
            pw[q][d][0] = 1.0;
            for (int i = 1; i <= p; ++i) {
                v = v * a / double(i);
                pw[q][d][i] = v;
            }
            gg[q][d] = double(gs[d * n + base + q]);
        }
        __syncthreads();
        for (int j = 0; j < kSlots; ++j) {
            const int t = threadIdx.x + 256 * j;
            if (t >= nt) break;
            const uint32_t k = terms[t];
            const int k0 = int(k & 0xff), k1 = int((k >> 8) & 0xff), k2 = int(k >> 16);
            for (int q = 0; q < m; ++q) {
                const double mono = pw[q][0][k0] * pw[q][1][k1] * pw[q][2][k2];
                for (int d = 0; d < 3; ++d) acc[j][d] += gg[q][d] * mono;
            }
        }
    }
    for (int j = 0; j < kSlots; ++j) {
        const int t = threadIdx.x + 256 * j;
        if (t >= nt) break;
        for (int d = 0; d < 3; ++d) lv.M[(int64_t(cell) * 3 + d) * nt + t] = acc[j][d];
    }
    // the M2L's batched reads run up to kM2lOverrun terms past a cell's last moment: after the
    // level's last cell they find zeros, not memory that no cell writes
    if (cell == *count - 1 && int(threadIdx.x) < kM2lOverrun) lv.M[int64_t(cell + 1) * 3 * nt + threadIdx.x] = 0.0;
}

// One axis of a separable Taylor shift of 3 x nt coefficients (mpos order, [3][nt]) held in
// LDS, with pw[i] = dl^i / i! along axis ax.  Moments (UP = false):
//   out(k) = sum_{i <= k_ax} in(k - i e_ax) pw[i];
// local expansions (UP = true):
//   out(n) = sum_{i <= p - |n|} in(n + i e_ax) pw[i].
// The three-dimensional shift is the product of the three axes' (the shift factor dl^q/q! is
// a product over the axes), and each axis keeps the set |n| <= p.  The term t's result is
// returned in o[3] (t < nt).
template <bool UP>
__device__ __forceinline__ void shift_axis_term(const double* in, const double* pw, int ax, int p, int nt,
                                                uint32_t k, double (&o)[3]) {
    const int n[3] = {int(k & 0xff), int((k >> 8) & 0xff), int(k >> 16)};
    const int cnt = UP ? p - (n[0] + n[1] + n[2]) : n[ax];
    o[0] = o[1] = o[2] = 0.0;
    for (int i = 0; i <= cnt; ++i) {
        int m[3] = {n[0], n[1], n[2]};
        m[ax] += UP ? i : -i;
        const int s = mpos(m[0], m[1], m[2]);
        const double f = pw[i];
        o[0] += in[s] * f;
        o[1] += in[nt + s] * f;
        o[2] += in[2 * nt + s] * f;
    }
}
template <bool UP>
__device__ __forceinline__ void shift_axis(const double* in, double* out, const double* pw, int ax, int p, int nt,
                                           const uint32_t* __restrict__ terms) {
    for (int t = threadIdx.x; t < nt; t += blockDim.x) {
        double o[3];
        shift_axis_term<UP>(in, pw, ax, p, nt, terms[t], o);
        out[t] = o[0];
        out[nt + t] = o[1];
        out[2 * nt + t] = o[2];
    }
}

// Parents at level l from their children at level l + 1: each child's moments are shifted by
// dl = c_child - c_parent one axis at a time in LDS (dynamic: 2 x 3 nt doubles) and added.
__global__ __launch_bounds__(256) void k_fmm_m2m(FmmLevel par, FmmLevel chi, const int32_t* __restrict__ count, int l,
                                                 const double* __restrict__ box, int p,
                                                 const uint32_t* __restrict__ terms) {
    const int cell = blockIdx.x;
    if (cell >= *count) return;
    const int nt = nterms(p);
    extern __shared__ double sShift[];
    double* bufA = sShift;
    double* bufB = sShift + 3 * nt;
    __shared__ double pw[3][kMaxOrder + 1];
    const int c0 = par.first[cell], c1 = par.first[cell + 1];
    int ip[3];
    cell_coords(par.code[cell], ip);
    double acc[kSlots][3];
    for (int j = 0; j < kSlots; ++j)
        for (int d = 0; d < 3; ++d) acc[j][d] = 0.0;
    for (int q = c0; q < c1; ++q) {
        __syncthreads();
        if (threadIdx.x < 3) {
            const int d = threadIdx.x;
            int ic[3];
            cell_coords(chi.code[q], ic);
            const double dl = cell_centre(box, d, ic[d], l + 1) - cell_centre(box, d, ip[d], l);
            double v = 1.0;
            pw[d][0] = 1.0;
            for (int i = 1; i <= p; ++i) {
                v = v * dl / double(i);
                pw[d][i] = v;
            }
        }
        const double* Mc = chi.M + int64_t(q) * 3 * nt;
        for (int i = threadIdx.x; i < 3 * nt; i += 256) bufA[i] = Mc[i];
        __syncthreads();
        shift_axis<false>(bufA, bufB, pw[0], 0, p, nt, terms);
        __syncthreads();
        shift_axis<false>(bufB, bufA, pw[1], 1, p, nt, terms);
        __syncthreads();
        for (int j = 0; j < kSlots; ++j) {
            const int t = threadIdx.x + 256 * j;
            if (t >= nt) break;
            double o[3];
            shift_axis_term<false>(bufA, pw[2], 2, p, nt, terms[t], o);
            for (int d = 0; d < 3; ++d) acc[j][d] += o[d];
        }
    }
    for (int j = 0; j < kSlots; ++j) {
        const int t = threadIdx.x + 256 * j;
        if (t >= nt) break;
        for (int d = 0; d < 3; ++d) par.M[(int64_t(cell) * 3 + d) * nt + t] = acc[j][d];
    }
    // zeros after the level's last cell for the M2L's batched reads (as in k_fmm_p2m)
    if (cell == *count - 1 && int(threadIdx.x) < kM2lOverrun) par.M[int64_t(cell + 1) * 3 * nt + threadIdx.x] = 0.0;
}

// ---------------------------------------------------------------- M2L and L2L
// LDS of one M2L group in doubles: the (p + 1)^3 grid and its zero; with MLDS also the source
// cell's moments (3 nt, and kM2lOverrun zeros after them) and the grid index of every term (nt,
// and kM2lOverrun more, as ints).  At least 3 nt for the group's sums at the end.
__host__ __device__ inline int m2l_group_doubles(int p, bool mlds) {
    const int nt = nterms(p);
    int g = (p + 1) * (p + 1) * (p + 1) + 1;
    if (mlds) g += 3 * nt + kM2lOverrun + (nt + kM2lOverrun + 1) / 2;
    return g > 3 * nt ? g : 3 * nt;
}

// Work units of the high-order M2L (orders whose grid fills the LDS, one group per cell).
// The terms n are cut into blocks of 64 (one wavefront's lanes, in degree order); block b's
// lanes walk the same k, up to the prefix length of its lowest-degree term.  Those walks are
// very uneven (at order 18 from 1330 steps for the first block down to 1), so each block's walk
// is cut into pieces, and the pieces are dealt to the wavefronts longest first (each to the
// least loaded wavefront with a free slot).  A piece is (block, k0, k1); the partial sums of a
// block's pieces are added in k order at the end.  Built on the host, passed by value.
constexpr int kUnitWaves = 16;                       // 1024 lanes
constexpr int kUnitSlots = 4;                        // pieces per wavefront
constexpr int kMaxUnits = kUnitWaves * kUnitSlots;   // 64
constexpr int kMaxBlocks = (kMaxTerms + 63) / 64;    // 28
struct M2lUnits {
    int16_t blk[kMaxUnits], k0[kMaxUnits], k1[kMaxUnits];  // pieces, sorted by (block, k0)
    int8_t wave_unit[kMaxUnits];                            // [wave * kUnitSlots + slot]: piece or -1
    int16_t first[kMaxBlocks + 1];                          // pieces of block b: [first[b], first[b + 1])
    int32_t n;                                              // number of pieces
};

// Degree of term t in the degree order (terms of degree d: (d + 1)(d + 2)/2 of them).
inline int term_degree_host(int t) {
    int d = 0;
    while (t >= (d + 1) * (d + 2) / 2) {
        t -= (d + 1) * (d + 2) / 2;
        ++d;
    }
    return d;
}

// Returns false when the order's walks do not fit kUnitWaves x kUnitSlots pieces.
inline bool m2l_units(int p, M2lUnits& u) {
    const int nt = nterms(p);
    const int nblk = (nt + 63) / 64;
    if (nblk > kMaxBlocks) return false;
    int steps[kMaxBlocks];
    int smax = 0;
    for (int b = 0; b < nblk; ++b) {
        steps[b] = nterms(p - term_degree_host(64 * b));
        smax = steps[b] > smax ? steps[b] : smax;
    }
    struct Piece { int len, b, k0, k1; };
    long best = -1;
    for (int umax = 8; umax <= smax + 8; umax += 8) {
        Piece pc[kMaxUnits];
        int np = 0;
        bool fits = true;
        for (int b = 0; b < nblk && fits; ++b) {
            const int parts = (steps[b] + umax - 1) / umax;
            int len = (steps[b] + parts - 1) / parts;
            len = (len + 7) / 8 * 8;
            for (int k = 0; k < steps[b]; k += len) {
                if (np == kMaxUnits) {
                    fits = false;
                    break;
                }
                const int k1 = k + len < steps[b] ? k + len : steps[b];
                pc[np++] = Piece{k1 - k, b, k, k1};
            }
        }
        if (!fits) continue;
        // longest first; ties in (block, k0) order
        for (int i = 1; i < np; ++i)
            for (int j = i; j > 0; --j) {
                const Piece& a = pc[j - 1];
                const Piece& c = pc[j];
                const bool swap = c.len > a.len || (c.len == a.len && (c.b < a.b || (c.b == a.b && c.k0 < a.k0)));
                if (!swap) break;
                const Piece t = pc[j - 1];
                pc[j - 1] = pc[j];
                pc[j] = t;
            }
        long load[kUnitWaves] = {};
        int cnt[kUnitWaves] = {};
        int owner[kMaxUnits], slot[kMaxUnits];
        for (int i = 0; i < np && fits; ++i) {
            int w = -1;
            for (int c = 0; c < kUnitWaves; ++c)
                if (cnt[c] < kUnitSlots && (w < 0 || load[c] < load[w])) w = c;
            if (w < 0) {
                fits = false;
                break;
            }
            owner[i] = w;
            slot[i] = cnt[w]++;
            load[w] += pc[i].len;
        }
        if (!fits) continue;
        // wavefronts share a SIMD four ways (wavefront w on SIMD w % 4)
        long score = 0;
        for (int sm = 0; sm < 4; ++sm) {
            long l = 0;
            for (int w = sm; w < kUnitWaves; w += 4) l += load[w];
            score = l > score ? l : score;
        }
        if (best >= 0 && score >= best) continue;
        best = score;
        // store sorted by (block, k0)
        int order[kMaxUnits];
        for (int i = 0; i < np; ++i) order[i] = i;
        for (int i = 1; i < np; ++i)
            for (int j = i; j > 0; --j) {
                const Piece& a = pc[order[j - 1]];
                const Piece& c = pc[order[j]];
                if (c.b < a.b || (c.b == a.b && c.k0 < a.k0)) {
                    const int t = order[j - 1];
                    order[j - 1] = order[j];
                    order[j] = t;
                } else {
                    break;
                }
            }
        for (int i = 0; i < kMaxUnits; ++i) u.wave_unit[i] = -1;
        for (int i = 0; i < np; ++i) {
            const Piece& c = pc[order[i]];
            u.blk[i] = int16_t(c.b);
            u.k0[i] = int16_t(c.k0);
            u.k1[i] = int16_t(c.k1);
            u.wave_unit[owner[order[i]] * kUnitSlots + slot[order[i]]] = int8_t(i);
        }
        for (int b = 0, i = 0; b <= nblk; ++b) {
            while (i < np && u.blk[i] < b) ++i;
            u.first[b] = int16_t(i);
        }
        u.n = np;
    }
    return best >= 0;
}

typedef __attribute__((address_space(4))) const double* CDouble;
typedef __attribute__((address_space(4))) const uint32_t* CUint;

// One workgroup per target cell of level l: L = M2L over the interaction list (written, not
// added: the parent's shifted expansion is added afterwards by k_fmm_l2l).  With the
// unit-spacing table D of the offset and the cell width w,
//   L_n = w^(-1-|n|)/(4 pi) sum_k D_{n+k} (-1/w)^|k| M_k = (-1)^|n|/(4 pi w) sum_k D'_{n+k} M_k,
//   D'_m = (-1/w)^|m| D_m.
// The workgroup is G groups of glanes lanes (a multiple of 64); group g takes interactions
// g, g + G, ...  Each interaction's D' is staged in the group's LDS grid of (p + 1)^3 entries
// (plus one zero), where the index of n + k is the sum of the indices of n and k.  Lanes own
// terms n (t = lane + glanes j, j < SLOTS); the terms k with |k| <= p - |n| are a prefix of the
// degree order, so the lanes of a wavefront walk the same k, whose M_k and grid index are
// uniform (scalar loads), and a lane past its prefix reads the zero.  Per lane and k: one LDS
// read and three FMAs.  The groups' sums are added in group order at the end (deterministic).
// Low orders take several 256-lane groups (interactions in parallel).  High orders, whose grids
// fill the LDS, take one group of kUnitWaves wavefronts (MLDS), which also stages the source
// cell's moments and the terms' grid indices in LDS, so that the walk over k reads LDS (in
// order, pipelined) instead of waiting on a batch of scalar loads every eight steps; there the
// walks of the blocks of 64 terms are cut into pieces dealt evenly to the wavefronts
// (M2lUnits), and each term adds its pieces' partial sums in k order at the end.
template <int SLOTS, bool MLDS>
__global__ __launch_bounds__(1024) void k_fmm_m2l(FmmLevel lv, const int32_t* __restrict__ count, int l,
                                                  const double* __restrict__ box, int p,
                                                  const uint32_t* __restrict__ terms, const double* __restrict__ dtab,
                                                  int glanes, const M2lUnits units) {
    const int cell = blockIdx.x;
    const int ncell = *count;
    if (cell >= ncell) return;
    const int nt = nterms(p);
    const int ngroup = int(blockDim.x) / glanes;
    // the group is uniform over each wavefront (groups of whole wavefronts)
    const int grp = __builtin_amdgcn_readfirstlane(int(threadIdx.x) / glanes), gt = int(threadIdx.x) % glanes;
    const int gsize = (p + 1) * (p + 1) * (p + 1) + 1;  // grid + the zero
    const int gstride = m2l_group_doubles(p, MLDS);
    extern __shared__ double sDyn[];                    // ngroup grids; reused for the final sum
    double* sDg = sDyn + grp * gstride;
    double* sM = sDg + gsize;                                   // MLDS: [3][nt] + zeros
    int32_t* sG = reinterpret_cast<int32_t*>(sM + 3 * nt + kM2lOverrun);  // MLDS: [nt] + zeros
    __shared__ int32_t cand[216];
    __shared__ int32_t list_src[216];
    __shared__ int32_t list_off[216];
    __shared__ int32_t nlist;
    __shared__ double sc[kMaxOrder + 1];
    int ic[3];
    cell_coords(lv.code[cell], ic);
    const int side = 1 << l;
    const double w = ldexp(2.0 * box[3], -l);
    if (threadIdx.x < 216) {
        const int pn = threadIdx.x / 8, ch = threadIdx.x % 8;
        const int pc[3] = {(ic[0] >> 1) + pn / 9 - 1, (ic[1] >> 1) + (pn / 3) % 3 - 1, (ic[2] >> 1) + pn % 3 - 1};
        const int s[3] = {2 * pc[0] + (ch >> 2), 2 * pc[1] + ((ch >> 1) & 1), 2 * pc[2] + (ch & 1)};
        int idx = -1;
        const bool inside = pc[0] >= 0 && pc[1] >= 0 && pc[2] >= 0 && 2 * pc[0] < side && 2 * pc[1] < side &&
                            2 * pc[2] < side;
        const bool adjacent = abs(s[0] - ic[0]) <= 1 && abs(s[1] - ic[1]) <= 1 && abs(s[2] - ic[2]) <= 1;
        if (inside && !adjacent) idx = find_code(lv.code, ncell, cell_code(s[0], s[1], s[2]));
        cand[threadIdx.x] = idx;
        if (idx >= 0)
            list_off[threadIdx.x] = (ic[0] - s[0] + 3) * 49 + (ic[1] - s[1] + 3) * 7 + (ic[2] - s[2] + 3);
    }
    if (threadIdx.x <= p) {
        // (-1/w)^k
        double v = 1.0;
        for (int k = 0; k < int(threadIdx.x); ++k) v *= -1.0 / w;
        sc[threadIdx.x] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int m = 0;
        for (int t = 0; t < 216; ++t)
            if (cand[t] >= 0) {
                list_src[m] = cand[t];
                list_off[m] = list_off[t];
                ++m;
            }
        nlist = m;
    }
    const CUint gidx = (CUint)(terms + kMaxTerms);
    const int zero_at = gsize - 1;  // the staging never writes there
    if (gt == 0) sDg[zero_at] = 0.0;
    if constexpr (MLDS) {
        for (int t = gt; t < nt + kM2lOverrun; t += glanes) sG[t] = t < nt ? int(terms[kMaxTerms + t]) : 0;
        if (gt < kM2lOverrun) sM[3 * nt + gt] = 0.0;
    }
    if constexpr (MLDS) {
        // one group of kUnitWaves wavefronts; wavefront w walks the pieces units.wave_unit[w][.]
        const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6), lane = int(threadIdx.x) & 63;
        int uid[kUnitSlots], nb[kUnitSlots], lim[kUnitSlots], k0[kUnitSlots], k1[kUnitSlots];
        double acc[kUnitSlots][3];
#pragma unroll
        for (int j = 0; j < kUnitSlots; ++j) {
            uid[j] = units.wave_unit[wave * kUnitSlots + j];
            nb[j] = 0;
            lim[j] = 0;
            k0[j] = 0;
            k1[j] = 0;
            if (uid[j] >= 0) {
                k0[j] = units.k0[uid[j]];
                k1[j] = units.k1[uid[j]];
                const int t = 64 * int(units.blk[uid[j]]) + lane;
                if (t < nt) {
                    const uint32_t k = terms[t];
                    const int dg = int(k & 0xff) + int((k >> 8) & 0xff) + int(k >> 16);
                    nb[j] = int(terms[kMaxTerms + t]);
                    const int c = nterms(p - dg);
                    lim[j] = c < k1[j] ? c : k1[j];
                }
            }
            for (int d = 0; d < 3; ++d) acc[j][d] = 0.0;
        }
        __syncthreads();
        for (int e = 0; e < nlist; ++e) {
            __syncthreads();
            {
                const double* D = dtab + int64_t(list_off[e]) * nt;
                for (int t = gt; t < nt; t += glanes) {
                    const uint32_t k = terms[t];
                    sDg[terms[kMaxTerms + t]] = D[t] * sc[int(k & 0xff) + int((k >> 8) & 0xff) + int(k >> 16)];
                }
                const double* Ms = lv.M + int64_t(list_src[e]) * 3 * nt;
                for (int t = gt; t < 3 * nt; t += glanes) sM[t] = Ms[t];
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < kUnitSlots; ++j) {
                // the piece's k range in batches of eight: the batch may read up to seven terms
                // past k1 (into the zeros after the staged moments and grid indices), and lanes
                // past their own limit read the zero after the grid
                for (int s0 = k0[j]; s0 < k1[j]; s0 += 8) {
                    int ks[8];
                    double m[3][8];
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        ks[i] = sG[s0 + i];
                        m[0][i] = sM[s0 + i];
                        m[1][i] = sM[nt + s0 + i];
                        m[2][i] = sM[2 * nt + s0 + i];
                    }
                    double Dv[8];
#pragma unroll
                    for (int i = 0; i < 8; ++i) Dv[i] = sDg[s0 + i < lim[j] ? nb[j] + ks[i] : zero_at];
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        acc[j][0] += Dv[i] * m[0][i];
                        acc[j][1] += Dv[i] * m[1][i];
                        acc[j][2] += Dv[i] * m[2][i];
                    }
                }
            }
        }
        // each piece's partial sums through LDS (64 lanes x 3 per piece), then every term adds
        // its block's pieces in k order
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kUnitSlots; ++j)
            if (uid[j] >= 0)
                for (int d = 0; d < 3; ++d) sDyn[(uid[j] * 64 + lane) * 3 + d] = acc[j][d];
        __syncthreads();
        for (int idx = threadIdx.x; idx < 3 * nt; idx += blockDim.x) {
            const int d = idx / nt, t = idx - d * nt;
            const int b = t >> 6, ln = t & 63;
            double v = 0.0;
            for (int q = units.first[b]; q < units.first[b + 1]; ++q) v += sDyn[(q * 64 + ln) * 3 + d];
            const uint32_t k = terms[t];
            const int dg = int(k & 0xff) + int((k >> 8) & 0xff) + int(k >> 16);
            const double f = ((dg & 1) ? -kInv4Pi : kInv4Pi) / w;
            lv.L[(int64_t(cell) * 3 + d) * nt + t] = v * f;
        }
        return;
    } else {
        int nb[SLOTS], cnt[SLOTS], smax[SLOTS], deg[SLOTS];
        double acc[SLOTS][3];
#pragma unroll
        for (int j = 0; j < SLOTS; ++j) {
            const int t = gt + glanes * j;
            nb[j] = 0;
            cnt[j] = 0;
            deg[j] = 0;
            if (t < nt) {
                const uint32_t k = terms[t];
                deg[j] = int(k & 0xff) + int((k >> 8) & 0xff) + int(k >> 16);
                nb[j] = int(terms[kMaxTerms + t]);
                cnt[j] = nterms(p - deg[j]);
            }
            // lane 0 of the wavefront owns its lowest degree, hence the longest prefix
            smax[j] = __builtin_amdgcn_readfirstlane(cnt[j]);
            for (int d = 0; d < 3; ++d) acc[j][d] = 0.0;
        }
        __syncthreads();
        const int rounds = (nlist + ngroup - 1) / ngroup;
        for (int r = 0; r < rounds; ++r) {
            const int e = r * ngroup + grp;
            const bool has = e < nlist;
            __syncthreads();
            if (has) {
                const double* D = dtab + int64_t(list_off[e]) * nt;
                for (int t = gt; t < nt; t += glanes) {
                    const uint32_t k = terms[t];
                    sDg[terms[kMaxTerms + t]] = D[t] * sc[int(k & 0xff) + int((k >> 8) & 0xff) + int(k >> 16)];
                }
            }
            __syncthreads();
            if (!has) continue;
            const int src = __builtin_amdgcn_readfirstlane(list_src[e]);
            const CDouble M0 = (CDouble)(lv.M + int64_t(src) * 3 * nt);
#pragma unroll
            for (int j = 0; j < SLOTS; ++j) {
                // 8 steps per batch of scalar loads, which may read up to 7 terms past a lane's
                // prefix; those lanes multiply by the zero.  Past a cell's first two components the
                // reads find the next component's moments, past the third the next cell's, or the
                // zeros that the moments' writers leave after the level's last cell: always finite.
                for (int s0 = 0; s0 < smax[j]; s0 += 8) {
                    int ks[8];
                    double m[3][8];
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        ks[i] = int(gidx[s0 + i]);
                        m[0][i] = M0[s0 + i];
                        m[1][i] = M0[nt + s0 + i];
                        m[2][i] = M0[2 * nt + s0 + i];
                    }
                    // lanes past their prefix read the zero after the grid (no branch, so that the
                    // eight reads are in flight together)
                    double Dv[8];
#pragma unroll
                    for (int i = 0; i < 8; ++i) Dv[i] = sDg[s0 + i < cnt[j] ? nb[j] + ks[i] : zero_at];
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        acc[j][0] += Dv[i] * m[0][i];
                        acc[j][1] += Dv[i] * m[1][i];
                        acc[j][2] += Dv[i] * m[2][i];
                    }
                }
            }
        }
        // add the groups' sums in group order through LDS (3 nt doubles per group)
        __syncthreads();
        for (int j = 0; j < SLOTS; ++j) {
            const int t = gt + glanes * j;
            if (t >= nt) break;
            for (int d = 0; d < 3; ++d) sDyn[(grp * 3 + d) * nt + t] = acc[j][d];
        }
        __syncthreads();
        for (int idx = threadIdx.x; idx < 3 * nt; idx += blockDim.x) {
            const int d = idx / nt, t = idx - d * nt;
            double v = 0.0;
            for (int g2 = 0; g2 < ngroup; ++g2) v += sDyn[(g2 * 3 + d) * nt + t];
            const uint32_t k = terms[t];
            const int dg = int(k & 0xff) + int((k >> 8) & 0xff) + int(k >> 16);
            const double f = ((dg & 1) ? -kInv4Pi : kInv4Pi) / w;
            lv.L[(int64_t(cell) * 3 + d) * nt + t] = v * f;
        }
    }
}

// Children at level l += shifted expansion of their parents at level l - 1 (one axis at a time
// in LDS, as k_fmm_m2m).
__global__ __launch_bounds__(256) void k_fmm_l2l(FmmLevel chi, FmmLevel par, const int32_t* __restrict__ count, int l,
                                                 const double* __restrict__ box, int p,
                                                 const uint32_t* __restrict__ terms) {
    const int cell = blockIdx.x;
    if (cell >= *count) return;
    const int nt = nterms(p);
    extern __shared__ double sShift[];
    double* bufA = sShift;
    double* bufB = sShift + 3 * nt;
    __shared__ double pw[3][kMaxOrder + 1];
    const int pa = chi.parent[cell];
    if (threadIdx.x < 3) {
        const int d = threadIdx.x;
        int ic[3], ip[3];
        cell_coords(chi.code[cell], ic);
        cell_coords(par.code[pa], ip);
        const double dl = cell_centre(box, d, ic[d], l) - cell_centre(box, d, ip[d], l - 1);
        double v = 1.0;
        pw[d][0] = 1.0;
        for (int i = 1; i <= p; ++i) {
            v = v * dl / double(i);
            pw[d][i] = v;
        }
    }
    const double* Lp = par.L + int64_t(pa) * 3 * nt;
    for (int i = threadIdx.x; i < 3 * nt; i += 256) bufA[i] = Lp[i];
    __syncthreads();
    shift_axis<true>(bufA, bufB, pw[0], 0, p, nt, terms);
    __syncthreads();
    shift_axis<true>(bufB, bufA, pw[1], 1, p, nt, terms);
    __syncthreads();
    for (int t = threadIdx.x; t < nt; t += 256) {
        double o[3];
        shift_axis_term<true>(bufA, pw[2], 2, p, nt, terms[t], o);
        for (int d = 0; d < 3; ++d) chi.L[(int64_t(cell) * 3 + d) * nt + t] += o[d];
    }
}

// ---------------------------------------------------------------- near field + evaluation
// Work items: chunks of kNearTile consecutive targets of one leaf (one workgroup).
__global__ __launch_bounds__(1024) void k_fmm_items(const int32_t* __restrict__ count, const int32_t* __restrict__ pstart,
                                                    int32_t* __restrict__ item_leaf, int32_t* __restrict__ item_t0,
                                                    int32_t* __restrict__ nitems) {
    __shared__ int32_t part[1024];
    const int64_t nl = *count;
    const int tid = threadIdx.x;
    const int64_t chunk = (nl + 1023) / 1024;
    const int64_t b = int64_t(tid) * chunk;
    const int64_t e = b + chunk < nl ? b + chunk : nl;
    int32_t cnt = 0;
    for (int64_t i = b; i < e; ++i) cnt += (pstart[i + 1] - pstart[i] + kNearTile - 1) / kNearTile;
    part[tid] = cnt;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int32_t v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int32_t pos = part[tid] - cnt;
    for (int64_t i = b; i < e; ++i)
        for (int32_t t0 = pstart[i]; t0 < pstart[i + 1]; t0 += kNearTile) {
            item_leaf[pos] = int32_t(i);
            item_t0[pos] = t0;
            ++pos;
        }
    if (tid == 1023) *nitems = part[1023];
}

struct NearArgs {
    const void* xs;
    const void* gs;
    const void* ss;
    const int32_t* perm;
    int64_t n;
    FmmLevel leaf;
    const int32_t* count;
    const int32_t* item_leaf;
    const int32_t* item_t0;
    const int32_t* nitems;
    const double* box;
    int level;
    int p;
    const double* far;  // [15][n] far field (u, dgamma, J) in sorted order, or null
    void* u;
    void* dg;
    void* grad;         // [9][ldo] velocity gradient, or null
    int64_t ldo;
};

// Far field at the targets of one work item from their leaf's local expansion (FP64):
// far[0..2] = curl psi, far[3..5] = J^T Gamma_i (transposed) or J Gamma_i (classical),
// far[6..14] = J (row-major) when the gradient is wanted.
// Two targets per lane (the item's targets t0 + tid and t0 + tid + 128, 128 lanes): every
// coefficient read from LDS (a broadcast, all lanes walk the same terms) serves both, which
// halves the LDS traffic that bounds this kernel (27 reads per term and target before).
constexpr int kL2pLanes = 128;
template <typename T, bool CLASSICAL>
__global__ __launch_bounds__(kL2pLanes) void k_fmm_l2p(NearArgs a, double* __restrict__ far) {
    const int item = blockIdx.x;
    if (item >= *a.nitems) return;
    const T* __restrict__ xs = static_cast<const T*>(a.xs);
    const T* __restrict__ gs = static_cast<const T*>(a.gs);
    const int64_t n = a.n;
    const int leaf = a.item_leaf[item];
    const int q0 = a.item_t0[item] + int(threadIdx.x);
    const int qend = a.leaf.pstart[leaf + 1];
    const int nt = nterms(a.p);
    extern __shared__ double sLx[];  // the leaf's expansion, [3][nt] (dynamic: 3 nt doubles)
    for (int t = threadIdx.x; t < nt; t += kL2pLanes)
        for (int d = 0; d < 3; ++d) sLx[d * nt + t] = a.leaf.L[(int64_t(leaf) * 3 + d) * nt + t];
    __syncthreads();
    if (q0 >= qend) return;
    int ic[3];
    cell_coords(a.leaf.code[leaf], ic);
    // the second target repeats the first where the item ends (computed, not written)
    const int qs[2] = {q0, q0 + kL2pLanes < qend ? q0 + kL2pLanes : q0};
    double av[2][3];
    for (int r = 0; r < 2; ++r)
        for (int d = 0; d < 3; ++d) av[r][d] = double(xs[d * n + qs[r]]) - cell_centre(a.box, d, ic[d], a.level);
    double gp[2][3][3], hp[2][6][3];  // d_b psi_c; d_e d_b psi_c for (e, b) in xx yy zz xy xz yz
    for (int r = 0; r < 2; ++r) {
        for (int b = 0; b < 3; ++b)
            for (int c = 0; c < 3; ++c) gp[r][b][c] = 0.0;
        for (int m = 0; m < 6; ++m)
            for (int c = 0; c < 3; ++c) hp[r][m][c] = 0.0;
    }
    const int p = a.p;
    double px[2] = {1.0, 1.0};
    for (int n0 = 0; n0 <= p - 1; ++n0) {
        double pxy[2] = {px[0], px[1]};
        for (int n1 = 0; n1 <= p - 1 - n0; ++n1) {
            double mono[2] = {pxy[0], pxy[1]};
            for (int n2 = 0; n2 <= p - 1 - n0 - n1; ++n2) {
                const int i0 = mpos(n0 + 1, n1, n2), i1 = mpos(n0, n1 + 1, n2), i2 = mpos(n0, n1, n2 + 1);
                for (int c = 0; c < 3; ++c) {
                    const double l0 = sLx[c * nt + i0], l1 = sLx[c * nt + i1], l2 = sLx[c * nt + i2];
                    for (int r = 0; r < 2; ++r) {
                        gp[r][0][c] += l0 * mono[r];
                        gp[r][1][c] += l1 * mono[r];
                        gp[r][2][c] += l2 * mono[r];
                    }
                }
                if (n0 + n1 + n2 <= p - 2) {
                    const int h[6] = {mpos(n0 + 2, n1, n2), mpos(n0, n1 + 2, n2), mpos(n0, n1, n2 + 2),
                                      mpos(n0 + 1, n1 + 1, n2), mpos(n0 + 1, n1, n2 + 1), mpos(n0, n1 + 1, n2 + 1)};
                    for (int m = 0; m < 6; ++m)
                        for (int c = 0; c < 3; ++c) {
                            const double lv = sLx[c * nt + h[m]];
                            for (int r = 0; r < 2; ++r) hp[r][m][c] += lv * mono[r];
                        }
                }
                for (int r = 0; r < 2; ++r) mono[r] = mono[r] * av[r][2] * kInvInt[n2 + 1];
            }
            for (int r = 0; r < 2; ++r) pxy[r] = pxy[r] * av[r][1] * kInvInt[n1 + 1];
        }
        for (int r = 0; r < 2; ++r) px[r] = px[r] * av[r][0] * kInvInt[n0 + 1];
    }
    for (int r = 0; r < 2; ++r) {
        const int q = qs[r];
        if (r == 1 && q == q0) break;  // no second target in this lane
        auto H = [&](int e, int b, int c) -> double {
            if (e == b) return hp[r][e][c];
            const int lo2 = e < b ? e : b, hi2 = e < b ? b : e;
            const int m = (lo2 == 0 && hi2 == 1) ? 3 : ((lo2 == 0 && hi2 == 2) ? 4 : 5);
            return hp[r][m][c];
        };
        // u_a = eps_abc d_b psi_c;  J_ae = eps_abc d_e d_b psi_c
        far[q] = gp[r][1][2] - gp[r][2][1];
        far[n + q] = gp[r][2][0] - gp[r][0][2];
        far[2 * n + q] = gp[r][0][1] - gp[r][1][0];
        double J[3][3];
        for (int e = 0; e < 3; ++e) {
            J[0][e] = H(e, 1, 2) - H(e, 2, 1);
            J[1][e] = H(e, 2, 0) - H(e, 0, 2);
            J[2][e] = H(e, 0, 1) - H(e, 1, 0);
        }
        const double Gi[3] = {double(gs[q]), double(gs[n + q]), double(gs[2 * n + q])};
        for (int c = 0; c < 3; ++c) {
            double sum = 0.0;
            for (int b = 0; b < 3; ++b) sum += (CLASSICAL ? J[c][b] : J[b][c]) * Gi[b];
            far[(3 + c) * n + q] = sum;
        }
        if (a.grad)
            for (int c = 0; c < 3; ++c)
                for (int e = 0; e < 3; ++e) far[(6 + 3 * c + e) * n + q] = J[c][e];
    }
}

// Keeps a value opaque to the optimiser (emits no instruction).
__device__ __forceinline__ float opaque_reg(float v) {
    asm volatile("" : "+v"(v));
    return v;
}
__device__ __forceinline__ double opaque_reg(double v) {
    asm volatile("" : "+v"(v));
    return v;
}

// One near-field pair.  Sums (as the direct kernel's):
//   plain:    U = sum G v (v = Gamma_j x r), A = sum G Gamma_j outside the cores,
//             B = sum Hn tau r (transposed, tau = Gamma_i . v) or sum Hn (r . Gamma_i) v
//             (classical), in-core cross terms G Gamma_i x Gamma_j put into B (x -1/3; the
//             classical sign is folded in);
//   gradient: U, A outside the cores, H = sum Hn v r^T (row-major), A of the in-core pairs,
//             C = sum over in-core pairs of G Gamma_i x Gamma_j.
// Sign-folded cross product (as in the direct kernel): the pair holds r' = (r_x, -r_y, r_z)
// and v' = (v_x, -v_y, -v_z), each component of v' a multiply and an accumulating
// multiply-add with the staged -Gamma_j,z, so no multiply-add needs a negated operand; the
// sums then hold some components negated (near_held_sign), which the epilogue undoes.
// p = (x_j, -Gamma_j,z), q = (Gamma_j, cut_j), w = (1/sigma_j, 1/sigma_j^2) (read only in a
// core); ngyi = -Gamma_i,y, ngzi = -Gamma_i,z.
template <typename T, bool CLASSICAL, bool GRAD, bool MAYCORE, typename V4, typename V2>
__device__ __forceinline__ void near_pair(T xi, T yi, T zi, T gxi, T gyi, T gzi, T ngyi, T ngzi, const V4& p,
                                          const V4& q, const V2* w, T* acc) {
    const T rx = xi - p.x, ryn = p.y - yi, rz = zi - p.z;
    const T s2 = rx * rx + ryn * ryn + rz * rz;
    const T vx = q.y * rz + q.z * ryn, vyn = p.w * rx + q.x * rz, vzn = q.x * ryn + q.y * rx;
    const T inv = rsqrt_fast(s2);
    const T inv2 = inv * inv;
    T G = inv * inv2, Hn = G * inv2;
    bool core = false;
    T Ga = G;  // weight of Gamma_j in A (plain mode)
    if constexpr (MAYCORE) {
        core = s2 < q.w;
        if (core) {
            const V2 iw = *w;
            core_weights_call(s2, iw.x, iw.y, G, Hn);
            if constexpr (!GRAD) {
                // transposed: G Gamma_i x Gamma_j, classical: G Gamma_j x Gamma_i, into B x -1/3
                // (held signs as B'), and nothing into A
                const T f = G * T(CLASSICAL ? 1.0 / 3.0 : -1.0 / 3.0);
                acc[6] += f * (gyi * q.z - gzi * q.y);
                acc[7] -= f * (gzi * q.x - gxi * q.z);
                if constexpr (CLASSICAL) acc[8] -= f * (gxi * q.y - gyi * q.x);
                else acc[8] += f * (gxi * q.y - gyi * q.x);
                Ga = T(0);
            }
        }
    }
    acc[0] += G * vx;
    acc[1] += G * vyn;
    acc[2] += G * vzn;
    if constexpr (GRAD) {
        const T hx = Hn * vx, hy = Hn * vyn, hz = Hn * vzn;
        acc[6] += hx * rx;
        acc[7] += hx * ryn;
        acc[8] += hx * rz;
        acc[9] += hy * rx;
        acc[10] += hy * ryn;
        acc[11] += hy * rz;
        acc[12] += hz * rx;
        acc[13] += hz * ryn;
        acc[14] += hz * rz;
        if constexpr (MAYCORE) {
            // A of the in-core pairs and A outside the cores go to different sums; the weights
            // are selected rather than the destinations (a selected destination becomes an
            // indexed array in scratch memory)
            const T Gc = core ? G : T(0), Go = core ? T(0) : G;
            acc[3] += Go * q.x;
            acc[4] += Go * q.y;
            acc[5] += Go * q.z;
            acc[15] += Gc * q.x;
            acc[16] += Gc * q.y;
            acc[17] += Gc * q.z;
            if (core) {
                acc[18] += G * (gyi * q.z - gzi * q.y);
                acc[19] += G * (gzi * q.x - gxi * q.z);
                acc[20] += G * (gxi * q.y - gyi * q.x);
            }
        } else {
            acc[3] += G * q.x;
            acc[4] += G * q.y;
            acc[5] += G * q.z;
        }
    } else {
        const T wgt = CLASSICAL ? Hn * (rx * gxi + ryn * ngyi + rz * gzi) : Hn * (gxi * vx + ngyi * vyn + ngzi * vzn);
        if constexpr (!CLASSICAL) {
            acc[6] += wgt * rx;
            acc[7] += wgt * ryn;
            acc[8] += wgt * rz;
        } else {
            acc[6] += wgt * vx;
            acc[7] += wgt * vyn;
            acc[8] += wgt * vzn;
        }
        acc[3] += Ga * q.x;
        acc[4] += Ga * q.y;
        acc[5] += Ga * q.z;
    }
}

// Signs that the near-field sums hold relative to the sums they stand for (near_pair):
// U' = (U_x, -U_y, -U_z); transposed B' = (B_x, -B_y, B_z); classical B' = (B_x, -B_y, -B_z);
// gradient H'_ab = s_a t_b H_ab with s = (+, -, -) from v and t = (+, -, +) from r.
__device__ constexpr double near_held_sign(bool classical, bool grad, int c) {
    return c == 1 || c == 2 ? -1.0
         : c < 6 ? 1.0
         : grad ? (c < 15 ? ((c - 6) / 3 == 0 ? 1.0 : -1.0) * ((c - 6) % 3 == 1 ? -1.0 : 1.0) : 1.0)
         : classical ? (c == 7 || c == 8 ? -1.0 : 1.0)
         : (c == 7 ? -1.0 : 1.0);
}

// Near field of one work item: the exact Gaussian pair sum over the 27 neighbouring leaves.
// Sources stream through LDS in tiles of 256; each wavefront tests every 64-source subtile
// against its own 64 targets and runs the loop without the core test where the boxes are
// farther apart than the subtile's largest core cut (rho_far sigma).  The epilogue adds the
// far field (if any) and writes in the caller's order.
template <typename T, bool CLASSICAL, bool GRAD>
__global__ __launch_bounds__(256, GRAD ? 4 : 1) void k_fmm_near(NearArgs a) {
    constexpr bool kComp = std::is_same<T, float>::value;
    constexpr int NA = GRAD ? 21 : 9;
    const int item = blockIdx.x;
    if (item >= *a.nitems) return;
    const T* __restrict__ xs = static_cast<const T*>(a.xs);
    const T* __restrict__ gs = static_cast<const T*>(a.gs);
    const T* __restrict__ ss = static_cast<const T*>(a.ss);
    const int64_t n = a.n;
    const int leaf = a.item_leaf[item];
    const int t0 = a.item_t0[item];
    const int tend = a.leaf.pstart[leaf + 1];
    const int q = t0 + int(threadIdx.x);
    const bool valid = q < tend;
    const int qq = valid ? q : t0;
    const int nleaf = *a.count;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int wq0 = t0 + 64 * wv;  // first target of this wavefront

    using V4 = typename std::conditional<kComp, float4, double4>::type;
    using V2 = typename std::conditional<kComp, float2, double2>::type;
    // per source: (x, -Gamma_z), (Gamma, cut) and (1/sigma, 1/sigma^2)
    __shared__ V4 sp[kNearTile], sq[kNearTile];
    __shared__ V2 sw[kNearTile];
    __shared__ T sbox[4][7];
    __shared__ int32_t nb_lo[27], nb_hi[27];
    int ic[3];
    cell_coords(a.leaf.code[leaf], ic);
    const int side = 1 << a.level;
    if (threadIdx.x < 27) {
        const int t = threadIdx.x;
        const int s[3] = {ic[0] + t / 9 - 1, ic[1] + (t / 3) % 3 - 1, ic[2] + t % 3 - 1};
        int idx = -1;
        if (s[0] >= 0 && s[1] >= 0 && s[2] >= 0 && s[0] < side && s[1] < side && s[2] < side)
            idx = find_code(a.leaf.code, nleaf, cell_code(s[0], s[1], s[2]));
        nb_lo[t] = idx >= 0 ? a.leaf.pstart[idx] : 0;
        nb_hi[t] = idx >= 0 ? a.leaf.pstart[idx + 1] : 0;
    }
    __syncthreads();

    const T xi = xs[qq], yi = xs[n + qq], zi = xs[2 * n + qq];
    const T gxi = gs[qq], gyi = gs[n + qq], gzi = gs[2 * n + qq];
    // (kept opaque so that their products stay plain multiplies by a register)
    const T ngyi = opaque_reg(-gyi), ngzi = opaque_reg(-gzi);
    // box of this wavefront's targets (lanes past the end repeat the item's first target)
    T tlo[3], thi[3], tcut;
    {
        const T pl[3] = {xi, yi, zi};
        wave_box(pl, pl, T(0), tlo, thi, tcut);
    }
    T acc[NA], hi[NA], lo[NA];
#pragma unroll
    for (int c = 0; c < NA; ++c) acc[c] = hi[c] = lo[c] = T(0);
    for (int nb = 0; nb < 27; ++nb) {
        const int lo_j = nb_lo[nb], hi_j = nb_hi[nb];
        for (int j0 = lo_j; j0 < hi_j; j0 += kNearTile) {
            const int cnt = hi_j - j0 < kNearTile ? hi_j - j0 : kNearTile;
            __syncthreads();
            {
                const bool has = int(threadIdx.x) < cnt;
                const int j = has ? j0 + threadIdx.x : j0;
                T pl[3];
                for (int d = 0; d < 3; ++d) pl[d] = xs[d * n + j];
                const T sj = ss[j];
                const T is = T(1) / sj;
                const T cut = Prec<T>::kFarRho2 * sj * sj;
                const T g0 = gs[j], g1 = gs[n + j], g2 = gs[2 * n + j];
                sp[threadIdx.x] = V4{pl[0], pl[1], pl[2], -g2};
                sq[threadIdx.x] = V4{g0, g1, g2, cut};
                sw[threadIdx.x] = V2{is, is * is};
                // subtile box of this wavefront's 64 staged sources (past the end: the tile's
                // first source again, which only makes the box larger)
                T blo[3], bhi[3], bcut;
                wave_box(pl, pl, cut, blo, bhi, bcut);
                if (lane == 0) {
                    for (int d = 0; d < 3; ++d) {
                        sbox[wv][d] = blo[d];
                        sbox[wv][3 + d] = bhi[d];
                    }
                    sbox[wv][6] = bcut;
                }
            }
            __syncthreads();
            for (int sub = 0; sub * 64 < cnt; ++sub) {
                const int jb = sub * 64;
                const int je = cnt - jb < 64 ? cnt : jb + 64;
                T d2 = T(0);
                for (int d = 0; d < 3; ++d) {
                    const T g1 = sbox[sub][d] - thi[d], g2 = tlo[d] - sbox[sub][3 + d];
                    const T gap = g1 > g2 ? g1 : g2;
                    d2 += gap > T(0) ? gap * gap : T(0);
                }
                // the self pairs of this wavefront's targets can only lie in a subtile whose
                // sources overlap their index range
                const bool self_sub = j0 + jb < wq0 + 64 && j0 + je > wq0;
                if (d2 >= sbox[sub][6]) {
                    // every pair of this wavefront and subtile is outside the cores
#pragma unroll 2
                    for (int jj = jb; jj < je; ++jj)
                        near_pair<T, CLASSICAL, GRAD, false>(xi, yi, zi, gxi, gyi, gzi, ngyi, ngzi, sp[jj], sq[jj],
                                                             sw + jj, acc);
                } else if (self_sub) {
                    for (int jj = jb; jj < je; ++jj) {
                        if (j0 + jj == qq) continue;  // self pair
                        near_pair<T, CLASSICAL, GRAD, true>(xi, yi, zi, gxi, gyi, gzi, ngyi, ngzi, sp[jj], sq[jj],
                                                            sw + jj, acc);
                    }
                } else {
                    for (int jj = jb; jj < je; ++jj)
                        near_pair<T, CLASSICAL, GRAD, true>(xi, yi, zi, gxi, gyi, gzi, ngyi, ngzi, sp[jj], sq[jj],
                                                            sw + jj, acc);
                }
            }
            if constexpr (kComp) {
#pragma unroll
                for (int c = 0; c < NA; ++c) {
                    T s, e;
                    two_sum(hi[c], acc[c], s, e);
                    hi[c] = s;
                    lo[c] += e;
                    acc[c] = T(0);
                }
            }
        }
    }
    if (!valid) return;
    double S[NA];
#pragma unroll
    for (int c = 0; c < NA; ++c)
        S[c] = near_held_sign(CLASSICAL, GRAD, c) * (kComp ? double(hi[c]) + double(lo[c]) : double(acc[c]));
    const double Gi[3] = {double(gxi), double(gyi), double(gzi)};
    double u[3] = {S[0] * kInv4Pi, S[1] * kInv4Pi, S[2] * kInv4Pi};
    double dgv[3];
    // Gamma_i x A
    const double cx = Gi[1] * S[5] - Gi[2] * S[4];
    const double cy = Gi[2] * S[3] - Gi[0] * S[5];
    const double cz = Gi[0] * S[4] - Gi[1] * S[3];
    double Jn[9];
    if constexpr (GRAD) {
        // stretching from the same sums: transposed (Gamma_i x A + C - 3 H^T Gamma_i)/4pi,
        // classical (A x Gamma_i - C - 3 H Gamma_i)/4pi; J = ([A + A_core]x - 3H)/4pi
        const double* H = S + 6;
        const double sgn = CLASSICAL ? -1.0 : 1.0;
        double hg[3];
        for (int r = 0; r < 3; ++r)
            hg[r] = CLASSICAL ? H[3 * r] * Gi[0] + H[3 * r + 1] * Gi[1] + H[3 * r + 2] * Gi[2]
                              : H[r] * Gi[0] + H[3 + r] * Gi[1] + H[6 + r] * Gi[2];
        dgv[0] = (sgn * (cx + S[18]) - 3.0 * hg[0]) * kInv4Pi;
        dgv[1] = (sgn * (cy + S[19]) - 3.0 * hg[1]) * kInv4Pi;
        dgv[2] = (sgn * (cz + S[20]) - 3.0 * hg[2]) * kInv4Pi;
        const double At0 = S[3] + S[15], At1 = S[4] + S[16], At2 = S[5] + S[17];
        const double X[9] = {0.0, -At2, At1, At2, 0.0, -At0, -At1, At0, 0.0};
        for (int c = 0; c < 9; ++c) Jn[c] = (X[c] - 3.0 * H[c]) * kInv4Pi;
    } else {
        // transposed (Gamma_i x A - 3B)/4pi; classical (A x Gamma_i - 3B)/4pi
        const double sgn = CLASSICAL ? -1.0 : 1.0;
        dgv[0] = (sgn * cx - 3.0 * S[6]) * kInv4Pi;
        dgv[1] = (sgn * cy - 3.0 * S[7]) * kInv4Pi;
        dgv[2] = (sgn * cz - 3.0 * S[8]) * kInv4Pi;
    }
    if (a.far) {
        for (int c = 0; c < 3; ++c) {
            u[c] += a.far[c * n + q];
            dgv[c] += a.far[(3 + c) * n + q];
        }
        if constexpr (GRAD)
            for (int c = 0; c < 9; ++c) Jn[c] += a.far[(6 + c) * n + q];
    }
    T* __restrict__ U = static_cast<T*>(a.u);
    T* __restrict__ DG = static_cast<T*>(a.dg);
    const int64_t o = a.perm[q];
    for (int c = 0; c < 3; ++c) {
        U[c * a.ldo + o] = T(u[c]);
        DG[c * a.ldo + o] = T(dgv[c]);
    }
    if constexpr (GRAD) {
        T* __restrict__ JO = static_cast<T*>(a.grad);
        for (int c = 0; c < 9; ++c) JO[c * a.ldo + o] = T(Jn[c]);
    }
}

// ---------------------------------------------------------------- workspace
size_t al256(size_t v) { return (v + 255) / 256 * 256; }

struct Layout {
    size_t keys, box, scan, xs, gs, ss, perm, lcode, terms, dtab, item_leaf, item_t0, counts, far;
    size_t code[kMaxLevel + 1], first[kMaxLevel + 1], pstart[kMaxLevel + 1], parent[kMaxLevel + 1];
    size_t M[kMaxLevel + 1], L[kMaxLevel + 1];
    int64_t cap[kMaxLevel + 1];
    int64_t items_cap;
    size_t total;
};

Layout layout(int64_t n, int level, int order, size_t es) {
    Layout y{};
    const int nt = nterms(order);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += al256(bytes);
        return at;
    };
    y.keys = take(size_t(sort_len(n)) * 8);
    y.box = take(8 * sizeof(double));
    const size_t nb = size_t((n + kScanChunk - 1) / kScanChunk);
    y.scan = take(nb * 4 > 6 * kBoxParts * sizeof(double) ? nb * 4 : 6 * kBoxParts * sizeof(double));
    y.xs = take(3 * size_t(n) * es);
    y.gs = take(3 * size_t(n) * es);
    y.ss = take(size_t(n) * es);
    y.perm = take(size_t(n) * 4);
    y.lcode = take(size_t(n) * 4);
    y.terms = take(size_t(2 * kMaxTerms + 8) * 4);  // + 8: M2L's batched reads past a prefix
    y.dtab = take(size_t(kOffsets) * nt * sizeof(double));
    y.items_cap = n / kNearTile + n + 1;
    y.item_leaf = take(size_t(y.items_cap) * 4);
    y.item_t0 = take(size_t(y.items_cap) * 4);
    y.counts = take(size_t(kMaxLevel + 2) * 4);
    y.far = take(15 * size_t(n) * sizeof(double));
    for (int l = 0; l <= level; ++l) {
        const int64_t full = int64_t(1) << (3 * l);
        const int64_t cap = full < n ? full : n;
        y.cap[l] = cap < 1 ? 1 : cap;
        y.code[l] = take(size_t(y.cap[l]) * 4);
        y.first[l] = take(size_t(y.cap[l] + 1) * 4);
        y.pstart[l] = take(size_t(y.cap[l] + 1) * 4);
        y.parent[l] = take(size_t(y.cap[l]) * 4);
        y.M[l] = take((size_t(y.cap[l]) * 3 * nt + kM2lOverrun) * sizeof(double));
        y.L[l] = take(size_t(y.cap[l]) * 3 * nt * sizeof(double));
    }
    y.total = o;
    return y;
}

template <typename T>
hipError_t run_fmm(int64_t n, const T* x, const T* g, const T* sg, int64_t ld, int level, int p, int classical,
                   T* u, T* dg, T* grad, int64_t ldo, unsigned char* ws, hipStream_t st) {
    const Layout y = layout(n, level, p, sizeof(T));
    uint64_t* keys = reinterpret_cast<uint64_t*>(ws + y.keys);
    double* box = reinterpret_cast<double*>(ws + y.box);
    T* xs = reinterpret_cast<T*>(ws + y.xs);
    T* gs = reinterpret_cast<T*>(ws + y.gs);
    T* ss = reinterpret_cast<T*>(ws + y.ss);
    int32_t* perm = reinterpret_cast<int32_t*>(ws + y.perm);
    uint32_t* lcode = reinterpret_cast<uint32_t*>(ws + y.lcode);
    uint32_t* terms = reinterpret_cast<uint32_t*>(ws + y.terms);
    double* dtab = reinterpret_cast<double*>(ws + y.dtab);
    int32_t* item_leaf = reinterpret_cast<int32_t*>(ws + y.item_leaf);
    int32_t* item_t0 = reinterpret_cast<int32_t*>(ws + y.item_t0);
    int32_t* counts = reinterpret_cast<int32_t*>(ws + y.counts);  // [level + 1] cells, then items
    FmmLevel lv[kMaxLevel + 1];
    for (int l = 0; l <= level; ++l) {
        lv[l].code = reinterpret_cast<uint32_t*>(ws + y.code[l]);
        lv[l].first = reinterpret_cast<int32_t*>(ws + y.first[l]);
        lv[l].pstart = reinterpret_cast<int32_t*>(ws + y.pstart[l]);
        lv[l].parent = reinterpret_cast<int32_t*>(ws + y.parent[l]);
        lv[l].M = reinterpret_cast<double*>(ws + y.M[l]);
        lv[l].L = reinterpret_cast<double*>(ws + y.L[l]);
        lv[l].cap = y.cap[l];
    }
    hipError_t e;
    const int64_t P = sort_len(n);
    {
        const int64_t want = (n + 2047) / 2048;
        const int nparts = int(want < kBoxParts ? want : kBoxParts);
        double* part = reinterpret_cast<double*>(ws + y.scan);
        hipLaunchKernelGGL(k_fmm_box_part<T>, dim3(unsigned(nparts)), dim3(256), 0, st, x, ld, n, part);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(k_fmm_box, dim3(1), dim3(256), 0, st, part, nparts, level, box);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_fmm_keys<T>, dim3(unsigned(P / 256)), dim3(256), 0, st, x, ld, n, level, box, keys, P);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = sort_keys(keys, P, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_fmm_gather<T>, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, x, g, sg, ld, n, keys, xs,
                       gs, ss, perm, lcode, level);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // leaves: distinct leaf codes of the sorted particles
    {
        const int64_t nb = (n + kScanChunk - 1) / kScanChunk;
        int32_t* bsum = reinterpret_cast<int32_t*>(ws + y.scan);
        hipLaunchKernelGGL(k_fmm_leaf_count, dim3(unsigned(nb)), dim3(256), 0, st, lcode, n, bsum);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(k_fmm_leaf_scan, dim3(1), dim3(1024), 0, st, bsum, nb, n, lv[level].pstart,
                           counts + level);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(k_fmm_leaf_scatter, dim3(unsigned(nb)), dim3(256), 0, st, lcode, n, bsum,
                           lv[level].code, lv[level].pstart);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // coarser levels: distinct parent codes of the level below
    for (int l = level - 1; l >= 0; --l) {
        hipLaunchKernelGGL(k_fmm_unique, dim3(1), dim3(1024), 0, st, lv[l + 1].code, counts + l + 1, int64_t(0), 3,
                           lv[l].code, lv[l].first, lv[l + 1].parent, counts + l, lv[l + 1].pstart, lv[l].pstart,
                           int32_t(n));
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_fmm_terms, dim3(1), dim3(64), 0, st, p, terms);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // M2L: as many groups of 256 lanes as 60 KiB of LDS allow (at most 4), each holding its grid
    // (or its 3 nt sums at the end if those are larger); where fewer than two fit, one group of
    // kUnitWaves wavefronts that share the terms' walks in balanced pieces (m2l_units)
    const size_t m2l_grid = size_t(m2l_group_doubles(p, false)) * sizeof(double);
    int m2l_groups = int((60 * 1024) / m2l_grid);
    m2l_groups = m2l_groups > 4 ? 4 : m2l_groups;
    int m2l_gsize = 256;
    M2lUnits units{};
    size_t m2l_lds = size_t(m2l_groups) * m2l_grid;
    if (m2l_groups < 2) {
        m2l_groups = 1;
        m2l_gsize = 64 * kUnitWaves;
        if (!m2l_units(p, units)) return hipErrorInvalidValue;
        // the group's grid, moments and indices, or the pieces' partial sums at the end
        const size_t grid = size_t(m2l_group_doubles(p, true));
        const size_t sums = size_t(units.n) * 64 * 3;
        m2l_lds = (grid > sums ? grid : sums) * sizeof(double);
    } else if (nterms(p) > 5 * m2l_gsize) {
        // every term has a lane: 5 per lane in 256-lane groups (two or more groups fit only
        // while 3 nt doubles take at most 30 KiB, nt <= 1280)
        return hipErrorInvalidValue;
    }
    const size_t shift_lds = size_t(6 * nterms(p)) * sizeof(double);  // M2M and L2L: two 3 nt buffers
    if (level >= 2) {
        hipLaunchKernelGGL(k_fmm_dtab, dim3(kOffsets), dim3(256), 0, st, p, terms, dtab);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(k_fmm_p2m<T>, dim3(unsigned(y.cap[level])), dim3(256), 0, st, xs, gs, n, lv[level],
                           counts + level, box, level, p, terms);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        for (int l = level - 1; l >= 2; --l) {
            hipLaunchKernelGGL(k_fmm_m2m, dim3(unsigned(y.cap[l])), dim3(256), shift_lds, st, lv[l], lv[l + 1],
                               counts + l, l, box, p, terms);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        for (int l = 2; l <= level; ++l) {
            if (m2l_gsize == 256)
                hipLaunchKernelGGL((k_fmm_m2l<5, false>), dim3(unsigned(y.cap[l])), dim3(256 * m2l_groups), m2l_lds, st, lv[l],
                               counts + l, l, box, p, terms, dtab, m2l_gsize, units);
            else
                hipLaunchKernelGGL((k_fmm_m2l<2, true>), dim3(unsigned(y.cap[l])), dim3(m2l_gsize), m2l_lds, st, lv[l],
                               counts + l, l, box, p, terms, dtab, m2l_gsize, units);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            if (l >= 3) {
                hipLaunchKernelGGL(k_fmm_l2l, dim3(unsigned(y.cap[l])), dim3(256), shift_lds, st, lv[l], lv[l - 1],
                                   counts + l, l, box, p, terms);
                if ((e = hipGetLastError()) != hipSuccess) return e;
            }
        }
    }
    hipLaunchKernelGGL(k_fmm_items, dim3(1), dim3(1024), 0, st, counts + level, lv[level].pstart, item_leaf, item_t0,
                       counts + level + 1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    NearArgs na;
    na.xs = xs;
    na.gs = gs;
    na.ss = ss;
    na.perm = perm;
    na.n = n;
    na.leaf = lv[level];
    na.count = counts + level;
    na.item_leaf = item_leaf;
    na.item_t0 = item_t0;
    na.nitems = counts + level + 1;
    na.box = box;
    na.level = level;
    na.p = p;
    na.far = nullptr;
    na.u = u;
    na.dg = dg;
    na.grad = grad;
    na.ldo = ldo;
    const unsigned grid = unsigned((n + kNearTile - 1) / kNearTile + y.cap[level]);
    if (level >= 2) {
        double* far = reinterpret_cast<double*>(ws + y.far);
        const size_t l2p_lds = size_t(3 * nterms(p)) * sizeof(double);
        if (classical)
            hipLaunchKernelGGL((k_fmm_l2p<T, true>), dim3(grid), dim3(kL2pLanes), l2p_lds, st, na, far);
        else
            hipLaunchKernelGGL((k_fmm_l2p<T, false>), dim3(grid), dim3(kL2pLanes), l2p_lds, st, na, far);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        na.far = far;
    }
    if (grad) {
        if (classical)
            hipLaunchKernelGGL((k_fmm_near<T, true, true>), dim3(grid), dim3(256), 0, st, na);
        else
            hipLaunchKernelGGL((k_fmm_near<T, false, true>), dim3(grid), dim3(256), 0, st, na);
    } else {
        if (classical)
            hipLaunchKernelGGL((k_fmm_near<T, true, false>), dim3(grid), dim3(256), 0, st, na);
        else
            hipLaunchKernelGGL((k_fmm_near<T, false, false>), dim3(grid), dim3(256), 0, st, na);
    }
    return hipGetLastError();
}

}  // namespace

size_t fmm_workspace(int64_t n, int level, int order, int dtype) {
    return layout(n, level, order, dtype == kDtypeF64 ? sizeof(double) : sizeof(float)).total;
}

hipError_t launch_fmm(int dtype, int64_t n, const void* x, const void* g, const void* sg, int64_t ld, int level,
                      int order, int classical, void* u, void* dg, void* grad, int64_t ldo, void* ws,
                      hipStream_t st) {
    if (n == 0) return hipSuccess;
    unsigned char* w = static_cast<unsigned char*>(ws);
    if (dtype == kDtypeF64)
        return run_fmm<double>(n, static_cast<const double*>(x), static_cast<const double*>(g),
                               static_cast<const double*>(sg), ld, level, order, classical, static_cast<double*>(u),
                               static_cast<double*>(dg), static_cast<double*>(grad), ldo, w, st);
    return run_fmm<float>(n, static_cast<const float*>(x), static_cast<const float*>(g), static_cast<const float*>(sg),
                          ld, level, order, classical, static_cast<float*>(u), static_cast<float*>(dg),
                          static_cast<float*>(grad), ldo, w, st);
}

}  // namespace vpm
