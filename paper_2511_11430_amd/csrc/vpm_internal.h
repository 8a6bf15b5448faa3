// Internal interface between the libvpm host layer (vpm_api.cpp) and its HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace vpm {

enum { kDtypeF64 = 0, kDtypeF32C = 1 };
enum { kModeTransposed = 0, kModeClassical = 1, kModeVelocity = 2, kModeGradient = 3 };

// Per-target accumulator count of each mode (see pair_forward.hip for the layouts).
constexpr int nacc_of(int mode) { return mode == kModeVelocity ? 3 : (mode == kModeGradient ? 21 : 9); }
constexpr int kMaxAcc = 21;

// Arguments of the particle-pair forward kernels.  Pointers are device pointers of the
// kernel's element type; 3-vectors are [3][ld].
struct FwdArgs {
    const void* xs;
    const void* gs;
    const void* ss;
    int64_t lds;
    const void* xt;
    const void* gt;
    const void* st;
    int64_t ldt;
    const int32_t* excl;  // per-target source index to skip (or nullptr)
    void* u;
    void* dg;
    void* grad;         // gradient mode: du_a/dx_b at [3a + b][ldo]
    int64_t ldo;
    int64_t src_begin, src_end;  // single-set launch
    int64_t tgt_begin, tgt_end;
    int32_t self;
    int32_t accumulate;
    int32_t classical;  // gradient mode: stretching output in the classical scheme
    // Source split (one set only): nchunk > 1 launches a 2-D grid whose y index picks a chunk of
    // `chunk` sources; each workgroup writes FP64 partial sums part[(ch * nacc + c) * n_tgt + t]
    // and launch_pair_fwd then runs the finishing kernel that adds the chunks in order.
    double* part;
    int64_t chunk;
    int32_t nchunk;
};

// Work queue of the persistent batched launch (lives in the caller's workspace).
struct BatchQueue {
    int* counter;            // zeroed before the launch
    const int2* items;       // (set, target block), decreasing cost
    const int64_t* src_off;  // [n_sets + 1]
    const int64_t* tgt_off;  // [n_sets + 1]
    int n_items;
};

struct FwdVariant {
    int k;       // targets per lane
    int wg;      // workgroup size
    int unroll;  // sources per inner-loop iteration
};
constexpr int kNumF32Variants = 8;
extern const FwdVariant kF32Variants[kNumF32Variants];
// The gradient mode has one FP32C shape: kF32Variants[kGradientVariant] = (1, 256, 2).
constexpr int kGradientVariant = 1;
constexpr int kF64TargetsPerBlock = 256;

// variant: 0-based index into kF32Variants (ignored for FP64; must be kGradientVariant in the
// gradient mode).  bq == nullptr: one set, grid = number of target blocks; otherwise
// persistent grid over bq.
hipError_t launch_pair_fwd(int dtype, int variant, int mode, bool sym, const FwdArgs& a,
                           const BatchQueue* bq, int grid, hipStream_t st);
// Scratch of the no-allocation entry point: a file-scope device array of this many bytes
// (noalloc.hip); noalloc_scratch returns its address on the current device.
constexpr size_t kNoAllocScratchBytes = size_t(32) << 20;
hipError_t noalloc_scratch(void** ptr);
int pair_fwd_occupancy(int dtype, int variant, int mode, bool sym, bool batched);

// ---------------------------------------------------------------- segments
struct SegArgs {
    const void* a;
    const void* b;
    const void* gam;
    int64_t ld_seg;
    int64_t n_seg;
    double rc;
    int32_t vn;
    const void* xt;
    int64_t ldt;
    int64_t n_tgt;
    void* u;
    int64_t ldo;
    int32_t accumulate;
    // gradient form only (launch_segments_gradient): outputs may be null
    const void* gt;  // target strengths [3][ldt] (needed for dg)
    void* grad;      // J[(3a+b)][ldo] = du_a/dx_b
    void* dg;        // stretching [3][ldo]: J^T gamma (transposed) or J gamma (classical)
    int32_t classical;
    // adjoint form only (launch_segments_vjp): seeds [3][ldb], gradients [3][ldo] (added to)
    const void* ub;  // may be null
    const void* db;  // may be null (then gt, gb unused)
    int64_t ldb;
    void* xb;
    void* gb;
};
hipError_t launch_segments(int dtype, const SegArgs& a, hipStream_t st);

// ---------------------------------------------------------------- key sort (viscous.hip)
// Smallest power of two >= max(n, 1024), and an ascending bitonic sort of P such keys.
int64_t sort_len(int64_t n);
hipError_t sort_keys(uint64_t* keys, int64_t P, hipStream_t st);

// ---------------------------------------------------------------- Cartesian FMM (fmm.hip)
size_t fmm_workspace(int64_t n, int level, int order, int dtype);
hipError_t launch_fmm(int dtype, int64_t n, const void* x, const void* g, const void* sg, int64_t ld, int level,
                      int order, int classical, void* u, void* dg, void* grad, int64_t ldo, void* ws,
                      hipStream_t st);
hipError_t launch_segments_gradient(int dtype, const SegArgs& a, hipStream_t st);
hipError_t launch_segments_vjp(int dtype, const SegArgs& a, hipStream_t st);

// ---------------------------------------------------------------- adjoint
// Gather form: each lane owns one particle of the "lane set" and loops over the "loop set".
//   role A: lane particle is the target (needs lane seeds); loop particles are sources.
//   role B: lane particle is the source; loop particles are targets (needs loop seeds).
struct BwdArgs {
    const void* xl;  // lane set
    const void* gl;
    const void* sl;
    const void* ubl;  // lane seeds (role A)
    const void* sbl;
    int64_t ldl;
    int64_t nl;
    const void* xo;  // loop set
    const void* go;
    const void* so;
    const void* ubo;  // loop seeds (role B)
    const void* sbo;
    int64_t ldo;
    int64_t no;
    void* xbar;  // += gradients of the lane set
    void* gbar;
    int64_t ldg;
    int32_t self;  // loop set == lane set, skip j == i
};
// Lane set per workgroup of the adjoint kernel.
constexpr int kBwdWG = 256;
// Persistent launch over a queue of (set, lane block) items (lane_is_tgt: the lane set of set
// b is its target range, the loop set its source range); grid = resident workgroups.
hipError_t launch_backward_batched(int dtype, bool role_a, bool role_b, bool stretch, bool sym, const BwdArgs& a,
                                   const BatchQueue& q, int grid, int lane_is_tgt, hipStream_t st);
int backward_occupancy(int dtype, bool role_a, bool role_b, bool stretch, bool sym);
hipError_t launch_backward(int dtype, bool role_a, bool role_b, bool stretch, bool sym,
                           const BwdArgs& a, hipStream_t st);

// ---------------------------------------------------------------- viscous terms
// PSE diffusion of the particles [begin, end) of one set; ws = device scratch of
// pse_workspace(end - begin, dtype) bytes (reused by the next set once this one is done).
hipError_t launch_pse(int dtype, int64_t begin, int64_t end, const void* x, const void* g, const void* sg,
                      const void* vol, const void* nut, int64_t ld, double nu, void* dg, int64_t ldo,
                      int accumulate, void* ws, hipStream_t st);
size_t pse_workspace(int64_t n, int dtype);
hipError_t launch_vreman(int dtype, int64_t n, const void* J, int64_t ld, const void* sg, double cv, void* nut,
                         hipStream_t st);

// ---------------------------------------------------------------- blade solve and wake management
hipError_t launch_aic(int64_t n, const double* c00, const double* c01, const double* c11, const double* c10,
                      int64_t ldr, const double* col, const double* nrm, int64_t ldc, double rc, int vn, double* A,
                      int64_t lda, hipStream_t st);
hipError_t launch_lu_factor(int64_t n, double* A, int64_t lda, int32_t* ipiv, int32_t* info, hipStream_t st);
hipError_t launch_lu_solve(int64_t n, const double* LU, int64_t lda, const int32_t* ipiv, double* b,
                           hipStream_t st);
hipError_t launch_wake_shed(int dtype, int n_blades, int n_span, const void* gb, const int32_t* te, void* prev,
                            void* trailed, void* shed, hipStream_t st);
hipError_t launch_aic_update(int64_t n, const double* base, int64_t ldb, double* out, int64_t ldo, const double* col,
                             const double* nrm, int64_t ldc, int64_t m, const double* r00, const double* r01,
                             const double* r11, const double* r10, int64_t ldr, const int32_t* ring_of_col,
                             double rc, int vn, hipStream_t st);
hipError_t launch_neumann_rhs(int dtype, int64_t n, const double* col, const double* nrm, int64_t ldc, const void* u,
                              int64_t ldu, const double* vinf, const double* omega, double* rhs, hipStream_t st);
size_t conv_workspace(int64_t n);
hipError_t launch_wake_convert(int dtype, int64_t n, const void* a, const void* b, int64_t ld, const void* dg,
                               const int32_t* tip, int n_tip, int n_max, double sigma, int64_t capacity, void* xo,
                               void* go, void* so, int64_t ldo, int64_t* count, void* ws, hipStream_t st);

// ---------------------------------------------------------------- RK3 and diagnostics
hipError_t launch_rk3_stage(int dtype, int state_dtype, int stage, int64_t n, double dt, void* x, void* g,
                            void* qx, void* qg, const void* u, const void* dg, int64_t ld, void* xe, void* ge,
                            hipStream_t st);
hipError_t launch_rk3_advect(int dtype, int stage, int64_t n, double dt, void* x, void* qx, const void* u, void* g,
                            void* qg, const void* dg, int64_t ld, const double* vinf, hipStream_t st);
hipError_t launch_rk3_stage_bwd(int dtype, int state_dtype, int stage, int64_t n, double dt, const void* xb,
                                const void* gb, void* qxb, void* qgb, void* us, void* ds, int64_t ld,
                                hipStream_t st);
hipError_t launch_convert(int src_dtype, int dst_dtype, int64_t n, const void* src, int64_t lds, void* dst,
                          int64_t ldd, int add, hipStream_t st);
constexpr int kDiagBlocks = 512;
constexpr int kDiagSlots = 16;  // doubles per block partial (13 used)
hipError_t launch_diagnostics(int dtype, int64_t n, const void* x, const void* g, const void* u,
                              const void* dg, int64_t ld, double* out, double* partials,
                              hipStream_t st);

hipError_t launch_validate(int dtype, int64_t n, const void* x, const void* g, const void* sg, int64_t ld,
                           double* out, double* partials, hipStream_t st);
hipError_t launch_axial_loss(int dtype, int64_t m, const void* u, int64_t ld, double* loss, void* ubar,
                             const double* loss_bar, hipStream_t st);

// ---------------------------------------------------------------- counter calibration
int fma_chain_count();
hipError_t launch_fma_chain(int64_t n, int fmas, int form, float* out, hipStream_t st);

}  // namespace vpm
