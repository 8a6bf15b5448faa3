/* vpm.h — C ABI of libvpm: the vortex-particle hot path on one AMD Instinct MI355X (gfx950).
 *
 * The library evaluates, by direct all-pairs summation on the GPU, the right-hand side of
 * the vortex-particle equations of Fu & Laurendeau, "Nonlinear Unsteady Vortex-Lattice
 * Vortex-Particle Method with Adaptive Wake Conversion for Rotorcraft Aerodynamics":
 *
 *   particle field   w(x) = sum_j Gamma_j zeta_sigma(x - x_j)              Sec. II.B, Eq. 2
 *   Gaussian blob    zeta_sigma(rho) = (2 pi sigma^2)^(-3/2) exp(-rho^2/2)  Eq. 3
 *   convection       dx_i/dt = u_i                                          Eq. 4
 *   stretching       dGamma_i/dt = (Gamma_i . grad^T) u_i + nu lap(Gamma_i)  Eq. 5
 *
 * with u_i = sum_{j != i} g(|r|) Gamma_j x r, r = x_i - x_j, g(s) = q(s/sigma)/(4 pi s^3),
 * q(rho) = erf(rho/sqrt 2) - sqrt(2/pi) rho exp(-rho^2/2) (the Biot-Savart law of the field
 * of Eq. 2), and the stretching
 *   transposed: sum_{j != i} [ g Gamma_i x Gamma_j + h (Gamma_i . (Gamma_j x r)) r ],
 *   classical:  sum_{j != i} [ g Gamma_j x Gamma_i + h (r . Gamma_i) (Gamma_j x r) ],
 * h(s) = g'(s)/s.  It also evaluates the velocity that straight vortex segments (vortex-ring
 * edges of the lattice, Sec. II.A) induce with a Vatistas core, a hand-written adjoint of
 * the particle sums, one stage of the low-storage third-order Runge-Kutta scheme used to
 * advance (x_i, Gamma_i) (Sec. II.B) and its adjoint, FP64 invariant diagnostics, and the
 * viscous term of Eq. 5: the velocity gradient, Vreman's eddy viscosity and particle strength
 * exchange (Sec. II.B).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Device arrays are owned by the caller; the library never frees or keeps them.
 *  - A 3-vector array is component-major [3][ld]: component c of item i is at p[c*ld + i],
 *    ld >= the item count.  Scalars per item (sigma, segment circulation) are [n].
 *  - dtype VPM_F64: every float array is double and the sums run in FP64.
 *    dtype VPM_F32C: every float array is float; pair arithmetic is FP32 and each target's
 *    sums are carried as compensated FP32 pairs (hi, lo) across source chunks (TwoSum, or
 *    FastTwoSum with the error carried forward in the particle forward kernel).
 *  - Units are SI: x in m, Gamma in m^3/s, sigma in m, segment circulation in m^2/s.
 *  - Every call is asynchronous on `stream` (a hipStream_t passed as void*; NULL = the null
 *    stream).  Results are valid once the stream is synchronised.  Calls that overlap in
 *    time must not share output buffers.
 *  - Arguments are validated on the host before any HIP call; a bad argument returns its
 *    status and launches nothing.  A launch failure returns VPM_ERR_HIP.  The library
 *    prints nothing and never aborts.
 *  - The library allocates no device memory per call.  Where scratch is needed the caller
 *    passes `workspace` of at least the size the matching *_workspace_size call returns.
 */
#ifndef VPM_H
#define VPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum vpm_status {
    VPM_OK = 0,
    VPM_ERR_NULL = 1,        /* a required pointer is NULL */
    VPM_ERR_SIZE = 2,        /* a count < 0, ld < count, or a size above the supported range */
    VPM_ERR_DTYPE = 3,       /* dtype is not VPM_F64 / VPM_F32C */
    VPM_ERR_ENUM = 4,        /* scheme, sigma rule, stage, Vatistas exponent or form out of range */
    VPM_ERR_ALIAS = 5,       /* an output overlaps an input or another output */
    VPM_ERR_OFFSETS = 6,     /* batch offsets not starting at 0, decreasing, or mismatched */
    VPM_ERR_WORKSPACE = 7,   /* workspace NULL or smaller than required */
    VPM_ERR_HIP = 8,         /* the HIP runtime reported an error */
    VPM_ERR_INPUT = 9,       /* invalid input values found on the device (vpm_check_inputs) */
    VPM_ERR_UNSUPPORTED = 10 /* valid combination that this library does not implement */
} vpm_status;

typedef enum vpm_dtype { VPM_F64 = 0, VPM_F32C = 1 } vpm_dtype;

/* Eq. 5 writes (Gamma . grad^T) u: the transposed scheme is the default reading. */
typedef enum vpm_scheme { VPM_STRETCH_TRANSPOSED = 0, VPM_STRETCH_CLASSICAL = 1 } vpm_scheme;

/* Core size of a pair.  SOURCE: sigma_j of the source particle (the literal field of Eq. 2;
 * the only rule for targets that carry no sigma).  SYMMETRIC: sigma_ij^2 = (sigma_i^2 +
 * sigma_j^2)/2, which makes the pair terms antisymmetric when cores differ. */
typedef enum vpm_sigma_rule { VPM_SIGMA_SOURCE = 0, VPM_SIGMA_SYMMETRIC = 1 } vpm_sigma_rule;

typedef struct vpm_options {
    int32_t scheme;      /* vpm_scheme */
    int32_t sigma_rule;  /* vpm_sigma_rule */
    int32_t self;        /* 1: the targets are the sources (target t is source t of the same
                            batch) and the pair j == t is skipped; target arrays may be NULL */
    int32_t accumulate;  /* 1: outputs += result; 0: outputs = result */
    int32_t variant;     /* 0: tuned/default kernel shape; k > 0: variant k of
                            vpm_variant_count() (used by the tuner and the tests) */
    int32_t gradient;    /* 1: the layout is for vpm_eval_velocity_gradient (read by
                            vpm_workspace_size; vpm_eval_velocity_stretching requires 0) */
    int32_t reserved[2]; /* must be 0 */
} vpm_options;

/* ---------------------------------------------------------------------------------------
 * vpm_eval_velocity_stretching — u_t and dGamma_t/dt at every target from every source of
 * its batch (Eqs. 2-5 as above; the viscous term of Eq. 5 is vpm_eval_diffusion).
 *
 *  dtype            VPM_F64 or VPM_F32C.
 *  n_batch          number of independent particle sets (wakes), >= 1.
 *  src_off,tgt_off  host int64[n_batch+1]; batch b owns sources [src_off[b], src_off[b+1])
 *                   and targets [tgt_off[b], tgt_off[b+1]).  Must start at 0 and not
 *                   decrease.  tgt_off may be NULL with opt->self (then equals src_off).
 *  x_src [3][ld_src], gamma_src [3][ld_src], sigma_src [ld_src]: source particles; every
 *                   sigma must be > 0.
 *  x_tgt [3][ld_tgt], gamma_tgt [3][ld_tgt], sigma_tgt [ld_tgt]: targets.  gamma_tgt NULL:
 *                   velocity only (e.g. blade control points), dgamma_out must be NULL too.
 *                   sigma_tgt is read only with VPM_SIGMA_SYMMETRIC.  With opt->self the
 *                   target pointers must be NULL or equal to the source pointers.
 *  tgt_exclude      NULL, or device int32[n_tgt]: for target t the index (global, into the
 *                   source arrays) of one source to skip, -1 for none.  Used to evaluate a
 *                   subset of particles as targets without their self pair.  Ignored with
 *                   opt->self.
 *  u_out [3][ld_out], dgamma_out [3][ld_out]: results; must not overlap any input.
 *  opt              NULL = defaults (transposed, source rule, self = 0, overwrite).
 *  workspace        device scratch of vpm_workspace_size(...) bytes.  Required for n_batch > 1
 *                   (work queue).  For n_batch == 1 it holds per-chunk partial sums when the
 *                   target set is too small to fill the GPU (the sources are then split into
 *                   chunks); without it (NULL or smaller) such a set runs unsplit, correct but
 *                   slower.  Must not overlap any other argument.
 * Returns VPM_OK or the first violated condition. */
vpm_status vpm_eval_velocity_stretching(int32_t dtype, int32_t n_batch, const int64_t* src_off,
                                        const int64_t* tgt_off, const void* x_src,
                                        const void* gamma_src, const void* sigma_src,
                                        int64_t ld_src, const void* x_tgt, const void* gamma_tgt,
                                        const void* sigma_tgt, int64_t ld_tgt,
                                        const int32_t* tgt_exclude, void* u_out, void* dgamma_out,
                                        int64_t ld_out, const vpm_options* opt, void* workspace,
                                        size_t ws_bytes, void* stream);

/* vpm_eval_velocity_stretching_noalloc — vpm_eval_velocity_stretching for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same arguments without the workspace, one set only (n_batch == 1;
 * VPM_ERR_UNSUPPORTED otherwise, since the batched queue is staged from host memory).  Source-
 * split partial sums of small target sets go to a static device array of
 * vpm_noalloc_scratch_bytes() bytes (32 MiB) that the library holds on each GPU it runs on for
 * the life of the process; when the split would need more, it uses as many source chunks as
 * the array holds (results then differ from the workspace form only in summation order).  The
 * call allocates nothing (no hipMalloc, hipFree or allocating library routine; its first call
 * on a device looks up the array's address).  Every call on one GPU shares that GPU's array:
 * calls that overlap in time on one GPU (different streams, or different host threads) race
 * and must be serialised by the caller.  Errors as vpm_eval_velocity_stretching. */
vpm_status vpm_eval_velocity_stretching_noalloc(int32_t dtype, int32_t n_batch, const int64_t* src_off,
                                                const int64_t* tgt_off, const void* x_src, const void* gamma_src,
                                                const void* sigma_src, int64_t ld_src, const void* x_tgt,
                                                const void* gamma_tgt, const void* sigma_tgt, int64_t ld_tgt,
                                                const int32_t* tgt_exclude, void* u_out, void* dgamma_out,
                                                int64_t ld_out, const vpm_options* opt, void* stream);
size_t vpm_noalloc_scratch_bytes(void);

/* ---------------------------------------------------------------------------------------
 * vpm_eval_velocity_gradient — as vpm_eval_velocity_stretching, and also the velocity
 * gradient at every target, the input of the sub-grid model of Sec. II.B:
 *   J_t[a][b] = d u_a / d x_b = sum_j [ g [Gamma_j]_x + h (Gamma_j x r) r^T ]   ([w]_x y = w x y)
 * (the derivative of the Biot-Savart velocity of Eq. 2 at the target, sources fixed).  The
 * stretching output is J^T Gamma_t (transposed) or J Gamma_t (classical), the same quantity
 * vpm_eval_velocity_stretching returns.
 *
 *  Arguments as for vpm_eval_velocity_stretching, except:
 *  gamma_tgt        required (the targets are particles); dgamma_out is required.
 *  grad_out [9][ld_out]: J, row-major per target: element (a, b) of target t at
 *                   grad_out[(3a + b) ld_out + t]; must not overlap any other argument.
 *  opt->variant     ignored: the gradient kernel has one shape per dtype.
 *  workspace        vpm_workspace_size with opt->gradient = 1.
 * Returns VPM_OK or the first violated condition. */
vpm_status vpm_eval_velocity_gradient(int32_t dtype, int32_t n_batch, const int64_t* src_off,
                                      const int64_t* tgt_off, const void* x_src, const void* gamma_src,
                                      const void* sigma_src, int64_t ld_src, const void* x_tgt,
                                      const void* gamma_tgt, const void* sigma_tgt, int64_t ld_tgt,
                                      const int32_t* tgt_exclude, void* u_out, void* dgamma_out,
                                      void* grad_out, int64_t ld_out, const vpm_options* opt,
                                      void* workspace, size_t ws_bytes, void* stream);

/* Bytes of workspace vpm_eval_velocity_stretching (opt->gradient = 0) or
 * vpm_eval_velocity_gradient (opt->gradient = 1) uses for this layout and kernel shape
 * (opt->variant): the work queue for n_batch > 1, the source-split partials for a small single
 * target set, else 0.  Depends on sizes only (no HIP call).  Returns 0 also for invalid
 * arguments; the evaluation then reports them. */
size_t vpm_workspace_size(int32_t dtype, int32_t n_batch, const int64_t* src_off,
                          const int64_t* tgt_off, const vpm_options* opt);

/* ---------------------------------------------------------------------------------------
 * vpm_sgs_vreman — Vreman's sub-grid eddy viscosity per particle (Sec. II.B uses Vreman's
 * model with C_V = 0.07), with the particle's core size as the filter width:
 *   nu_t = c_v sqrt(B_beta / (alpha_ab alpha_ab)),  alpha_ab = d u_b / d x_a,
 *   beta = sigma^2 alpha^T alpha,  B_beta = b11 b22 - b12^2 + b11 b33 - b13^2 + b22 b33 - b23^2,
 * and nu_t = 0 where alpha = 0.
 *
 *  grad [9][ld]     velocity gradients as written by vpm_eval_velocity_gradient.
 *  sigma [ld]       filter width per particle (its core size), > 0.
 *  c_v              model constant (0.07 in the paper), >= 0.
 *  nu_t_out [ld]    result, m^2/s; must not overlap grad or sigma.
 * Arithmetic is FP64 for both dtypes. */
vpm_status vpm_sgs_vreman(int32_t dtype, int64_t n, const void* grad, const void* sigma, int64_t ld, double c_v,
                          void* nu_t_out, void* stream);

/* ---------------------------------------------------------------------------------------
 * vpm_eval_diffusion — the viscous term nu lap(Gamma_i) of Eq. 5 by particle strength
 * exchange (PSE, Sec. II.B) with the Gaussian of Eq. 3 as the exchange kernel, within each
 * particle set of the batch:
 *   dGamma_i/dt = sum_{j != i} (2 nu_ij / sigma_ij^2) (V_i Gamma_j - V_j Gamma_i) zeta_{sigma_ij}(|x_i - x_j|)
 *   sigma_ij^2 = (sigma_i^2 + sigma_j^2)/2,  nu_ij = nu + (nu_t,i + nu_t,j)/2,
 * which conserves sum_i Gamma_i.  Pairs beyond rho_ij = 7 (FP32C) or 9.5 (FP64) are skipped:
 * the Gaussian there is below the working precision.
 *
 *  off              host int64[n_batch+1] set offsets (as src_off above).
 *  x [3][ld], gamma [3][ld], sigma [ld]: particles (sigma > 0).
 *  vol [ld]         particle volumes V_i (> 0), m^3.
 *  nu_t [ld]        eddy viscosity per particle (vpm_sgs_vreman), or NULL for none.
 *  nu               kinematic viscosity, >= 0.
 *  dgamma_out [3][ld_out]: result (accumulate = 1: added to it, e.g. to the stretching of
 *                   vpm_eval_velocity_stretching); must not overlap any input.
 *  workspace        vpm_diffusion_workspace_size(...) bytes, required: each set is put in
 *                   Morton order there (sort keys, packed particle records and bounding boxes,
 *                   about 56 B per particle of the largest set in FP32C, 104 B in FP64), so the
 *                   cost follows the number of near pairs whatever order the particles come in.
 *                   Results are written to the particles' own indices.
 * Returns VPM_OK or the first violated condition. */
vpm_status vpm_eval_diffusion(int32_t dtype, int32_t n_batch, const int64_t* off, const void* x,
                              const void* gamma, const void* sigma, const void* vol, const void* nu_t,
                              int64_t ld, double nu, void* dgamma_out, int64_t ld_out, int32_t accumulate,
                              void* workspace, size_t ws_bytes, void* stream);
size_t vpm_diffusion_workspace_size(int32_t dtype, int32_t n_batch, const int64_t* off);  /* 0 if invalid */

/* ---------------------------------------------------------------------------------------
 * vpm_eval_segments — velocity at n_tgt points induced by n_seg straight vortex segments
 * a->b of circulation gamma_seg (vortex-ring edges and wake lines, Sec. II.A), with the
 * Vatistas core of radius core_radius and exponent vatistas_n:
 *   u(P) += gamma/(4 pi) (r1 x r2) [r0 . (r1/|r1| - r2/|r2|)] / (|r0|^2 (d^2n + rc^2n)^(1/n))
 * r1 = P - a, r2 = P - b, r0 = b - a, d = |r1 x r2| / |r0| (distance to the line).  A segment
 * whose length or either arm is below 1e-12 max(|r0|, 1 m) contributes nothing, and so does
 * a point with a zero denominator (on the line with core_radius == 0).
 *  a, b [3][ld_seg], gamma_seg [ld_seg]; x_tgt [3][ld_tgt]; u_out [3][ld_out].
 *  core_radius >= 0 (m); vatistas_n >= 1 (2 is the usual choice).
 *  accumulate: 1 = u_out += result, 0 = u_out = result. */
vpm_status vpm_eval_segments(int32_t dtype, int64_t n_seg, const void* a, const void* b,
                             const void* gamma_seg, int64_t ld_seg, double core_radius,
                             int32_t vatistas_n, int64_t n_tgt, const void* x_tgt, int64_t ld_tgt,
                             void* u_out, int64_t ld_out, int32_t accumulate, void* stream);

/* vpm_eval_segments_gradient — the segments' velocity, its gradient and the stretching they
 * impose on particles at the targets (Sec. II.A segment law; the stretching term of the
 * particle equations, Sec. II.B, with the segments' share of the velocity):
 *   J[a][b](P) = du_a/dP_b of the vpm_eval_segments law, differentiated exactly (the core
 *   factor included); pairs that law drops contribute nothing.
 *   dgamma = J^T gamma_tgt (VPM_STRETCH_TRANSPOSED) or J gamma_tgt (VPM_STRETCH_CLASSICAL).
 *  Segment arguments, core_radius, vatistas_n as vpm_eval_segments; x_tgt, gamma_tgt [3][ld_tgt]
 *  (gamma_tgt only read when dgamma_out is given).
 *  u_out [3][ld_out], grad_out [9][ld_out] (row 3a + b holds du_a/dx_b), dgamma_out
 *  [3][ld_out]: each may be NULL, not all three (unless n_tgt == 0); outputs must not overlap
 *  inputs or each other.
 *  accumulate: 1 = outputs += result, 0 = outputs = result.
 * Returns VPM_OK or the first violated condition. */
vpm_status vpm_eval_segments_gradient(int32_t dtype, int64_t n_seg, const void* a, const void* b,
                                      const void* gamma_seg, int64_t ld_seg, double core_radius,
                                      int32_t vatistas_n, int64_t n_tgt, const void* x_tgt, const void* gamma_tgt,
                                      int64_t ld_tgt, int32_t scheme, void* u_out, void* grad_out,
                                      void* dgamma_out, int64_t ld_out, int32_t accumulate, void* stream);

/* vpm_segments_backward — vector-Jacobian product of vpm_eval_segments_gradient's velocity
 * and stretching with respect to the target particles (segments held fixed): given seeds
 * u_bar and dgamma_bar on u and on s = J^T gamma_tgt (transposed) or J gamma_tgt (classical),
 * ADD to the particle gradients
 *   x_bar     += J^T u_bar + d/dx [dgamma_bar . s]   (second derivatives of the segment law),
 *   gamma_bar += J dgamma_bar (transposed) or J^T dgamma_bar (classical).
 * Used where segments (blade rings, frozen wake lines) act on particles inside a
 * differentiated time integration.
 *  Segment arguments, core_radius, vatistas_n as vpm_eval_segments; x_tgt, gamma_tgt
 *  [3][ld_tgt]; u_bar, dgamma_bar [3][ld_bar] (either may be NULL, not both); x_bar,
 *  gamma_bar [3][ld_grad].  Without dgamma_bar, gamma_tgt and gamma_bar are not used.
 *  Gradient arrays must not overlap the inputs or each other.
 * Returns VPM_OK or the first violated condition. */
vpm_status vpm_segments_backward(int32_t dtype, int64_t n_seg, const void* a, const void* b,
                                 const void* gamma_seg, int64_t ld_seg, double core_radius, int32_t vatistas_n,
                                 int64_t n_tgt, const void* x_tgt, const void* gamma_tgt, int64_t ld_tgt,
                                 int32_t scheme, const void* u_bar, const void* dgamma_bar, int64_t ld_bar,
                                 void* x_bar, void* gamma_bar, int64_t ld_grad, void* stream);

/* ---------------------------------------------------------------------------------------
 * vpm_fmm_eval — the self-interaction of n particles (velocity u and stretching dGamma/dt, as
 * vpm_eval_velocity_stretching with self = 1 and the source core rule) by a Cartesian fast
 * multipole method (Sec. II.B: the paper accelerates the velocity and its gradient with one):
 *  - a uniform octree of depth `level` over the particles' bounding cube (centre of the box,
 *    half of its largest extent); each particle belongs to the leaf floor((x - corner)/w);
 *  - each leaf's 27 neighbouring leaves are summed directly with the exact Gaussian kernel;
 *  - all other pairs through Taylor expansions of total order `order` of the vector
 *    potential of the point-vortex kernel (P2M, M2M, M2L from level 2 on, L2L, L2P), which
 *    the Gaussian equals to 2e-9 beyond seven core radii: choose the level so that the leaf
 *    width is at least seven times the largest sigma.
 * The error of the far field falls geometrically with the order (about x0.6 per order on
 * rotor wakes).  Expansions are FP64 for both dtypes; VPM_F32C sums the near field in FP32
 * with compensation.
 *  x, gamma [3][ld], sigma [ld]; u_out, dgamma_out [3][ld_out] (written, in the input order);
 *  grad_out [9][ld_out] (row 3a + b = du_a/dx_b, near pairs exact, far field from the local
 *  expansions) or NULL: the velocity gradient the paper's FMM also provides (Vreman's model).
 *  0 <= level <= 10, 1 <= order <= 20, n < 2^30.
 *  workspace        vpm_fmm_workspace_size(dtype, n, level, order) bytes (0 if invalid);
 *                   holds the sorted particles, the tree and the expansions.
 * Returns VPM_OK or the first violated condition. */
vpm_status vpm_fmm_eval(int32_t dtype, int64_t n, const void* x, const void* gamma, const void* sigma, int64_t ld,
                        int32_t level, int32_t order, int32_t scheme, void* u_out, void* dgamma_out, void* grad_out,
                        int64_t ld_out, void* workspace, size_t ws_bytes, void* stream);
size_t vpm_fmm_workspace_size(int32_t dtype, int64_t n, int32_t level, int32_t order);

/* ---------------------------------------------------------------------------------------
 * vpm_backward — vector-Jacobian product of vpm_eval_velocity_stretching (Eqs. 2-5, both
 * stretching schemes of opt->scheme, both core rules, one set or n_batch independent sets):
 * given seeds u_bar [3][ld_tgt] and dgamma_bar [3][ld_tgt] on the outputs, ADD dL/dx and
 * dL/dGamma to the gradient arrays.  sigma is not differentiated.
 *  With opt->self: sources are targets; the gradients are x_src_bar and gamma_src_bar, each
 *  particle gathering its contributions both as target and as source.  x_tgt_bar and
 *  gamma_tgt_bar must be NULL.
 *  Without self: x_src_bar/gamma_src_bar receive the source gradients (required);
 *  x_tgt_bar/gamma_tgt_bar receive the target gradients (both NULL to skip).
 *  dgamma_bar NULL: only velocities are seeded (gamma_tgt may then be NULL).
 *  n_batch > 1: sets b = [src_off[b], src_off[b+1]) (targets by tgt_off, or the same sets
 *  with self) do not interact; one persistent launch per lane role pops (set, block) items in
 *  decreasing cost from a queue kept in the workspace, which must hold
 *  vpm_backward_workspace_size() bytes and is overwritten.  The classical scheme with
 *  stretching seeds runs three launches per set (its pair term is the transposed one with
 *  the target strength and its seed exchanged) and needs no workspace.
 * Gradient arrays are [3][ld_src] / [3][ld_tgt] and must not overlap inputs or the workspace.
 * Errors: VPM_ERR_DTYPE, VPM_ERR_ENUM (options), VPM_ERR_SIZE (n_batch < 1, ld < n, more than
 * INT32_MAX particles), VPM_ERR_OFFSETS, VPM_ERR_NULL, VPM_ERR_ALIAS, VPM_ERR_WORKSPACE
 * (n_batch > 1 with a missing or short workspace), VPM_ERR_HIP. */
vpm_status vpm_backward(int32_t dtype, int32_t n_batch, const int64_t* src_off,
                        const int64_t* tgt_off, const void* x_src, const void* gamma_src,
                        const void* sigma_src, int64_t ld_src, const void* x_tgt,
                        const void* gamma_tgt, const void* sigma_tgt, int64_t ld_tgt,
                        const void* u_bar, const void* dgamma_bar, void* x_src_bar,
                        void* gamma_src_bar, void* x_tgt_bar, void* gamma_tgt_bar,
                        const vpm_options* opt, void* workspace, size_t ws_bytes, void* stream);

/* vpm_backward_workspace_size — bytes of workspace vpm_backward needs for these offsets
 * (0 for one set; tgt_off NULL: the sets of src_off); 0 also for invalid arguments. */
size_t vpm_backward_workspace_size(int32_t dtype, int32_t n_batch, const int64_t* src_off, const int64_t* tgt_off);

/* ---------------------------------------------------------------------------------------
 * Blade solve and wake management of one NL-UVLM-VPM step (Sec. II.A; Sec. II.C, Eqs. 6-8).
 *
 * vpm_aic_assemble — FP64 influence matrix of a vortex-ring lattice (the Neumann condition
 * at the collocation points, Sec. II.A):
 *   aic[i * ld_aic + j] = n_i . u_j(c_i),
 * u_j = velocity of ring j with unit circulation on the closed path c00 -> c01 -> c11 -> c10,
 * each edge by the finite-segment law with the Vatistas core (core_radius, vatistas_n), as in
 * vpm_eval_segments.
 *  c00, c01, c11, c10 [3][ld_ring]: ring corners (double); colloc, normal [3][ld_col]:
 *  collocation points (centre of each panel's 3/4-chord line) and unit normals (double).
 *  aic [n][ld_aic] (double, row-major): output; must not overlap any input.  1 <= n <= 32768. */
vpm_status vpm_aic_assemble(int64_t n, const double* c00, const double* c01, const double* c11, const double* c10,
                            int64_t ld_ring, const double* colloc, const double* normal, int64_t ld_col,
                            double core_radius, int32_t vatistas_n, double* aic, int64_t ld_aic, void* stream);

/* vpm_lu_factor — in-place LU factorisation with partial pivoting of the FP64 matrix
 * a [n][lda] (row-major): P a = L U, L unit lower (below the diagonal), U upper.  ipiv
 * (device int32[n]): row swapped with row k at step k.  info (device int32): 0, or k + 1 for
 * the first column k without a nonzero pivot (the factorisation continues past it).  Meant
 * for the blade systems (a few hundred to a few thousand panels): blocked in panels of 16
 * columns up to n = 1024 (several launches on the stream), one workgroup beyond. */
vpm_status vpm_lu_factor(int64_t n, double* a, int64_t lda, int32_t* ipiv, int32_t* info, void* stream);

/* vpm_lu_solve — solves a x = b with the factors of vpm_lu_factor; b (device double[n]) is
 * overwritten by x.  The closed step factors and solves once per time step: the wake row at
 * the trailing edge (the Kutta rings) moves with the wake, so the matrix changes every step.
 * One workgroup; up to n = 1024 in blocks of 64 rows with b in LDS. */
vpm_status vpm_lu_solve(int64_t n, const double* lu, int64_t lda, const int32_t* ipiv, double* b, void* stream);

/* vpm_wake_shed — Kutta condition and the newest wake row (Sec. II.A; Eq. 7).  The new wake
 * row takes the trailing-edge panels' circulations gamma_blade[te_index[b * n_span + c]];
 * the wake is kept as straight lines of frozen strength:
 *   trailed_out[b * (n_span + 1) + c] = G(b, c - 1) - G(b, c)   (0 outside the blade),
 *   shed_out[b * n_span + c]          = gamma_te_prev[b * n_span + c] - G(b, c),
 * then gamma_te_prev is replaced by G (zeros before the first step: the starting vortex).
 * Trailed lines run downstream, shed lines outward along the span.  Arrays are of dtype
 * (double or float); te_index is device int32 [n_blades * n_span]. */
vpm_status vpm_wake_shed(int32_t dtype, int32_t n_blades, int32_t n_span, const void* gamma_blade,
                         const int32_t* te_index, void* gamma_te_prev, void* trailed_out, void* shed_out,
                         void* stream);

/* vpm_wake_convert — wake lines to particles, the adaptive conversion of Sec. II.C.
 * Line i runs a -> b with strength dgamma[i].  Its particle count is
 *   n_i = ceil(ds_i / ds_t * n_tip)   (Eq. 8)  when tip_index[i] >= 0,
 * with ds_i = |b_i - a_i| and ds_t the length of line tip_index[i] (the tip trailed line of
 * its row), capped at n_max; n_i = 1 when tip_index[i] < 0 (shed lines), and when ds_t = 0.
 * Counts are decided in FP64 as written.  Particles (Eq. 6) go to the midpoints of n_i equal
 * sub-segments with strength dgamma (b - a) / n_i and core size sigma, line after line, in
 * line order, into x_out, gamma_out [3][ld_out] and sigma_out [ld_out] from index 0.
 *  count_out (device int64): total particle count.  Lines that would pass capacity are left
 *  out whole (the count still reports the total, so the caller can tell).
 *  workspace        vpm_wake_convert_workspace_size(n_lines) bytes.
 * dtype applies to every float array. */
vpm_status vpm_wake_convert(int32_t dtype, int64_t n_lines, const void* a, const void* b, int64_t ld_line,
                            const void* dgamma, const int32_t* tip_index, int32_t n_tip, int32_t n_max,
                            double sigma, int64_t capacity, void* x_out, void* gamma_out, void* sigma_out,
                            int64_t ld_out, int64_t* count_out, void* workspace, size_t ws_bytes, void* stream);
size_t vpm_wake_convert_workspace_size(int64_t n_lines);

/* vpm_aic_update — the influence matrix of one time step: out = base plus, in every column j
 * with ring_of_col[j] = q >= 0, the influence n_i . u_q(c_i) of extra ring q (corners r00,
 * r01, r11, r10 [3][ld_ring], m rings).  Used for the wake row at the trailing edge, whose
 * rings carry the (unknown) circulation of the trailing-edge panel they hang from (the Kutta
 * condition, Sec. II.A).  base and out [n][ld] (double, row-major) may be the same array (same
 * ld); ring_of_col is device int32 [n] (-1: none).  Other arguments as vpm_aic_assemble. */
vpm_status vpm_aic_update(int64_t n, const double* base, int64_t ld_base, double* out, int64_t ld_out,
                          const double* colloc, const double* normal, int64_t ld_col, int64_t m, const double* r00,
                          const double* r01, const double* r11, const double* r10, int64_t ld_ring,
                          const int32_t* ring_of_col, double core_radius, int32_t vatistas_n, void* stream);

/* vpm_neumann_rhs — right-hand side of the Neumann system (Sec. II.A) for a lattice turning at
 * omega (host double[3], rad/s) in a free stream v_inf (host double[3], m/s):
 *   rhs[i] = -((v_inf - omega x c_i + u[i]) . n_i),
 * u [3][ld_u] (dtype) the velocity the wake and the particles induce at the collocation
 * points c (colloc, normal [3][ld_col], double).  rhs: device double[n]. */
vpm_status vpm_neumann_rhs(int32_t dtype, int64_t n, const double* colloc, const double* normal, int64_t ld_col,
                           const void* u, int64_t ld_u, const double* v_inf, const double* omega, double* rhs,
                           void* stream);

/* vpm_rk3_advect — stage k (0, 1, 2) of Williamson's low-storage third-order Runge-Kutta
 * scheme (Sec. II.B) for n points carried by the flow in a free stream (the wake-line points
 * and the particles of the closed step):
 *   Qx <- A_k Qx + dt (u + v_inf);   x <- x + B_k Qx,
 * and, when gamma is not NULL, Qg <- A_k Qg + dt dgamma;  gamma <- gamma + B_k Qg, with
 * A = (0, -5/9, -153/128), B = (1/3, 15/16, 8/15).  u and dgamma are the right-hand side at
 * the stage's state (evaluated at time t + (0, 1/3, 3/4)[k] dt).  x, qx, u, gamma, qg, dgamma:
 * [3][ld] device arrays of dtype, caller-owned; the registers qx, qg are read at stages 1 and 2
 * and only written at stage 0.  v_inf: host double[3] (m/s).  The update is computed in FP64
 * and stored in dtype.  Errors: VPM_ERR_DTYPE, VPM_ERR_ENUM (stage), VPM_ERR_SIZE (n < 0,
 * ld < n, non-finite dt), VPM_ERR_NULL (missing array, gamma without qg or dgamma),
 * VPM_ERR_ALIAS (overlapping arrays), VPM_ERR_HIP. */
vpm_status vpm_rk3_advect(int32_t dtype, int32_t stage, int64_t n, double dt, void* x, void* qx, const void* u,
                          void* gamma, void* qg, const void* dgamma, int64_t ld, const double* v_inf, void* stream);

/* ---------------------------------------------------------------------------------------
 * vpm_rk3_stage — stage k (0, 1, 2) of Williamson's low-storage third-order Runge-Kutta
 * scheme (Sec. II.B) on Y = (x, Gamma) with register Q = (qx, qg) and F = (u, dgamma):
 *     Q <- A_k Q + dt F;   Y <- Y + B_k Q,
 * A = (0, -5/9, -153/128), B = (1/3, 15/16, 8/15).  All arrays [3][ld], n items, in place.
 *  dtype        type of u, dgamma and of x_eval, gamma_eval.
 *  state_dtype  type of x, gamma, qx, qg: equal to dtype, or VPM_F64 with dtype VPM_F32C (a
 *               mixed program: FP64 state, FP32-compensated pair sums).
 *  x_eval, gamma_eval  both NULL, or [3][ld] arrays of dtype that receive the updated state
 *               rounded to dtype (the input of the next evaluation). */
vpm_status vpm_rk3_stage(int32_t dtype, int32_t state_dtype, int32_t stage, int64_t n, double dt, void* x,
                         void* gamma, void* qx, void* qg, const void* u, const void* dgamma, int64_t ld,
                         void* x_eval, void* gamma_eval, void* stream);

/* vpm_rk3_stage_backward — adjoint of vpm_rk3_stage.  In: x_bar, gamma_bar (adjoint of Y
 * after the stage, state_dtype), qx_bar, qg_bar (adjoint of Q after the stage, state_dtype).
 * Out, in place: qx_bar, qg_bar become the adjoint of Q before the stage; u_seed,
 * dgamma_seed (dtype) receive dt (Q_bar + B_k Y_bar), the seeds to pass to vpm_backward at
 * the stage's input state; its result, added to x_bar, gamma_bar (with vpm_convert when the
 * types differ), completes the adjoint of Y before the stage.  x_bar, gamma_bar are read
 * only. */
vpm_status vpm_rk3_stage_backward(int32_t dtype, int32_t state_dtype, int32_t stage, int64_t n, double dt,
                                  const void* x_bar, const void* gamma_bar, void* qx_bar, void* qg_bar,
                                  void* u_seed, void* dgamma_seed, int64_t ld, void* stream);

/* vpm_convert — dst = src (accumulate 0) or dst += src (accumulate 1) for [3][ld] arrays, with
 * element-type conversion between VPM_F64 and VPM_F32C data.  Used to hand an FP64 state to
 * the FP32 kernels and to add FP32 gradient contributions into an FP64 adjoint state. */
vpm_status vpm_convert(int32_t src_dtype, int32_t dst_dtype, int64_t n, const void* src, int64_t ld_src, void* dst,
                       int64_t ld_dst, int32_t accumulate, void* stream);

/* ---------------------------------------------------------------------------------------
 * vpm_diagnostics — FP64 invariants of one evaluation, reduced on the GPU (for the
 * vorticity-conservation check of Eq. 1): out (device double[13]) receives
 *   [0..2] sum_i Gamma_i, [3..5] sum_i dGamma_i/dt, [6..8] linear impulse 1/2 sum x_i x Gamma_i,
 *   [9..11] its rate 1/2 sum (u_i x Gamma_i + x_i x dGamma_i/dt), [12] number of non-finite
 *   entries among x, Gamma, u, dGamma/dt.
 * Inputs [3][ld] of dtype; workspace of vpm_diagnostics_workspace_size() bytes. */
vpm_status vpm_diagnostics(int32_t dtype, int64_t n, const void* x, const void* gamma, const void* u,
                           const void* dgamma, int64_t ld, double* out, void* workspace,
                           size_t ws_bytes, void* stream);
size_t vpm_diagnostics_workspace_size(void);

/* vpm_validate_inputs — device-side check of a particle set before an evaluation: out (device
 * double[13]) receives [0] the number of particles whose sigma is not finite and > 0, [1] the
 * number of non-finite entries among x and Gamma; [2..12] are 0.  Nothing is modified; the
 * caller decides (an evaluation on such inputs is not defined).  Workspace as for
 * vpm_diagnostics. */
vpm_status vpm_validate_inputs(int32_t dtype, int64_t n, const void* x, const void* gamma, const void* sigma,
                               int64_t ld, double* out, void* workspace, size_t ws_bytes, void* stream);

/* vpm_check_inputs — synchronous form of vpm_validate_inputs for callers that want a status:
 * runs the same device check, waits for the stream, and returns VPM_ERR_INPUT when any sigma
 * is not finite and positive or any entry of x or Gamma is not finite (VPM_OK otherwise).
 * workspace: device memory of vpm_check_inputs_workspace_size() bytes (overwritten). */
vpm_status vpm_check_inputs(int32_t dtype, int64_t n, const void* x, const void* gamma, const void* sigma,
                            int64_t ld, void* workspace, size_t ws_bytes, void* stream);
size_t vpm_check_inputs_workspace_size(void);

/* ---------------------------------------------------------------------------------------
 * vpm_axial_loss — the blade-point loss used for wake gradients: L = sum_c (u_c . z)^2 over
 * m control-point velocities u [3][ld] (u_c from vpm_eval_velocity_stretching with the
 * control points as velocity-only targets).  loss (device double, may be NULL) receives L in
 * FP64.  u_bar ([3][ld] of dtype, may be NULL) receives the seed loss_bar dL/du =
 * 2 loss_bar (0, 0, u_z); loss_bar is a device double or NULL for 1. */
vpm_status vpm_axial_loss(int32_t dtype, int64_t m, const void* u, int64_t ld, double* loss, void* u_bar,
                          const double* loss_bar, void* stream);

/* ---------------------------------------------------------------------------------------
 * Kernel-shape variants of the FP32C particle kernel (targets per lane x workgroup size x
 * sources per inner-loop iteration), for the tuner and the tests.  vpm_variant_info fills
 * targets-per-lane and workgroup size of variant k (1-based); returns VPM_ERR_ENUM for an
 * unknown k. */
int32_t vpm_variant_count(void);
vpm_status vpm_variant_info(int32_t k, int32_t* targets_per_lane, int32_t* workgroup);

/* vpm_autotune — the kernel-shape tuner (FP32C only): times every shape of the particle
 * kernel (vpm_variant_count of them) on the caller's particle set(s) — a self evaluation of
 * n_batch sets with offsets src_off (host int64[n_batch+1]), x, gamma, sigma [3][ld] — with
 * HIP events on `stream`, reps timed runs each after one untimed run, keeps the fastest
 * (minimum over the runs) and records it in the plan for launches of that many targets
 * (single-set or batched, as vpm_set_plan).  u_scratch, dgamma_scratch [3][ld] receive
 * results and are overwritten; workspace as for vpm_eval_velocity_stretching (required when
 * n_batch > 1).  variant_out (host, may be NULL) receives the chosen variant (1-based), ms_out
 * (host float[vpm_variant_count()], may be NULL) each shape's best time in ms.  A setup call:
 * it synchronises the stream after each timed run and creates (and destroys) two events; it
 * allocates no device memory.  Errors: VPM_ERR_DTYPE (not FP32C), VPM_ERR_SIZE (n_batch < 1,
 * no particle, reps outside 1..1000), those of vpm_eval_velocity_stretching, VPM_ERR_HIP. */
vpm_status vpm_autotune(int32_t dtype, int32_t n_batch, const int64_t* src_off, const void* x, const void* gamma,
                        const void* sigma, int64_t ld, void* u_scratch, void* dgamma_scratch, void* workspace,
                        size_t ws_bytes, int32_t reps, int32_t* variant_out, float* ms_out, void* stream);

/* Kernel-shape plan used when opt->variant is 0 (FP32C only): for target counts in
 * [n_lo, n_hi] (rounded out to powers of two), single-set (batched = 0) or batched
 * (batched = 1, counted over all sets) launches use variant k (0 restores the default, 1).
 * Written by the tuner; process-wide, thread-safe.  vpm_get_plan returns the variant a
 * launch of n targets would use. */
vpm_status vpm_set_plan(int32_t dtype, int32_t batched, int64_t n_lo, int64_t n_hi, int32_t variant);
int32_t vpm_get_plan(int32_t dtype, int32_t batched, int64_t n);

/* vpm_fma_chain — calibration kernel for hardware counters and for the FP32 FMA rate (not part
 * of the method): n_lanes lanes each run 8 independent chains of fmas_per_chain dependent FP32
 * fused multiply-adds (a multiple of 4) and store one float to out (device float[n_lanes]).
 * form 0: the accumulating form with per-lane register operands (a = b * d + a, v_fmac_f32),
 * which the particle kernels' sums use; form 1: one operand a kernel argument held in a
 * scalar register (a = a * s + t), a slower issue form on this GPU; form 2: the three-operand
 * encoding with register operands (a = a * b + d, v_fma_f32); form 3: fmas_per_chain FP32
 * matrix steps (v_mfma_f32_16x16x4f32, four independent accumulators) per wavefront instead;
 * form 4: forms 0 and 3 interleaved.  fma_instructions (host, may be NULL) receives the number
 * of FP32 FMA instructions the launch issues (a 16x16x4 matrix step counts as 16),
 * ceil(n_lanes / 64) x (8, 16 or 24) x fmas_per_chain wavefront instructions, against which counter
 * readings (e.g. rocprofv3's SQ_INSTS_VALU_FMA_F32) are scaled, and from which the achieved
 * FMA rate follows with a timing of the launch.  Errors: VPM_ERR_SIZE, VPM_ERR_ENUM (form),
 * VPM_ERR_NULL, VPM_ERR_HIP. */
vpm_status vpm_fma_chain(int64_t n_lanes, int32_t fmas_per_chain, int32_t form, float* out,
                         int64_t* fma_instructions, void* stream);

/* Human-readable name of a status code (static string). */
const char* vpm_status_string(int32_t status);

/* Library version string (static). */
const char* vpm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* VPM_H */
