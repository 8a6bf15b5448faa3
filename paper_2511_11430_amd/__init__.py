"""paper_2511_11430_amd — the vortex-particle hot path of Fu & Laurendeau's NL-UVLM-VPM
rotor solver (Sec. II.A-B) on one AMD Instinct MI355X.

The compute runs in libvpm.so (HIP kernels for gfx950, C ABI in include/vpm.h).  This
module is the thin Python binding: each ``vpm_*`` function has the name of the C entry
point it calls, takes torch CUDA tensors of shape (3, n) (component-major, unit stride
along n) or (n,), allocates the outputs it is not given, and passes pointers and the
current torch stream.  It computes nothing itself.

dtype follows the tensors: float64 -> the FP64 path, float32 -> the FP32-compensated path.
"""
import ctypes

from . import _lib

F64, F32C = 0, 1
ENUM_ERROR = 4  # VPM_ERR_ENUM
INPUT_ERROR = 9  # VPM_ERR_INPUT
TRANSPOSED, CLASSICAL = 0, 1
SIGMA_SOURCE, SIGMA_SYMMETRIC = 0, 1

__all__ = ["vpm_eval_velocity_stretching", "vpm_eval_segments", "vpm_eval_segments_gradient", "vpm_segments_backward", "vpm_fmm_eval", "vpm_fmm_workspace_size", "vpm_backward", "vpm_rk3_stage",
           "vpm_rk3_stage_backward", "vpm_diagnostics", "vpm_workspace_size", "vpm_variant_count",
           "vpm_variant_info", "vpm_axial_loss", "vpm_convert", "vpm_validate_inputs", "vpm_set_plan", "vpm_get_plan", "VpmError", "F64", "F32C", "TRANSPOSED", "CLASSICAL", "SIGMA_SOURCE",
           "SIGMA_SYMMETRIC"]


class VpmError(RuntimeError):
    """A libvpm call returned a non-zero status."""

    def __init__(self, fn, status):
        msg = _lib.load().vpm_status_string(status).decode()
        super().__init__(f"{fn}: {msg} (status {status})")
        self.status = status


def _check(fn, status):
    if status != 0:
        raise VpmError(fn, status)


def _torch():
    import torch
    return torch


def _code(t):
    torch = _torch()
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32C
    raise TypeError(f"unsupported dtype {t.dtype}; use float32 or float64")


def _vec(t, name, n=None, dtype=None):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA tensor")
    if t.dim() != 2 or t.shape[0] != 3 or (t.shape[1] > 1 and t.stride(1) != 1):
        raise ValueError(f"{name} must have shape (3, n) with unit stride along n")
    if n is not None and t.shape[1] != n:
        raise ValueError(f"{name} has {t.shape[1]} items, expected {n}")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} has dtype {t.dtype}, expected {dtype}")
    return t


def _scal(t, name, n=None, dtype=None):
    if t is None:
        return None
    if not t.is_cuda or t.dim() != 1 or (t.shape[0] > 1 and t.stride(0) != 1):
        raise ValueError(f"{name} must be a contiguous 1-D CUDA tensor")
    if n is not None and t.shape[0] != n:
        raise ValueError(f"{name} has {t.shape[0]} items, expected {n}")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} has dtype {t.dtype}, expected {dtype}")
    return t


def _ld(t):
    return int(t.stride(0)) if t is not None and t.shape[1] > 0 else (t.shape[1] if t is not None else 0)


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _offsets(off):
    arr = (ctypes.c_int64 * len(off))(*[int(v) for v in off])
    return arr


def _opts(scheme=TRANSPOSED, sigma_rule=SIGMA_SOURCE, self_eval=0, accumulate=0, variant=0, gradient=0):
    o = _lib.VpmOptions()
    o.scheme, o.sigma_rule, o.self_, o.accumulate, o.variant = int(scheme), int(sigma_rule), int(self_eval), \
        int(accumulate), int(variant)
    o.gradient = int(gradient)
    return o


def vpm_workspace_size(dtype, src_off, tgt_off=None, self_eval=True, variant=0, gradient=False):
    """Workspace bytes of a (batched) evaluation; see include/vpm.h."""
    lib = _lib.load()
    so = _offsets(src_off)
    to = None if tgt_off is None else _offsets(tgt_off)
    o = _opts(self_eval=int(self_eval), variant=variant, gradient=int(gradient))
    return int(lib.vpm_workspace_size(int(dtype), len(src_off) - 1, so, to, ctypes.byref(o)))


def vpm_eval_velocity_stretching(x_src, gamma_src, sigma_src, x_tgt=None, gamma_tgt=None, sigma_tgt=None, *,
                                 tgt_exclude=None, u_out=None, dgamma_out=None, velocity_only=False,
                                 scheme=TRANSPOSED, sigma_rule=SIGMA_SOURCE, accumulate=False, variant=0,
                                 src_off=None, tgt_off=None, workspace=None, stream=None):
    """u and dGamma/dt at the targets (Eqs. 2-5).  ``x_tgt`` None: the targets are the
    sources (self evaluation, self pair skipped).  ``gamma_tgt`` None with explicit targets,
    or ``velocity_only``: velocity only (dgamma returned as None).  ``src_off``/``tgt_off``:
    batch offsets (lists) for many independent sets in one persistent launch.
    Returns (u, dgamma)."""
    torch = _torch()
    lib = _lib.load()
    dt = _code(x_src)
    tdt = x_src.dtype
    _vec(x_src, "x_src", dtype=tdt)
    n_src = x_src.shape[1]
    _vec(gamma_src, "gamma_src", n_src, tdt)
    _scal(sigma_src, "sigma_src", n_src, tdt)
    self_eval = x_tgt is None
    if self_eval:
        n_tgt = n_src
        stretch = not velocity_only
    else:
        _vec(x_tgt, "x_tgt", dtype=tdt)
        n_tgt = x_tgt.shape[1]
        _vec(gamma_tgt, "gamma_tgt", n_tgt, tdt)
        _scal(sigma_tgt, "sigma_tgt", n_tgt, tdt)
        stretch = gamma_tgt is not None and not velocity_only
    dev = x_src.device
    if u_out is None:
        u_out = torch.empty((3, n_tgt), dtype=tdt, device=dev)
    if stretch and dgamma_out is None:
        dgamma_out = torch.empty((3, n_tgt), dtype=tdt, device=dev)
    if not stretch:
        dgamma_out = None
    _vec(u_out, "u_out", n_tgt, tdt)
    _vec(dgamma_out, "dgamma_out", n_tgt, tdt)
    if tgt_exclude is not None:
        _scal(tgt_exclude, "tgt_exclude", n_tgt, torch.int32)
    if src_off is None:
        src_off = [0, n_src]
    if tgt_off is None and not self_eval:
        tgt_off = [0, n_tgt]
    n_batch = len(src_off) - 1
    so = _offsets(src_off)
    to = None if tgt_off is None else _offsets(tgt_off)
    o = _opts(scheme, sigma_rule, self_eval, accumulate, variant)
    ws_need = int(lib.vpm_workspace_size(dt, n_batch, so, to, ctypes.byref(o)))
    if ws_need and workspace is None:
        workspace = torch.empty(ws_need, dtype=torch.uint8, device=dev)
    if workspace is not None and workspace.numel() == 0:
        workspace = None
    ws_bytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    ld_src = _ld(x_src)
    ld_tgt = 0 if self_eval else _ld(x_tgt)
    st = lib.vpm_eval_velocity_stretching(
        dt, n_batch, so, to, _p(x_src), _p(gamma_src), _p(sigma_src), ld_src,
        None if self_eval else _p(x_tgt), None if self_eval else _p(gamma_tgt),
        None if self_eval else _p(sigma_tgt), ld_tgt, _p(tgt_exclude), _p(u_out), _p(dgamma_out),
        _ld(u_out), ctypes.byref(o), _p(workspace), ws_bytes, _stream(stream))
    _check("vpm_eval_velocity_stretching", st)
    return u_out, dgamma_out


def vpm_eval_velocity_gradient(x_src, gamma_src, sigma_src, x_tgt=None, gamma_tgt=None, sigma_tgt=None, *,
                               tgt_exclude=None, u_out=None, dgamma_out=None, grad_out=None, scheme=TRANSPOSED,
                               sigma_rule=SIGMA_SOURCE, accumulate=False, src_off=None, tgt_off=None,
                               workspace=None, stream=None):
    """u, dGamma/dt and the velocity gradient J (shape (9, n): J[3a+b] = du_a/dx_b) at the
    targets; arguments as vpm_eval_velocity_stretching (targets must carry Gamma).
    Returns (u, dgamma, grad)."""
    torch = _torch()
    lib = _lib.load()
    dt = _code(x_src)
    tdt = x_src.dtype
    _vec(x_src, "x_src", dtype=tdt)
    n_src = x_src.shape[1]
    _vec(gamma_src, "gamma_src", n_src, tdt)
    _scal(sigma_src, "sigma_src", n_src, tdt)
    self_eval = x_tgt is None
    if self_eval:
        n_tgt = n_src
    else:
        _vec(x_tgt, "x_tgt", dtype=tdt)
        n_tgt = x_tgt.shape[1]
        if gamma_tgt is None:
            raise ValueError("vpm_eval_velocity_gradient: the targets must carry gamma_tgt")
        _vec(gamma_tgt, "gamma_tgt", n_tgt, tdt)
        _scal(sigma_tgt, "sigma_tgt", n_tgt, tdt)
    dev = x_src.device
    if u_out is None:
        u_out = torch.empty((3, n_tgt), dtype=tdt, device=dev)
    if dgamma_out is None:
        dgamma_out = torch.empty((3, n_tgt), dtype=tdt, device=dev)
    if grad_out is None:
        grad_out = torch.empty((9, n_tgt), dtype=tdt, device=dev)
    _vec(u_out, "u_out", n_tgt, tdt)
    _vec(dgamma_out, "dgamma_out", n_tgt, tdt)
    if (not grad_out.is_cuda or grad_out.dim() != 2 or grad_out.shape[0] != 9 or grad_out.shape[1] != n_tgt
            or grad_out.dtype != tdt or (n_tgt > 1 and grad_out.stride(1) != 1)):
        raise ValueError("grad_out must be a (9, n_tgt) CUDA tensor of the particle dtype, unit stride along n")
    if _ld(grad_out) != _ld(u_out) or _ld(dgamma_out) != _ld(u_out):
        raise ValueError("u_out, dgamma_out and grad_out must share one leading dimension")
    if tgt_exclude is not None:
        _scal(tgt_exclude, "tgt_exclude", n_tgt, torch.int32)
    if src_off is None:
        src_off = [0, n_src]
    if tgt_off is None and not self_eval:
        tgt_off = [0, n_tgt]
    n_batch = len(src_off) - 1
    so = _offsets(src_off)
    to = None if tgt_off is None else _offsets(tgt_off)
    o = _opts(scheme, sigma_rule, self_eval, accumulate, 0, gradient=1)
    ws_need = int(lib.vpm_workspace_size(dt, n_batch, so, to, ctypes.byref(o)))
    if ws_need and workspace is None:
        workspace = torch.empty(ws_need, dtype=torch.uint8, device=dev)
    if workspace is not None and workspace.numel() == 0:
        workspace = None
    ws_bytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    ld_src = _ld(x_src)
    ld_tgt = 0 if self_eval else _ld(x_tgt)
    st = lib.vpm_eval_velocity_gradient(
        dt, n_batch, so, to, _p(x_src), _p(gamma_src), _p(sigma_src), ld_src,
        None if self_eval else _p(x_tgt), None if self_eval else _p(gamma_tgt),
        None if self_eval else _p(sigma_tgt), ld_tgt, _p(tgt_exclude), _p(u_out), _p(dgamma_out), _p(grad_out),
        _ld(u_out), ctypes.byref(o), _p(workspace), ws_bytes, _stream(stream))
    _check("vpm_eval_velocity_gradient", st)
    return u_out, dgamma_out, grad_out


def vpm_sgs_vreman(grad, sigma, c_v=0.07, *, nu_t_out=None, stream=None):
    """Vreman eddy viscosity per particle from J (9, n) with filter width sigma (n,)."""
    torch = _torch()
    lib = _lib.load()
    dt = _code(grad)
    if not grad.is_cuda or grad.dim() != 2 or grad.shape[0] != 9:
        raise ValueError("grad must be a CUDA tensor of shape (9, n)")
    n = grad.shape[1]
    _scal(sigma, "sigma", n, grad.dtype)
    if nu_t_out is None:
        nu_t_out = torch.empty(n, dtype=grad.dtype, device=grad.device)
    _scal(nu_t_out, "nu_t_out", n, grad.dtype)
    if n > 0 and not grad.is_contiguous():
        raise ValueError("grad must be contiguous (9, n)")
    st = lib.vpm_sgs_vreman(dt, n, _p(grad), _p(sigma), n, float(c_v), _p(nu_t_out), _stream(stream))
    _check("vpm_sgs_vreman", st)
    return nu_t_out


def vpm_eval_diffusion(x, gamma, sigma, vol, nu, nu_t=None, *, dgamma_out=None, accumulate=False, off=None,
                       workspace=None, stream=None):
    """Viscous term of Eq. 5 by PSE within each set of ``off`` (default: one set).
    Returns dgamma_out (3, n)."""
    torch = _torch()
    lib = _lib.load()
    dt = _code(x)
    tdt = x.dtype
    _vec(x, "x", dtype=tdt)
    n = x.shape[1]
    _vec(gamma, "gamma", n, tdt)
    _scal(sigma, "sigma", n, tdt)
    _scal(vol, "vol", n, tdt)
    if nu_t is not None:
        _scal(nu_t, "nu_t", n, tdt)
    if dgamma_out is None:
        if accumulate:
            raise ValueError("accumulate needs dgamma_out")
        dgamma_out = torch.empty((3, n), dtype=tdt, device=x.device)
    _vec(dgamma_out, "dgamma_out", n, tdt)
    if _ld(gamma) != _ld(x):
        raise ValueError("x and gamma must share one leading dimension")
    if off is None:
        off = [0, n]
    oo = _offsets(off)
    nb = len(off) - 1
    need = int(lib.vpm_diffusion_workspace_size(dt, nb, oo))
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=x.device)
    ws_bytes = workspace.numel() * workspace.element_size()
    st = lib.vpm_eval_diffusion(dt, nb, oo, _p(x), _p(gamma), _p(sigma), _p(vol), _p(nu_t), _ld(x), float(nu),
                                _p(dgamma_out), _ld(dgamma_out), int(bool(accumulate)), _p(workspace), ws_bytes,
                                _stream(stream))
    _check("vpm_eval_diffusion", st)
    return dgamma_out


def vpm_aic_assemble(c00, c01, c11, c10, colloc, normal, core_radius, vatistas_n=2, *, aic_out=None, stream=None):
    """FP64 influence matrix (n, n) of a vortex-ring lattice at its collocation points
    (Sec. II.A); all inputs float64 CUDA tensors of shape (3, n)."""
    torch = _torch()
    lib = _lib.load()
    n = colloc.shape[1]
    for name, t in (("c00", c00), ("c01", c01), ("c11", c11), ("c10", c10), ("colloc", colloc), ("normal", normal)):
        _vec(t, name, n, torch.float64)
    if len({_ld(t) for t in (c00, c01, c11, c10)}) != 1 or _ld(colloc) != _ld(normal):
        raise ValueError("ring corners must share one leading dimension, and so must colloc and normal")
    if aic_out is None:
        aic_out = torch.empty((n, n), dtype=torch.float64, device=colloc.device)
    if aic_out.dim() != 2 or aic_out.shape != (n, n) or aic_out.stride(1) != 1 or aic_out.dtype != torch.float64:
        raise ValueError("aic_out must be a row-major (n, n) float64 tensor")
    st = lib.vpm_aic_assemble(n, _p(c00), _p(c01), _p(c11), _p(c10), _ld(c00), _p(colloc), _p(normal), _ld(colloc),
                              float(core_radius), int(vatistas_n), _p(aic_out), int(aic_out.stride(0)), _stream(stream))
    _check("vpm_aic_assemble", st)
    return aic_out


def vpm_lu_factor(a, *, ipiv=None, info=None, stream=None):
    """In-place LU with partial pivoting of a row-major (n, n) float64 CUDA tensor.
    Returns (ipiv int32 (n,), info int32 (1,)) as device tensors."""
    torch = _torch()
    lib = _lib.load()
    n = a.shape[0]
    if a.dim() != 2 or a.shape[1] != n or a.stride(1) != 1 or a.dtype != torch.float64 or not a.is_cuda:
        raise ValueError("a must be a row-major (n, n) float64 CUDA tensor")
    if ipiv is None:
        ipiv = torch.empty(n, dtype=torch.int32, device=a.device)
    if info is None:
        info = torch.empty(1, dtype=torch.int32, device=a.device)
    st = lib.vpm_lu_factor(n, _p(a), int(a.stride(0)), _p(ipiv), _p(info), _stream(stream))
    _check("vpm_lu_factor", st)
    return ipiv, info


def vpm_lu_solve(lu, ipiv, b, *, stream=None):
    """Solves with the factors of vpm_lu_factor; b (n,) float64 is overwritten by x."""
    lib = _lib.load()
    n = lu.shape[0]
    _scal(b, "b", n)
    st = lib.vpm_lu_solve(n, _p(lu), int(lu.stride(0)), _p(ipiv), _p(b), _stream(stream))
    _check("vpm_lu_solve", st)
    return b


def vpm_wake_shed(gamma_blade, te_index, gamma_te_prev, n_blades, n_span, *, trailed_out=None, shed_out=None,
                  stream=None):
    """Kutta condition and the newest wake row's line strengths (Eq. 7); updates
    gamma_te_prev.  Returns (trailed (n_blades * (n_span + 1),), shed (n_blades * n_span,))."""
    torch = _torch()
    lib = _lib.load()
    dt = _code(gamma_blade)
    _scal(gamma_te_prev, "gamma_te_prev", n_blades * n_span, gamma_blade.dtype)
    _scal(te_index, "te_index", n_blades * n_span, torch.int32)
    if trailed_out is None:
        trailed_out = torch.empty(n_blades * (n_span + 1), dtype=gamma_blade.dtype, device=gamma_blade.device)
    if shed_out is None:
        shed_out = torch.empty(n_blades * n_span, dtype=gamma_blade.dtype, device=gamma_blade.device)
    st = lib.vpm_wake_shed(dt, int(n_blades), int(n_span), _p(gamma_blade), _p(te_index), _p(gamma_te_prev),
                           _p(trailed_out), _p(shed_out), _stream(stream))
    _check("vpm_wake_shed", st)
    return trailed_out, shed_out


def vpm_wake_convert(a, b, dgamma, tip_index, n_tip, sigma, capacity, *, n_max=64, x_out=None, gamma_out=None,
                     sigma_out=None, count_out=None, workspace=None, stream=None):
    """Wake lines a -> b (3, n) with strengths dgamma (n,) to particles (Eqs. 6-8).
    Returns (x (3, capacity), gamma (3, capacity), sigma (capacity,), count (device int64))."""
    torch = _torch()
    lib = _lib.load()
    dt = _code(a)
    n = a.shape[1]
    _vec(a, "a", dtype=a.dtype)
    _vec(b, "b", n, a.dtype)
    _scal(dgamma, "dgamma", n, a.dtype)
    _scal(tip_index, "tip_index", n, torch.int32)
    if _ld(a) != _ld(b):
        raise ValueError("a and b must share one leading dimension")
    dev = a.device
    if x_out is None:
        x_out = torch.empty((3, capacity), dtype=a.dtype, device=dev)
    if gamma_out is None:
        gamma_out = torch.empty((3, capacity), dtype=a.dtype, device=dev)
    if sigma_out is None:
        sigma_out = torch.empty(capacity, dtype=a.dtype, device=dev)
    if count_out is None:
        count_out = torch.empty(1, dtype=torch.int64, device=dev)
    if _ld(gamma_out) != _ld(x_out):
        raise ValueError("x_out and gamma_out must share one leading dimension")
    need = int(lib.vpm_wake_convert_workspace_size(n))
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    ld_out = _ld(x_out) if capacity > 0 else 0
    st = lib.vpm_wake_convert(dt, n, _p(a), _p(b), _ld(a) if n > 0 else 0, _p(dgamma), _p(tip_index), int(n_tip),
                              int(n_max), float(sigma), int(capacity), _p(x_out), _p(gamma_out), _p(sigma_out),
                              ld_out, _p(count_out), _p(workspace), workspace.numel(), _stream(stream))
    _check("vpm_wake_convert", st)
    return x_out, gamma_out, sigma_out, count_out


def _host3(v):
    return (ctypes.c_double * 3)(*[float(c) for c in v])


def vpm_aic_update(base, colloc, normal, r00, r01, r11, r10, ring_of_col, core_radius, vatistas_n=2, *, out=None,
                   stream=None):
    """out = base + the influence of extra rings in the columns ring_of_col maps them to."""
    torch = _torch()
    lib = _lib.load()
    n = colloc.shape[1]
    m = r00.shape[1]
    for name, t in (("r00", r00), ("r01", r01), ("r11", r11), ("r10", r10)):
        _vec(t, name, m, torch.float64)
    _scal(ring_of_col, "ring_of_col", n, torch.int32)
    if out is None:
        out = torch.empty_like(base)
    ldr = _ld(r00) if m > 0 else 0
    st = lib.vpm_aic_update(n, _p(base), int(base.stride(0)), _p(out), int(out.stride(0)), _p(colloc), _p(normal),
                            _ld(colloc), m, _p(r00), _p(r01), _p(r11), _p(r10), ldr, _p(ring_of_col),
                            float(core_radius), int(vatistas_n), _stream(stream))
    _check("vpm_aic_update", st)
    return out


def vpm_neumann_rhs(colloc, normal, u, v_inf, omega, *, rhs_out=None, stream=None):
    """rhs_i = -((v_inf - omega x c_i + u_i) . n_i) (Neumann condition, Sec. II.A)."""
    torch = _torch()
    lib = _lib.load()
    n = colloc.shape[1]
    _vec(u, "u", n)
    if rhs_out is None:
        rhs_out = torch.empty(n, dtype=torch.float64, device=colloc.device)
    st = lib.vpm_neumann_rhs(_code(u), n, _p(colloc), _p(normal), _ld(colloc), _p(u), _ld(u), _host3(v_inf),
                             _host3(omega), _p(rhs_out), _stream(stream))
    _check("vpm_neumann_rhs", st)
    return rhs_out


def vpm_rk3_advect(stage, x, qx, u, dt, v_inf=(0.0, 0.0, 0.0), *, gamma=None, qg=None, dgamma=None,
                   stream=None):
    """RK3 stage `stage` in place: qx = A_k qx + dt (u + v_inf), x += B_k qx (and the same for
    gamma with qg, dgamma)."""
    lib = _lib.load()
    n = x.shape[1]
    for t, name in ((qx, "qx"), (u, "u")) + (((qg, "qg"), (dgamma, "dgamma")) if gamma is not None else ()):
        _vec(t, name, n, x.dtype)
        if _ld(t) != _ld(x):
            raise ValueError("x, qx, u (and gamma, qg, dgamma) must share one leading dimension")
    if gamma is not None and _ld(gamma) != _ld(x):
        raise ValueError("x, qx, u (and gamma, qg, dgamma) must share one leading dimension")
    st = lib.vpm_rk3_advect(_code(x), int(stage), n, float(dt), _p(x), _p(qx), _p(u), _p(gamma), _p(qg),
                            _p(dgamma), _ld(x), _host3(v_inf), _stream(stream))
    _check("vpm_rk3_advect", st)
    return x


def vpm_eval_segments(a, b, gamma_seg, x_tgt, core_radius, vatistas_n=2, *, u_out=None, accumulate=False,
                      stream=None):
    """Velocity at x_tgt induced by straight vortex segments a->b (Vatistas core, Sec. II.A)."""
    torch = _torch()
    lib = _lib.load()
    dt = _code(x_tgt)
    tdt = x_tgt.dtype
    _vec(x_tgt, "x_tgt", dtype=tdt)
    n_tgt = x_tgt.shape[1]
    _vec(a, "a", dtype=tdt)
    n_seg = a.shape[1]
    _vec(b, "b", n_seg, tdt)
    _scal(gamma_seg, "gamma_seg", n_seg, tdt)
    if a.shape[1] > 0 and (b.stride(0) != a.stride(0)):
        raise ValueError("a and b must share one leading dimension")
    if u_out is None:
        u_out = torch.empty((3, n_tgt), dtype=tdt, device=x_tgt.device)
    _vec(u_out, "u_out", n_tgt, tdt)
    st = lib.vpm_eval_segments(dt, n_seg, _p(a), _p(b), _p(gamma_seg), _ld(a) if n_seg else 0,
                               float(core_radius), int(vatistas_n), n_tgt, _p(x_tgt), _ld(x_tgt), _p(u_out),
                               _ld(u_out), int(accumulate), _stream(stream))
    _check("vpm_eval_segments", st)
    return u_out


def vpm_eval_segments_gradient(a, b, gamma_seg, x_tgt, core_radius, vatistas_n=2, *, gamma_tgt=None,
                               scheme=TRANSPOSED, want_u=True, want_grad=True, u_out=None, grad_out=None,
                               dgamma_out=None, accumulate=False, stream=None):
    """Velocity (3, n), gradient J (9, n; row 3a + b = du_a/dx_b) and, with gamma_tgt, the
    stretching J^T gamma (transposed) or J gamma (classical) that straight vortex segments
    impose at x_tgt (Vatistas core, Sec. II.A).  Outputs share one leading dimension; those
    not given are allocated with the leading dimension of a given one.  Returns
    (u, J, dgamma), None where not requested."""
    torch = _torch()
    lib = _lib.load()
    dt = _code(x_tgt)
    tdt = x_tgt.dtype
    _vec(x_tgt, "x_tgt", dtype=tdt)
    n_tgt = x_tgt.shape[1]
    _vec(a, "a", dtype=tdt)
    n_seg = a.shape[1]
    _vec(b, "b", n_seg, tdt)
    _scal(gamma_seg, "gamma_seg", n_seg, tdt)
    if a.shape[1] > 0 and (b.stride(0) != a.stride(0)):
        raise ValueError("a and b must share one leading dimension")
    if gamma_tgt is not None:
        _vec(gamma_tgt, "gamma_tgt", n_tgt, tdt)
        if gamma_tgt.stride(0) != x_tgt.stride(0):
            raise ValueError("x_tgt and gamma_tgt must share one leading dimension")
    given = [t for t in (u_out, grad_out, dgamma_out) if t is not None]
    ld = _ld(given[0]) if given else n_tgt
    if any(_ld(t) != ld for t in given):
        raise ValueError("u_out, grad_out and dgamma_out must share one leading dimension")
    ld = max(ld, 1)

    def alloc(rows):
        return torch.zeros((rows, ld), dtype=tdt, device=x_tgt.device)[:, :n_tgt]
    if want_u and u_out is None:
        u_out = alloc(3)
    if want_grad and grad_out is None:
        grad_out = alloc(9)
    if gamma_tgt is not None and dgamma_out is None:
        dgamma_out = alloc(3)
    for t, nm, rows in ((u_out, "u_out", 3), (grad_out, "grad_out", 9), (dgamma_out, "dgamma_out", 3)):
        if t is not None:
            if t.dim() != 2 or t.shape[0] != rows or t.shape[1] != n_tgt or t.dtype != tdt or t.stride(1) != 1:
                raise ValueError(f"{nm} must be ({rows}, {n_tgt}) {tdt} with unit stride along points")
    if dgamma_out is not None and gamma_tgt is None:
        raise ValueError("dgamma_out needs gamma_tgt")
    st = lib.vpm_eval_segments_gradient(dt, n_seg, _p(a), _p(b), _p(gamma_seg), _ld(a) if n_seg else 0,
                                        float(core_radius), int(vatistas_n), n_tgt, _p(x_tgt),
                                        _p(gamma_tgt) if gamma_tgt is not None else None, _ld(x_tgt), int(scheme),
                                        _p(u_out) if u_out is not None else None,
                                        _p(grad_out) if grad_out is not None else None,
                                        _p(dgamma_out) if dgamma_out is not None else None, ld, int(accumulate),
                                        _stream(stream))
    _check("vpm_eval_segments_gradient", st)
    return u_out, grad_out, dgamma_out


def vpm_segments_backward(a, b, gamma_seg, x_tgt, core_radius, vatistas_n=2, u_bar=None, dgamma_bar=None, *,
                          gamma_tgt=None, scheme=TRANSPOSED, x_bar=None, gamma_bar=None, stream=None):
    """Vector-Jacobian product of :func:`vpm_eval_segments_gradient`'s velocity and stretching
    with respect to the target particles.  Gradients are ADDED to x_bar and gamma_bar
    (zero-initialised when allocated here).  Returns (x_bar, gamma_bar); gamma_bar is None
    without dgamma_bar."""
    torch = _torch()
    lib = _lib.load()
    dt = _code(x_tgt)
    tdt = x_tgt.dtype
    _vec(x_tgt, "x_tgt", dtype=tdt)
    n_tgt = x_tgt.shape[1]
    _vec(a, "a", dtype=tdt)
    n_seg = a.shape[1]
    _vec(b, "b", n_seg, tdt)
    _scal(gamma_seg, "gamma_seg", n_seg, tdt)
    if a.shape[1] > 0 and (b.stride(0) != a.stride(0)):
        raise ValueError("a and b must share one leading dimension")
    if u_bar is None and dgamma_bar is None:
        raise ValueError("give u_bar, dgamma_bar or both")
    for t, nm in ((u_bar, "u_bar"), (dgamma_bar, "dgamma_bar")):
        if t is not None:
            _vec(t, nm, n_tgt, tdt)
    if u_bar is not None and dgamma_bar is not None and _ld(u_bar) != _ld(dgamma_bar):
        raise ValueError("u_bar and dgamma_bar must share one leading dimension")
    ld_bar = _ld(u_bar if u_bar is not None else dgamma_bar)
    if dgamma_bar is not None:
        if gamma_tgt is None:
            raise ValueError("dgamma_bar needs gamma_tgt")
        _vec(gamma_tgt, "gamma_tgt", n_tgt, tdt)
        if gamma_tgt.stride(0) != x_tgt.stride(0):
            raise ValueError("x_tgt and gamma_tgt must share one leading dimension")
    if x_bar is None:
        x_bar = torch.zeros((3, n_tgt), dtype=tdt, device=x_tgt.device)
    _vec(x_bar, "x_bar", n_tgt, tdt)
    if dgamma_bar is not None:
        if gamma_bar is None:
            gamma_bar = torch.zeros((3, max(_ld(x_bar), 1)), dtype=tdt, device=x_tgt.device)[:, :n_tgt]
        _vec(gamma_bar, "gamma_bar", n_tgt, tdt)
        if _ld(gamma_bar) != _ld(x_bar):
            raise ValueError("x_bar and gamma_bar must share one leading dimension")
    else:
        gamma_bar = None
    st = lib.vpm_segments_backward(dt, n_seg, _p(a), _p(b), _p(gamma_seg), _ld(a) if n_seg else 0,
                                   float(core_radius), int(vatistas_n), n_tgt, _p(x_tgt), _p(gamma_tgt),
                                   _ld(x_tgt), int(scheme), _p(u_bar), _p(dgamma_bar), ld_bar, _p(x_bar),
                                   _p(gamma_bar), _ld(x_bar), _stream(stream))
    _check("vpm_segments_backward", st)
    return x_bar, gamma_bar


def vpm_fmm_workspace_size(n, level, order, dtype=None):
    """Workspace bytes of :func:`vpm_fmm_eval` (dtype: torch.float64 or torch.float32)."""
    torch = _torch()
    lib = _lib.load()
    code = F64 if (dtype or torch.float64) == torch.float64 else F32C
    return int(lib.vpm_fmm_workspace_size(code, int(n), int(level), int(order)))


def vpm_fmm_eval(x, gamma, sigma, level, order, *, scheme=TRANSPOSED, u_out=None, dgamma_out=None, want_grad=False,
                 grad_out=None, workspace=None, stream=None):
    """Self-interaction (u, dgamma) of the particles by the Cartesian FMM (Sec. II.B): uniform
    octree of depth ``level``, expansions of order ``order``, exact Gaussian kernel over each
    leaf's 27 neighbours.  Returns (u, dgamma), or (u, dgamma, J) with ``want_grad`` (J of
    shape (9, n), row 3a + b = du_a/dx_b)."""
    torch = _torch()
    lib = _lib.load()
    dt = _code(x)
    tdt = x.dtype
    _vec(x, "x", dtype=tdt)
    n = x.shape[1]
    _vec(gamma, "gamma", n, tdt)
    _scal(sigma, "sigma", n, tdt)
    if n > 0 and gamma.stride(0) != x.stride(0):
        raise ValueError("x and gamma must share one leading dimension")
    if u_out is None:
        u_out = torch.empty((3, n), dtype=tdt, device=x.device)
    if dgamma_out is None:
        dgamma_out = torch.empty((3, max(_ld(u_out), 1)), dtype=tdt, device=x.device)[:, :n]
    _vec(u_out, "u_out", n, tdt)
    _vec(dgamma_out, "dgamma_out", n, tdt)
    if n > 0 and _ld(u_out) != _ld(dgamma_out):
        raise ValueError("u_out and dgamma_out must share one leading dimension")
    if want_grad and grad_out is None:
        grad_out = torch.empty((9, max(_ld(u_out), 1)), dtype=tdt, device=x.device)[:, :n]
    if grad_out is not None:
        if grad_out.dim() != 2 or grad_out.shape != (9, n) or grad_out.dtype != tdt or (n > 1 and grad_out.stride(1) != 1):
            raise ValueError(f"grad_out must be (9, {n}) {tdt} with unit stride along points")
        if n > 0 and _ld(grad_out) != _ld(u_out):
            raise ValueError("grad_out and u_out must share one leading dimension")
    need = int(lib.vpm_fmm_workspace_size(dt, n, int(level), int(order)))
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=x.device)
    ws_bytes = workspace.numel() * workspace.element_size()
    st = lib.vpm_fmm_eval(dt, n, _p(x), _p(gamma), _p(sigma), _ld(x), int(level), int(order), int(scheme), _p(u_out),
                          _p(dgamma_out), _p(grad_out), _ld(u_out), _p(workspace), ws_bytes, _stream(stream))
    _check("vpm_fmm_eval", st)
    return (u_out, dgamma_out, grad_out) if grad_out is not None else (u_out, dgamma_out)


def vpm_backward(x_src, gamma_src, sigma_src, u_bar, dgamma_bar=None, x_tgt=None, gamma_tgt=None,
                 sigma_tgt=None, *, x_src_bar=None, gamma_src_bar=None, x_tgt_bar=None, gamma_tgt_bar=None,
                 want_target_grads=False, scheme=TRANSPOSED, sigma_rule=SIGMA_SOURCE, src_off=None, tgt_off=None,
                 workspace=None, stream=None):
    """Vector-Jacobian product of :func:`vpm_eval_velocity_stretching` (either stretching
    scheme; src_off / tgt_off: many independent sets, as in the forward call).  Gradients are
    accumulated into the given arrays (zero-initialised when allocated here).
    Returns (x_src_bar, gamma_src_bar, x_tgt_bar, gamma_tgt_bar)."""
    torch = _torch()
    lib = _lib.load()
    dt = _code(x_src)
    tdt = x_src.dtype
    n_src = x_src.shape[1]
    _vec(x_src, "x_src", dtype=tdt)
    _vec(gamma_src, "gamma_src", n_src, tdt)
    _scal(sigma_src, "sigma_src", n_src, tdt)
    self_eval = x_tgt is None
    n_tgt = n_src if self_eval else x_tgt.shape[1]
    if not self_eval:
        _vec(x_tgt, "x_tgt", dtype=tdt)
        _vec(gamma_tgt, "gamma_tgt", n_tgt, tdt)
        _scal(sigma_tgt, "sigma_tgt", n_tgt, tdt)
    _vec(u_bar, "u_bar", n_tgt, tdt)
    _vec(dgamma_bar, "dgamma_bar", n_tgt, tdt)
    dev = x_src.device
    if x_src_bar is None:
        x_src_bar = torch.zeros((3, n_src), dtype=tdt, device=dev)
    if gamma_src_bar is None:
        gamma_src_bar = torch.zeros((3, n_src), dtype=tdt, device=dev)
    if not self_eval and want_target_grads:
        if x_tgt_bar is None:
            x_tgt_bar = torch.zeros((3, n_tgt), dtype=tdt, device=dev)
        if gamma_tgt_bar is None and dgamma_bar is not None:
            gamma_tgt_bar = torch.zeros((3, n_tgt), dtype=tdt, device=dev)
    so = _offsets([0, n_src] if src_off is None else src_off)
    nb = len(so) - 1
    if self_eval:
        to = None
    else:
        to = _offsets([0, n_tgt] if tgt_off is None else tgt_off)
        if len(to) != len(so):
            raise ValueError("src_off and tgt_off must have the same length")
    if nb > 1 and workspace is None:
        need = lib.vpm_backward_workspace_size(dt, nb, so, to)
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    o = _opts(scheme, sigma_rule, self_eval, 1, 0)
    st = lib.vpm_backward(dt, nb, so, to, _p(x_src), _p(gamma_src), _p(sigma_src), _ld(x_src),
                          None if self_eval else _p(x_tgt), None if self_eval else _p(gamma_tgt),
                          None if self_eval else _p(sigma_tgt), 0 if self_eval else _ld(x_tgt), _p(u_bar),
                          _p(dgamma_bar), _p(x_src_bar), _p(gamma_src_bar), _p(x_tgt_bar), _p(gamma_tgt_bar),
                          ctypes.byref(o), _p(workspace), 0 if workspace is None else workspace.numel(),
                          _stream(stream))
    _check("vpm_backward", st)
    return x_src_bar, gamma_src_bar, x_tgt_bar, gamma_tgt_bar


def _same_ld(ref, arrays, n):
    for t, nm in arrays:
        if t is None:
            continue
        _vec(t, nm, n)
        if n and t.stride(0) != ref.stride(0):
            raise ValueError("all stage arrays must share one leading dimension")


def vpm_rk3_stage(stage, dt_step, x, gamma, qx, qg, u, dgamma, *, x_eval=None, gamma_eval=None, stream=None):
    """One low-storage RK3 stage in place: Q <- A_k Q + dt F, Y <- Y + B_k Q (Sec. II.B).
    The state (x, gamma, qx, qg) may be float64 with float32 F (mixed program); x_eval and
    gamma_eval then receive the updated state in F's type."""
    lib = _lib.load()
    dt, sdt = _code(u), _code(x)
    n = x.shape[1]
    _same_ld(x, [(x, "x"), (gamma, "gamma"), (qx, "qx"), (qg, "qg"), (u, "u"), (dgamma, "dgamma"),
                 (x_eval, "x_eval"), (gamma_eval, "gamma_eval")], n)
    st = lib.vpm_rk3_stage(dt, sdt, int(stage), n, float(dt_step), _p(x), _p(gamma), _p(qx), _p(qg), _p(u),
                           _p(dgamma), _ld(x), _p(x_eval), _p(gamma_eval), _stream(stream))
    _check("vpm_rk3_stage", st)


def vpm_rk3_stage_backward(stage, dt_step, x_bar, gamma_bar, qx_bar, qg_bar, u_seed, dgamma_seed, *, stream=None):
    """Adjoint of one RK3 stage (see include/vpm.h); seeds take u_seed's type."""
    lib = _lib.load()
    dt, sdt = _code(u_seed), _code(x_bar)
    n = x_bar.shape[1]
    _same_ld(x_bar, [(x_bar, "x_bar"), (gamma_bar, "gamma_bar"), (qx_bar, "qx_bar"), (qg_bar, "qg_bar"),
                     (u_seed, "u_seed"), (dgamma_seed, "dgamma_seed")], n)
    st = lib.vpm_rk3_stage_backward(dt, sdt, int(stage), n, float(dt_step), _p(x_bar), _p(gamma_bar),
                                    _p(qx_bar), _p(qg_bar), _p(u_seed), _p(dgamma_seed), _ld(x_bar),
                                    _stream(stream))
    _check("vpm_rk3_stage_backward", st)


def vpm_convert(src, dst, *, accumulate=False, stream=None):
    """dst = src or dst += src for (3, n) arrays, converting float64 <-> float32."""
    lib = _lib.load()
    n = src.shape[1]
    _vec(src, "src")
    _vec(dst, "dst", n)
    st = lib.vpm_convert(_code(src), _code(dst), n, _p(src), _ld(src), _p(dst), _ld(dst), int(accumulate),
                         _stream(stream))
    _check("vpm_convert", st)


def vpm_diagnostics(x, gamma, u, dgamma, *, out=None, workspace=None, stream=None):
    """FP64 invariants reduced on the GPU; returns a float64 CUDA tensor of 13 values
    (sum Gamma, sum dGamma/dt, impulse, impulse rate, non-finite count)."""
    torch = _torch()
    lib = _lib.load()
    dt = _code(x)
    n = x.shape[1]
    for t, nm in ((x, "x"), (gamma, "gamma"), (u, "u"), (dgamma, "dgamma")):
        _vec(t, nm, n, x.dtype)
        if n and t.stride(0) != x.stride(0):
            raise ValueError("all arrays must share one leading dimension")
    if out is None:
        out = torch.empty(13, dtype=torch.float64, device=x.device)
    need = int(lib.vpm_diagnostics_workspace_size())
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=x.device)
    st = lib.vpm_diagnostics(dt, n, _p(x), _p(gamma), _p(u), _p(dgamma), _ld(x), _p(out), _p(workspace),
                             workspace.numel() * workspace.element_size(), _stream(stream))
    _check("vpm_diagnostics", st)
    return out


def vpm_validate_inputs(x, gamma, sigma, *, out=None, workspace=None, stream=None):
    """Counts of invalid inputs on the GPU: returns a float64 CUDA tensor whose [0] is the
    number of non-positive or non-finite sigma and [1] the number of non-finite x, Gamma."""
    torch = _torch()
    lib = _lib.load()
    dt = _code(x)
    n = x.shape[1]
    _vec(x, "x", dtype=x.dtype)
    _vec(gamma, "gamma", n, x.dtype)
    _scal(sigma, "sigma", n, x.dtype)
    if n and gamma.stride(0) != x.stride(0):
        raise ValueError("x and gamma must share one leading dimension")
    if out is None:
        out = torch.empty(13, dtype=torch.float64, device=x.device)
    need = int(lib.vpm_diagnostics_workspace_size())
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=x.device)
    st = lib.vpm_validate_inputs(dt, n, _p(x), _p(gamma), _p(sigma), _ld(x), _p(out), _p(workspace),
                                 workspace.numel() * workspace.element_size(), _stream(stream))
    _check("vpm_validate_inputs", st)
    return out


def vpm_axial_loss(u_ctrl, *, loss=None, u_bar=None, loss_bar=None, want_seed=True, stream=None):
    """L = sum_c (u_c . z)^2 (float64 device scalar) and the seed 2 loss_bar (0, 0, u_z) on u_ctrl.
    Returns (loss, u_bar)."""
    torch = _torch()
    lib = _lib.load()
    dt = _code(u_ctrl)
    _vec(u_ctrl, "u_ctrl")
    m = u_ctrl.shape[1]
    if loss is None:
        loss = torch.empty((), dtype=torch.float64, device=u_ctrl.device)
    if want_seed and u_bar is None:
        u_bar = torch.empty_like(u_ctrl)
    _vec(u_bar, "u_bar", m, u_ctrl.dtype)
    if u_bar is not None and m and u_bar.stride(0) != u_ctrl.stride(0):
        raise ValueError("u_bar must share u_ctrl's leading dimension")
    if loss_bar is not None and (loss_bar.dtype != torch.float64 or loss_bar.numel() != 1 or not loss_bar.is_cuda):
        raise ValueError("loss_bar must be a float64 CUDA scalar")
    st = lib.vpm_axial_loss(dt, m, _p(u_ctrl), _ld(u_ctrl), _p(loss), _p(u_bar), _p(loss_bar), _stream(stream))
    _check("vpm_axial_loss", st)
    return loss, u_bar


def vpm_set_plan(batched, n_lo, n_hi, variant):
    """Kernel shape for FP32C launches of n_lo..n_hi targets when no variant is given."""
    _check("vpm_set_plan", _lib.load().vpm_set_plan(F32C, int(batched), int(n_lo), int(n_hi), int(variant)))


def vpm_get_plan(batched, n):
    return int(_lib.load().vpm_get_plan(F32C, int(batched), int(n)))


def vpm_check_inputs(x, gamma, sigma, *, workspace=None, stream=None):
    """Synchronous input check: True when every sigma is finite and positive and every entry of
    x and Gamma is finite, False when the library reports VPM_ERR_INPUT."""
    torch = _torch()
    lib = _lib.load()
    n = x.shape[1]
    _vec(x, "x", dtype=x.dtype)
    _vec(gamma, "gamma", n, x.dtype)
    _scal(sigma, "sigma", n, x.dtype)
    if n and gamma.stride(0) != x.stride(0):
        raise ValueError("x and gamma must share one leading dimension")
    if workspace is None:
        workspace = torch.empty(int(lib.vpm_check_inputs_workspace_size()), dtype=torch.uint8, device=x.device)
    st = lib.vpm_check_inputs(_code(x), n, _p(x), _p(gamma), _p(sigma), _ld(x), _p(workspace),
                              workspace.numel() * workspace.element_size(), _stream(stream))
    if st == INPUT_ERROR:
        return False
    _check("vpm_check_inputs", st)
    return True


def vpm_autotune(x, gamma, sigma, *, src_off=None, reps=3, u_scratch=None, dgamma_scratch=None, workspace=None,
                 stream=None):
    """Times every FP32C kernel shape on these particles (self evaluation; src_off: many sets)
    inside the library and records the fastest in its plan.  Returns (variant, [ms per shape])."""
    torch = _torch()
    lib = _lib.load()
    n = x.shape[1]
    _vec(x, "x", dtype=torch.float32)
    _vec(gamma, "gamma", n, torch.float32)
    _scal(sigma, "sigma", n, torch.float32)
    if u_scratch is None:
        u_scratch = torch.empty_like(x)
    if dgamma_scratch is None:
        dgamma_scratch = torch.empty_like(x)
    off = [0, n] if src_off is None else list(src_off)
    so = _offsets(off)
    if workspace is None and len(off) > 2:
        workspace = torch.empty(max(vpm_workspace_size(F32C, off), 1), dtype=torch.uint8, device=x.device)
    nv = vpm_variant_count()
    ms = (ctypes.c_float * nv)()
    v = ctypes.c_int32()
    st = lib.vpm_autotune(F32C, len(off) - 1, so, _p(x), _p(gamma), _p(sigma), _ld(x), _p(u_scratch),
                          _p(dgamma_scratch), _p(workspace), 0 if workspace is None else workspace.numel(),
                          int(reps), ctypes.byref(v), ms, _stream(stream))
    _check("vpm_autotune", st)
    return v.value, [float(t) for t in ms]


def vpm_variant_count():
    return int(_lib.load().vpm_variant_count())


def vpm_variant_info(k):
    a, b = ctypes.c_int32(), ctypes.c_int32()
    _check("vpm_variant_info", _lib.load().vpm_variant_info(int(k), ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value
