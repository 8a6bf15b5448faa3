"""FP64 CPU oracle for the vortex-particle hot path — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may import this package.  It wraps ``liboracle.so`` (built from ``oracle.cpp`` by
``oracle/build.py``) with numpy; it never touches the GPU library and shares no code
with it.  Every function follows the paper (Fu & Laurendeau, Sec. II.B Eqs. 2-5 and
Sec. II.A for the Vatistas-cored segments); ``oracle.cpp`` states the definitions.

All 3-vector arrays are float64 of shape (3, n) (component-major), the same layout the
GPU library takes.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

TRANSPOSED, CLASSICAL = 0, 1
SIGMA_SOURCE, SIGMA_SYMMETRIC = 0, 1
STORE_F64, STORE_F32_EVAL, STORE_F32 = 0, 1, 2  # storage models of the RK3 program

_dp = ctypes.POINTER(ctypes.c_double)
_lp = ctypes.POINTER(ctypes.c_int64)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(_LIB_PATH)
        i64, i32, dbl = ctypes.c_int64, ctypes.c_int, ctypes.c_double
        lib.orc_weights.argtypes = [dbl, _dp, _dp, _dp]
        lib.orc_ghk.argtypes = [dbl, dbl, _dp, _dp, _dp]
        lib.orc_eval.argtypes = [i64, _dp, _dp, _dp, i64, _dp, _dp, _dp, _lp, i32, i32, _dp, _dp, i32]
        lib.orc_eval_jvp.argtypes = [i64, _dp, _dp, _dp, _dp, _dp, i64, _dp, _dp, _dp, _dp, _dp, _lp,
                                     i32, i32, _dp, _dp, _dp, _dp, i32]
        lib.orc_segments.argtypes = [i64, _dp, _dp, _dp, dbl, i32, i64, _dp, _dp, i32]
        lat = [i64, _dp, _dp, _dp, dbl, i32]
        lib.orc_rk3_program.argtypes = [i64, _dp, _dp, _dp, i32, dbl, i32, i32, i64, _dp, _dp, _dp, i32] + lat + [i32]
        lib.orc_rk3_program_jvp.argtypes = [i64, _dp, _dp, _dp, _dp, _dp, i32, dbl, i32, i32, i64, _dp,
                                            _dp, _dp, i32] + lat + [i32]
        lib.orc_segments_vjp.argtypes = [i64, _dp, _dp, _dp, dbl, i32, i64, _dp, _dp, _dp, _dp, i32, _dp, _dp, i32]
        lib.orc_fmm.argtypes = [i64, _dp, _dp, _dp, i32, i32, i32, _dp, _dp, _dp, i32]
        lib.orc_inv_r_taylor.argtypes = [_dp, i32, _dp, ctypes.POINTER(ctypes.c_int)]
        lib.orc_diagnostics.argtypes = [i64, _dp, _dp, _dp, _dp, _dp]
        lib.orc_gradient.argtypes = [i64, _dp, _dp, _dp, i64, _dp, _dp, _lp, i32, _dp, i32]
        lib.orc_vreman.argtypes = [i64, _dp, _dp, dbl, _dp]
        lib.orc_pse.argtypes = [i64, _dp, _dp, _dp, _dp, _dp, dbl, _dp, i32]
        lib.orc_pse_at.argtypes = [i64, _dp, _dp, _dp, _dp, _dp, dbl, i64, _lp, _dp, i32]
        lib.orc_segments_gradient.argtypes = [i64, _dp, _dp, _dp, dbl, i32, i64, _dp, _dp, i32]
        for f in ("orc_weights", "orc_ghk", "orc_eval", "orc_eval_jvp", "orc_segments",
                  "orc_rk3_program", "orc_rk3_program_jvp", "orc_diagnostics", "orc_gradient",
                  "orc_vreman", "orc_pse", "orc_pse_at", "orc_segments_gradient", "orc_segments_vjp", "orc_fmm", "orc_inv_r_taylor"):
            getattr(lib, f).restype = ctypes.c_int
        _lib = lib
    return _lib


def _d(a):
    """float64 C-contiguous view (or copy) and its pointer."""
    if a is None:
        return None, None
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def _vec(a, name):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.ndim != 2 or a.shape[0] != 3:
        raise ValueError(f"{name} must have shape (3, n), got {a.shape}")
    return a


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what}: bad arguments (code {rc})")


def weights(rho):
    """Dimensionless blob weights (Gw, Hw, Kw) = (q/rho^3, (rho q'-3q)/rho^5,
    (rho^2 q''-7 rho q'+15 q)/rho^7) of the Gaussian of Eq. 3 at one rho."""
    lib = _load()
    a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(lib.orc_weights(float(rho), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)), "weights")
    return a.value, b.value, c.value


def ghk(s, sigma):
    """g(s), h(s) = g'(s)/s and k(s) = h'(s)/s for core size sigma (Eqs. 2-3)."""
    lib = _load()
    a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(lib.orc_ghk(float(s), float(sigma), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)), "ghk")
    return a.value, b.value, c.value


def _excl(excl, nt):
    if excl is None:
        return None, None
    e = np.ascontiguousarray(excl, dtype=np.int64)
    if e.shape != (nt,):
        raise ValueError("excl must have one entry per target")
    return e, e.ctypes.data_as(_lp)


def eval_pairs(x_src, gam_src, sig_src, x_tgt=None, gam_tgt=None, sig_tgt=None, excl=None,
               scheme=TRANSPOSED, sigma_rule=SIGMA_SOURCE, self_eval=None, nthreads=0):
    """Velocity u and stretching dGamma/dt at the targets (Eqs. 2-5), FP64, direct sums.

    With ``x_tgt`` None the targets are the sources themselves and the self pair is
    excluded (unless ``excl`` is given).  ``gam_tgt`` None with explicit targets: velocity
    only (dGamma/dt returned as None).  ``excl[t]`` is the source index skipped for target
    t (-1: none).  Returns (u, dgamma), each (3, n_tgt).
    """
    lib = _load()
    xs = _vec(x_src, "x_src")
    gs = _vec(gam_src, "gam_src")
    ss = np.ascontiguousarray(sig_src, dtype=np.float64).reshape(-1)
    ns = xs.shape[1]
    if x_tgt is None:
        xt, gt, st = xs, gs, ss
        if excl is None:
            excl = np.arange(ns, dtype=np.int64)
    else:
        xt = _vec(x_tgt, "x_tgt")
        gt = None if gam_tgt is None else _vec(gam_tgt, "gam_tgt")
        st = None if sig_tgt is None else np.ascontiguousarray(sig_tgt, dtype=np.float64).reshape(-1)
    nt = xt.shape[1]
    u = np.zeros((3, nt))
    dg = np.zeros((3, nt)) if gt is not None else None
    e, ep = _excl(excl, nt)
    rc = lib.orc_eval(ns, xs.ctypes.data_as(_dp), gs.ctypes.data_as(_dp), ss.ctypes.data_as(_dp), nt,
                      xt.ctypes.data_as(_dp), None if gt is None else gt.ctypes.data_as(_dp),
                      None if st is None else st.ctypes.data_as(_dp), ep, int(scheme), int(sigma_rule),
                      u.ctypes.data_as(_dp), None if dg is None else dg.ctypes.data_as(_dp), int(nthreads))
    _check(rc, "eval")
    return u, dg


def eval_pairs_jvp(x, gam, sig, x_dot, gam_dot, scheme=TRANSPOSED, sigma_rule=SIGMA_SOURCE,
                   x_tgt=None, gam_tgt=None, sig_tgt=None, x_tgt_dot=None, gam_tgt_dot=None,
                   excl=None, nthreads=0):
    """Forward-mode tangent of :func:`eval_pairs` on dual numbers.

    Self evaluation (``x_tgt`` None): one direction (x_dot, gam_dot) moves sources and
    targets together.  Returns (u, dgamma, u_dot, dgamma_dot).
    """
    lib = _load()
    xs, gs = _vec(x, "x"), _vec(gam, "gam")
    ss = np.ascontiguousarray(sig, dtype=np.float64).reshape(-1)
    xsd, gsd = _vec(x_dot, "x_dot"), _vec(gam_dot, "gam_dot")
    ns = xs.shape[1]
    if x_tgt is None:
        xt, gt, st, xtd, gtd = xs, gs, ss, xsd, gsd
        if excl is None:
            excl = np.arange(ns, dtype=np.int64)
    else:
        xt = _vec(x_tgt, "x_tgt")
        gt = None if gam_tgt is None else _vec(gam_tgt, "gam_tgt")
        st = None if sig_tgt is None else np.ascontiguousarray(sig_tgt, dtype=np.float64).reshape(-1)
        xtd = np.zeros_like(xt) if x_tgt_dot is None else _vec(x_tgt_dot, "x_tgt_dot")
        gtd = None if gt is None else (np.zeros_like(gt) if gam_tgt_dot is None else _vec(gam_tgt_dot, "g"))
    nt = xt.shape[1]
    u, ud = np.zeros((3, nt)), np.zeros((3, nt))
    dg = np.zeros((3, nt)) if gt is not None else None
    dgd = np.zeros((3, nt)) if gt is not None else None
    e, ep = _excl(excl, nt)
    P = lambda a: None if a is None else a.ctypes.data_as(_dp)
    rc = lib.orc_eval_jvp(ns, P(xs), P(gs), P(ss), P(xsd), P(gsd), nt, P(xt), P(gt), P(st), P(xtd),
                          P(gtd), ep, int(scheme), int(sigma_rule), P(u), P(dg), P(ud), P(dgd),
                          int(nthreads))
    _check(rc, "eval_jvp")
    return u, dg, ud, dgd


def segments(a, b, gam_seg, x_tgt, core_radius, vatistas_n=2, nthreads=0):
    """Velocity at targets induced by straight segments a->b of circulation gam_seg
    with the Vatistas core (Sec. II.A).  Returns u of shape (3, n_tgt)."""
    lib = _load()
    A, B = _vec(a, "a"), _vec(b, "b")
    g = np.ascontiguousarray(gam_seg, dtype=np.float64).reshape(-1)
    xt = _vec(x_tgt, "x_tgt")
    u = np.zeros_like(xt)
    rc = lib.orc_segments(A.shape[1], A.ctypes.data_as(_dp), B.ctypes.data_as(_dp), g.ctypes.data_as(_dp),
                          float(core_radius), int(vatistas_n), xt.shape[1], xt.ctypes.data_as(_dp),
                          u.ctypes.data_as(_dp), int(nthreads))
    _check(rc, "segments")
    return u


def segments_gradient(a, b, gam_seg, x_tgt, core_radius, vatistas_n=2, nthreads=0):
    """Velocity gradient J[a, b] = du_a/dx_b (3, 3, n_tgt) of straight segments with the
    Vatistas core (Sec. II.A) at the targets, by forward-mode differentiation of the segment law."""
    lib = _load()
    A, B = _vec(a, "a"), _vec(b, "b")
    g = np.ascontiguousarray(gam_seg, dtype=np.float64).reshape(-1)
    xt = _vec(x_tgt, "x_tgt")
    J = np.zeros((9, xt.shape[1]))
    rc = lib.orc_segments_gradient(A.shape[1], A.ctypes.data_as(_dp), B.ctypes.data_as(_dp), g.ctypes.data_as(_dp),
                                   float(core_radius), int(vatistas_n), xt.shape[1], xt.ctypes.data_as(_dp),
                                   J.ctypes.data_as(_dp), int(nthreads))
    _check(rc, "segments_gradient")
    return J.reshape(3, 3, -1)


def _lattice(segments):
    """(a, b, gamma_seg, core_radius, vatistas_n) or None -> the trailing C arguments and the
    arrays they point into (kept alive by the caller)."""
    if segments is None:
        return [0, None, None, None, 0.0, 2], ()
    a, b, g, rc, vn = segments
    A, B = _vec(a, "seg_a"), _vec(b, "seg_b")
    G = np.ascontiguousarray(g, dtype=np.float64).reshape(-1)
    if B.shape != A.shape or G.shape[0] != A.shape[1]:
        raise ValueError("segments: a, b must be (3, n) and gamma (n,)")
    return [A.shape[1], A.ctypes.data_as(_dp), B.ctypes.data_as(_dp), G.ctypes.data_as(_dp), float(rc),
            int(vn)], (A, B, G)


def fmm(x, gam, sig, level, order, scheme=TRANSPOSED, nthreads=0, want_grad=False):
    """Cartesian FMM (Sec. II.B) of the self-interaction: uniform octree of depth ``level``
    over the bounding cube, Taylor expansions of the vector potential of order ``order``,
    exact Gaussian kernel over each leaf's 27 neighbours.  Returns (u, dgamma), plus the
    velocity gradient J (3, 3, n) with ``want_grad``."""
    lib = _load()
    X, G = _vec(x, "x"), _vec(gam, "gam")
    s = np.ascontiguousarray(sig, dtype=np.float64).reshape(-1)
    u, d = np.zeros_like(X), np.zeros_like(X)
    J = np.zeros((9, X.shape[1])) if want_grad else None
    rc = lib.orc_fmm(X.shape[1], X.ctypes.data_as(_dp), G.ctypes.data_as(_dp), s.ctypes.data_as(_dp), int(level),
                     int(order), int(scheme), u.ctypes.data_as(_dp), d.ctypes.data_as(_dp),
                     None if J is None else J.ctypes.data_as(_dp), int(nthreads))
    _check(rc, "fmm")
    return (u, d, J.reshape(3, 3, -1)) if want_grad else (u, d)


def inv_r_taylor(R, Q):
    """Taylor coefficients of 1/|R + h| in h up to total degree Q: (coef, multi-indices (T, 3))."""
    lib = _load()
    from math import comb
    nt = comb(Q + 3, 3)
    c = np.zeros(nt)
    idx = np.zeros((nt, 3), dtype=np.int32)
    Rv = np.ascontiguousarray(R, dtype=np.float64)
    _check(lib.orc_inv_r_taylor(Rv.ctypes.data_as(_dp), int(Q), c.ctypes.data_as(_dp),
                                idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int))), "inv_r_taylor")
    return c, idx


def segments_vjp(a, b, gam_seg, x_tgt, core_radius, vatistas_n, u_bar, dgamma_bar=None, gam_tgt=None,
                 scheme=TRANSPOSED, nthreads=0):
    """Vector-Jacobian product of the segments' velocity u(x) and stretching s (J^T Gamma,
    transposed; J Gamma, classical) at particles (x_tgt, gam_tgt) with seeds u_bar and
    dgamma_bar: returns (x_bar, gam_bar) of L = sum u_bar . u + dgamma_bar . s (gam_bar None
    without dgamma_bar).  Second derivatives by hyper-dual numbers."""
    lib = _load()
    A, B = _vec(a, "a"), _vec(b, "b")
    g = np.ascontiguousarray(gam_seg, dtype=np.float64).reshape(-1)
    xt = _vec(x_tgt, "x_tgt")
    ub = _vec(u_bar, "u_bar")
    db = None if dgamma_bar is None else _vec(dgamma_bar, "dgamma_bar")
    gt = None if dgamma_bar is None else _vec(gam_tgt, "gam_tgt")
    xb = np.zeros_like(xt)
    gb = None if db is None else np.zeros_like(xt)
    p = lambda v: None if v is None else v.ctypes.data_as(_dp)
    rc = lib.orc_segments_vjp(A.shape[1], p(A), p(B), p(g), float(core_radius), int(vatistas_n), xt.shape[1], p(xt),
                              p(gt), p(ub), p(db), int(scheme), p(xb), p(gb), int(nthreads))
    _check(rc, "segments_vjp")
    return xb, gb


def rk3_program(x, gam, sig, n_steps, dt, y_ctrl=None, scheme=TRANSPOSED, sigma_rule=SIGMA_SOURCE,
                nthreads=0, segments=None, storage=STORE_F64):
    """n_steps of low-storage RK3 (Williamson) on (x, Gamma), then the velocity at the
    control points y_ctrl and L = sum_c (u_c . z)^2.  Returns (x, gam, u_ctrl, L).
    ``segments`` = (a, b, gamma_seg, core_radius, vatistas_n): a fixed lattice whose velocity
    and stretching act on the particles and whose velocity adds at the control points.
    ``storage``: STORE_F64 (the exact program), STORE_F32_EVAL (every evaluation reads the
    state rounded to FP32 and returns FP32 results; FP64 state) or STORE_F32 (state and
    registers also rounded to FP32 after every update)."""
    lib = _load()
    lat, keep = _lattice(segments)
    X, G = _vec(x, "x").copy(), _vec(gam, "gam").copy()
    s = np.ascontiguousarray(sig, dtype=np.float64).reshape(-1)
    m = 0 if y_ctrl is None else _vec(y_ctrl, "y_ctrl").shape[1]
    Y = None if y_ctrl is None else _vec(y_ctrl, "y_ctrl")
    uc = np.zeros((3, max(m, 1)))
    L = ctypes.c_double()
    rc = lib.orc_rk3_program(X.shape[1], X.ctypes.data_as(_dp), G.ctypes.data_as(_dp), s.ctypes.data_as(_dp),
                             int(n_steps), float(dt), int(scheme), int(sigma_rule), m,
                             None if Y is None else Y.ctypes.data_as(_dp), uc.ctypes.data_as(_dp),
                             ctypes.byref(L), int(nthreads), *lat, int(storage))
    _check(rc, "rk3_program")
    del keep
    return X, G, uc[:, :m], L.value


def rk3_program_jvp(x, gam, sig, x_dot, gam_dot, n_steps, dt, y_ctrl, scheme=TRANSPOSED,
                    sigma_rule=SIGMA_SOURCE, nthreads=0, segments=None, storage=STORE_F64):
    """Loss of :func:`rk3_program` and its directional derivative along (x_dot, gam_dot)
    (rounding, under the FP32 storage models, passes tangents through unchanged)."""
    lib = _load()
    lat, keep = _lattice(segments)
    X, G = _vec(x, "x"), _vec(gam, "gam")
    Xd, Gd = _vec(x_dot, "x_dot"), _vec(gam_dot, "gam_dot")
    s = np.ascontiguousarray(sig, dtype=np.float64).reshape(-1)
    Y = _vec(y_ctrl, "y_ctrl")
    L, dL = ctypes.c_double(), ctypes.c_double()
    rc = lib.orc_rk3_program_jvp(X.shape[1], X.ctypes.data_as(_dp), G.ctypes.data_as(_dp),
                                 s.ctypes.data_as(_dp), Xd.ctypes.data_as(_dp), Gd.ctypes.data_as(_dp),
                                 int(n_steps), float(dt), int(scheme), int(sigma_rule), Y.shape[1],
                                 Y.ctypes.data_as(_dp), ctypes.byref(L), ctypes.byref(dL), int(nthreads), *lat,
                                 int(storage))
    _check(rc, "rk3_program_jvp")
    del keep
    return L.value, dL.value


def diagnostics(x, gam, u, dgam):
    """FP64 invariants: dict with sum_gamma, sum_dgamma, impulse, impulse_rate (3-vectors)
    and nonfinite (count)."""
    lib = _load()
    X, G, U, D = (_vec(a, n) for a, n in ((x, "x"), (gam, "gam"), (u, "u"), (dgam, "dgam")))
    out = np.zeros(13)
    _check(lib.orc_diagnostics(X.shape[1], X.ctypes.data_as(_dp), G.ctypes.data_as(_dp),
                               U.ctypes.data_as(_dp), D.ctypes.data_as(_dp), out.ctypes.data_as(_dp)),
           "diagnostics")
    return {"sum_gamma": out[0:3], "sum_dgamma": out[3:6], "impulse": out[6:9],
            "impulse_rate": out[9:12], "nonfinite": int(out[12])}


def velocity_gradient(x_src, gam_src, sig_src, x_tgt=None, sig_tgt=None, excl=None, sigma_rule=SIGMA_SOURCE,
                      nthreads=0):
    """Velocity gradient J[a, b] = du_a/dx_b at the targets (sources fixed), shape (3, 3, n_tgt):
    J = sum_j [g [Gamma_j]_x + h (Gamma_j x r) r^T] (derivative of Eq. 2's Biot-Savart
    velocity).  With ``x_tgt`` None the targets are the sources and the self pair is skipped."""
    lib = _load()
    xs = _vec(x_src, "x_src")
    gs = _vec(gam_src, "gam_src")
    ss = np.ascontiguousarray(sig_src, dtype=np.float64).reshape(-1)
    ns = xs.shape[1]
    if x_tgt is None:
        xt, st = xs, ss
        if excl is None:
            excl = np.arange(ns, dtype=np.int64)
    else:
        xt = _vec(x_tgt, "x_tgt")
        st = None if sig_tgt is None else np.ascontiguousarray(sig_tgt, dtype=np.float64).reshape(-1)
    nt = xt.shape[1]
    e, ep = _excl(excl, nt)
    J = np.zeros((9, nt))
    _, stp = _d(st)
    _check(lib.orc_gradient(ns, xs.ctypes.data_as(_dp), gs.ctypes.data_as(_dp), ss.ctypes.data_as(_dp), nt,
                            xt.ctypes.data_as(_dp), stp, ep, int(sigma_rule), J.ctypes.data_as(_dp), int(nthreads)),
           "gradient")
    return J.reshape(3, 3, nt)


def vreman(J, sigma, c_v=0.07):
    """Vreman eddy viscosity per particle from J (3, 3, n) with filter width sigma (n,)
    (Sec. II.B: Vreman's model, C_V = 0.07)."""
    lib = _load()
    J = np.ascontiguousarray(np.asarray(J, dtype=np.float64).reshape(9, -1))
    n = J.shape[1]
    sg = np.ascontiguousarray(sigma, dtype=np.float64).reshape(-1)
    if sg.shape != (n,):
        raise ValueError("sigma must have one entry per particle")
    nut = np.zeros(n)
    _check(lib.orc_vreman(n, J.ctypes.data_as(_dp), sg.ctypes.data_as(_dp), float(c_v), nut.ctypes.data_as(_dp)),
           "vreman")
    return nut


def pse(x, gam, sigma, vol, nu, nu_t=None, targets=None, nthreads=0):
    """Viscous term nu lap(Gamma_i) of Eq. 5 by particle strength exchange with the Gaussian
    of Eq. 3, for one particle set: returns dGamma/dt (3, n), or (3, len(targets)) at the
    listed particle indices only."""
    lib = _load()
    x = _vec(x, "x")
    g = _vec(gam, "gam")
    n = x.shape[1]
    sg = np.ascontiguousarray(sigma, dtype=np.float64).reshape(-1)
    vo = np.ascontiguousarray(vol, dtype=np.float64).reshape(-1)
    if sg.shape != (n,) or vo.shape != (n,):
        raise ValueError("sigma and vol must have one entry per particle")
    nt_, ntp = _d(None if nu_t is None else np.asarray(nu_t, dtype=np.float64).reshape(-1))
    if nt_ is not None and nt_.shape != (n,):
        raise ValueError("nu_t must have one entry per particle")
    if targets is not None:
        tg = np.ascontiguousarray(targets, dtype=np.int64).reshape(-1)
        dg = np.zeros((3, tg.shape[0]))
        _check(lib.orc_pse_at(n, x.ctypes.data_as(_dp), g.ctypes.data_as(_dp), sg.ctypes.data_as(_dp),
                              vo.ctypes.data_as(_dp), ntp, float(nu), tg.shape[0], tg.ctypes.data_as(_lp),
                              dg.ctypes.data_as(_dp), int(nthreads)), "pse_at")
        return dg
    dg = np.zeros((3, n))
    _check(lib.orc_pse(n, x.ctypes.data_as(_dp), g.ctypes.data_as(_dp), sg.ctypes.data_as(_dp),
                       vo.ctypes.data_as(_dp), ntp, float(nu), dg.ctypes.data_as(_dp), int(nthreads)), "pse")
    return dg
