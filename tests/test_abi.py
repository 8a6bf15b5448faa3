"""The C ABI without a GPU: the library loads, exports every entry point include/vpm.h
declares, and rejects bad arguments on the host before any HIP call (fake device
pointers are never dereferenced on these paths)."""
import ctypes
import os
import re

import pytest

from paper_2511_11430_amd import _lib

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "vpm.h")

OK, NULL, SIZE, DTYPE, ENUM, ALIAS, OFFSETS, WORKSPACE, HIP, INPUT, UNSUPPORTED = range(11)
F64, F32C = 0, 1


def declared_functions():
    text = open(HDR).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vpm_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_expected_entry_points():
    names = declared_functions()
    for n in ("vpm_eval_velocity_stretching", "vpm_eval_segments", "vpm_backward", "vpm_rk3_stage",
              "vpm_rk3_stage_backward", "vpm_diagnostics", "vpm_workspace_size", "vpm_status_string"):
        assert n in names


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) == set(_lib.SIGNATURES)


def test_status_strings_and_version():
    lib = _lib.load()
    assert lib.vpm_status_string(0) == b"ok"
    assert b"NULL" in lib.vpm_status_string(1)
    assert lib.vpm_status_string(99) == b"unknown status"
    assert b"gfx950" in lib.vpm_version()
    assert lib.vpm_variant_count() == 8
    a, b = ctypes.c_int32(), ctypes.c_int32()
    assert lib.vpm_variant_info(1, ctypes.byref(a), ctypes.byref(b)) == OK and (a.value, b.value) == (2, 256)
    assert lib.vpm_variant_info(0, ctypes.byref(a), ctypes.byref(b)) == ENUM


# Fake, distinct, never-dereferenced device addresses.
def P(k):
    return ctypes.c_void_p(0x100000 * (k + 1))


def off(*v):
    return (ctypes.c_int64 * len(v))(*v)


def opts(**kw):
    o = _lib.VpmOptions()
    fields = {f[0] for f in _lib.VpmOptions._fields_}
    for k, v in kw.items():
        assert k in fields, k  # a misspelt field would be set silently on the ctypes struct
        setattr(o, k, v)
    return o


def evs(dtype=F32C, n_batch=1, so=None, to=None, xs=P(0), gs=P(1), ss=P(2), lds=100, xt=P(3), gt=P(4), st=P(5),
        ldt=50, ex=None, u=P(6), dg=P(7), ldo=50, o=None, ws=None, wsb=0):
    lib = _lib.load()
    so = off(0, 100) if so is None else so
    to = off(0, 50) if to is None else to
    o = opts() if o is None else o
    return lib.vpm_eval_velocity_stretching(dtype, n_batch, so, to, xs, gs, ss, lds, xt, gt, st, ldt, ex, u, dg, ldo,
                                            ctypes.byref(o), ws, wsb, None)


def test_eval_validation_paths():
    assert evs(dtype=7) == DTYPE
    assert evs(n_batch=0) == SIZE
    lib = _lib.load()
    o = opts()
    assert lib.vpm_eval_velocity_stretching(F32C, 1, None, off(0, 50), P(0), P(1), P(2), 100, P(3), P(4), P(5), 50,
                                            None, P(6), P(7), 50, ctypes.byref(o), None, 0, None) == NULL
    assert evs(so=off(1, 100)) == OFFSETS
    assert evs(n_batch=2, so=off(0, 60, 40), to=off(0, 20, 50)) == OFFSETS
    assert evs(lds=99) == SIZE
    assert evs(ldo=10) == SIZE
    assert evs(xs=None) == NULL
    assert evs(u=None) == NULL
    assert evs(gt=None) == NULL                    # stretching needs target strengths
    assert evs(o=opts(scheme=2)) == ENUM
    assert evs(o=opts(sigma_rule=3)) == ENUM
    assert evs(o=opts(variant=9)) == ENUM
    o = opts()
    o.reserved[1] = 1
    assert evs(o=o) == ENUM
    assert evs(o=opts(sigma_rule=1), st=None) == NULL
    assert evs(u=P(0)) == ALIAS                     # output on an input
    assert evs(dg=P(6)) == ALIAS                    # two outputs on one buffer
    assert evs(o=opts(self_=1), to=off(0, 100), xt=P(9)) == ALIAS   # self with other targets
    assert evs(o=opts(self_=1), to=off(0, 50)) == OFFSETS
    assert evs(n_batch=2, so=off(0, 60, 100), to=off(0, 20, 50)) == WORKSPACE
    # empty target set: nothing to launch, succeeds without touching the GPU
    assert evs(to=off(0, 0), ldt=0) == OK


def test_workspace_size():
    lib = _lib.load()
    o = opts()
    assert lib.vpm_workspace_size(F32C, 1, off(0, 100), off(0, 100), ctypes.byref(o)) == 0
    n = lib.vpm_workspace_size(F32C, 3, off(0, 1000, 3000, 9000), off(0, 1000, 3000, 9000), ctypes.byref(o))
    assert n >= 256 + 2 * 32 + 8 * (9000 // 128)
    assert lib.vpm_workspace_size(F32C, 2, off(0, 5, 3), off(0, 5, 3), ctypes.byref(o)) == 0


def test_segments_validation():
    lib = _lib.load()
    f = lib.vpm_eval_segments
    assert f(9, 10, P(0), P(1), P(2), 10, 0.02, 2, 5, P(3), 5, P(4), 5, 0, None) == DTYPE
    assert f(F32C, -1, P(0), P(1), P(2), 10, 0.02, 2, 5, P(3), 5, P(4), 5, 0, None) == SIZE
    assert f(F32C, 10, P(0), P(1), P(2), 9, 0.02, 2, 5, P(3), 5, P(4), 5, 0, None) == SIZE
    assert f(F32C, 10, P(0), P(1), P(2), 10, -1.0, 2, 5, P(3), 5, P(4), 5, 0, None) == SIZE
    assert f(F32C, 10, P(0), P(1), P(2), 10, 0.02, 0, 5, P(3), 5, P(4), 5, 0, None) == ENUM
    assert f(F32C, 10, None, P(1), P(2), 10, 0.02, 2, 5, P(3), 5, P(4), 5, 0, None) == NULL
    assert f(F32C, 10, P(0), P(1), P(2), 10, 0.02, 2, 5, P(3), 5, P(3), 5, 0, None) == ALIAS
    assert f(F32C, 10, P(0), P(1), P(2), 10, 0.02, 2, 0, P(3), 0, P(4), 0, 0, None) == OK


def test_backward_validation():
    lib = _lib.load()
    o = opts(self_=1)
    b = lib.vpm_backward
    args = lambda **k: [k.get("dt", F32C), k.get("nb", 1), k.get("so", off(0, 100)), None, P(0), P(1), P(2), 100,
                        None, None, None, 0, P(3), P(4), k.get("xb", P(5)), P(6), None, None,
                        ctypes.byref(k.get("o", o)), k.get("ws", None), k.get("wsb", 0), None]
    assert b(*args(dt=4)) == DTYPE
    # many sets need the queue workspace, of the size the library reports
    two = off(0, 50, 100)
    need = lib.vpm_backward_workspace_size(F32C, 2, two, None)
    assert need > 0 and lib.vpm_backward_workspace_size(F32C, 1, off(0, 100), None) == 0
    assert lib.vpm_backward_workspace_size(F32C, 2, off(0, 60, 50), None) == 0
    assert b(*args(nb=2, so=two)) == WORKSPACE
    assert b(*args(nb=2, so=two, ws=P(9), wsb=need - 1)) == WORKSPACE
    assert b(*args(nb=2, so=two, ws=P(5), wsb=need)) == ALIAS
    assert b(*args(nb=2, so=off(0, 60, 50), ws=P(9), wsb=need)) == OFFSETS
    assert b(*args(o=opts(self_=1, scheme=2))) == ENUM
    assert b(*args(xb=None)) == NULL
    assert b(*args(xb=P(0))) == ALIAS


def test_rk3_and_diagnostics_validation():
    lib = _lib.load()
    r = lib.vpm_rk3_stage
    assert r(F32C, F32C, 3, 10, 0.1, P(0), P(1), P(2), P(3), P(4), P(5), 10, None, None, None) == ENUM
    assert r(F32C, F32C, 0, 10, 0.1, P(0), P(1), P(2), P(3), P(4), P(5), 9, None, None, None) == SIZE
    assert r(F32C, F32C, 0, 10, 0.1, P(0), P(0), P(2), P(3), P(4), P(5), 10, None, None, None) == ALIAS
    assert r(F32C, F32C, 0, 10, 0.1, None, P(1), P(2), P(3), P(4), P(5), 10, None, None, None) == NULL
    assert r(F64, F32C, 0, 10, 0.1, P(0), P(1), P(2), P(3), P(4), P(5), 10, None, None, None) == DTYPE
    assert r(F32C, F64, 0, 10, 0.1, P(0), P(1), P(2), P(3), P(4), P(5), 10, P(6), None, None) == NULL
    assert r(F32C, F64, 0, 0, 0.1, None, None, None, None, None, None, 0, None, None, None) == OK
    rb = lib.vpm_rk3_stage_backward
    assert rb(F32C, F32C, -1, 10, 0.1, P(0), P(1), P(2), P(3), P(4), P(5), 10, None) == ENUM
    cv = lib.vpm_convert
    assert cv(F32C, F64, 10, P(0), 9, P(1), 10, 0, None) == SIZE
    assert cv(F32C, F64, 10, P(0), 10, P(0), 10, 0, None) == ALIAS
    assert cv(F32C, F64, 10, P(0), 10, P(1), 10, 2, None) == ENUM
    d = lib.vpm_diagnostics
    need = lib.vpm_diagnostics_workspace_size()
    assert need >= 13 * 8
    assert d(F32C, 10, P(0), P(1), P(2), P(3), 10, P(4), P(5), need - 1, None) == WORKSPACE
    assert d(F32C, 10, P(0), P(1), P(2), P(3), 10, None, P(5), need, None) == NULL


def test_plan_table():
    lib = _lib.load()
    assert lib.vpm_get_plan(F32C, 0, 1000) >= 1
    assert lib.vpm_set_plan(F64, 0, 0, 10, 2) == DTYPE
    assert lib.vpm_set_plan(F32C, 2, 0, 10, 2) == ENUM
    assert lib.vpm_set_plan(F32C, 0, 0, 10, 9) == ENUM
    assert lib.vpm_set_plan(F32C, 0, 10, 5, 2) == SIZE
    old = lib.vpm_get_plan(F32C, 0, 3000)
    assert lib.vpm_set_plan(F32C, 0, 2049, 4096, 3) == OK
    assert lib.vpm_get_plan(F32C, 0, 3000) == 3
    assert lib.vpm_get_plan(F32C, 0, 5000) != 3 or old == 3
    assert lib.vpm_set_plan(F32C, 0, 2049, 4096, old) == OK


def test_validate_inputs_validation():
    lib = _lib.load()
    v = lib.vpm_validate_inputs
    need = lib.vpm_diagnostics_workspace_size()
    assert v(5, 10, P(0), P(1), P(2), 10, P(3), P(4), need, None) == DTYPE
    assert v(F32C, 10, P(0), P(1), P(2), 9, P(3), P(4), need, None) == SIZE
    assert v(F32C, 10, P(0), P(1), None, 10, P(3), P(4), need, None) == NULL
    assert v(F32C, 10, P(0), P(1), P(2), 10, P(3), P(4), 8, None) == WORKSPACE
    assert v(F32C, 10, P(0), P(1), P(2), 10, P(0), P(4), need, None) == ALIAS


def test_check_inputs_validation():
    lib = _lib.load()
    c = lib.vpm_check_inputs
    need = lib.vpm_check_inputs_workspace_size()
    assert need >= lib.vpm_diagnostics_workspace_size() + 13 * 8
    assert c(F32C, 10, P(0), P(1), P(2), 10, P(4), need - 1, None) == WORKSPACE
    assert c(F32C, 10, P(0), P(1), P(2), 10, None, need, None) == WORKSPACE
    assert c(5, 10, P(0), P(1), P(2), 10, P(4), need, None) == DTYPE
    assert c(F32C, 10, P(0), P(1), None, 10, P(4), need, None) == NULL
    assert c(F32C, 10, P(0), P(1), P(2), 9, P(4), need, None) == SIZE
    assert c(F32C, 10, P(0), P(1), P(2), 10, P(0), need, None) == ALIAS


def test_autotune_validation():
    lib = _lib.load()
    t = lib.vpm_autotune
    v = ctypes.c_int32(-1)

    def call(dt=F32C, nb=1, so=None, reps=3, ws=None, wsb=0):
        so = off(0, 100) if so is None else so
        return t(dt, nb, so, P(0), P(1), P(2), 100, P(3), P(4), ws, wsb, reps, ctypes.byref(v), None, None)

    assert call(dt=F64) == DTYPE
    assert call(nb=0) == SIZE
    assert call(reps=0) == SIZE and call(reps=1001) == SIZE
    assert t(F32C, 1, None, P(0), P(1), P(2), 100, P(3), P(4), None, 0, 3, None, None, None) == NULL
    assert call(so=off(0, 0)) == SIZE
    assert call(nb=2, so=off(0, 60, 50)) == OFFSETS
    assert call(nb=2, so=off(0, 50, 100)) == WORKSPACE  # the batched evaluation needs its queue
    assert v.value == -1  # nothing chosen by a rejected call


def gvs(dtype=F32C, n_batch=1, so=None, to=None, xs=P(0), gs=P(1), ss=P(2), lds=100, xt=P(3), gt=P(4), st=P(5),
        ldt=50, ex=None, u=P(6), dg=P(7), J=P(8), ldo=50, o=None, ws=None, wsb=0):
    lib = _lib.load()
    so = off(0, 100) if so is None else so
    to = off(0, 50) if to is None else to
    o = opts() if o is None else o
    return lib.vpm_eval_velocity_gradient(dtype, n_batch, so, to, xs, gs, ss, lds, xt, gt, st, ldt, ex, u, dg, J,
                                          ldo, ctypes.byref(o), ws, wsb, None)


def test_gradient_validation_paths():
    assert evs(o=opts(gradient=1)) == ENUM         # the stretching entry point has no gradient output
    assert gvs(dtype=5) == DTYPE
    assert gvs(J=None) == NULL
    assert gvs(dg=None) == NULL                     # the gradient call returns the stretching too
    assert gvs(gt=None) == NULL
    assert gvs(J=P(0)) == ALIAS                     # gradient on an input
    assert gvs(J=P(6)) == ALIAS                     # gradient on the velocity output
    assert gvs(o=opts(gradient=2)) == ENUM
    assert gvs(o=opts(variant=9)) == ENUM
    assert gvs(ldo=10) == SIZE
    assert gvs(to=off(0, 0), ldt=0) == OK
    lib = _lib.load()
    # small single sets split their sources: the gradient's partials need 21 sums per target
    o0, o1 = opts(), opts(gradient=1)
    a = lib.vpm_workspace_size(F32C, 1, off(0, 1 << 20), off(0, 64), ctypes.byref(o0))
    b = lib.vpm_workspace_size(F32C, 1, off(0, 1 << 20), off(0, 64), ctypes.byref(o1))
    assert a > 0 and b > a


def test_vreman_validation():
    lib = _lib.load()
    f = lib.vpm_sgs_vreman
    assert f(3, 10, P(0), P(1), 10, 0.07, P(2), None) == DTYPE
    assert f(F32C, -1, P(0), P(1), 10, 0.07, P(2), None) == SIZE
    assert f(F32C, 10, P(0), P(1), 9, 0.07, P(2), None) == SIZE
    assert f(F32C, 10, P(0), P(1), 10, -0.1, P(2), None) == SIZE
    assert f(F32C, 10, None, P(1), 10, 0.07, P(2), None) == NULL
    assert f(F32C, 10, P(0), P(1), 10, 0.07, P(0), None) == ALIAS
    assert f(F32C, 0, None, None, 0, 0.07, None, None) == OK


def test_diffusion_validation():
    lib = _lib.load()
    f = lib.vpm_eval_diffusion
    ws = lib.vpm_diffusion_workspace_size(F32C, 1, off(0, 1000))
    assert ws >= 1024 * 8 + 1000 * 48                 # sort keys and packed records
    big = lib.vpm_diffusion_workspace_size(F64, 2, off(0, 1000, 5000))
    assert big >= 4096 * 8 + 4000 * 96                # the largest set decides
    assert lib.vpm_diffusion_workspace_size(F32C, 1, off(3, 10)) == 0

    def call(dtype=F32C, nb=1, o=None, x=P(0), g=P(1), s=P(2), v=P(3), nut=None, ld=1000, nu=1.5e-5, dg=P(5),
             ldo=1000, acc=0, w=P(6), wsb=ws):
        o = off(0, 1000) if o is None else o
        return f(dtype, nb, o, x, g, s, v, nut, ld, nu, dg, ldo, acc, w, wsb, None)

    assert call(dtype=4) == DTYPE
    assert call(nb=0) == SIZE
    assert call(o=off(1, 1000)) == OFFSETS
    assert call(ld=999) == SIZE
    assert call(nu=-1.0) == SIZE
    assert call(acc=2) == ENUM
    assert call(v=None) == NULL
    assert call(w=None) == WORKSPACE
    assert call(wsb=ws - 1) == WORKSPACE
    assert call(dg=P(0)) == ALIAS
    assert call(w=P(1)) == ALIAS
    assert call(o=off(0, 0), ld=0, ldo=0) == OK


def test_uvlm_validation():
    lib = _lib.load()
    f = lib.vpm_aic_assemble
    assert f(0, P(0), P(1), P(2), P(3), 10, P(4), P(5), 10, 0.0, 2, P(6), 10, None) == SIZE
    assert f(10, P(0), P(1), P(2), P(3), 9, P(4), P(5), 10, 0.0, 2, P(6), 10, None) == SIZE
    assert f(10, P(0), P(1), P(2), P(3), 10, P(4), P(5), 10, -1.0, 2, P(6), 10, None) == SIZE
    assert f(10, P(0), P(1), P(2), P(3), 10, P(4), P(5), 10, 0.0, 0, P(6), 10, None) == ENUM
    assert f(10, None, P(1), P(2), P(3), 10, P(4), P(5), 10, 0.0, 2, P(6), 10, None) == NULL
    assert f(10, P(0), P(1), P(2), P(3), 10, P(4), P(5), 10, 0.0, 2, P(4), 10, None) == ALIAS
    assert lib.vpm_lu_factor(0, P(0), 1, P(1), P(2), None) == SIZE
    assert lib.vpm_lu_factor(5, P(0), 4, P(1), P(2), None) == SIZE
    assert lib.vpm_lu_factor(5, P(0), 5, None, P(2), None) == NULL
    assert lib.vpm_lu_factor(5, P(0), 5, P(0), P(2), None) == ALIAS
    assert lib.vpm_lu_solve(5, P(0), 5, P(1), None, None) == NULL
    assert lib.vpm_lu_solve(5, P(0), 5, P(1), P(0), None) == ALIAS
    sh = lib.vpm_wake_shed
    assert sh(9, 2, 8, P(0), P(1), P(2), P(3), P(4), None) == DTYPE
    assert sh(F64, 0, 8, P(0), P(1), P(2), P(3), P(4), None) == SIZE
    assert sh(F64, 2, 8, P(0), None, P(2), P(3), P(4), None) == NULL
    assert sh(F64, 2, 8, P(0), P(1), P(2), P(2), P(4), None) == ALIAS
    cw = lib.vpm_wake_convert
    need = lib.vpm_wake_convert_workspace_size(100)
    assert need >= 100 * 4 + 101 * 8

    def conv(dtype=F64, n=100, a=P(0), b=P(1), ld=100, dg=P(2), tip=P(3), nt=2, nmax=64, sig=0.01, cap=500,
             x=P(4), g=P(5), s=P(6), ldo=500, cnt=P(7), w=P(8), wsb=need):
        return cw(dtype, n, a, b, ld, dg, tip, nt, nmax, sig, cap, x, g, s, ldo, cnt, w, wsb, None)

    assert conv(dtype=3) == DTYPE
    assert conv(ld=99) == SIZE
    assert conv(ldo=499) == SIZE
    assert conv(nt=0) == SIZE
    assert conv(sig=0.0) == SIZE
    assert conv(cnt=None) == NULL
    assert conv(tip=None) == NULL
    assert conv(w=None) == WORKSPACE
    assert conv(wsb=need - 1) == WORKSPACE
    assert conv(x=P(0)) == ALIAS
    assert conv(g=P(4)) == ALIAS


def test_step_kernels_validation():
    lib = _lib.load()
    v3 = (ctypes.c_double * 3)(0.0, 0.0, -1.0)
    u = lib.vpm_aic_update
    assert u(0, P(0), 1, P(1), 1, P(2), P(3), 1, 0, None, None, None, None, 0, P(4), 0.0, 2, None) == SIZE
    assert u(8, None, 8, P(1), 8, P(2), P(3), 8, 0, None, None, None, None, 0, P(4), 0.0, 2, None) == NULL
    assert u(8, P(0), 8, P(1), 8, P(2), P(3), 8, 4, None, P(6), P(7), P(8), 4, P(4), 0.0, 2, None) == NULL
    assert u(8, P(0), 8, P(0) , 7, P(2), P(3), 8, 0, None, None, None, None, 0, P(4), 0.0, 2, None) == SIZE
    assert u(8, P(0), 8, P(2), 8, P(2), P(3), 8, 0, None, None, None, None, 0, P(4), 0.0, 2, None) == ALIAS
    r = lib.vpm_neumann_rhs
    assert r(7, 8, P(0), P(1), 8, P(2), 8, v3, v3, P(3), None) == DTYPE
    assert r(F64, 8, P(0), P(1), 7, P(2), 8, v3, v3, P(3), None) == SIZE
    assert r(F64, 8, P(0), P(1), 8, P(2), 8, None, v3, P(3), None) == NULL
    assert r(F64, 8, P(0), P(1), 8, P(2), 8, v3, v3, P(0), None) == ALIAS
    assert r(F64, 0, None, None, 0, None, 0, v3, v3, None, None) == OK
    a = lib.vpm_rk3_advect
    assert a(F64, 0, 8, 0.1, P(0), P(5), P(1), None, None, None, 7, v3, None) == SIZE
    assert a(F64, 3, 8, 0.1, P(0), P(5), P(1), None, None, None, 8, v3, None) == ENUM
    assert a(7, 0, 8, 0.1, P(0), P(5), P(1), None, None, None, 8, v3, None) == DTYPE
    assert a(F64, 0, 8, 0.1, P(0), P(5), None, None, None, None, 8, v3, None) == NULL
    assert a(F64, 0, 8, 0.1, P(0), None, P(1), None, None, None, 8, v3, None) == NULL
    assert a(F64, 0, 8, 0.1, P(0), P(5), P(1), P(2), None, P(3), 8, v3, None) == NULL
    assert a(F64, 0, 8, 0.1, P(0), P(5), P(1), P(2), P(4), None, 8, v3, None) == NULL
    assert a(F64, 0, 8, 0.1, P(0), P(5), P(1), None, None, None, 8, None, None) == NULL
    assert a(F64, 0, 8, 0.1, P(0), P(5), P(0), None, None, None, 8, v3, None) == ALIAS
    assert a(F64, 0, 8, 0.1, P(0), P(5), P(1), P(2), P(4), P(2), 8, v3, None) == ALIAS
    assert a(F64, 1, 0, 0.1, None, None, None, None, None, None, 0, v3, None) == OK


def test_segments_gradient_validation():
    lib = _lib.load()
    f = lib.vpm_eval_segments_gradient

    def args(**k):
        return [k.get("dt", F32C), k.get("ns", 10), P(0), P(1), P(2), 10, k.get("rc", 0.02), k.get("vn", 2), 5, P(3),
                k.get("gt", P(4)), 5, k.get("sch", 0), k.get("u", P(5)), k.get("j", P(6)), k.get("dg", P(7)),
                k.get("ldo", 5), k.get("acc", 0), None]
    assert f(*args(dt=7)) == DTYPE
    assert f(*args(ns=-1)) == SIZE
    assert f(*args(ldo=4)) == SIZE
    assert f(*args(rc=-0.1)) == SIZE
    assert f(*args(vn=0)) == ENUM
    assert f(*args(sch=2)) == ENUM
    assert f(*args(acc=3)) == ENUM
    assert f(*args(u=None, j=None, dg=None)) == NULL
    assert f(*args(gt=None)) == NULL          # stretching needs the target strengths
    assert f(*args(j=P(3))) == ALIAS          # gradient over the targets
    assert f(*args(dg=P(4))) == ALIAS         # stretching over the target strengths
    assert f(*args(u=P(6))) == ALIAS          # two outputs on one array
    args0 = args(gt=None, dg=None)
    args0[8] = 0
    args0[11] = 0
    args0[16] = 0
    assert f(*args0) == OK                    # no targets: nothing to launch


def test_segments_backward_validation():
    lib = _lib.load()
    f = lib.vpm_segments_backward

    def args(**k):
        return [k.get("dt", F32C), 10, P(0), P(1), P(2), 10, k.get("rc", 0.02), k.get("vn", 2), 5, P(3),
                k.get("gt", P(4)), 5, k.get("sch", 0), k.get("ub", P(5)), k.get("db", P(6)), k.get("ldb", 5),
                k.get("xb", P(7)), k.get("gb", P(8)), 5, None]
    assert f(*args(dt=3)) == DTYPE
    assert f(*args(ldb=4)) == SIZE
    assert f(*args(vn=17)) == ENUM
    assert f(*args(sch=-1)) == ENUM
    assert f(*args(ub=None, db=None)) == NULL    # no seed
    assert f(*args(xb=None)) == NULL
    assert f(*args(gb=None)) == NULL             # dgamma_bar needs gamma_bar
    assert f(*args(gt=None)) == NULL             # and gamma_tgt
    assert f(*args(xb=P(3))) == ALIAS            # gradient over the positions
    assert f(*args(gb=P(6))) == ALIAS            # gradient over a seed
    assert f(*args(gb=P(7))) == ALIAS            # the two gradients on one array


def test_fmm_validation():
    lib = _lib.load()
    f = lib.vpm_fmm_eval
    ws = lib.vpm_fmm_workspace_size
    assert ws(F32C, 1000, 4, 8) > 0 and ws(F32C, 1000, 11, 8) == 0 and ws(F32C, 1000, 4, 21) == 0
    assert ws(F32C, 1000, 4, 20) > ws(F32C, 1000, 4, 16) > 0
    assert ws(7, 1000, 4, 8) == 0 and ws(F64, 1000, 4, 8) > ws(F32C, 1000, 4, 8)

    def args(**k):
        return [k.get("dt", F32C), k.get("n", 100), P(0), P(1), P(2), k.get("ld", 100), k.get("lev", 3),
                k.get("ord", 8), k.get("sch", 0), k.get("u", P(3)), k.get("d", P(4)), k.get("j", None),
                k.get("ldo", 100), k.get("w", P(5)), k.get("wb", 1 << 40), None]
    assert f(*args(dt=2)) == DTYPE
    assert f(*args(ld=99)) == SIZE
    assert f(*args(lev=11)) == ENUM
    assert f(*args(ord=0)) == ENUM
    assert f(*args(ord=21)) == ENUM
    assert f(*args(sch=3)) == ENUM
    assert f(*args(u=None)) == NULL
    assert f(*args(u=P(0))) == ALIAS
    assert f(*args(d=P(3))) == ALIAS
    assert f(*args(j=P(4))) == ALIAS   # gradient over the stretching
    assert f(*args(j=P(1))) == ALIAS   # gradient over the strengths
    assert f(*args(wb=16)) == WORKSPACE
    assert f(*args(w=None)) == WORKSPACE
    assert f(*args(n=0, ld=0, ldo=0, w=None, wb=0)) == OK


def test_tuning_cache_matches_the_kernel_sources():
    """The shipped tuning cache is applied only when its hash matches the pair-kernel sources;
    a stale cache would silently fall back to the default shapes."""
    import json
    from paper_2511_11430_amd import tune
    with open(tune.DEFAULT_CACHE) as f:
        cache = json.load(f)
    assert cache["source_hash"] == tune.source_hash()
    assert {p["batched"] for p in cache["plans"]} == {0, 1}


def test_fma_chain_validation():
    lib = _lib.load()
    f = lib.vpm_fma_chain
    n = ctypes.c_int64(-1)
    assert f(0, 8, 0, P(0), ctypes.byref(n), None) == SIZE
    assert f(64, 6, 0, P(0), ctypes.byref(n), None) == SIZE   # not a multiple of 4
    assert f(64, 8, 5, P(0), ctypes.byref(n), None) == ENUM
    assert f(64, 8, -1, P(0), ctypes.byref(n), None) == ENUM
    assert f(64, 8, 0, None, ctypes.byref(n), None) == NULL
    assert n.value == -1  # nothing counted by a rejected call


def test_noalloc_validation():
    lib = _lib.load()
    f = lib.vpm_eval_velocity_stretching_noalloc
    assert lib.vpm_noalloc_scratch_bytes() == 32 << 20

    def call(dtype=F32C, nb=1, so=None, xs=P(0), u=P(6), dg=P(7), o=None):
        so = off(0, 100) if so is None else so
        o = opts(self_=1) if o is None else o
        return f(dtype, nb, so, None, xs, P(1), P(2), 100, None, None, None, 0, None, u, dg, 100, ctypes.byref(o), None)

    assert call(dtype=7) == DTYPE
    assert call(nb=0) == SIZE
    assert call(nb=2, so=off(0, 50, 100)) == UNSUPPORTED  # one set per call
    assert call(xs=None) == NULL
    assert call(u=P(0)) == ALIAS
    assert call(o=opts(self_=1, gradient=1)) == ENUM  # the gradient has its own entry point
