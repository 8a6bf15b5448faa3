"""The no-allocation entry point (vpm_eval_velocity_stretching_noalloc, through the C ABI)
against the workspace form of the same evaluation: two calls in a row, the second with a
smaller input, in both precisions.  Where a call's source split needs more partial sums than
the library's scratch array holds (the first call: 36 MiB in FP64, 72 MiB in FP32C with the
shape fixed to two targets per lane and 256 lanes, so that the case does not depend on the
tuned plan), the entry
point uses fewer chunks: the same sums in another order, checked to the parity tolerance (FP64:
differences in the last bits; FP32C: the FP32 partial sums of each chunk start at other
sources, so the outputs differ at the level of FP32 rounding, rel-L2 3.5e-8 here); where it
fits (the second call), the chunks are the same and so are the bits."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2511_11430_amd as vpm
from paper_2511_11430_amd import _lib
from paper_2511_11430_amd import workloads as W

from gpu_helpers import TOL, host, per_target, rel_l2, say

pytestmark = pytest.mark.gpu


def _noalloc(x_src, g_src, s_src, x_tgt=None, g_tgt=None, velocity_only=False, variant=0):
    lib = _lib.load()
    self_eval = x_tgt is None
    n_src = x_src.shape[1]
    n_tgt = n_src if self_eval else x_tgt.shape[1]
    u = torch.empty((3, n_tgt), dtype=x_src.dtype, device=x_src.device)
    d = None if velocity_only else torch.empty_like(u)
    o = vpm._opts(self_eval=int(self_eval), variant=variant)
    P = lambda t: None if t is None else ctypes.c_void_p(t.data_ptr())
    so = vpm._offsets([0, n_src])
    to = None if self_eval else vpm._offsets([0, n_tgt])
    st = lib.vpm_eval_velocity_stretching_noalloc(
        vpm._code(x_src), 1, so, to, P(x_src), P(g_src), P(s_src), x_src.stride(0),
        None if self_eval else P(x_tgt), None if (self_eval or velocity_only) else P(g_tgt), None,
        0 if self_eval else x_tgt.stride(0), None, P(u), P(d), u.stride(0), ctypes.byref(o),
        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, vpm._lib.load().vpm_status_string(st)
    return u, d


@pytest.mark.parametrize("kind", ["f64", "f32c"])
def test_noalloc_matches_the_workspace_form(kind, gpu):
    dt = torch.float64 if kind == "f64" else torch.float32
    T = lambda a: torch.tensor(np.ascontiguousarray(a if kind == "f64" else W.to_f32(a)), dtype=dt, device="cuda")
    lib = _lib.load()
    assert lib.vpm_noalloc_scratch_bytes() == 32 << 20
    # call 1: 65,536-particle self evaluation (its split needs more than the scratch holds)
    c = W.config3(n=65536)
    x, g, s = T(c["x"]), T(c["gamma"]), T(c["sigma"])
    v = 0 if kind == "f64" else 1  # FP32C: (2 targets per lane, 256 lanes)
    u1, d1 = _noalloc(x, g, s, variant=v)
    need = vpm.vpm_workspace_size(vpm._code(x), [0, 65536], variant=v)
    ws = torch.empty(max(1, need), dtype=torch.uint8, device="cuda")
    ur, dr = vpm.vpm_eval_velocity_stretching(x, g, s, workspace=ws, variant=v)
    eu, ed = rel_l2(host(u1), host(ur)), rel_l2(host(d1), host(dr))
    pu, pd = per_target(host(u1), host(ur)), per_target(host(d1), host(dr))
    say(f"{kind} call 1 (65536 self, split needs {need >> 20} MiB): rel-L2 u {eu:.2e} dgamma {ed:.2e}, "
        f"worst target {pu:.2e} {pd:.2e}")
    if need > lib.vpm_noalloc_scratch_bytes():
        assert max(eu, ed, pu, pd) <= TOL[kind]
    else:
        assert torch.equal(u1, ur) and torch.equal(d1, dr)
    assert need > lib.vpm_noalloc_scratch_bytes()  # the reduced-chunk path is exercised
    # call 2, smaller: 4096 velocity-only points against 16,384 sources (the split fits)
    c2 = W.config3(n=16384)
    x2, g2, s2 = T(c2["x"]), T(c2["gamma"]), T(c2["sigma"])
    y = T(np.random.default_rng(3).uniform(-1.0, 3.0, (3, 4096)))
    u2, _ = _noalloc(x2, g2, s2, y, velocity_only=True)
    ws2 = torch.empty(max(1, vpm.vpm_workspace_size(vpm._code(x2), [0, 16384], [0, 4096], self_eval=False)),
                      dtype=torch.uint8, device="cuda")
    ur2, _ = vpm.vpm_eval_velocity_stretching(x2, g2, s2, y, workspace=ws2)
    say(f"{kind} call 2 (4096 points x 16384): rel-L2 u {rel_l2(host(u2), host(ur2)):.2e}")
    assert torch.equal(u2, ur2)
    # and a repeat of the first call after the second reuses the scratch correctly
    u3, d3 = _noalloc(x, g, s, variant=v)
    assert torch.equal(u3, u1) and torch.equal(d3, d1)


def test_noalloc_rejects_many_sets(gpu):
    lib = _lib.load()
    o = vpm._opts(self_eval=1)
    st = lib.vpm_eval_velocity_stretching_noalloc(1, 2, vpm._offsets([0, 5, 10]), None, ctypes.c_void_p(16),
                                                  ctypes.c_void_p(4096), ctypes.c_void_p(8192), 10, None, None,
                                                  None, 0, None, ctypes.c_void_p(12288), ctypes.c_void_p(16384),
                                                  10, ctypes.byref(o), None)
    assert st == 10  # VPM_ERR_UNSUPPORTED
