"""GPU parity of one closed blade / wake / particle step (Sec. II.A; Sec. II.C, Eqs. 6-8;
Sec. II.B with its low-storage RK3) against the FP64 oracle of the same step, over several
steps that shed rows and convert the oldest ones into particles, in FP64 and with an FP32C
wake (FP32 state, compensated sums), and the closure of the vorticity (the wake lines, the
open line along the youngest boundary and the particles form closed loops)."""
import numpy as np
import pytest

from oracle import uvlm
from paper_2511_11430_amd import workloads as W

from gpu_helpers import host, rel_l2, say

pytestmark = pytest.mark.gpu

ARGS = dict(omega=40.0, v_inf=[0.0, 0.0, -1.0], dt=0.005, core_radius=0.02, vatistas_n=2, sigma_p=0.03, n_tip=2,
            n_rows=3)


def _vort(lines, gprev_pending, gp):
    a, b, g = lines
    return (g * (b - a)).sum(1) + gp.sum(1)


def test_closed_step_matches_oracle(gpu):
    from paper_2511_11430_amd.solver import Step
    geom = W.blade_rings(n_blades=2, n_chord=4, n_span=8)
    gs = Step(geom, capacity=4096, **ARGS)
    go = uvlm.StepOracle(geom, **ARGS)
    first_conversion = None
    for k in range(9):
        gam_g = host(gs.step())
        gam_o = go.step()
        xg, gg, sg = (host(t) for t in gs.particles())
        say(f"step {k}: rows {len(gs.rows)} particles {xg.shape[1]} gamma rel-L2 {rel_l2(gam_g, gam_o):.2e}")
        assert rel_l2(gam_g, gam_o) <= 1e-10
        assert len(gs.rows) == len(go.rows) and len(gs.bounds) == len(go.bounds)
        assert xg.shape[1] == go.xp.shape[1]
        for bg, bo in zip(gs.bounds, go.bounds):
            assert rel_l2(host(bg), bo) <= 1e-10
        if xg.shape[1]:
            assert rel_l2(xg, go.xp) <= 1e-10 and rel_l2(gg, go.gp) <= 1e-9
            assert np.allclose(sg, ARGS["sigma_p"])
            if first_conversion is None:
                first_conversion = k
        # closure of the vorticity holds exactly until the converted particles start moving on
        # their own: their strengths are then stretched by the rings' and lines' field as well,
        # which the line ends do not balance exactly
        if first_conversion is None or k == first_conversion:
            wl = gs.lines(gs.gprev)
            tot = np.zeros(3) if wl is None else (host(wl[2]) * (host(wl[1]) - host(wl[0]))).sum(1)
            tot = tot + gg.sum(1) if xg.shape[1] else tot
            scale = np.abs(gam_g).max() * 0.1
            assert np.abs(tot).max() <= 1e-12 * scale
    assert first_conversion is not None


@pytest.mark.parametrize("kind", ["f64", "f32c"])
def test_step_in_an_existing_wake_matches_oracle(gpu, kind):
    """The hover lattice's small cousin turning inside a 2048-particle hover wake: every RK3
    stage moves and stretches the particles, conversions add more; FP64 to 1e-10, the FP32C
    wake (FP32 positions, strengths and registers) to the FP32C gate."""
    import torch
    from paper_2511_11430_amd.solver import Step
    c = W.config2(n=2048)
    geom = W.blade_rings(n_blades=2, n_chord=4, n_span=8)
    kw = dict(omega=W.OMEGA, v_inf=(0.0, 0.0, -0.5), dt=W.DT, core_radius=0.02, vatistas_n=2, sigma_p=0.02,
              n_tip=2, n_rows=2)
    x0, g0, s0 = (c["x"], c["gamma"], c["sigma"]) if kind == "f64" else (W.to_f32(c["x"]), W.to_f32(c["gamma"]),
                                                                          W.to_f32(c["sigma"]))
    dt_t = torch.float64 if kind == "f64" else torch.float32
    T = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=dt_t, device="cuda")
    gs = Step(geom, capacity=8192, dtype=dt_t, **kw)
    gs.add_particles(T(x0), T(g0), T(s0))
    go = uvlm.StepOracle(geom, **kw)
    go.add_particles(x0, g0, s0)
    tol_x, tol_g = (1e-10, 1e-9) if kind == "f64" else (1e-5, 1e-5)
    for k in range(6):
        gam_g = host(gs.step())
        gam_o = go.step()
        xg, gg, _ = (host(t) for t in gs.particles())
        ex, eg = rel_l2(xg, go.xp), rel_l2(gg, go.gp)
        eb = max(rel_l2(host(bg), bo) for bg, bo in zip(gs.bounds, go.bounds))
        say(f"{kind} step {k}: particles {xg.shape[1]} gamma {rel_l2(gam_g, gam_o):.2e} bounds {eb:.2e} "
            f"x {ex:.2e} Gamma {eg:.2e}")
        assert xg.shape[1] == go.xp.shape[1]
        assert rel_l2(gam_g, gam_o) <= tol_g and eb <= tol_x and ex <= tol_x and eg <= tol_g
    assert xg.shape[1] > 2048


def test_streams_give_the_bits_of_one_stream(gpu):
    """The hover lattice in its 65,536-particle FP32C wake: the particle sums on streams of
    their own beside the blade solve give the same bits, step after step (conversions
    included), as the same calls in order on one stream."""
    import torch
    from paper_2511_11430_amd.solver import Step
    c2 = W.config2()
    geom = W.blade_rings()
    f32 = lambda a: torch.tensor(np.ascontiguousarray(W.to_f32(a)), dtype=torch.float32, device="cuda")
    kw = dict(omega=W.OMEGA, v_inf=(0.0, 0.0, 0.0), dt=W.DT, core_radius=c2["core_radius"], vatistas_n=2,
              sigma_p=0.02 * W.R, n_tip=2, n_rows=2, dtype=torch.float32, capacity=1 << 17)
    steps = [Step(geom, overlap=ov, **kw) for ov in (True, False)]
    for st in steps:
        st.add_particles(f32(c2["x"]), f32(c2["gamma"]), f32(c2["sigma"]))
    for k in range(5):
        gam = [st.step() for st in steps]
        say(f"step {k}: particles {steps[0].np} / {steps[1].np}")
        assert steps[0].np == steps[1].np
        assert torch.equal(gam[0], gam[1])
        for p, q in zip(steps[0].particles(), steps[1].particles()):
            assert torch.equal(p, q)
        assert all(torch.equal(a, b) for a, b in zip(steps[0].bounds, steps[1].bounds))
    assert steps[0].np > 65536  # rows were converted
