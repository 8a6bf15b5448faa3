"""GPU parity of the segments' velocity gradient and the stretching they impose on particles
(segment law of Sec. II.A, differentiated; the stretching term of Sec. II.B) against the FP64
oracle, which differentiates the same law in forward mode."""
import numpy as np
import pytest

import oracle
import paper_2511_11430_amd as vpm
from paper_2511_11430_amd import workloads as W

from gpu_helpers import TOL, dev, host, prepare, rel_l2, say

pytestmark = pytest.mark.gpu
KINDS = ["f64", "f32c"]


def _stretch(J, g, classical):
    """J (3, 3, n) applied to particle strengths g (3, n)."""
    return np.einsum("abn,an->bn", J, g) if not classical else np.einsum("abn,bn->an", J, g)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("rc,vn", [(0.02, 2), (0.0, 2), (0.02, 1), (0.03, 3)])
def test_segments_gradient_matches_oracle(kind, rc, vn, gpu):
    c = W.config2(n=3000)
    a, b, gs, x, g = prepare([c["seg_a"], c["seg_b"], c["seg_gamma"], c["x"], c["gamma"]], kind)
    say(f"segments gradient {kind} rc={rc} n={vn}")
    u, J, d = vpm.vpm_eval_segments_gradient(dev(a, kind), dev(b, kind), dev(gs, kind), dev(x, kind), rc, vn,
                                             gamma_tgt=dev(g, kind))
    Jo = oracle.segments_gradient(a, b, gs, x, rc, vn)
    assert rel_l2(host(u), oracle.segments(a, b, gs, x, rc, vn)) <= TOL[kind]
    assert rel_l2(host(J), Jo.reshape(9, -1)) <= TOL[kind]
    assert rel_l2(host(d), _stretch(Jo, g, False)) <= TOL[kind]


@pytest.mark.parametrize("kind", KINDS)
def test_segments_classical_stretching_and_accumulate(kind, gpu):
    import torch
    c = W.config2(n=2000)
    a, b, gs, x, g = prepare([c["seg_a"], c["seg_b"], c["seg_gamma"], c["x"], c["gamma"]], kind)
    rng = np.random.default_rng(2)
    u0, d0 = rng.normal(size=(3, x.shape[1])), rng.normal(size=(3, x.shape[1]))
    # preallocated outputs with a leading dimension wider than the point count
    ld = x.shape[1] + 37
    U = torch.zeros((3, ld), dtype=torch.float64 if kind == "f64" else torch.float32, device="cuda")
    D = torch.zeros_like(U)
    U[:, :x.shape[1]] = dev(u0, kind)
    D[:, :x.shape[1]] = dev(d0, kind)
    u0, d0 = host(U[:, :x.shape[1]]), host(D[:, :x.shape[1]])
    u, J, d = vpm.vpm_eval_segments_gradient(dev(a, kind), dev(b, kind), dev(gs, kind), dev(x, kind), 0.02, 2,
                                             gamma_tgt=dev(g, kind), scheme=vpm.CLASSICAL, want_grad=False,
                                             u_out=U[:, :x.shape[1]], dgamma_out=D[:, :x.shape[1]], accumulate=True)
    assert J is None
    Jo = oracle.segments_gradient(a, b, gs, x, 0.02, 2)
    uo = oracle.segments(a, b, gs, x, 0.02, 2)
    assert rel_l2(host(u) - u0, uo) <= TOL[kind] * 10
    assert rel_l2(host(d) - d0, _stretch(Jo, g, True)) <= TOL[kind] * 10
    assert np.all(host(U)[:, x.shape[1]:] == 0) and np.all(host(D)[:, x.shape[1]:] == 0)


@pytest.mark.parametrize("kind", KINDS)
def test_segments_gradient_full_size_sampled(kind, gpu):
    """All particles of the 65,536-particle hover wake with the 4096 lattice segments; the
    oracle checks 2048 sampled particles."""
    c = W.config2()
    a, b, gs, x, g = prepare([c["seg_a"], c["seg_b"], c["seg_gamma"], c["x"], c["gamma"]], kind)
    _, J, d = vpm.vpm_eval_segments_gradient(dev(a, kind), dev(b, kind), dev(gs, kind), dev(x, kind), 0.02, 2,
                                             gamma_tgt=dev(g, kind), want_u=False)
    idx = np.sort(np.random.default_rng(5).choice(x.shape[1], 2048, replace=False))
    Jo = oracle.segments_gradient(a, b, gs, x[:, idx], 0.02, 2)
    say(f"segments gradient full {kind}: J rel-L2 {rel_l2(host(J)[:, idx], Jo.reshape(9, -1)):.2e}")
    assert rel_l2(host(J)[:, idx], Jo.reshape(9, -1)) <= TOL[kind]
    assert rel_l2(host(d)[:, idx], _stretch(Jo, g[:, idx], False)) <= TOL[kind]
    # the cored field is divergence-free: trace J = 0 at every particle
    Jh = host(J)
    tr = Jh[0] + Jh[4] + Jh[8]
    assert np.abs(tr).max() <= (1e-10 if kind == "f64" else 1e-4) * np.abs(Jh).max()


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("n", [16384, 16385, 196608, 196609])
def test_segments_gradient_on_either_side_of_the_lane_splits(n, kind, gpu):
    """Target counts on either side of those where the kernel changes the number of lanes that
    share a target's segments (16 below 16,385 targets, 4 below 196,609, then 1); the oracle
    checks 512 sampled targets, the first and the last among them."""
    c = W.config2(n=n)
    a, b, gs, x, g = prepare([c["seg_a"], c["seg_b"], c["seg_gamma"], c["x"], c["gamma"]], kind)
    say(f"segments gradient {kind} n_tgt={n}")
    u, J, d = vpm.vpm_eval_segments_gradient(dev(a, kind), dev(b, kind), dev(gs, kind), dev(x, kind), 0.02, 2,
                                             gamma_tgt=dev(g, kind))
    rng = np.random.default_rng(n)
    idx = np.unique(np.concatenate([[0, n - 1], rng.choice(n, 510, replace=False)]))
    Jo = oracle.segments_gradient(a, b, gs, x[:, idx], 0.02, 2)
    assert rel_l2(host(u)[:, idx], oracle.segments(a, b, gs, x[:, idx], 0.02, 2)) <= TOL[kind]
    assert rel_l2(host(J)[:, idx], Jo.reshape(9, -1)) <= TOL[kind]
    assert rel_l2(host(d)[:, idx], _stretch(Jo, g[:, idx], False)) <= TOL[kind]


@pytest.mark.parametrize("kind", KINDS)
def test_segments_gradient_degenerate_cases(kind, gpu):
    """A zero-length segment, a target on a segment's end point and on its line without a
    core contribute nothing; no segments give zeros; no targets launch nothing."""
    import torch
    a = np.array([[0.0, 0.0], [0.0, 0.0], [0.0, 0.0]])
    b = np.array([[1.0, 0.0], [0.0, 0.0], [0.0, 0.0]])  # segment 1 has zero length
    gs = np.array([1.5, 2.0])
    x = np.array([[0.0, 1.0, 0.5, 0.3], [0.0, 0.0, 0.0, 0.4], [0.0, 0.0, 0.0, -0.2]])
    g = np.ones((3, 4))
    for rc in (0.0, 0.05):
        u, J, d = vpm.vpm_eval_segments_gradient(dev(a, kind), dev(b, kind), dev(gs, kind), dev(x, kind), rc, 2,
                                                 gamma_tgt=dev(g, kind))
        Jo = oracle.segments_gradient(a, b, gs, x, rc, 2).reshape(9, -1)
        Jh = host(J)
        assert np.all(np.isfinite(Jh)) and np.all(np.isfinite(host(d)))
        assert np.all(Jh[:, :2] == 0) and np.all(host(u)[:, :2] == 0)   # end points
        if rc == 0.0:
            assert np.all(Jh[:, 2] == 0)                                # on the line, no core
        assert rel_l2(Jh, Jo) <= TOL[kind]
    z = lambda r, n: torch.zeros((r, n), dtype=torch.float64 if kind == "f64" else torch.float32, device="cuda")
    u, J, _ = vpm.vpm_eval_segments_gradient(z(3, 0), z(3, 0), z(1, 0)[0], dev(x, kind), 0.02, 2)
    assert np.all(host(u) == 0) and np.all(host(J) == 0)
    u, J, _ = vpm.vpm_eval_segments_gradient(dev(a, kind), dev(b, kind), dev(gs, kind), z(3, 0), 0.02, 2)
    assert u.shape == (3, 0) and J.shape == (9, 0)
