"""GPU parity of the segments' vector-Jacobian product at particles (the adjoint of their
velocity and stretching, Sec. II.A segment law inside the Sec. II.B right-hand side) against
the FP64 oracle, whose second derivatives come from hyper-dual numbers."""
import numpy as np
import pytest

import oracle
import paper_2511_11430_amd as vpm
from paper_2511_11430_amd import workloads as W

from gpu_helpers import TOL, dev, host, prepare, rel_l2, say

pytestmark = pytest.mark.gpu
KINDS = ["f64", "f32c"]


def _case(kind, n=2500, seed=3):
    c = W.config2(n=n)
    rng = np.random.default_rng(seed)
    ub = rng.normal(size=c["x"].shape)
    db = rng.normal(size=c["x"].shape)
    return prepare([c["seg_a"], c["seg_b"], c["seg_gamma"], c["x"], c["gamma"], ub, db], kind)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("scheme", [vpm.TRANSPOSED, vpm.CLASSICAL])
@pytest.mark.parametrize("rc,vn", [(0.02, 2), (0.0, 2), (0.02, 1), (0.03, 3)])
def test_segments_vjp_matches_oracle(kind, scheme, rc, vn, gpu):
    a, b, gs, x, g, ub, db = _case(kind)
    say(f"segments vjp {kind} scheme={scheme} rc={rc} n={vn}")
    xb, gb = vpm.vpm_segments_backward(dev(a, kind), dev(b, kind), dev(gs, kind), dev(x, kind), rc, vn,
                                       dev(ub, kind), dev(db, kind), gamma_tgt=dev(g, kind), scheme=scheme)
    xo, go = oracle.segments_vjp(a, b, gs, x, rc, vn, ub, db, g, scheme)
    assert rel_l2(host(xb), xo) <= TOL[kind]
    assert rel_l2(host(gb), go) <= TOL[kind]


@pytest.mark.parametrize("kind", KINDS)
def test_segments_vjp_seeds_alone_and_accumulation(kind, gpu):
    """Velocity seeds only, stretching seeds only, and gradients added to what the arrays hold."""
    import torch
    a, b, gs, x, g, ub, db = _case(kind, n=1500, seed=4)
    A, B, Gs, X, G = (dev(v, kind) for v in (a, b, gs, x, g))
    xb, gb = vpm.vpm_segments_backward(A, B, Gs, X, 0.02, 2, dev(ub, kind))
    assert gb is None
    xo, _ = oracle.segments_vjp(a, b, gs, x, 0.02, 2, ub)
    assert rel_l2(host(xb), xo) <= TOL[kind]
    x0 = torch.randn_like(X)
    g0 = torch.randn_like(X)
    xb2, gb2 = vpm.vpm_segments_backward(A, B, Gs, X, 0.02, 2, None, dev(db, kind), gamma_tgt=G,
                                         x_bar=x0.clone(), gamma_bar=g0.clone())
    xo2, go2 = oracle.segments_vjp(a, b, gs, x, 0.02, 2, np.zeros_like(x), db, g)
    assert rel_l2(host(xb2) - host(x0), xo2) <= TOL[kind] * 10
    assert rel_l2(host(gb2) - host(g0), go2) <= TOL[kind] * 10


@pytest.mark.parametrize("kind", KINDS)
def test_segments_vjp_full_size_sampled(kind, gpu):
    """All 65,536 particles of the hover wake with the 4096 lattice segments; 1024 sampled."""
    a, b, gs, x, g, ub, db = _case(kind, n=65536, seed=5)
    xb, gb = vpm.vpm_segments_backward(dev(a, kind), dev(b, kind), dev(gs, kind), dev(x, kind), 0.02, 2,
                                       dev(ub, kind), dev(db, kind), gamma_tgt=dev(g, kind))
    idx = np.sort(np.random.default_rng(6).choice(x.shape[1], 1024, replace=False))
    xo, go = oracle.segments_vjp(a, b, gs, x[:, idx], 0.02, 2, ub[:, idx], db[:, idx], g[:, idx])
    say(f"segments vjp full {kind}: x_bar rel-L2 {rel_l2(host(xb)[:, idx], xo):.2e}")
    assert rel_l2(host(xb)[:, idx], xo) <= TOL[kind]
    assert rel_l2(host(gb)[:, idx], go) <= TOL[kind]


@pytest.mark.parametrize("kind", KINDS)
def test_segments_vjp_degenerate_points(kind, gpu):
    """Particles on a segment's end points and a zero-length segment give finite zeros."""
    a = np.array([[0.0, 0.0], [0.0, 0.0], [0.0, 0.0]])
    b = np.array([[1.0, 0.0], [0.0, 0.0], [0.0, 0.0]])
    gs = np.array([1.5, 2.0])
    x = np.array([[0.0, 1.0, 0.3], [0.0, 0.0, 0.4], [0.0, 0.0, -0.2]])
    one = np.ones((3, 3))
    xb, gb = vpm.vpm_segments_backward(dev(a, kind), dev(b, kind), dev(gs, kind), dev(x, kind), 0.05, 2,
                                       dev(one, kind), dev(one, kind), gamma_tgt=dev(one, kind))
    assert np.all(np.isfinite(host(xb))) and np.all(np.isfinite(host(gb)))
    assert np.all(host(xb)[:, :2] == 0) and np.all(host(gb)[:, :2] == 0)
    xo, go = oracle.segments_vjp(a, b, gs, x, 0.05, 2, one, one, one)
    assert rel_l2(host(xb), xo) <= TOL[kind] and rel_l2(host(gb), go) <= TOL[kind]


def _lattice_program(kind):
    """36 particles of a hover tip helix right behind the 2 x 8 x 32 blade lattice (4096
    segments, r_c = 0.02 R), two control points near the helix."""
    rng = np.random.default_rng(3)
    c = W.config4(n=36)
    c2 = W.config2(n=16)
    x, g, s = c["x"], c["gamma"], c["sigma"]
    y = x[:, :2] + np.array([[0.0], [0.0], [-0.03]]) + rng.normal(scale=0.005, size=(3, 2))
    arrs = prepare([x, g, s, y, c2["seg_a"], c2["seg_b"], c2["seg_gamma"]], kind)
    return arrs, 0.02 * W.R


@pytest.mark.parametrize("kind", ["f64", "mixed"])
def test_rk3_program_with_lattice_gradient_vs_oracle_tangents(kind, gpu):
    """Gradient of the differentiated RK3 program with the blade lattice acting on the
    particles (velocity and stretching in every stage, velocity at the control points)
    against the oracle's tangents of the same program: <grad L, v> = dL/dv for random dense
    directions and for unit directions at the particles nearest the lattice.  'mixed': FP64
    state, FP32-compensated sums."""
    from paper_2511_11430_amd import autograd as AG
    ek = "f64" if kind == "f64" else "f32c"
    (x, g, s, y, sa, sb, sg), rc = _lattice_program(ek)
    steps, dt = 2, 2e-4
    lat_o = (sa, sb, sg, rc, 2)
    lat_d = (dev(sa, ek), dev(sb, ek), dev(sg, ek), rc, 2)
    say(f"RK3 program with lattice, {kind}")
    X, G = dev(x, "f64").requires_grad_(True), dev(g, "f64").requires_grad_(True)
    L = AG.rk3_program_loss(X, G, dev(s, ek), steps, dt, dev(y, ek), segments=lat_d)
    L.backward()
    # mixed: compared with the oracle's program under the same storage model (evaluation
    # inputs and results rounded to FP32, FP64 state), to the FP32C gate; how far that model
    # itself is from the exact program (FP32 positions near 1 m, 0.017 m from the nearest
    # segment; 3.6e-5 at the unit directions) is printed.  What remains against the model
    # (4.2e-6 at a unit direction next to the lattice, 1e-7 on the loss) is the FP32 evaluation
    # itself: the rings' shared edges carry opposite circulations, whose large contributions
    # cancel at a particle that close
    st = oracle.STORE_F64 if kind == "f64" else oracle.STORE_F32_EVAL
    Lo = oracle.rk3_program(x, g, s, steps, dt, y, segments=lat_o, storage=st)[3]
    Lx = oracle.rk3_program(x, g, s, steps, dt, y, segments=lat_o)[3]
    say(f"  loss {abs(L.item() - Lo) / abs(Lo):.2e} against the storage model; model vs exact "
        f"{abs(Lo - Lx) / abs(Lx):.2e}")
    tol = 1e-10 if kind == "f64" else TOL[ek]
    assert abs(L.item() - Lo) <= (1e-12 if kind == "f64" else 1e-6) * abs(Lo)
    gx, gg = host(X.grad), host(G.grad)
    rng = np.random.default_rng(17)
    dirs = [(rng.normal(size=x.shape), np.zeros_like(g)) for _ in range(3)]
    dirs += [(np.zeros_like(x), rng.normal(size=g.shape)) for _ in range(3)]
    near = np.argsort(np.min(np.linalg.norm(x[:, :, None] - sa[:, None, :], axis=0), axis=1))[:4]
    for i in near:
        for c in range(3):
            xd = np.zeros_like(x)
            xd[c, i] = 1.0
            dirs.append((xd, np.zeros_like(g)))
    worst = worst_model = 0.0
    for xd, gd in dirs:
        ref = oracle.rk3_program_jvp(x, g, s, xd, gd, steps, dt, y, segments=lat_o, storage=st)[1]
        got = float((gx * xd).sum() + (gg * gd).sum())
        worst = max(worst, abs(got - ref) / max(abs(ref), 1e-30))
        if kind != "f64":
            ex = oracle.rk3_program_jvp(x, g, s, xd, gd, steps, dt, y, segments=lat_o)[1]
            worst_model = max(worst_model, abs(ref - ex) / max(abs(ex), 1e-30))
    say(f"  worst relative error over {len(dirs)} directions {worst:.2e} (storage model vs exact "
        f"{worst_model:.2e})")
    assert worst <= tol
    # the lattice is felt by the gradient, not only by the loss
    X2, G2 = dev(x, "f64").requires_grad_(True), dev(g, "f64").requires_grad_(True)
    AG.rk3_program_loss(X2, G2, dev(s, ek), steps, dt, dev(y, ek)).backward()
    assert rel_l2(host(X2.grad), gx) > 1e-3  # 0.46 % here
