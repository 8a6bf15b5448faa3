"""GPU parity of the blade solve and the wake management (Sec. II.A; Sec. II.C, Eqs. 6-8)
against the FP64 oracle: the ring influence matrix element by element, the LU solve against a
library dense solve, a steady flat wing's lift slope against thin-airfoil theory, Kutta
shedding exactly, and the adaptive panel-to-particle conversion (counts bit-exact, particles
to rounding)."""
import math

import numpy as np
import pytest

import oracle
import paper_2511_11430_amd as vpm
from oracle import uvlm
from paper_2511_11430_amd import workloads as W

from gpu_helpers import TOL, dev, host, prepare, rel_l2, say

pytestmark = pytest.mark.gpu


def _d64(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _ring_inputs(g):
    return [_d64(g[k]) for k in ("c00", "c01", "c11", "c10", "colloc", "normal")]


@pytest.mark.parametrize("rc,vn", [(0.02, 2), (0.0, 2), (0.02, 1), (0.03, 3)])
def test_aic_matches_oracle(rc, vn, gpu):
    g = W.blade_rings(n_blades=2, n_chord=4, n_span=16)
    say(f"aic rc={rc} n={vn} panels={g['colloc'].shape[1]}")
    A = host(vpm.vpm_aic_assemble(*_ring_inputs(g), rc, vn))
    Ao = uvlm.aic(g["c00"], g["c01"], g["c11"], g["c10"], g["colloc"], g["normal"], rc, vn)
    assert rel_l2(A, Ao) <= 1e-13
    assert np.abs(A - Ao).max() <= 1e-12 * np.abs(Ao).max()


def test_aic_full_blade_lattice(gpu):
    """The 2 x 8 x 32 lattice of the hover workload (512 panels)."""
    g = W.blade_rings()
    A = host(vpm.vpm_aic_assemble(*_ring_inputs(g), 0.02 * W.R, 2))
    Ao = uvlm.aic(g["c00"], g["c01"], g["c11"], g["c10"], g["colloc"], g["normal"], 0.02 * W.R, 2)
    say(f"aic 512 panels rel-L2 {rel_l2(A, Ao):.2e}")
    assert rel_l2(A, Ao) <= 1e-13


@pytest.mark.parametrize("n", [1, 7, 16, 17, 33, 300, 512, 1024, 1025, 1100])
def test_lu_solve_matches_library_solve(n, gpu):
    rng = np.random.default_rng(n)
    M = rng.normal(size=(n, n)) + n ** 0.5 * np.eye(n) * rng.choice([-1, 1], size=n)
    b = rng.normal(size=n)
    say(f"lu n={n}")
    A = _d64(M)
    ipiv, info = vpm.vpm_lu_factor(A)
    x = vpm.vpm_lu_solve(A, ipiv, _d64(b))
    xo = np.linalg.solve(M, b)
    assert int(info.item()) == 0
    assert rel_l2(host(x), xo) <= 1e-11
    assert np.linalg.norm(M @ host(x) - b) <= 1e-12 * np.linalg.norm(M) * np.linalg.norm(host(x))


def test_lu_reports_a_singular_column(gpu):
    M = np.random.default_rng(1).normal(size=(50, 50))
    M[:, 17] = 0.0
    _, info = vpm.vpm_lu_factor(_d64(M))
    assert int(info.item()) == 18


def _exact_lu_case(n, seed, ties):
    """A with rows of L U in the order perm, L unit lower with entries in {0, +-1/2, +-1}, U with
    small integers and a diagonal in {+-1, +-2}: every value elimination forms is a multiple of
    1/2 far below 2^52, so LU with partial pivoting is exact in FP64 and its factors are L and U
    themselves.  ties: perm = identity and |l_ik| = 1 for about half the rows below the diagonal,
    whose magnitude then equals the pivot's (the diagonal row, the first of them, must win);
    otherwise |l_ik| <= 1/2 and perm is random, so each pivot is unique and sits anywhere."""
    rng = np.random.default_rng(seed)
    if ties:
        Lv = rng.choice([-1.0, -0.5, 0.0, 0.5, 1.0], p=[0.25, 0.15, 0.2, 0.15, 0.25], size=(n, n))
    else:
        Lv = rng.choice([-0.5, 0.0, 0.5], size=(n, n))
    L = np.tril(Lv, -1) + np.eye(n)
    U = np.triu(rng.integers(-2, 3, size=(n, n)).astype(np.float64), 1) + np.diag(
        rng.choice([-2.0, -1.0, 1.0, 2.0], size=n))
    perm = np.arange(n) if ties else rng.permutation(n)
    A = np.empty((n, n))
    A[perm] = L @ U
    # pivot rows by the textbook exchange sequence: row k of L U sits at position perm[k]
    cur = np.argsort(perm)            # cur[p] = row of L U now at position p
    ipiv = np.empty(n, dtype=np.int64)
    for k in range(n):
        q = int(np.nonzero(cur == k)[0][0])
        ipiv[k] = q
        cur[[k, q]] = cur[[q, k]]
    return A, np.tril(L, -1) + U, ipiv


@pytest.mark.parametrize("ties", [True, False])
@pytest.mark.parametrize("n", [40, 600, 1024, 1100])
def test_lu_exact_on_dyadic_systems(n, ties, gpu):
    """Bit-exact factors, pivot sequence and solution where elimination is exact: the first row
    wins a tie (within a wavefront and across wavefronts of the panel), pivots found at any
    position, both the blocked path (n <= 1024) and the column-by-column one."""
    A, F, ipiv_ref = _exact_lu_case(n, 1000 + n, ties)
    x_ref = np.random.default_rng(n).integers(-3, 4, size=n).astype(np.float64)
    b = A @ x_ref
    say(f"lu exact n={n} ties={ties}")
    Ad = _d64(A)
    ipiv, info = vpm.vpm_lu_factor(Ad)
    x = host(vpm.vpm_lu_solve(Ad, ipiv, _d64(b)))
    assert int(info.item()) == 0
    assert np.array_equal(host(ipiv).astype(np.int64), ipiv_ref)
    assert np.array_equal(host(Ad), F)
    assert np.array_equal(x, x_ref)


def test_blade_system_solve(gpu):
    """The hover lattice's Neumann system with a rotor-like right-hand side."""
    g = W.blade_rings()
    rc = 0.02 * W.R
    A = vpm.vpm_aic_assemble(*_ring_inputs(g), rc, 2)
    Ao = uvlm.aic(g["c00"], g["c01"], g["c11"], g["c10"], g["colloc"], g["normal"], rc, 2)
    # relative air of a rotor at Omega = 1 rad/s plus a small inflow: -(Omega x c) - 0.05 z
    c = g["colloc"]
    v = np.stack([c[1], -c[0], -0.05 * np.ones(c.shape[1])])
    rhs = -(v * g["normal"]).sum(0)
    ipiv, info = vpm.vpm_lu_factor(A)
    x = host(vpm.vpm_lu_solve(A, ipiv, _d64(rhs)))
    xo = uvlm.solve(Ao, rhs)
    assert int(info.item()) == 0
    assert rel_l2(x, xo) <= 1e-11


def test_steady_flat_wing_lift_slope_on_gpu(gpu):
    """Thin-airfoil lift slope 2 pi at mid-span of an AR = 400 flat wing: GPU influence
    matrix plus its steady wake rings, GPU LU solve."""
    import sys
    import os
    sys.path.insert(0, os.path.dirname(__file__))
    from test_oracle_uvlm import _flat_wing
    n_chord, n_span, alpha = 4, 40, math.radians(2.0)
    g, w, ys = _flat_wing(400.0, n_chord, n_span)
    A = vpm.vpm_aic_assemble(*_ring_inputs(g), 0.0, 2)
    col, nrm = _d64(g["colloc"]), g["normal"]
    for k in range(n_span):
        a, b, gm = uvlm.ring_edges(*(w[nm][:, k:k + 1] for nm in ("c00", "c01", "c11", "c10")))
        u = host(vpm.vpm_eval_segments(_d64(a), _d64(b), _d64(gm), col, 0.0, 2))
        A[:, (n_chord - 1) * n_span + k] += _d64((u * nrm).sum(0))
    v = np.array([math.cos(alpha), 0.0, math.sin(alpha)])
    ipiv, _ = vpm.vpm_lu_factor(A)
    gam = host(vpm.vpm_lu_solve(A, ipiv, _d64(-(v[:, None] * nrm).sum(0))))
    cl_mid = 2.0 * gam[(n_chord - 1) * n_span + n_span // 2]
    say(f"flat wing c_l / alpha = {cl_mid / alpha:.4f} (2 pi = {2 * math.pi:.4f})")
    assert cl_mid / alpha == pytest.approx(2 * math.pi, rel=0.01)


@pytest.mark.parametrize("kind", ["f64", "f32c"])
def test_wake_shed_exact(kind, gpu):
    import torch
    nb, ns = 3, 24
    rng = np.random.default_rng(5)
    gb, prev = prepare([rng.normal(size=nb * 8 * ns), rng.normal(size=nb * ns)], kind)
    te = np.array([(b * 8 + 7) * ns + k for b in range(nb) for k in range(ns)], dtype=np.int32)
    P = dev(prev, kind)
    tr, sh = vpm.vpm_wake_shed(dev(gb, kind), torch.tensor(te, device="cuda"), P, nb, ns)
    for b in range(nb):
        gnow = gb[te[b * ns:(b + 1) * ns]]
        to, so = uvlm.shed(gnow, prev[b * ns:(b + 1) * ns])
        if kind == "f32c":
            to, so = to.astype(np.float32), so.astype(np.float32)
        assert np.array_equal(host(tr)[b * (ns + 1):(b + 1) * (ns + 1)], to.astype(np.float64))
        assert np.array_equal(host(sh)[b * ns:(b + 1) * ns], so.astype(np.float64))
        assert np.array_equal(host(P)[b * ns:(b + 1) * ns], gnow)


@pytest.mark.parametrize("kind", ["f64", "f32c"])
def test_wake_convert_counts_and_particles(kind, gpu):
    import torch
    rng = np.random.default_rng(6)
    n = 333
    a = rng.normal(size=(3, n)) * 0.5
    b = a + rng.normal(size=(3, n)) * rng.uniform(0.001, 0.2, n)
    dg = rng.normal(size=n)
    tip = np.where(rng.random(n) < 0.7, rng.integers(0, n, n), -1).astype(np.int32)
    a, b, dg = prepare([a, b, dg], kind)
    cnt_o = uvlm.particle_counts(a, b, tip, 3)
    cap = int(np.minimum(cnt_o, 64).sum())
    say(f"convert {kind} lines={n} particles={cap}")
    x, g, s, c = vpm.vpm_wake_convert(dev(a, kind), dev(b, kind), dev(dg, kind), torch.tensor(tip, device="cuda"),
                                      3, 0.02, cap, n_max=64)
    assert int(c.item()) == cap
    tip_capped = tip.copy()
    xo, go, so, co = uvlm.convert(a, b, dg, tip_capped, 3, 0.02)
    assert np.array_equal(np.minimum(co, 64), np.minimum(cnt_o, 64))
    if np.all(co <= 64):
        tol = 1e-15 if kind == "f64" else 2e-7
        assert np.abs(host(x) - xo).max() <= tol * max(1.0, np.abs(xo).max())
        assert rel_l2(host(g), go) <= tol * 10
        assert np.allclose(host(s), 0.02, rtol=1e-7)
    # total vorticity of the lines is carried over (Eq. 6)
    assert np.allclose(host(g).sum(1), (dg * (b - a)).sum(1), rtol=0, atol=1e-5 if kind == "f32c" else 1e-12)


def test_wake_convert_capacity_and_empty(gpu):
    import torch
    a = np.zeros((3, 3))
    b = np.zeros((3, 3))
    b[0] = [0.1, 0.3, 0.05]
    tip = np.array([0, 0, -1], dtype=np.int32)
    # counts 2, 6, 1 = 9; with capacity 5 only the first line (2) fits ahead of the second
    x, g, s, c = vpm.vpm_wake_convert(_d64(a), _d64(b), _d64([1.0, 1.0, 1.0]), torch.tensor(tip, device="cuda"),
                                      2, 0.01, 5)
    assert int(c.item()) == 9
    assert np.allclose(host(x)[0, :2], [0.025, 0.075])
    _, _, _, c0 = vpm.vpm_wake_convert(_d64(np.zeros((3, 0))), _d64(np.zeros((3, 0))), _d64(np.zeros(0)),
                                       torch.zeros(0, dtype=torch.int32, device="cuda"), 2, 0.01, 0)
    assert int(c0.item()) == 0
