"""Pins of the oracle's blade solve and wake management (Sec. II.A; Sec. II.C, Eqs. 6-8)
against things other than the oracle itself: thin-airfoil theory (a flat plate's lift slope
2 pi in the two-dimensional limit), lifting-line theory for a finite wing, the closed-form
field of a square ring, hand-worked Eq. 8 counts, conservation of the converted vorticity,
the far field of a line against its particles, and Kelvin's theorem for the shed lines."""
import math

import numpy as np
import pytest

import oracle
from oracle import uvlm


def _flat_wing(ar, n_chord=4, n_span=40, chord=1.0, wake_len=2000.0):
    """Planar rectangular wing in z = 0, chord along +x (LE -> TE), span along y, rings a
    quarter panel aft; one long trailing ring per strip behind the trailing edge (steady
    wake).  Returns geometry and the strip wake rings."""
    span = ar * chord
    cp = chord / n_chord
    ys = np.linspace(-span / 2, span / 2, n_span + 1)
    c = {k: [] for k in ("c00", "c01", "c11", "c10")}
    col, nrm = [], []
    for i in range(n_chord):
        x0, x1 = i * cp + cp / 4, (i + 1) * cp + cp / 4
        for k in range(n_span):
            c["c00"].append([x0, ys[k], 0.0])
            c["c01"].append([x0, ys[k + 1], 0.0])
            c["c11"].append([x1, ys[k + 1], 0.0])
            c["c10"].append([x1, ys[k], 0.0])
            col.append([i * cp + 0.75 * cp, 0.5 * (ys[k] + ys[k + 1]), 0.0])
            nrm.append([0.0, 0.0, 1.0])
    g = {k: np.array(v).T for k, v in c.items()}
    g["colloc"], g["normal"] = np.array(col).T, np.array(nrm).T
    xt = chord + cp / 4
    w = {"c00": np.array([[xt, ys[k], 0.0] for k in range(n_span)]).T,
         "c01": np.array([[xt, ys[k + 1], 0.0] for k in range(n_span)]).T,
         "c11": np.array([[xt + wake_len, ys[k + 1], 0.0] for k in range(n_span)]).T,
         "c10": np.array([[xt + wake_len, ys[k], 0.0] for k in range(n_span)]).T}
    return g, w, ys


def _steady_lift(ar, alpha, n_chord=4, n_span=40):
    """Sectional lift coefficients c_l(y) and C_L of the steady flat wing (unit chord, unit
    speed): Neumann system with the Kutta condition (each strip's wake ring carries the
    trailing-edge panel's circulation), Kutta-Joukowski on the bound vortices."""
    g, w, ys = _flat_wing(ar, n_chord, n_span)
    A = uvlm.aic(g["c00"], g["c01"], g["c11"], g["c10"], g["colloc"], g["normal"], 0.0)
    # wake ring of strip k moves with the trailing-edge panel (n_chord - 1, k)
    for k in range(n_span):
        a, b, _ = uvlm.ring_edges(*(w[n][:, k:k + 1] for n in ("c00", "c01", "c11", "c10")))
        u = oracle.segments(a, b, np.ones(4), g["colloc"], 0.0)
        A[:, (n_chord - 1) * n_span + k] += (u * g["normal"]).sum(0)
    v = np.array([math.cos(alpha), 0.0, math.sin(alpha)])
    gam = uvlm.solve(A, -(v[:, None] * g["normal"]).sum(0))
    gte = gam[(n_chord - 1) * n_span:]  # sum of the bound vortices of each strip
    dy = np.diff(ys)
    cl = 2.0 * gte
    CL = 2.0 * (gte * dy).sum() / (ar * 1.0)
    return cl, CL, ys


def test_thin_airfoil_lift_slope_in_the_2d_limit():
    """Vortex at the panel quarter-chord, collocation at its three-quarter chord: the
    lattice gives a flat plate the thin-airfoil lift slope 2 pi (Sec. II.A)."""
    alpha = math.radians(2.0)
    cl, _, _ = _steady_lift(ar=400.0, alpha=alpha, n_span=40)
    mid = cl[len(cl) // 2]
    assert mid / alpha == pytest.approx(2 * math.pi, rel=0.01)


def test_finite_wing_matches_lifting_line():
    """Lift slope of a rectangular wing of aspect ratio 8 against Helmbold's lifting-surface
    estimate 2 pi AR / (2 + sqrt(AR^2 + 4)) = 4.91/rad.  The estimate itself is good to a few
    per cent; the lattice converges to 4.63/rad (4x32 and 8x64 panels agree to 0.1 %), so the
    check is loose (6 %) and mainly catches sign and factor errors in the assembly."""
    ar, alpha = 8.0, math.radians(3.0)
    _, CL, _ = _steady_lift(ar, alpha, n_chord=4, n_span=32)
    ref = 2 * math.pi * ar / (2 + math.sqrt(ar * ar + 4))
    assert CL / alpha == pytest.approx(ref, rel=0.06)
    assert CL / alpha < ref  # a finite flat wing lifts less than the estimate, never more


def test_square_ring_self_influence():
    """At the centre of a square ring of side a the normal velocity is 2 sqrt2 / (pi a)."""
    a = 0.3
    h = a / 2
    c00, c01 = np.array([[-h], [-h], [0.0]]), np.array([[-h], [h], [0.0]])
    c11, c10 = np.array([[h], [h], [0.0]]), np.array([[h], [-h], [0.0]])
    A = uvlm.aic(c00, c01, c11, c10, np.zeros((3, 1)), np.array([[0.0], [0.0], [1.0]]), 0.0)
    assert abs(A[0, 0]) == pytest.approx(2 * math.sqrt(2) / (math.pi * a), rel=1e-13)


def test_eq8_counts_hand_example():
    """Tip line 0.1 long with n_t = 2: lines of 0.1, 0.25, 0.05, 0.3 and 0.2 get
    ceil(2, 5, 1, 6, 4) particles; a shed line gets one; a degenerate tip gives one."""
    lens = [0.1, 0.25, 0.05, 0.3, 0.2, 0.07]
    a = np.zeros((3, 6))
    b = np.zeros((3, 6))
    b[0] = lens
    tip = np.array([0, 0, 0, 0, 0, -1])
    assert uvlm.particle_counts(a, b, tip, 2).tolist() == [2, 5, 1, 6, 4, 1]
    b2 = b.copy()
    b2[0, 0] = 0.0
    assert uvlm.particle_counts(a, b2, np.array([0, 0]), 3).tolist()[:2] == [1, 1]


def test_conversion_positions_strengths_and_conservation():
    rng = np.random.default_rng(3)
    n = 40
    a = rng.normal(size=(3, n))
    b = a + rng.normal(size=(3, n)) * 0.2
    dg = rng.normal(size=n)
    tip = np.where(np.arange(n) < 30, 7, -1)
    x, g, s, cnt = uvlm.convert(a, b, dg, tip, 3, 0.02)
    assert x.shape[1] == cnt.sum() == g.shape[1] == s.shape[0]
    # total vorticity of the converted lines is conserved (Eq. 6)
    assert np.allclose(g.sum(1), (dg * (b - a)).sum(1), rtol=0, atol=1e-14)
    # one line, four particles: midpoints of quarters, equal strengths
    x1, g1, _, c1 = uvlm.convert(np.zeros((3, 1)), np.array([[1.0], [0.0], [0.0]]), [2.0], [0], 4, 0.01)
    assert c1.tolist() == [4]
    assert np.allclose(x1[0], [0.125, 0.375, 0.625, 0.875]) and np.allclose(x1[1:], 0)
    assert np.allclose(g1, [[0.5] * 4, [0] * 4, [0] * 4])


def test_converted_particles_reproduce_the_line_far_away():
    """Far from a line of strength dGamma, its n particles (Eq. 6) induce the line's
    velocity with an error of order (|dl| / (n s))^2: doubling n quarters it."""
    a = np.array([[0.0], [0.0], [0.0]])
    b = np.array([[0.4], [0.1], [0.0]])
    y = np.array([[0.3], [1.5], [0.4]])
    u_line = oracle.segments(a, b, [1.3], y, 0.0)
    errs = []
    for n in (2, 4, 8):
        x, g, s, _ = uvlm.convert(a, b, [1.3], [0], n, 1e-3)
        u, _ = oracle.eval_pairs(x, g, s, x_tgt=y)
        errs.append(np.linalg.norm(u - u_line) / np.linalg.norm(u_line))
    assert errs[0] < 2e-3
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


def test_shedding_kelvin_and_kutta():
    rng = np.random.default_rng(4)
    g_now = rng.normal(size=16)
    g_prev = rng.normal(size=16)
    tr, sh = uvlm.shed(g_now, g_prev)
    assert tr.shape == (17,) and sh.shape == (16,)
    # the trailed lines of a row close on themselves: their strengths sum to zero
    assert abs(tr.sum()) <= 1e-15 * np.abs(tr).sum()
    # Kelvin: each strip sheds the opposite of its change of bound circulation
    assert np.allclose(sh, g_prev - g_now, rtol=0, atol=0)
    # tips: the "neighbour absent" case of Eq. 7
    assert tr[0] == -g_now[0] and tr[-1] == g_now[-1]
    # starting vortex: nothing shed before
    _, sh0 = uvlm.shed(g_now, np.zeros(16))
    assert np.array_equal(sh0, -g_now)
