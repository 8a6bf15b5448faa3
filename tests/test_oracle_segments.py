"""Pins for the oracle's straight-segment velocity with the Vatistas core (Sec. II.A).

The finite-segment Biot-Savart part is checked by quadrature of the line integral and by
the centre of a square vortex ring; the Vatistas factor by the swirl profile of a long
straight vortex; plus orientation, additivity and the far-field particle limit (Eq. 6
with one particle per element).
"""
import math

import numpy as np
import pytest

import oracle
from oracle import brute_mp


def _seg(a, b):
    return np.array(a, dtype=float).reshape(3, 1), np.array(b, dtype=float).reshape(3, 1)


@pytest.mark.parametrize("p", [(0.3, 0.2, 0.1), (-0.5, 0.05, 0.0), (1.5, -0.2, 0.7), (0.5, 0.0, 1e-3)])
def test_singular_segment_by_quadrature(p):
    a, b = _seg((0.0, 0.0, 0.0), (1.0, 0.2, -0.1))
    u = oracle.segments(a, b, [0.7], np.array(p).reshape(3, 1), core_radius=0.0)
    ub = brute_mp.segment_velocity_singular(a[:, 0], b[:, 0], 0.7, p)
    assert np.allclose(u[:, 0], ub, rtol=1e-13, atol=1e-15 * np.abs(ub).max())


def test_square_ring_centre():
    """Centre of a square ring of side a and circulation G: |u| = 2 sqrt(2) G / (pi a), along the normal."""
    side, G = 0.4, 1.3
    c = [(0, 0, 0), (side, 0, 0), (side, side, 0), (0, side, 0)]
    A = np.array([c[0], c[1], c[2], c[3]]).T
    B = np.array([c[1], c[2], c[3], c[0]]).T
    u = oracle.segments(A, B, [G] * 4, np.array([[side / 2], [side / 2], [0.0]]), core_radius=0.0)
    assert u[2, 0] == pytest.approx(2 * math.sqrt(2) * G / (math.pi * side), rel=1e-14)
    assert abs(u[0, 0]) < 1e-14 and abs(u[1, 0]) < 1e-14


@pytest.mark.parametrize("n", [1, 2, 3])
@pytest.mark.parametrize("d", [0.002, 0.02, 0.05, 0.3])
def test_long_segment_vatistas_profile(n, d):
    """Far from its ends a segment is an infinite line vortex with the Vatistas swirl
    G d / (2 pi (rc^(2n) + d^(2n))^(1/n))."""
    rc, G = 0.02, 0.5
    a, b = _seg((-1e5, 0, 0), (1e5, 0, 0))
    u = oracle.segments(a, b, [G], np.array([[0.0], [d], [0.0]]), core_radius=rc, vatistas_n=n)
    expect = G * d / (2 * math.pi * (rc ** (2 * n) + d ** (2 * n)) ** (1.0 / n))
    assert np.linalg.norm(u[:, 0]) == pytest.approx(expect, rel=1e-9)
    assert u[2, 0] == pytest.approx(expect, rel=1e-9)  # right-handed about +x at +y gives +z


def test_swapping_ends_negates():
    rng = np.random.default_rng(3)
    A, B = rng.normal(size=(3, 20)), rng.normal(size=(3, 20))
    g = rng.normal(0.5, 0.1, 20)
    P = rng.normal(size=(3, 30))
    u1 = oracle.segments(A, B, g, P, core_radius=0.05)
    u2 = oracle.segments(B, A, g, P, core_radius=0.05)
    assert np.allclose(u1, -u2, rtol=1e-14, atol=1e-16)


@pytest.mark.parametrize("rc", [0.0, 0.03])
def test_collinear_split_is_additive(rc):
    """The core factor depends only on the distance to the line, so splitting a segment at an
    interior point leaves the velocity unchanged."""
    a, b = np.array([0.1, -0.2, 0.3]), np.array([0.7, 0.4, -0.1])
    m = a + 0.37 * (b - a)
    P = np.random.default_rng(4).normal(scale=0.5, size=(3, 16))
    whole = oracle.segments(a.reshape(3, 1), b.reshape(3, 1), [0.9], P, core_radius=rc)
    parts = oracle.segments(np.stack([a, m], 1), np.stack([m, b], 1), [0.9, 0.9], P, core_radius=rc)
    assert np.allclose(whole, parts, rtol=1e-12, atol=1e-15)


def test_far_field_is_a_particle():
    """Far away, a segment acts like one point vortex Gamma_s dl at its midpoint (Eq. 6 with
    one particle); the relative gap closes as (|dl|/s)^2."""
    a, b = np.array([0.0, 0.0, 0.0]), np.array([0.1, 0.05, 0.02])
    mid, dl = 0.5 * (a + b), b - a
    direction = np.array([0.3, 0.8, -0.52])
    direction /= np.linalg.norm(direction)
    gaps = []
    for dist in (1.0, 2.0, 4.0):
        P = mid + dist * direction
        u = oracle.segments(a.reshape(3, 1), b.reshape(3, 1), [0.8], P.reshape(3, 1), core_radius=0.01)[:, 0]
        r = P - mid
        up = 0.8 * np.cross(dl, r) / (4 * math.pi * np.linalg.norm(r) ** 3)
        gaps.append(np.linalg.norm(u - up) / np.linalg.norm(up))
    assert 3.6 < gaps[0] / gaps[1] < 4.4 and 3.6 < gaps[1] / gaps[2] < 4.4


def test_degenerate_segments_contribute_nothing():
    """Zero-length segments and targets on an end point give zero; a target on the line
    with a core gives zero."""
    A = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    B = np.array([[0.0, 1.0, 1.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    P = np.array([[0.0, 0.5, 1.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    u = oracle.segments(A, B, [1.0, 1.0, 1.0], P, core_radius=0.02)
    assert np.all(u == 0)


# ------------------------------------------------------------------ velocity gradient (lattice on particles)

@pytest.mark.parametrize("rc,vn", [(0.0, 2), (0.05, 2), (0.05, 1), (0.08, 3)])
def test_segment_gradient_matches_central_differences(rc, vn):
    rng = np.random.default_rng(11)
    a = rng.normal(size=(3, 20))
    b = a + rng.normal(size=(3, 20)) * 0.3
    g = rng.normal(size=20)
    y = rng.normal(size=(3, 6))
    J = oracle.segments_gradient(a, b, g, y, rc, vn)
    h = 1e-6
    Jf = np.zeros_like(J)
    for c in range(3):
        yp, ym = y.copy(), y.copy()
        yp[c] += h
        ym[c] -= h
        Jf[:, c, :] = (oracle.segments(a, b, g, yp, rc, vn) - oracle.segments(a, b, g, ym, rc, vn)) / (2 * h)
    assert np.abs(J - Jf).max() <= 1e-8 * np.abs(J).max()


def test_segment_gradient_is_divergence_free():
    """The core factor depends only on the distance to the line, across which the velocity is
    azimuthal, so the cored field stays divergence free: tr J = 0."""
    rng = np.random.default_rng(12)
    a = rng.normal(size=(3, 50))
    b = a + rng.normal(size=(3, 50)) * 0.2
    J = oracle.segments_gradient(a, b, rng.normal(size=50), rng.normal(size=(3, 40)), 0.05, 2)
    assert np.abs(np.einsum("aat->t", J)).max() <= 1e-13 * np.abs(J).max()


def test_segment_gradient_infinite_line_profile():
    """A long line along z (Vatistas n = 2): u_y(x) = G x / (2 pi sqrt(rc^4 + x^4)), so
    du_y/dx = G (rc^4 - x^4) / (2 pi (rc^4 + x^4)^(3/2)) on the x axis."""
    G, rc, L = 1.7, 0.05, 1e4
    a, b = np.array([[0.0], [0.0], [-L]]), np.array([[0.0], [0.0], [L]])
    for d in (0.01, 0.05, 0.2):
        J = oracle.segments_gradient(a, b, [G], np.array([[d], [0.0], [0.0]]), rc, 2)
        ref = G * (rc ** 4 - d ** 4) / (2 * math.pi * (rc ** 4 + d ** 4) ** 1.5)
        assert J[1, 0, 0] == pytest.approx(ref, rel=1e-7, abs=1e-8 * G / rc ** 2)


def _vjp_case(seed=7, n=12):
    rng = np.random.default_rng(seed)
    a = rng.uniform(-0.2, 0.2, (3, 6))
    b = a + rng.normal(size=(3, 6)) * 0.1
    gs = rng.normal(size=6)
    x = rng.uniform(-0.25, 0.25, (3, n))
    g = rng.normal(size=(3, n))
    ub = rng.normal(size=(3, n))
    db = rng.normal(size=(3, n))
    return a, b, gs, x, g, ub, db


def _seg_loss(a, b, gs, x, g, ub, db, rc, scheme):
    """L = sum ub . u + db . s from the oracle's velocity and first-derivative routines."""
    u = oracle.segments(a, b, gs, x, rc, 2)
    J = oracle.segments_gradient(a, b, gs, x, rc, 2)
    s = np.einsum("abn,an->bn", J, g) if scheme == oracle.TRANSPOSED else np.einsum("abn,bn->an", J, g)
    return float((ub * u).sum() + (db * s).sum())


@pytest.mark.parametrize("scheme", [oracle.TRANSPOSED, oracle.CLASSICAL])
@pytest.mark.parametrize("rc", [0.0, 0.03])
def test_segment_vjp_matches_central_differences(scheme, rc):
    """x_bar (which needs the segment law's second derivatives) against central differences
    of L built from the velocity and its first derivative."""
    a, b, gs, x, g, ub, db = _vjp_case()
    xb, _ = oracle.segments_vjp(a, b, gs, x, rc, 2, ub, db, g, scheme)
    h = 1e-6
    for t in (0, 5, 11):
        for c in range(3):
            xp, xm = x.copy(), x.copy()
            xp[c, t] += h
            xm[c, t] -= h
            fd = (_seg_loss(a, b, gs, xp, g, ub, db, rc, scheme) - _seg_loss(a, b, gs, xm, g, ub, db, rc, scheme))
            fd /= 2 * h
            assert xb[c, t] == pytest.approx(fd, rel=2e-6, abs=1e-6 * np.abs(xb).max())


@pytest.mark.parametrize("scheme", [oracle.TRANSPOSED, oracle.CLASSICAL])
def test_segment_vjp_strength_gradient_is_exact_by_linearity(scheme):
    """L is linear in the particle strengths, so L(G + D) - L(G) = D . G_bar to rounding."""
    a, b, gs, x, g, ub, db = _vjp_case(8)
    _, gb = oracle.segments_vjp(a, b, gs, x, 0.02, 2, ub, db, g, scheme)
    D = np.random.default_rng(9).normal(size=g.shape)
    dL = _seg_loss(a, b, gs, x, g + D, ub, db, 0.02, scheme) - _seg_loss(a, b, gs, x, g, ub, db, 0.02, scheme)
    assert dL == pytest.approx(float((D * gb).sum()), rel=1e-12)


def test_segment_hessian_is_symmetric():
    """The second-derivative term is H w with H the Hessian of Gamma . u at each particle, so
    v . (H w) = w . (H v) point by point (a swapped index would break it)."""
    a, b, gs, x, g, _, _ = _vjp_case(10)
    rng = np.random.default_rng(11)
    v, w = rng.normal(size=x.shape), rng.normal(size=x.shape)
    z = np.zeros_like(x)
    Hw, _ = oracle.segments_vjp(a, b, gs, x, 0.02, 2, z, w, g, oracle.TRANSPOSED)
    Hv, _ = oracle.segments_vjp(a, b, gs, x, 0.02, 2, z, v, g, oracle.TRANSPOSED)
    lhs, rhs = (v * Hw).sum(0), (w * Hv).sum(0)
    assert np.allclose(lhs, rhs, rtol=1e-10, atol=1e-12 * np.abs(lhs).max())
    # the two schemes swap the roles of the particle strength and the stretching seed
    Hc, _ = oracle.segments_vjp(a, b, gs, x, 0.02, 2, z, g, w, oracle.CLASSICAL)
    assert np.allclose(Hc, Hw, rtol=1e-12, atol=1e-14 * np.abs(Hw).max())
