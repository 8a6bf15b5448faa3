"""Pins for the oracle's particle sums: velocity and stretching (Eqs. 2-5, Sec. II.B).

The oracle is checked against an independent arbitrary-precision route (the vector
potential of the Gaussian field, differentiated numerically), the point-vortex limit,
solid-body rotation inside a core, exact invariants of the transposed scheme, and the
velocity gradient taken by finite differences.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import brute_mp

C0 = math.sqrt(2.0 / math.pi)


def _small_set(n, seed, spread=0.1):
    rng = np.random.default_rng([7, seed])
    x = rng.uniform(-spread, spread, (3, n))
    g = rng.normal(0, 1e-3, (3, n))
    s = rng.uniform(0.02, 0.06, n)
    return x, g, s


@pytest.mark.parametrize("scheme", [oracle.TRANSPOSED, oracle.CLASSICAL])
@pytest.mark.parametrize("rule", [oracle.SIGMA_SOURCE, oracle.SIGMA_SYMMETRIC])
def test_against_potential_brute_force(scheme, rule):
    """Whole oracle vs 30-digit curl/gradient of the vector potential, N = 8."""
    x, g, s = _small_set(8, 1)
    u, d = oracle.eval_pairs(x, g, s, scheme=scheme, sigma_rule=rule)
    ub, db = brute_mp.particle_sums(x.T, g.T, s, scheme=scheme, sigma_rule=rule)
    ub, db = np.array(ub).T, np.array(db).T
    assert np.linalg.norm(u - ub) <= 1e-14 * np.linalg.norm(ub)
    assert np.linalg.norm(d - db) <= 1e-14 * np.linalg.norm(db)


def test_brute_force_spread_set():
    """Mixed near and far pairs (rho from ~0.1 to ~60) against the potential route."""
    x, g, s = _small_set(10, 2, spread=1.0)
    s = s * 0.5
    u, d = oracle.eval_pairs(x, g, s)
    ub, db = brute_mp.particle_sums(x.T, g.T, s)
    ub, db = np.array(ub).T, np.array(db).T
    assert np.linalg.norm(u - ub) <= 1e-14 * np.linalg.norm(ub)
    assert np.linalg.norm(d - db) <= 1e-14 * np.linalg.norm(db)


def test_far_pair_is_singular_biot_savart():
    """Two particles 12 cores apart: u_1 = Gamma_2 x r / (4 pi s^3) exactly in FP64."""
    x = np.array([[0.0, 0.3], [0.0, 0.4], [0.0, -0.1]])
    g = np.array([[1e-3, -2e-3], [5e-4, 1e-3], [2e-3, 3e-4]])
    s = np.full(2, 0.5 / 12)
    u, _ = oracle.eval_pairs(x, g, s)
    r = x[:, 0] - x[:, 1]
    expect = np.cross(g[:, 1], r) / (4 * math.pi * np.linalg.norm(r) ** 3)
    assert np.allclose(u[:, 0], expect, rtol=1e-15, atol=0)
    assert np.allclose(u[:, 1], -np.cross(g[:, 0], r) / (4 * math.pi * np.linalg.norm(r) ** 3), rtol=1e-15)


def test_solid_body_rotation_inside_core():
    """A target deep inside a source's core turns rigidly: u = g(0) Gamma x r, g(0) = c0/(12 pi sigma^3)."""
    sigma = 0.05
    xs = np.zeros((3, 1))
    gs = np.array([[0.0], [0.0], [1e-3]])
    xt = np.array([[1e-6], [2e-6], [0.0]])
    u, _ = oracle.eval_pairs(xs, gs, [sigma], x_tgt=xt)
    expect = C0 / (12 * math.pi * sigma ** 3) * np.cross(gs[:, 0], xt[:, 0])
    assert np.allclose(u[:, 0], expect, rtol=1e-9)


def test_coincident_distinct_particles():
    """Two different particles at one point: no velocity, stretching g(0) Gamma_i x Gamma_j."""
    x = np.zeros((3, 2))
    g = np.array([[1e-3, 0.0], [0.0, 2e-3], [0.0, 0.0]])
    s = np.full(2, 0.04)
    u, d = oracle.eval_pairs(x, g, s)
    g0 = C0 / (12 * math.pi * 0.04 ** 3)
    assert np.all(u == 0)
    assert np.allclose(d[:, 0], g0 * np.cross(g[:, 0], g[:, 1]), rtol=1e-15)
    assert np.allclose(d[:, 1], g0 * np.cross(g[:, 1], g[:, 0]), rtol=1e-15)


def test_pair_velocity_kernel_is_odd():
    """The velocity kernel is odd in r: swapping target and source (same Gamma, same sigma) negates u."""
    x = np.array([[0.0, 0.03], [0.0, -0.01], [0.0, 0.02]])
    g = np.array([[1e-3, 1e-3], [2e-3, 2e-3], [-1e-3, -1e-3]])
    u, _ = oracle.eval_pairs(x, g, np.full(2, 0.02))
    assert np.allclose(u[:, 0], -u[:, 1], rtol=1e-15, atol=0)


@pytest.mark.parametrize("rule,uniform", [(oracle.SIGMA_SYMMETRIC, False), (oracle.SIGMA_SOURCE, True)])
def test_total_vorticity_conserved_transposed(rule, uniform):
    """Transposed scheme with a symmetric core: sum_i dGamma_i/dt = 0 (pairwise antisymmetric terms)."""
    x, g, s = _small_set(200, 3, spread=0.3)
    if uniform:
        s = np.full_like(s, 0.04)
    u, d = oracle.eval_pairs(x, g, s, sigma_rule=rule)
    scale = np.abs(d).sum()
    assert np.abs(d.sum(axis=1)).max() <= 1e-14 * scale


def test_classical_scheme_does_not_conserve():
    """The classical scheme has no such identity; the sum is O(1) relative to the terms."""
    x, g, s = _small_set(200, 3, spread=0.3)
    _, d = oracle.eval_pairs(x, g, s, scheme=oracle.CLASSICAL, sigma_rule=oracle.SIGMA_SYMMETRIC)
    assert np.abs(d.sum(axis=1)).max() > 1e-3 * np.abs(d).sum()


def test_impulse_rate_identity():
    """Transposed scheme, symmetric cores: d/dt (1/2 sum x_i x Gamma_i) = sum_{i<j} g_ij r_ij x (Gamma_i x Gamma_j)
    (Jacobi identity on the pair terms)."""
    x, g, s = _small_set(60, 4, spread=0.2)
    u, d = oracle.eval_pairs(x, g, s, sigma_rule=oracle.SIGMA_SYMMETRIC)
    rate = oracle.diagnostics(x, g, u, d)["impulse_rate"]
    expect = np.zeros(3)
    n = x.shape[1]
    for i in range(n):
        for j in range(i + 1, n):
            r = x[:, i] - x[:, j]
            sig = math.sqrt(0.5 * (s[i] ** 2 + s[j] ** 2))
            gij, _, _ = oracle.ghk(float(np.linalg.norm(r)), sig)
            expect += gij * np.cross(r, np.cross(g[:, i], g[:, j]))
    assert np.allclose(rate, expect, rtol=1e-12, atol=1e-13 * np.abs(expect).max())


def test_impulse_nearly_conserved_on_closed_ring():
    """A discretised, non-planar closed vortex ring (sum Gamma = 0 exactly) keeps its linear
    impulse to a residual that is a discretisation error: it falls ~4x per halving of the
    particle spacing at fixed core size (second order)."""
    res = []
    for n in (32, 64, 128):
        th = 2 * math.pi * np.arange(n + 1) / n
        rad = 0.3 * (1 + 0.15 * np.cos(3 * th))
        nodes = np.stack([rad * np.cos(th), rad * np.sin(th), 0.05 * np.sin(2 * th)])
        x = 0.5 * (nodes[:, :-1] + nodes[:, 1:])
        g = 0.1 * (nodes[:, 1:] - nodes[:, :-1])
        u, d = oracle.eval_pairs(x, g, np.full(n, 0.06))
        diag = oracle.diagnostics(x, g, u, d)
        assert np.abs(diag["sum_gamma"]).max() < 1e-16
        res.append(np.linalg.norm(diag["impulse_rate"]) / np.linalg.norm(diag["impulse"]))
    assert 3.5 < res[0] / res[1] < 4.5 and 3.5 < res[1] / res[2] < 4.5


def test_stretching_is_transposed_velocity_gradient():
    """dGamma_i/dt = J(x_i)^T Gamma_i (and J Gamma_i for the classical scheme), J = grad u by
    central differences of the velocity with particle i removed."""
    x, g, s = _small_set(12, 5, spread=0.08)
    i = 3
    others = [j for j in range(12) if j != i]
    hstep = 1e-6
    J = np.zeros((3, 3))
    for l in range(3):
        e = np.zeros((3, 1))
        e[l, 0] = hstep
        up, _ = oracle.eval_pairs(x[:, others], g[:, others], s[others], x_tgt=x[:, [i]] + e)
        um, _ = oracle.eval_pairs(x[:, others], g[:, others], s[others], x_tgt=x[:, [i]] - e)
        J[:, l] = (up[:, 0] - um[:, 0]) / (2 * hstep)
    _, dT = oracle.eval_pairs(x, g, s, scheme=oracle.TRANSPOSED)
    _, dC = oracle.eval_pairs(x, g, s, scheme=oracle.CLASSICAL)
    assert np.allclose(dT[:, i], J.T @ g[:, i], rtol=1e-7, atol=1e-9 * np.abs(dT[:, i]).max())
    assert np.allclose(dC[:, i], J @ g[:, i], rtol=1e-7, atol=1e-9 * np.abs(dC[:, i]).max())


def test_explicit_targets_match_self_evaluation():
    """Evaluating at explicit targets with per-target exclusion equals the self evaluation."""
    x, g, s = _small_set(40, 6)
    u, d = oracle.eval_pairs(x, g, s)
    idx = np.array([0, 7, 39, 12])
    u2, d2 = oracle.eval_pairs(x, g, s, x_tgt=x[:, idx], gam_tgt=g[:, idx], excl=idx)
    assert np.array_equal(u2, u[:, idx]) and np.array_equal(d2, d[:, idx])


def test_tangent_matches_finite_differences():
    """Dual-number tangent of (u, dGamma/dt) vs central differences of the oracle."""
    x, g, s = _small_set(16, 7)
    rng = np.random.default_rng(11)
    xd = rng.normal(size=x.shape)
    gd = rng.normal(size=g.shape) * 1e-3
    u, d, ud, dd = oracle.eval_pairs_jvp(x, g, s, xd, gd)
    eps = 1e-7
    up, dp = oracle.eval_pairs(x + eps * xd, g + eps * gd, s)
    um, dm = oracle.eval_pairs(x - eps * xd, g - eps * gd, s)
    assert np.allclose(ud, (up - um) / (2 * eps), rtol=1e-6, atol=1e-6 * np.abs(ud).max())
    assert np.allclose(dd, (dp - dm) / (2 * eps), rtol=1e-6, atol=1e-6 * np.abs(dd).max())
