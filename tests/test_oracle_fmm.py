"""Pins of the oracle's Cartesian FMM (Sec. II.B names a Cartesian FMM for the velocity and
its gradient) against things other than itself: the direct sums (the FMM reduces to them
when every leaf is a neighbour of every other, and converges to them geometrically in the
expansion order), closed forms of the derivatives of 1/r, and Laplace's equation."""
import math

import numpy as np
import pytest

import oracle
from paper_2511_11430_amd import workloads as W


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_inv_r_taylor_closed_forms():
    R = np.array([0.7, -1.3, 0.4])
    r = np.linalg.norm(R)
    c, idx = oracle.inv_r_taylor(R, 6)
    tab = {tuple(i): v for i, v in zip(idx, c)}
    assert tab[(0, 0, 0)] == pytest.approx(1 / r, rel=1e-15)
    for a in range(3):
        e = [0, 0, 0]
        e[a] = 1
        assert tab[tuple(e)] == pytest.approx(-R[a] / r ** 3, rel=1e-14)          # D_a / 1!
        e[a] = 2
        assert tab[tuple(e)] == pytest.approx((3 * R[a] ** 2 - r * r) / r ** 5 / 2, rel=1e-13)  # D_aa / 2!
    assert tab[(1, 1, 0)] == pytest.approx(3 * R[0] * R[1] / r ** 5, rel=1e-13)
    assert tab[(1, 1, 1)] == pytest.approx(-15 * R[0] * R[1] * R[2] / r ** 7, rel=1e-12)


def test_inv_r_taylor_is_harmonic_and_homogeneous():
    """sum_a D_(n + 2 e_a) = 0 for every n (1/r is harmonic), and D_n(lambda R) =
    lambda^(-1-|n|) D_n(R)."""
    R = np.array([-2.1, 0.9, 1.7])
    c, idx = oracle.inv_r_taylor(R, 10)
    tab = {tuple(i): v for i, v in zip(idx, c)}
    fact = math.factorial
    for n in idx:
        if n.sum() > 8:
            continue
        s, scale = 0.0, 0.0
        for a in range(3):
            m = n.copy()
            m[a] += 2
            D = tab[tuple(m)] * fact(m[0]) * fact(m[1]) * fact(m[2])
            s += D
            scale += abs(D)
        assert abs(s) <= 1e-12 * max(scale, 1e-300)
    c2, _ = oracle.inv_r_taylor(2.5 * R, 10)
    deg = idx.sum(1)
    ref = c * 2.5 ** (-1.0 - deg)
    for k in range(11):
        m = deg == k
        assert np.abs(c2[m] - ref[m]).max() <= 1e-13 * np.abs(ref[m]).max()


@pytest.mark.parametrize("level", [0, 1])
@pytest.mark.parametrize("scheme", [oracle.TRANSPOSED, oracle.CLASSICAL])
def test_fmm_without_far_field_is_the_direct_sum(level, scheme):
    """At depth 0 and 1 every leaf neighbours every other: the FMM is the direct sum."""
    rng = np.random.default_rng(1)
    x = rng.uniform(-1, 1, (3, 400))
    g = rng.normal(size=(3, 400))
    s = rng.uniform(0.02, 0.2, 400)
    u, d = oracle.fmm(x, g, s, level, 4, scheme)
    uo, do = oracle.eval_pairs(x, g, s, scheme=scheme)
    assert _rel(u, uo) <= 1e-14 and _rel(d, do) <= 1e-14


@pytest.mark.parametrize("scheme", [oracle.TRANSPOSED, oracle.CLASSICAL])
def test_fmm_converges_to_the_direct_sum_with_order(scheme):
    """Forward-flight wake sample (sigma up to 0.05R, leaf width 26 sigma_max): the error of
    the far field falls geometrically with the order."""
    c = W.config3(n=6000)
    x, g, s = c["x"], c["gamma"], c["sigma"]
    uo, do = oracle.eval_pairs(x, g, s, scheme=scheme)
    errs = []
    for p in (2, 4, 6, 8, 10):
        u, d = oracle.fmm(x, g, s, 4, p, scheme)
        errs.append(max(_rel(u, uo), _rel(d, do)))
    assert all(b < a for a, b in zip(errs, errs[1:]))
    assert errs[-1] < errs[0] / 30
    assert errs[-1] < 2e-4


def test_fmm_keeps_converging_up_to_the_highest_order():
    """Orders 14 to 20 on the same wake sample at depth 3: the error of u and of the stretching
    against the direct sum keeps falling with every two orders (no loss of accuracy in the
    high-order terms), and order 20 is below 3e-7 for both."""
    c = W.config3(n=4999)
    x, g, s = c["x"], c["gamma"], c["sigma"]
    uo, do = oracle.eval_pairs(x, g, s)
    eu, ed = [], []
    for p in (14, 16, 18, 20):
        u, d = oracle.fmm(x, g, s, 3, p)
        eu.append(_rel(u, uo))
        ed.append(_rel(d, do))
    assert all(b < a for a, b in zip(eu, eu[1:])), eu
    assert all(b < a for a, b in zip(ed, ed[1:])), ed
    assert eu[-1] < 3e-7 and ed[-1] < 3e-7


def test_fmm_far_field_of_separated_clusters():
    """Two compact clusters far apart: with the order raised to 16 the far field matches the
    singular kernel's direct sum to 1e-9."""
    rng = np.random.default_rng(2)
    a = rng.normal(scale=0.02, size=(3, 60)) + np.array([[-1.0], [0.0], [0.0]])
    b = rng.normal(scale=0.02, size=(3, 60)) + np.array([[1.0], [0.3], [0.0]])
    x = np.concatenate([a, b], 1)
    g = rng.normal(size=(3, 120))
    s = np.full(120, 1e-3)
    u, d = oracle.fmm(x, g, s, 3, 16)
    uo, do = oracle.eval_pairs(x, g, s)
    assert _rel(u, uo) <= 1e-9 and _rel(d, do) <= 1e-9


@pytest.mark.parametrize("level", [1, 4])
def test_fmm_velocity_gradient(level):
    """J from the FMM: the direct sums' gradient at depth 1 (no far field), and at depth 4
    within the truncation error of the velocity; its trace vanishes (div u = 0) up to that
    error, and J^T Gamma_i equals the transposed stretching the FMM returns."""
    c = W.config3(n=3000)
    x, g, s = c["x"], c["gamma"], c["sigma"]
    u, d, J = oracle.fmm(x, g, s, level, 10, want_grad=True)
    Jo = oracle.velocity_gradient(x, g, s)
    e = _rel(J.reshape(9, -1), Jo.reshape(9, -1))
    assert e <= (1e-14 if level == 1 else 1e-3)
    assert np.allclose(np.einsum("abn,an->bn", J, g), d, rtol=0, atol=1e-10 * np.abs(d).max())
    tr = J[0, 0] + J[1, 1] + J[2, 2]
    assert np.abs(tr).max() <= (1e-12 if level == 1 else 1e-3) * np.abs(J).max()
