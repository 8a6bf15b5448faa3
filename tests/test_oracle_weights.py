"""Pins for the oracle's Gaussian-blob kernel weights (Eq. 3, Sec. II.B).

Each weight is checked against something other than the oracle's own formula:
quadrature of the blob, derivatives of the textbook potential of a Gaussian, the
singular point-vortex limit, and closed-form values at the origin.
"""
import math

import numpy as np
import pytest
import mpmath as mp

import oracle
from oracle import brute_mp

C0 = math.sqrt(2.0 / math.pi)


def zeta1(t):
    """Unit-core 3-D Gaussian of Eq. 3 at rho = t."""
    return (2 * math.pi) ** -1.5 * math.exp(-t * t / 2)


@pytest.mark.parametrize("rho", [1e-4, 0.05, 0.3, 0.9, 0.999999, 1.0, 1.000001, 1.7, 3.0, 6.0, 9.0])
def test_q_by_quadrature(rho):
    """q(rho) = Gw * rho^3 is the blob mass inside radius rho: int_0^rho 4 pi t^2 zeta(t) dt
    (30-digit quadrature)."""
    Gw, _, _ = oracle.weights(rho)
    with mp.workdps(30):
        z = lambda t: 4 * mp.pi * t * t * (2 * mp.pi) ** mp.mpf(-1.5) * mp.exp(-t * t / 2)
        q_quad = float(mp.quad(z, [0, mp.mpf(rho)]))
    assert abs(Gw * rho ** 3 - q_quad) <= 2e-15 * q_quad


@pytest.mark.parametrize("rho", [0.2, 0.7, 1.3, 2.5, 5.0])
def test_hw_kw_by_quadrature(rho):
    """Hw and Kw from the blob's radial moments: rho q' = 4 pi rho^3 zeta, q'' = d/drho (4 pi rho^2 zeta)."""
    Gw, Hw, Kw = oracle.weights(rho)
    q = Gw * rho ** 3
    qp = 4 * math.pi * rho ** 2 * zeta1(rho)
    qpp = 4 * math.pi * (2 * rho - rho ** 3) * zeta1(rho)
    assert Hw == pytest.approx((rho * qp - 3 * q) / rho ** 5, rel=1e-13)
    assert Kw == pytest.approx((rho ** 2 * qpp - 7 * rho * qp + 15 * q) / rho ** 7, rel=1e-12)


def test_series_and_closed_form_meet_at_rho_1():
    """The two branches (series below 1, closed form above) agree across the switch."""
    lo = np.array(oracle.weights(1.0 - 4e-15))
    hi = np.array(oracle.weights(1.0))
    assert np.allclose(lo, hi, rtol=1e-13, atol=0)


@pytest.mark.parametrize("s,sigma", [(1e-5, 0.05), (0.01, 0.05), (0.049, 0.05), (0.07, 0.05),
                                     (0.2, 0.05), (0.02, 0.01), (0.3, 0.1)])
def test_ghk_against_potential(s, sigma):
    """g = -G'(s)/s, h = g'/s, k = h'/s of the Gaussian's potential erf(s/(sqrt2 sigma))/(4 pi s),
    differentiated numerically at 40 digits."""
    g, h, k = oracle.ghk(s, sigma)
    gb, hb, kb = brute_mp.kernel_weights(s, sigma)
    assert g == pytest.approx(gb, rel=2e-14)
    assert h == pytest.approx(hb, rel=2e-14)
    assert k == pytest.approx(kb, rel=1e-13)


def test_limits_at_origin():
    """g(0) = c0/(12 pi sigma^3), h(0) = -c0/(20 pi sigma^5), k(0) = c0/(28 pi sigma^7)."""
    sigma = 0.03
    g, h, k = oracle.ghk(0.0, sigma)
    assert g == pytest.approx(C0 / (12 * math.pi * sigma ** 3), rel=1e-15)
    assert h == pytest.approx(-C0 / (20 * math.pi * sigma ** 5), rel=1e-15)
    assert k == pytest.approx(C0 / (28 * math.pi * sigma ** 7), rel=1e-15)


@pytest.mark.parametrize("rho", [9.5, 11.0, 20.0, 100.0])
def test_far_field_is_point_vortex(rho):
    """Beyond rho = 9.5 the blob is a singular Biot-Savart point vortex to FP64 rounding:
    g = 1/(4 pi s^3), h = -3/(4 pi s^5), k = 15/(4 pi s^7)."""
    sigma = 0.02
    s = rho * sigma
    g, h, k = oracle.ghk(s, sigma)
    assert g == pytest.approx(1 / (4 * math.pi * s ** 3), rel=4e-16)
    assert h == pytest.approx(-3 / (4 * math.pi * s ** 5), rel=1e-15)
    assert k == pytest.approx(15 / (4 * math.pi * s ** 7), rel=1e-14)


def test_far_threshold_fp32():
    """At rho = 7 the point-vortex weights differ from the blob's by less than half an FP32 ulp,
    which is what lets the FP32 path drop erf/exp beyond it."""
    for rho in (7.0, 7.5):
        Gw, Hw, _ = oracle.weights(rho)
        assert abs(Gw * rho ** 3 - 1) < 2 ** -25
        assert abs(Hw * rho ** 5 / -3 - 1) < 2 ** -25
