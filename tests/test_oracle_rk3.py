"""Pins for the oracle's time integration (low-storage RK3 of Sec. II.B) and its tangent.

A co-rotating pair of parallel blobs has a closed-form motion (rigid rotation about the
midpoint at a rate fixed by g(d)); the program must converge to it at third order.  The
dual-number tangent of the whole program is checked by central differences.
"""
import math

import numpy as np
import pytest

import oracle


def _pair(d=0.04, gz=2e-3, sigma=0.03):
    x = np.array([[-d / 2, d / 2], [0.0, 0.0], [0.0, 0.0]])
    g = np.array([[0.0, 0.0], [0.0, 0.0], [gz, gz]])
    return x, g, np.full(2, sigma)


def test_corotating_pair_third_order():
    x0, g0, s = _pair()
    d = 0.04
    gd, _, _ = oracle.ghk(d, 0.03)
    omega = 2 * gd * 2e-3          # |u| = g d |Gamma| on a circle of radius d/2
    T = 2.0 / omega                # about a third of a turn
    errs = []
    for nsteps in (8, 16, 32):
        x, g, _, _ = oracle.rk3_program(x0, g0, s, nsteps, T / nsteps)
        ang = omega * T
        exact = np.array([[-d / 2 * math.cos(ang), d / 2 * math.cos(ang)],
                          [-d / 2 * math.sin(ang), d / 2 * math.sin(ang)], [0.0, 0.0]])
        assert np.array_equal(g, g0)  # parallel filaments do not stretch each other
        errs.append(np.abs(x - exact).max())
    assert 7.0 < errs[0] / errs[1] < 9.0 and 7.0 < errs[1] / errs[2] < 9.0


# Butcher form of the 2N-storage coefficients A = (0, -5/9, -153/128), B = (1/3, 15/16, 8/15),
# obtained by expanding the three register updates by hand.
BUTCHER_A = ((0.0, 0.0), (1.0 / 3.0, 0.0), (-3.0 / 16.0, 15.0 / 16.0))
BUTCHER_B = (1.0 / 6.0, 3.0 / 10.0, 8.0 / 15.0)


def test_butcher_form_has_third_order():
    """The four order conditions up to third order hold for the expanded tableau."""
    c = [sum(row) for row in BUTCHER_A]
    b = BUTCHER_B
    assert sum(b) == pytest.approx(1.0, abs=1e-15)
    assert sum(bi * ci for bi, ci in zip(b, c)) == pytest.approx(0.5, abs=1e-15)
    assert sum(bi * ci * ci for bi, ci in zip(b, c)) == pytest.approx(1.0 / 3.0, abs=1e-15)
    assert b[2] * BUTCHER_A[2][1] * c[1] == pytest.approx(1.0 / 6.0, abs=1e-15)


def test_single_step_is_williamson_rk3():
    """One program step equals the three-stage Butcher form evaluated with the oracle's RHS."""
    rng = np.random.default_rng(5)
    x = rng.uniform(-0.05, 0.05, (3, 5))
    g = rng.normal(0, 1e-3, (3, 5))
    s = np.full(5, 0.03)
    dt = 0.7

    def F(x, g):
        return oracle.eval_pairs(x, g, s)

    A, b = BUTCHER_A, BUTCHER_B
    k1 = F(x, g)
    k2 = F(x + dt * A[1][0] * k1[0], g + dt * A[1][0] * k1[1])
    k3 = F(x + dt * (A[2][0] * k1[0] + A[2][1] * k2[0]), g + dt * (A[2][0] * k1[1] + A[2][1] * k2[1]))
    xe = x + dt * (b[0] * k1[0] + b[1] * k2[0] + b[2] * k3[0])
    ge = g + dt * (b[0] * k1[1] + b[1] * k2[1] + b[2] * k3[1])
    x1, g1, _, _ = oracle.rk3_program(x, g, s, 1, dt)
    assert np.allclose(x1, xe, rtol=1e-13, atol=1e-16)
    assert np.allclose(g1, ge, rtol=1e-12, atol=1e-18)


def test_program_tangent_matches_central_differences():
    rng = np.random.default_rng(6)
    n = 24
    x = rng.uniform(-0.1, 0.1, (3, n))
    g = rng.normal(0, 1e-3, (3, n))
    s = np.full(n, 0.04)
    y = rng.uniform(-0.1, 0.1, (3, 5))
    xd = rng.normal(size=x.shape)
    gd = rng.normal(size=g.shape) * 1e-3
    dt, nsteps = 0.5, 3
    L, dL = oracle.rk3_program_jvp(x, g, s, xd, gd, nsteps, dt, y)
    h = 1e-6
    Lp = oracle.rk3_program(x + h * xd, g + h * gd, s, nsteps, dt, y)[3]
    Lm = oracle.rk3_program(x - h * xd, g - h * gd, s, nsteps, dt, y)[3]
    _, _, _, L0 = oracle.rk3_program(x, g, s, nsteps, dt, y)
    assert L == pytest.approx(L0, rel=1e-15)
    assert dL == pytest.approx((Lp - Lm) / (2 * h), rel=1e-6)


def _lattice(rng):
    a = rng.uniform(-0.12, 0.12, (3, 8))
    b = a + rng.normal(size=(3, 8)) * 0.05
    return a, b, rng.normal(size=8) * 1e-3


@pytest.mark.parametrize("scheme", [oracle.TRANSPOSED, oracle.CLASSICAL])
def test_single_step_with_lattice_is_williamson_rk3(scheme):
    """With a fixed lattice the right-hand side gains the segments' velocity and stretching
    (J^T Gamma or J Gamma); one program step equals the Butcher form built from the
    oracle's separate particle, segment and segment-gradient routines."""
    rng = np.random.default_rng(12)
    x = rng.uniform(-0.05, 0.05, (3, 5))
    g = rng.normal(0, 1e-3, (3, 5))
    s = np.full(5, 0.03)
    sa, sb, sg = _lattice(rng)
    dt = 0.7

    def F(x, g):
        u, d = oracle.eval_pairs(x, g, s, scheme=scheme)
        u = u + oracle.segments(sa, sb, sg, x, 0.02, 2)
        J = oracle.segments_gradient(sa, sb, sg, x, 0.02, 2)
        d = d + (np.einsum("abn,an->bn", J, g) if scheme == oracle.TRANSPOSED else np.einsum("abn,bn->an", J, g))
        return u, d

    A, b = BUTCHER_A, BUTCHER_B
    k1 = F(x, g)
    k2 = F(x + dt * A[1][0] * k1[0], g + dt * A[1][0] * k1[1])
    k3 = F(x + dt * (A[2][0] * k1[0] + A[2][1] * k2[0]), g + dt * (A[2][0] * k1[1] + A[2][1] * k2[1]))
    xe = x + dt * (b[0] * k1[0] + b[1] * k2[0] + b[2] * k3[0])
    ge = g + dt * (b[0] * k1[1] + b[1] * k2[1] + b[2] * k3[1])
    y = rng.uniform(-0.1, 0.1, (3, 3))
    x1, g1, uc, _ = oracle.rk3_program(x, g, s, 1, dt, y, scheme=scheme, segments=(sa, sb, sg, 0.02, 2))
    assert np.allclose(x1, xe, rtol=1e-13, atol=1e-16)
    assert np.allclose(g1, ge, rtol=1e-12, atol=1e-18)
    uc_e = oracle.eval_pairs(x1, g1, s, x_tgt=y)[0] + oracle.segments(sa, sb, sg, y, 0.02, 2)
    assert np.allclose(uc, uc_e, rtol=1e-13, atol=1e-18)


@pytest.mark.parametrize("scheme", [oracle.TRANSPOSED, oracle.CLASSICAL])
def test_program_with_lattice_tangent_matches_central_differences(scheme):
    rng = np.random.default_rng(13)
    n = 16
    x = rng.uniform(-0.1, 0.1, (3, n))
    g = rng.normal(0, 1e-3, (3, n))
    s = np.full(n, 0.04)
    y = rng.uniform(-0.1, 0.1, (3, 5))
    lat = (*_lattice(rng), 0.02, 2)
    xd = rng.normal(size=x.shape)
    gd = rng.normal(size=g.shape) * 1e-3
    dt, nsteps = 0.5, 3
    L, dL = oracle.rk3_program_jvp(x, g, s, xd, gd, nsteps, dt, y, scheme=scheme, segments=lat)
    h = 1e-6
    Lp = oracle.rk3_program(x + h * xd, g + h * gd, s, nsteps, dt, y, scheme=scheme, segments=lat)[3]
    Lm = oracle.rk3_program(x - h * xd, g - h * gd, s, nsteps, dt, y, scheme=scheme, segments=lat)[3]
    L0 = oracle.rk3_program(x, g, s, nsteps, dt, y, scheme=scheme, segments=lat)[3]
    assert L == pytest.approx(L0, rel=1e-15)
    assert dL == pytest.approx((Lp - Lm) / (2 * h), rel=1e-6)
    # without the lattice the loss differs (the lattice is felt)
    assert abs(oracle.rk3_program(x, g, s, nsteps, dt, y, scheme=scheme)[3] - L0) > 1e-3 * abs(L0)


def test_fp32_storage_models_do_what_they_state():
    """The program's FP32 storage models (test instruments that separate the GPU kernels' error
    from the cost of FP32 storage): with the state and registers stored in FP32 every returned
    state value is an FP32 number; with FP32 evaluations only the state stays FP64; both stay
    within FP32 rounding of the exact program on a short program; with no step, the loss is
    the sum of squares of the FP32-rounded control-point velocities."""
    rng = np.random.default_rng(11)
    n = 20
    x = rng.uniform(-0.1, 0.1, (3, n)).astype(np.float32).astype(np.float64)
    g = rng.normal(0, 1e-3, (3, n)).astype(np.float32).astype(np.float64)
    s = np.full(n, 0.03)
    y = rng.uniform(-0.1, 0.1, (3, 4))
    dt = 2e-4
    x0, g0, uc0, L0 = oracle.rk3_program(x, g, s, 3, dt, y)
    x1, g1, uc1, L1 = oracle.rk3_program(x, g, s, 3, dt, y, storage=oracle.STORE_F32_EVAL)
    x2, g2, uc2, L2 = oracle.rk3_program(x, g, s, 3, dt, y, storage=oracle.STORE_F32)
    f32 = lambda a: a.astype(np.float32).astype(np.float64)
    assert np.array_equal(x2, f32(x2)) and np.array_equal(g2, f32(g2))
    assert not np.array_equal(x1, f32(x1))  # FP64 state under FP32 evaluations
    assert np.array_equal(uc1, f32(uc1)) and np.array_equal(uc2, f32(uc2))
    for L in (L1, L2):
        assert abs(L - L0) <= 1e-5 * abs(L0) and L != L0
    assert np.abs(x1 - x0).max() <= 1e-6 and np.abs(x2 - x0).max() <= 1e-6
    # no step: the loss of the rounded velocities
    _, _, ucz, Lz = oracle.rk3_program(x, g, s, 0, dt, y, storage=oracle.STORE_F32_EVAL)
    _, _, ucx, _ = oracle.rk3_program(x, g, s, 0, dt, y)
    assert np.array_equal(ucz, f32(ucx))
    assert Lz == pytest.approx(float((f32(ucx)[2] ** 2).sum()), rel=1e-15)
    # a tangent passes the rounding unchanged: the storage models' tangents stay close to the
    # exact program's
    xd, gd = rng.normal(size=x.shape), rng.normal(size=x.shape) * 1e-3
    d0 = oracle.rk3_program_jvp(x, g, s, xd, gd, 3, dt, y)[1]
    d1 = oracle.rk3_program_jvp(x, g, s, xd, gd, 3, dt, y, storage=oracle.STORE_F32_EVAL)[1]
    assert abs(d1 - d0) <= 1e-4 * abs(d0)
