"""Pins of the oracle's velocity gradient, Vreman eddy viscosity and PSE diffusion
(Sec. II.B: the viscous term of Eq. 5 by particle strength exchange, Vreman's sub-grid
model with C_V = 0.07) against things other than the oracle itself: arbitrary-precision
derivatives of the blob potential, finite differences, divergence-free velocity, the
singular-value form of Vreman's invariant and closed-form flows, and the closed-form
Gaussian convolution that the PSE sum approximates on a lattice."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import brute_mp

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def _cloud(n, seed, spread=0.08, sig=0.05):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(3, n)) * spread
    g = rng.normal(size=(3, n)) * 1e-3
    s = sig * (1.0 + 0.5 * rng.random(n))
    return x, g, s


# ------------------------------------------------------------------ velocity gradient

@pytest.mark.parametrize("rule", [O.SIGMA_SOURCE, O.SIGMA_SYMMETRIC])
def test_gradient_matches_potential_derivatives(rule):
    """J from the second derivatives of the blob's vector potential at 30 digits."""
    x, g, s = _cloud(6, 1)
    J = O.velocity_gradient(x, g, s, sigma_rule=rule)
    _, _, jb = brute_mp.particle_sums(x.T, g.T, s, sigma_rule=rule, want_grad=True)
    Jb = np.array(jb).transpose(1, 2, 0)
    assert np.abs(J - Jb).max() <= 1e-13 * np.abs(Jb).max()


def test_gradient_matches_central_differences():
    """du_a/dx_b by central differences of the oracle velocity at targets off the sources."""
    x, g, s = _cloud(40, 2)
    rng = np.random.default_rng(3)
    y = rng.normal(size=(3, 12)) * 0.08
    J = O.velocity_gradient(x, g, s, x_tgt=y)
    h = 1e-6
    Jfd = np.zeros_like(J)
    for b in range(3):
        yp, ym = y.copy(), y.copy()
        yp[b] += h
        ym[b] -= h
        up, _ = O.eval_pairs(x, g, s, yp)
        um, _ = O.eval_pairs(x, g, s, ym)
        Jfd[:, b, :] = (up - um) / (2 * h)
    assert np.abs(J - Jfd).max() <= 1e-7 * np.abs(J).max()


def test_gradient_trace_is_zero():
    """The Biot-Savart velocity is divergence free: tr J = 0 at every target."""
    x, g, s = _cloud(200, 4)
    J = O.velocity_gradient(x, g, s)
    tr = np.einsum("aat->t", J)
    assert np.abs(tr).max() <= 1e-14 * np.abs(J).max()


def test_gradient_gives_both_stretching_schemes():
    """Eq. 5's stretching is J^T Gamma_i (transposed) or J Gamma_i (classical)."""
    x, g, s = _cloud(100, 5)
    J = O.velocity_gradient(x, g, s)
    _, dt = O.eval_pairs(x, g, s, scheme=O.TRANSPOSED)
    _, dc = O.eval_pairs(x, g, s, scheme=O.CLASSICAL)
    assert np.abs(np.einsum("bat,bt->at", J, g) - dt).max() <= 1e-14 * np.abs(dt).max()
    assert np.abs(np.einsum("abt,bt->at", J, g) - dc).max() <= 1e-14 * np.abs(dc).max()


# ------------------------------------------------------------------ Vreman

def _svd_vreman(J, delta, cv):
    """Vreman's invariant through the singular values of J: B_beta = delta^4 e2(s^2),
    alpha:alpha = sum s^2 (B_beta is the second invariant of delta^2 J J^T)."""
    sv = np.linalg.svd(J, compute_uv=False) ** 2
    aa = sv.sum()
    if aa == 0.0:
        return 0.0
    B = delta ** 4 * (sv[0] * sv[1] + sv[0] * sv[2] + sv[1] * sv[2])
    return cv * math.sqrt(B / aa)


def test_vreman_matches_singular_value_form():
    rng = np.random.default_rng(6)
    n = 64
    J = rng.normal(size=(3, 3, n)) * 10.0 ** rng.uniform(-3, 3, size=n)
    sig = 10.0 ** rng.uniform(-3, -1, size=n)
    nut = O.vreman(J, sig, 0.07)
    ref = np.array([_svd_vreman(J[:, :, i], sig[i], 0.07) for i in range(n)])
    assert np.abs(nut - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.all(np.abs(nut - ref) <= 1e-12 * ref + 1e-300)


def test_vreman_closed_form_flows():
    d, cv = 0.02, 0.07
    # pure shear u = (y, 0, 0): the model vanishes
    J = np.zeros((3, 3, 1))
    J[0, 1, 0] = 3.0
    assert O.vreman(J, [d], cv)[0] == 0.0
    # zero gradient
    assert O.vreman(np.zeros((3, 3, 1)), [d], cv)[0] == 0.0
    # solid-body rotation about z at rate W: nu_t = C d^2 W / sqrt 2
    W = 5.0
    J = np.zeros((3, 3, 1))
    J[0, 1, 0], J[1, 0, 0] = -W, W
    assert O.vreman(J, [d], cv)[0] == pytest.approx(cv * d * d * W / math.sqrt(2), rel=1e-14)
    # axisymmetric strain diag(-a/2, -a/2, a): nu_t = C d^2 a sqrt(3/8)
    a = 2.0
    J = np.zeros((3, 3, 1))
    J[0, 0, 0], J[1, 1, 0], J[2, 2, 0] = -a / 2, -a / 2, a
    assert O.vreman(J, [d], cv)[0] == pytest.approx(cv * d * d * a * math.sqrt(3 / 8), rel=1e-14)


def test_vreman_rotation_invariant_and_scaling():
    rng = np.random.default_rng(7)
    J = rng.normal(size=(3, 3))
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    a = O.vreman(J[:, :, None], [0.03], 0.07)[0]
    b = O.vreman((q @ J @ q.T)[:, :, None], [0.03], 0.07)[0]
    c = O.vreman((2.0 * J)[:, :, None], [0.06], 0.07)[0]
    assert b == pytest.approx(a, rel=1e-13)
    assert c == pytest.approx(8.0 * a, rel=1e-13)  # nu_t ~ delta^2 |J|


# ------------------------------------------------------------------ PSE

def _lattice(M, h):
    k = np.arange(-M, M + 1) * h
    X, Y, Z = np.meshgrid(k, k, k, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()])


def test_pse_matches_gaussian_convolution_on_a_lattice():
    """For a Gaussian vorticity field sampled on a lattice (Gamma_i = omega(x_i) h^3,
    V_i = h^3) the PSE sum is (2 nu / sigma^2) [(zeta_sigma * omega)(x_i) - omega(x_i)] up
    to the lattice quadrature error, which is spectrally small for h < sigma; the
    convolution of two Gaussians is a Gaussian in closed form."""
    h, sig, L, nu, w0 = 1.0, 1.5, 2.0, 1.5e-5, 0.7
    x = _lattice(14, h)
    n = x.shape[1]
    r2 = (x ** 2).sum(0)
    om = w0 * np.exp(-r2 / (2 * L * L))
    gam = np.zeros((3, n))
    gam[2] = om * h ** 3
    dg = O.pse(x, gam, np.full(n, sig), np.full(n, h ** 3), nu)
    conv = w0 * (L * L / (L * L + sig * sig)) ** 1.5 * np.exp(-r2 / (2 * (L * L + sig * sig)))
    ref = 2 * nu / sig ** 2 * (conv - om) * h ** 3
    inner = r2 <= (2 * L) ** 2
    assert np.abs(dg[2, inner] - ref[inner]).max() <= 1e-9 * np.abs(ref[inner]).max()
    assert np.abs(dg[:2]).max() == 0.0
    # ... and that limit approaches nu lap(omega) as sigma/L -> 0 (second order)
    errs = []
    for s_ in (0.4, 0.2):
        c = w0 * (L * L / (L * L + s_ * s_)) ** 1.5 * np.exp(-r2[inner] / (2 * (L * L + s_ * s_)))
        lim = 2 * nu / s_ ** 2 * (c - om[inner])
        lap = nu * om[inner] * (r2[inner] / L ** 4 - 3 / L ** 2)
        errs.append(np.abs(lim - lap).max() / np.abs(lap).max())
    assert 3.5 < errs[0] / errs[1] < 4.5


def test_pse_conserves_total_strength():
    """The exchange is antisymmetric in (i, j), so sum_i dGamma_i/dt = 0 for any
    volumes, core sizes and eddy viscosities."""
    x, g, s = _cloud(300, 8, spread=0.05)
    rng = np.random.default_rng(9)
    vol = s ** 3 * (0.5 + rng.random(300))
    nut = 1e-4 * rng.random(300)
    dg = O.pse(x, g, s, vol, 1.5e-5, nut)
    scale = np.abs(dg).sum()
    assert np.abs(dg.sum(1)).max() <= 1e-15 * scale


def test_pse_eddy_viscosity_enters_as_pair_average():
    x, g, s = _cloud(80, 10, spread=0.05)
    vol = s ** 3
    c = 3e-5
    a = O.pse(x, g, s, vol, 1.5e-5, np.full(80, c))
    b = O.pse(x, g, s, vol, 1.5e-5 + c)
    assert np.abs(a - b).max() <= 1e-14 * np.abs(b).max()
    # two particles with different nu_t: the pair uses nu + (nu_t1 + nu_t2)/2
    x2, g2, s2 = x[:, :2], g[:, :2], s[:2]
    a2 = O.pse(x2, g2, s2, vol[:2], 1e-5, np.array([2e-5, 6e-5]))
    b2 = O.pse(x2, g2, s2, vol[:2], 1e-5 + 4e-5)
    assert np.abs(a2 - b2).max() <= 1e-15 * np.abs(b2).max()
    assert np.abs(a2[:, 0] + a2[:, 1]).max() <= 1e-18


def test_pse_uniform_field_is_still():
    """Equal omega = Gamma/V everywhere: nothing diffuses."""
    x, _, s = _cloud(50, 11)
    vol = s ** 3
    g = np.outer([0.3, -0.2, 0.5], vol)
    dg = O.pse(x, g, s, vol, 1e-3)
    assert np.abs(dg).max() <= 1e-15 * np.abs(g).max() * 1e-3 / s.min() ** 2


def test_pse_at_listed_targets_matches_full():
    x, g, s = _cloud(120, 12, spread=0.05)
    vol = s ** 3
    idx = np.array([0, 7, 119, 7])
    full = O.pse(x, g, s, vol, 1e-5)
    part = O.pse(x, g, s, vol, 1e-5, targets=idx)
    assert np.array_equal(part, full[:, idx])
