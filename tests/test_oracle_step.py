"""Pins of the closed-step oracle's time loop (Sec. II.B: the particles' positions and
strengths advance with the low-storage third-order Runge-Kutta scheme; Sec. II.A and
Sec. II.C, Eqs. 6-8, for the blade and the wake lines) against things other than the step
itself:

* with the lattice switched off (zero prescribed circulation, no shedding) the step moves a
  co-rotating pair of parallel blobs along its closed-form circle, converging at third order;
* a rotating lattice with prescribed circulations acting on free particles (a right-hand side
  that depends on time through the blade's azimuth) converges at third order under step
  halving, which fixes the stage times of the blade as well as the RK3 coefficients;
* over one interval the wake of a shedding rotor (boundary points, lines, particles) has the
  fourth-order local error of a third-order scheme against the same interval in sub-steps;
* the vortex system the stages see (blade rings, the Kutta row, the lines and the open line
  along the youngest boundary) is closed at every vertex, so its total vorticity is zero, and
  carries no net vorticity along the trailing edge (the Kutta condition) at every azimuth.
"""
import copy
import math

import numpy as np

import oracle
from oracle import uvlm
from paper_2511_11430_amd import workloads as W

ARGS = dict(omega=40.0, v_inf=[0.0, 0.0, -1.0], core_radius=0.02, vatistas_n=2, sigma_p=0.03, n_tip=2,
            n_rows=3)


def _geom():
    return W.blade_rings(n_blades=2, n_chord=2, n_span=4)


def _free_particles(rng, n=6):
    r = rng.uniform(0.3, 0.9, n)
    th = rng.uniform(0, 2 * np.pi, n)
    x = np.array([r * np.cos(th), r * np.sin(th), rng.uniform(-0.15, -0.05, n)])
    return x, rng.normal(0, 1e-3, (3, n)), np.full(n, 0.03)


def test_lattice_off_corotating_pair_third_order():
    d, gz, sig = 0.04, 2e-3, 0.03
    gd, _, _ = oracle.ghk(d, sig)
    rate = 2 * gd * gz  # |u| = g(d) d |Gamma| on a circle of radius d/2
    T = 2.0 / rate
    x0 = np.array([[-d / 2, d / 2], [0.0, 0.0], [0.0, 0.0]])
    g0 = np.array([[0.0, 0.0], [0.0, 0.0], [gz, gz]])
    errs = []
    for nsteps in (8, 16, 32):
        kw = dict(ARGS, v_inf=[0.0, 0.0, 0.0])
        o = uvlm.StepOracle(_geom(), dt=T / nsteps, prescribed_gamma=np.zeros(16), shed=False, **kw)
        o.add_particles(x0, g0, np.full(2, sig))
        for _ in range(nsteps):
            o.step()
        ang = rate * T
        exact = np.array([[-d / 2 * math.cos(ang), d / 2 * math.cos(ang)],
                          [-d / 2 * math.sin(ang), d / 2 * math.sin(ang)], [0.0, 0.0]])
        assert np.array_equal(o.gp, g0)  # parallel blobs do not stretch each other
        assert abs(o.psi - ARGS["omega"] * T) < 1e-12
        errs.append(np.abs(o.xp - exact).max())
    assert 7.0 < errs[0] / errs[1] < 9.0 and 7.0 < errs[1] / errs[2] < 9.0


def test_prescribed_rotating_lattice_third_order():
    rng = np.random.default_rng(3)
    gam = rng.normal(0.5, 0.1, 16)
    xp, gp, sp = _free_particles(rng)
    T = 0.02  # the blade turns 0.8 rad
    res = []
    for nsteps in (4, 8, 16, 32):
        o = uvlm.StepOracle(_geom(), dt=T / nsteps, prescribed_gamma=gam, shed=False, **ARGS)
        o.add_particles(xp, gp, sp)
        for _ in range(nsteps):
            o.step()
        res.append((o.xp.copy(), o.gp.copy()))
    # successive differences shrink by 2^3 per halving (a first-order treatment of the blade's
    # motion, e.g. the blade held at the step's azimuth, would shrink them by 2)
    for q in (0, 1):
        ratios = []
        for i in (1, 2):
            e0 = np.abs(res[i - 1][q] - res[i][q]).max()
            e1 = np.abs(res[i][q] - res[i + 1][q]).max()
            ratios.append(e0 / e1)
        assert 6.5 < ratios[0] < 10.5 and 7.0 < ratios[1] < 9.0, (q, ratios)


def _advance(o, h, m):
    c = copy.deepcopy(o)
    for _ in range(m):
        c.advance(h / m)
    return np.concatenate(c.bounds, 1), c.xp, c.gp


def test_wake_interval_has_fourth_order_local_error():
    rng = np.random.default_rng(3)
    o = uvlm.StepOracle(_geom(), dt=0.005, **ARGS)
    o.add_particles(*_free_particles(rng))
    for _ in range(5):
        o.step()
    assert len(o.rows) == 3 and o.xp.shape[1] > 6  # lines, shed lines and converted particles
    errs = []
    for h in (0.0008, 0.0001):
        one = _advance(o, h, 1)
        ref = _advance(o, h, 8)
        errs.append([np.abs(a - b).max() for a, b in zip(one, ref)])
    # three halvings: a fourth-order local error shrinks 4096x, a third-order one 512x
    for q in range(3):
        assert errs[0][q] / errs[1][q] > 1500.0, (q, errs)


def _node_balance(a, b, g):
    """Net strength leaving every vertex of a set of straight vortex elements."""
    net = {}
    for i in range(g.size):
        ka, kb = tuple(a[:, i]), tuple(b[:, i])
        net[ka] = net.get(ka, 0.0) + g[i]
        net[kb] = net.get(kb, 0.0) - g[i]
    return np.array(list(net.values()))


def test_vortex_system_is_closed_and_the_trailing_edge_free_at_every_stage():
    """Kirchhoff at every vertex (the elements form closed loops: Kelvin) and, the Kutta
    condition, no net vorticity along the trailing edge at any stage's azimuth."""
    o = uvlm.StepOracle(_geom(), dt=0.005, **ARGS)
    ns1 = o.ns + 1
    for k in range(3):  # rows shed, no particle yet (n_rows = 3)
        o.step()
        assert o.xp.shape[1] == 0
        for c in uvlm.RK3_C:
            psi = o.psi + c * o.omega * o.dt
            a, b, g = o.vortex_system(psi)
            scale = np.abs(g).max()
            assert np.abs(_node_balance(a, b, g)).max() <= 1e-14 * scale
            tot = (g * (b - a)).sum(1)
            assert np.abs(tot).max() <= 1e-13 * scale * np.abs(b - a).max(), (k, c, tot)
            _, T = o._geom(psi)
            for bl in range(o.nb):
                for s in range(o.ns):
                    p, q = T[:, bl * ns1 + s], T[:, bl * ns1 + s + 1]
                    fwd = np.all(a == p[:, None], 0) & np.all(b == q[:, None], 0)
                    bwd = np.all(a == q[:, None], 0) & np.all(b == p[:, None], 0)
                    assert fwd.sum() + bwd.sum() >= 2  # the blade's edge and the Kutta row's
                    assert abs(g[fwd].sum() - g[bwd].sum()) <= 1e-15 * scale


def test_stage_nodes_are_the_schemes_butcher_nodes():
    """The stage times follow from the 2N-storage coefficients: c_1 = 0, c_2 = B_1,
    c_3 = B_1 + B_2 (1 + A_2) (the register keeps A_2 of the first stage's slope)."""
    A, B, C = uvlm.RK3_A, uvlm.RK3_B, uvlm.RK3_C
    assert C[0] == 0.0
    assert abs(C[1] - B[0]) < 1e-16
    assert abs(C[2] - (B[0] + B[1] * (1.0 + A[1]))) < 1e-15
