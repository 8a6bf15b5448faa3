"""FP64 CPU oracle for the blade solve and the wake management of one NL-UVLM-VPM step
— TEST INFRASTRUCTURE ONLY (only tests/, the smoke check and the benchmark's CPU legs use
it; it shares nothing with the GPU library).

What it computes (Fu & Laurendeau, Sec. II.A and Sec. II.C):

* Blade vortex-ring lattice: ring j has corners (c00, c01, c11, c10) and unit circulation
  on the closed path c00 -> c01 -> c11 -> c10 -> c00; the velocity of each straight edge is
  the Katz-Plotkin segment law with the Vatistas core (``oracle.segments``).  The Neumann
  condition at the collocation point c_i (centre of the panel's 3/4-chord line, normal n_i)
  gives the influence matrix AIC[i, j] = n_i . u_ring_j(c_i) and the system
  AIC Gamma = -(V_rel(c_i) . n_i).
* Kutta condition and shedding: the newest wake row takes the trailing-edge panels'
  circulations, so the trailing-edge line carries nothing.  The wake is kept as straight
  lines with frozen strengths equal to the circulation difference across them (Eq. 7):
      trailed line at span station c (downstream):  Gamma_now(c-1) - Gamma_now(c)
      shed line of strip c (spanwise, outward):       Gamma_prev(c) - Gamma_now(c)
  with Gamma = 0 outside the blade (the "neighbour absent" case of Eq. 7) and Gamma_prev = 0
  before the first step (the starting vortex).
* Conversion of a line a -> b with strength dGamma into n particles (Eq. 6): positions at
  the midpoints of n equal sub-segments, strengths dGamma (b - a) / n.  Trailed lines take
  n = ceil(ds / ds_t * n_t) (Eq. 8), ds the line's length and ds_t the length of its row's
  tip line; shed lines take n = 1 (the conventional count).
"""
import math

import numpy as np

from . import segments as _segments


def ring_edges(c00, c01, c11, c10, gamma=None):
    """The four edges of every ring as segments a -> b (shape (3, 4n)) with the ring's
    circulation (1 when gamma is None), ordered ring by ring."""
    c = [np.asarray(v, dtype=np.float64) for v in (c00, c01, c11, c10)]
    n = c[0].shape[1]
    a = np.empty((3, 4 * n))
    b = np.empty((3, 4 * n))
    for e in range(4):
        a[:, e::4] = c[e]
        b[:, e::4] = c[(e + 1) % 4]
    g = np.repeat(np.ones(n) if gamma is None else np.asarray(gamma, dtype=np.float64), 4)
    return a, b, g


def aic(c00, c01, c11, c10, colloc, normal, core_radius, vatistas_n=2):
    """AIC[i, j] = n_i . (velocity of ring j with unit circulation at collocation point i)."""
    colloc = np.asarray(colloc, dtype=np.float64)
    normal = np.asarray(normal, dtype=np.float64)
    n = colloc.shape[1]
    A = np.empty((n, n))
    a, b, _ = ring_edges(c00, c01, c11, c10)
    for j in range(n):
        u = _segments(a[:, 4 * j:4 * j + 4], b[:, 4 * j:4 * j + 4], np.ones(4), colloc, core_radius, vatistas_n)
        A[:, j] = (u * normal).sum(0)
    return A


def solve(A, rhs):
    """Ring circulations from the Neumann system (a library dense solve)."""
    return np.linalg.solve(np.asarray(A, dtype=np.float64), np.asarray(rhs, dtype=np.float64))


def shed(gamma_te_now, gamma_te_prev):
    """Strengths of the newest wake row's lines (Eq. 7): (trailed, shed) with n_s + 1
    trailed lines and n_s shed lines per blade."""
    g = np.asarray(gamma_te_now, dtype=np.float64)
    gp = np.asarray(gamma_te_prev, dtype=np.float64)
    trailed = np.concatenate(([0.0], g)) - np.concatenate((g, [0.0]))
    return trailed, gp - g


def particle_counts(a, b, tip_index, n_tip):
    """Eq. 8 for every line: ceil(ds / ds_t * n_t) for trailed lines (tip_index >= 0 names
    the row's tip line), 1 for shed lines (tip_index < 0).  A tip line of zero length gives 1.
    Lengths and the quotient are FP64, evaluated as written."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = b - a
    ds = np.sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2])
    n = np.ones(a.shape[1], dtype=np.int64)
    for i, t in enumerate(np.asarray(tip_index)):
        if t < 0:
            continue
        if ds[t] == 0.0:
            n[i] = 1
            continue
        n[i] = int(math.ceil(ds[i] / ds[t] * float(n_tip)))
    return n


def convert(a, b, dgamma, tip_index, n_tip, sigma):
    """Particles from lines (Eqs. 6-8): returns (x (3, m), gamma (3, m), sigma (m,), counts)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    dg = np.asarray(dgamma, dtype=np.float64)
    counts = particle_counts(a, b, tip_index, n_tip)
    xs, gs = [], []
    for i, n in enumerate(counts):
        dl = b[:, i] - a[:, i]
        for k in range(n):
            xs.append(a[:, i] + (k + 0.5) / n * dl)
            gs.append(dg[i] * dl / n)
    m = len(xs)
    x = np.array(xs).T if m else np.zeros((3, 0))
    g = np.array(gs).T if m else np.zeros((3, 0))
    return x, g, np.full(m, float(sigma)), counts
