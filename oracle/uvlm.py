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
from . import segments_gradient as _segments_gradient


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


def te_points(c10, c11, n_blades, n_chord, n_span):
    """Trailing-edge stations of every blade, (3, n_blades * (n_span + 1)): the downstream
    corners of the last chordwise row of rings, station k of blade b at b * (n_span + 1) + k."""
    out = np.empty((3, n_blades * (n_span + 1)))
    for b in range(n_blades):
        p0 = (b * n_chord + n_chord - 1) * n_span
        out[:, b * (n_span + 1):b * (n_span + 1) + n_span] = c10[:, p0:p0 + n_span]
        out[:, b * (n_span + 1) + n_span] = c11[:, p0 + n_span - 1]
    return out


def rot_z(psi):
    c, s = math.cos(psi), math.sin(psi)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


# Williamson's low-storage third-order Runge-Kutta scheme (Sec. II.B), in its 2N-storage
# form: per stage k, register Q <- A_k Q + dt F(Y, t + C_k dt) and state Y <- Y + B_k Q.
# C holds the nodes of the same scheme's Butcher form (the times at which stage k evaluates).
RK3_A = (0.0, -5.0 / 9.0, -153.0 / 128.0)
RK3_B = (1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0)
RK3_C = (0.0, 1.0 / 3.0, 3.0 / 4.0)


class StepOracle:
    """One time step of the closed blade/wake/particle loop, FP64 on the CPU.

    Blade: the ring lattice `geom` (body frame at azimuth 0) turning at omega about z in the
    free stream v_inf.  Wake: boundaries B_1 (youngest free row of points) ... B_m; trailed
    lines of the row between B_r and B_r+1; shed lines along B_r; particles.

    step():
     1. blade geometry at the current azimuth (rotation about z);
     2. influence matrix: the blade's (rotation invariant) plus, once a wake exists, the ring
        (T_k, T_k+1, B_1,k+1, B_1,k) in the column of trailing-edge panel k (Kutta: the wake
        row at the trailing edge carries that panel's circulation);
     3. velocity at the collocation points from the particles, the wake lines and the line
        along B_1 holding the circulation of the last shed row (still open), Neumann
        right-hand side, dense solve for the ring circulations (or the prescribed ones);
     4. the trailing-edge points become the youngest boundary; when a wake existed, the row
        between them and B_1 becomes lines (Eq. 7), the line along B_1 closes with
        Gamma_prev - Gamma_now, and Gamma_prev <- Gamma_now (before the first shed row
        Gamma_prev = 0: the starting vortex);
     5. advance(dt): the boundary points and the particles (x, Gamma) move through the three
        stages of the low-storage RK3 (Sec. II.B); the circulations of step 3 and the line
        strengths stay fixed over the step, the blade follows its prescribed rotation;
     6. when more than n_rows line rows exist, the oldest row's trailed lines and the shed line
        along the oldest boundary become particles (Eqs. 6-8, tip line = station n_span of the
        same blade and row; shed lines one particle each).

    prescribed_gamma: ring circulations used instead of the solve (steps 2-3 skipped);
    shed=False: the blade leaves no wake (steps 4 and 6 skipped), it only acts on particles.
    """

    def __init__(self, geom, omega, v_inf, dt, core_radius, vatistas_n, sigma_p, n_tip, n_rows, n_max=64,
                 prescribed_gamma=None, shed=True):
        self.g = {k: np.asarray(geom[k], dtype=np.float64) for k in ("c00", "c01", "c11", "c10", "colloc", "normal")}
        self.nb, self.nc, self.ns = geom["n_blades"], geom["n_chord"], geom["n_span"]
        self.te = np.asarray(geom["te"])
        self.omega, self.v_inf, self.dt = float(omega), np.asarray(v_inf, dtype=np.float64), float(dt)
        self.rc, self.vn, self.sig, self.n_tip, self.n_rows, self.n_max = (float(core_radius), int(vatistas_n),
                                                                           float(sigma_p), int(n_tip),
                                                                           int(n_rows), int(n_max))
        self.fixed = None if prescribed_gamma is None else np.asarray(prescribed_gamma, dtype=np.float64).copy()
        self.shed = bool(shed)
        self.A0 = None
        if self.fixed is None:
            self.A0 = aic(self.g["c00"], self.g["c01"], self.g["c11"], self.g["c10"], self.g["colloc"],
                          self.g["normal"], self.rc, self.vn)
        self.psi = 0.0
        self.bounds, self.rows, self.sheds = [], [], []  # sheds[r] along bounds[r] (None: not yet)
        self.gprev = np.zeros(self.nb * self.ns)
        self.xp, self.gp = np.zeros((3, 0)), np.zeros((3, 0))
        self.sp = np.zeros(0)
        self.gamma = None

    def _geom(self, psi=None):
        Rm = rot_z(self.psi if psi is None else psi)
        rg = {k: Rm @ v for k, v in self.g.items()}
        T = te_points(rg["c10"], rg["c11"], self.nb, self.nc, self.ns)
        return rg, T

    def add_particles(self, x, g, s):
        self.xp = np.concatenate([self.xp, np.asarray(x, dtype=np.float64)], 1)
        self.gp = np.concatenate([self.gp, np.asarray(g, dtype=np.float64)], 1)
        self.sp = np.concatenate([self.sp, np.asarray(s, dtype=np.float64)])

    def lines(self, pending=None):
        """All wake lines as (a, b, strength); `pending` adds the line along B_1."""
        A, B, G = [], [], []
        ns1 = self.ns + 1
        for r, tr in enumerate(self.rows):
            A.append(self.bounds[r])
            B.append(self.bounds[r + 1])
            G.append(tr)
        for r, sh in enumerate(self.sheds):
            if sh is None:
                continue
            p = self.bounds[r]
            for bl in range(self.nb):
                A.append(p[:, bl * ns1:bl * ns1 + self.ns])
                B.append(p[:, bl * ns1 + 1:bl * ns1 + ns1])
            G.append(sh)
        if pending is not None and self.bounds:
            p = self.bounds[0]
            for bl in range(self.nb):
                A.append(p[:, bl * ns1:bl * ns1 + self.ns])
                B.append(p[:, bl * ns1 + 1:bl * ns1 + ns1])
            G.append(pending)
        if not A:
            return np.zeros((3, 0)), np.zeros((3, 0)), np.zeros(0)
        return np.concatenate(A, 1), np.concatenate(B, 1), np.concatenate(G)

    def _induced(self, y, with_pending):
        u = np.zeros_like(y)
        if self.xp.shape[1]:
            u += _eval_pairs(self.xp, self.gp, self.sp, x_tgt=y)[0]
        a, b, g = self.lines(self.gprev if with_pending else None)
        if a.shape[1]:
            u += _segments(a, b, g, y, self.rc, self.vn)
        return u

    def _kutta_rings(self, T, gam):
        """The wake row between the trailing edge T and the youngest boundary B_1, one ring per
        trailing-edge panel carrying that panel's circulation: (T_k, T_k+1, B_1,k+1, B_1,k)."""
        ns1 = self.ns + 1
        B1 = self.bounds[0]
        cs = [[], [], [], []]
        for bl in range(self.nb):
            lo = np.arange(bl * ns1, bl * ns1 + self.ns)
            cs[0].append(T[:, lo])
            cs[1].append(T[:, lo + 1])
            cs[2].append(B1[:, lo + 1])
            cs[3].append(B1[:, lo])
        return ring_edges(*(np.concatenate(c, 1) for c in cs), gam[self.te])

    def vortex_system(self, psi):
        """Every straight vortex element at azimuth psi during a step, as (a, b, strength): the
        blade rings with the circulations of the step, the Kutta row from the trailing edge to
        B_1, the wake lines and the line along B_1 with Gamma_prev.  The Kutta row's front edges
        cancel the blade's trailing-edge edges and its back edges cancel the line along B_1
        (once a row has been shed), so the trailing edge carries no vorticity and the lines
        stay attached to it while the blade turns."""
        rg, T = self._geom(psi)
        parts = [ring_edges(rg["c00"], rg["c01"], rg["c11"], rg["c10"], self.gamma)]
        if self.bounds:
            parts.append(self._kutta_rings(T, self.gamma))
            parts.append(self.lines(self.gprev))
        return tuple(np.concatenate([p[i] for p in parts], -1) for i in range(3))

    def _rhs(self, psi):
        """Velocity at every boundary point, velocity and stretching rate of every particle."""
        a, b, g = self.vortex_system(psi)
        pts = np.concatenate(self.bounds, 1) if self.bounds else np.zeros((3, 0))
        up = _segments(a, b, g, pts, self.rc, self.vn) if pts.shape[1] else np.zeros((3, 0))
        uq, dq = np.zeros((3, 0)), np.zeros((3, 0))
        if self.xp.shape[1]:
            if pts.shape[1]:
                up += _eval_pairs(self.xp, self.gp, self.sp, x_tgt=pts)[0]
            uq, dq = _eval_pairs(self.xp, self.gp, self.sp)
            uq += _segments(a, b, g, self.xp, self.rc, self.vn)
            # stretching by the rings' and lines' share of the velocity gradient (transposed)
            J = _segments_gradient(a, b, g, self.xp, self.rc, self.vn)
            dq += np.einsum("abn,an->bn", J, self.gp)
        return up, uq, dq

    def advance(self, h):
        """Move the boundary points and the particles over the interval h (three RK3 stages,
        the blade at its azimuth at each stage's time) and turn the blade by omega h."""
        nbp = self.nb * (self.ns + 1)
        qp = np.zeros((3, nbp * len(self.bounds)))
        qx, qg = np.zeros_like(self.xp), np.zeros_like(self.gp)
        vinf = self.v_inf[:, None]
        for k in range(3):
            up, uq, dq = self._rhs(self.psi + RK3_C[k] * self.omega * h)
            if self.bounds:
                qp = RK3_A[k] * qp + h * (up + vinf)
                pts = np.concatenate(self.bounds, 1) + RK3_B[k] * qp
                self.bounds = [pts[:, i * nbp:(i + 1) * nbp] for i in range(len(self.bounds))]
            if self.xp.shape[1]:
                qx = RK3_A[k] * qx + h * (uq + vinf)
                qg = RK3_A[k] * qg + h * dq
                self.xp = self.xp + RK3_B[k] * qx
                self.gp = self.gp + RK3_B[k] * qg
        self.psi += self.omega * h

    def step(self):
        rg, T = self._geom()
        ns1 = self.ns + 1
        if self.fixed is None:
            A = self.A0.copy()
            if self.bounds:
                B1 = self.bounds[0]
                for bl in range(self.nb):
                    for k in range(self.ns):
                        i0, i1 = bl * ns1 + k, bl * ns1 + k + 1
                        cs = [T[:, i0:i0 + 1], T[:, i1:i1 + 1], B1[:, i1:i1 + 1], B1[:, i0:i0 + 1]]
                        a, b, _ = ring_edges(*cs)
                        u = _segments(a, b, np.ones(4), rg["colloc"], self.rc, self.vn)
                        A[:, self.te[bl * self.ns + k]] += (u * rg["normal"]).sum(0)
            u = self._induced(rg["colloc"], with_pending=True)
            w = np.array([0.0, 0.0, self.omega])
            vrel = self.v_inf[:, None] - np.cross(w, rg["colloc"].T).T + u
            gam = solve(A, -(vrel * rg["normal"]).sum(0))
        else:
            gam = self.fixed.copy()
        self.gamma = gam
        if self.shed:
            # the trailing-edge points join the wake as its youngest boundary
            had_wake = bool(self.bounds)
            self.bounds.insert(0, T.copy())
            self.sheds.insert(0, None)
            if had_wake:
                trs, shs = [], []
                for bl in range(self.nb):
                    gte = gam[self.te[bl * self.ns:(bl + 1) * self.ns]]
                    tr, sh = shed(gte, self.gprev[bl * self.ns:(bl + 1) * self.ns])
                    trs.append(tr)
                    shs.append(sh)
                self.rows.insert(0, np.concatenate(trs))  # between the trailing edge and B_1
                self.sheds[1] = np.concatenate(shs)      # along B_1
                self.gprev = gam[self.te].copy()
        self.advance(self.dt)
        # conversion of the oldest row
        if self.shed and len(self.rows) > self.n_rows:
            r = len(self.rows) - 1
            a = [self.bounds[r]]
            b = [self.bounds[r + 1]]
            tip = [np.repeat(np.arange(self.nb) * ns1 + self.ns, ns1)]
            dg = [self.rows[r]]
            p = self.bounds[r + 1]
            for bl in range(self.nb):
                a.append(p[:, bl * ns1:bl * ns1 + self.ns])
                b.append(p[:, bl * ns1 + 1:bl * ns1 + ns1])
            dg.append(self.sheds[r + 1])
            tip.append(-np.ones(self.nb * self.ns, dtype=np.int64))
            x, g, s, _ = convert(np.concatenate(a, 1), np.concatenate(b, 1), np.concatenate(dg), np.concatenate(tip),
                                 self.n_tip, self.sig)
            self.add_particles(x, g, s)
            del self.rows[r]
            del self.bounds[r + 1]
            del self.sheds[r + 1]
        return gam

    def total_vorticity(self):
        """sum over lines of strength x (b - a), plus the particles, plus the line along B_1 that
        the next shed row closes (Gamma_prev): zero for a closed system of rings."""
        a, b, g = self.lines(self.gprev)
        return (g * (b - a)).sum(1) + self.gp.sum(1)


def _eval_pairs(*args, **kw):
    from . import eval_pairs
    return eval_pairs(*args, **kw)
