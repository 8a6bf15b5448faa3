"""One time step of the closed blade / wake / particle loop on the GPU (Sec. II.A, the
adaptive conversion of Sec. II.C, the particle right-hand side and the low-storage RK3 time
integration of Sec. II.B).

``Step`` keeps the state in device memory and sequences libvpm calls; it does no arithmetic
of its own beyond gathering and concatenating arrays (the blade's prescribed rotation is
applied to its body-frame geometry on the host, as input kinematics).  The blade lattice
turns at omega about z in the free stream v_inf:

 1. blade geometry at the current azimuth;
 2. influence matrix: the blade's own (assembled once; rotation leaves it unchanged) updated
    with the ring (T_k, T_k+1, B_1,k+1, B_1,k) in the column of trailing-edge panel k once a
    wake exists (Kutta: the wake row at the trailing edge carries that panel's circulation),
    then LU (vpm_aic_update, vpm_lu_factor);
 3. velocity at the collocation points from the particles, the wake lines and the line along
    B_1 that holds the circulation of the last shed row, Neumann right-hand side and solve
    (vpm_eval_velocity_stretching, vpm_eval_segments, vpm_neumann_rhs, vpm_lu_solve);
 4. the trailing-edge points become the youngest boundary; when a wake existed, the row
    between them and B_1 becomes lines (vpm_wake_shed, Eq. 7);
 5. three stages of Williamson's low-storage RK3 move the boundary points and the particles
    (x, Gamma) with vpm_rk3_advect.  Stage k evaluates at t + (0, 1/3, 3/4)[k] dt: the blade
    at that azimuth with the circulations of step 3, the Kutta row from its trailing edge to
    B_1 carrying the trailing-edge circulations, the wake lines with the line along B_1, and
    the particles; velocity at every boundary point and particle, particle stretching by the
    whole field (the particles' share and J^T Gamma with J the gradient of the segments'
    velocity, vpm_eval_segments_gradient);
 6. beyond n_rows line rows, the oldest row and the shed line along the oldest boundary
    become particles (vpm_wake_convert, Eqs. 6-8);
 7. azimuth += omega dt.

Boundaries B_r are (3, n_blades * (n_span + 1)) point sets, station k of blade b at
b * (n_span + 1) + k; trailed lines of the row between B_r and B_r+1 run downstream at every
station, shed lines run outward along a boundary.
"""
import math

import numpy as np
import torch

from . import (vpm_aic_assemble, vpm_aic_update, vpm_eval_segments, vpm_eval_segments_gradient,
               vpm_eval_velocity_stretching, vpm_lu_factor, vpm_lu_solve, vpm_neumann_rhs, vpm_rk3_advect,
               vpm_wake_convert, vpm_wake_shed)

# Butcher nodes of the three-stage low-storage RK3: the times t + C_k dt of its stages.
RK3_C = (0.0, 1.0 / 3.0, 3.0 / 4.0)


def _rot_z(psi):
    c, s = math.cos(psi), math.sin(psi)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


class Step:
    def __init__(self, geom, omega, v_inf, dt, core_radius, vatistas_n, sigma_p, n_tip, n_rows, n_max=64,
                 dtype=torch.float64, capacity=1 << 20, device="cuda", overlap=True):
        self.dev = torch.device(device)
        self.dt_t = dtype
        self.g0 = {k: np.asarray(geom[k], dtype=np.float64) for k in ("c00", "c01", "c11", "c10", "colloc",
                                                                      "normal")}
        self.nb, self.nc, self.ns = int(geom["n_blades"]), int(geom["n_chord"]), int(geom["n_span"])
        self.n_panels = self.g0["colloc"].shape[1]
        self.te = np.asarray(geom["te"], dtype=np.int64)
        self.te_d = torch.tensor(self.te, dtype=torch.int32, device=self.dev)
        self.omega, self.v_inf, self.dt = float(omega), [float(v) for v in v_inf], float(dt)
        self.rc, self.vn, self.sig = float(core_radius), int(vatistas_n), float(sigma_p)
        self.n_tip, self.n_rows, self.n_max = int(n_tip), int(n_rows), int(n_max)
        d64 = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=self.dev)
        self.A0 = vpm_aic_assemble(*(d64(self.g0[k]) for k in ("c00", "c01", "c11", "c10", "colloc", "normal")),
                                   self.rc, self.vn)
        self.A = torch.empty_like(self.A0)
        # column of every trailing-edge panel -> its wake ring (b * n_span + k)
        roc = -np.ones(self.n_panels, dtype=np.int32)
        roc[self.te] = np.arange(self.te.size, dtype=np.int32)
        self.ring_of_col = torch.tensor(roc, device=self.dev)
        self.psi = 0.0
        self.bounds, self.rows, self.sheds = [], [], []
        self.gprev = torch.zeros(self.nb * self.ns, dtype=dtype, device=self.dev)
        self.cap = int(capacity)
        self.xp = torch.zeros((3, self.cap), dtype=dtype, device=self.dev)
        self.gp = torch.zeros_like(self.xp)
        self.sp = torch.zeros(self.cap, dtype=dtype, device=self.dev)
        self.uq = torch.zeros_like(self.xp)
        self.dq = torch.zeros_like(self.xp)
        self.qx = torch.zeros_like(self.xp)  # RK3 registers of the particles
        self.qg = torch.zeros_like(self.xp)
        # two more streams (default priority) for the particle sums, which run beside the blade
        # solve (its LU keeps a few compute units busy at a time)
        # (overlap=False: everything on the caller's stream, in the same order)
        self.side = torch.cuda.Stream(device=self.dev) if overlap else None
        self.side2 = torch.cuda.Stream(device=self.dev) if overlap else None
        self.np = 0
        self.gamma = None
        ns1 = self.ns + 1
        self.tip_row = torch.tensor(np.repeat(np.arange(self.nb) * ns1 + self.ns, ns1).astype(np.int32),
                                    device=self.dev)
        self.tip_shed = torch.full((self.nb * self.ns,), -1, dtype=torch.int32, device=self.dev)
        lo = np.concatenate([np.arange(b * ns1, b * ns1 + self.ns) for b in range(self.nb)])
        self.span_lo = torch.tensor(lo, device=self.dev)
        self.span_hi = self.span_lo + 1

    # ------------------------------------------------------------------ helpers
    def _geometry(self, psi):
        Rm = _rot_z(psi)
        g = {k: Rm @ v for k, v in self.g0.items()}
        ns1 = self.ns + 1
        T = np.empty((3, self.nb * ns1))
        for b in range(self.nb):
            p0 = (b * self.nc + self.nc - 1) * self.ns
            T[:, b * ns1:b * ns1 + self.ns] = g["c10"][:, p0:p0 + self.ns]
            T[:, b * ns1 + self.ns] = g["c11"][:, p0 + self.ns - 1]
        d64 = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=self.dev)
        return {k: d64(v) for k, v in g.items()}, d64(T)

    def _span(self, p):
        """Shed-line end points along a boundary: (a, b) of shape (3, n_blades * n_span)."""
        return p[:, self.span_lo].contiguous(), p[:, self.span_hi].contiguous()

    def lines(self, pending=None):
        """All wake lines (a, b, strength); `pending` adds the line along B_1."""
        A, B, G = [], [], []
        for r, tr in enumerate(self.rows):
            A.append(self.bounds[r])
            B.append(self.bounds[r + 1])
            G.append(tr)
        for r, sh in enumerate(self.sheds):
            if sh is None:
                continue
            a, b = self._span(self.bounds[r])
            A.append(a)
            B.append(b)
            G.append(sh)
        if pending is not None and self.bounds:
            a, b = self._span(self.bounds[0])
            A.append(a)
            B.append(b)
            G.append(pending)
        if not A:
            return None
        return torch.cat(A, 1).contiguous(), torch.cat(B, 1).contiguous(), torch.cat(G).contiguous()

    # ------------------------------------------------------------------ the step
    def vortex_system(self, g, T):
        """Segments (a, b, strength) of every vortex element during the step, with the blade at
        the geometry g (trailing edge T): its rings carrying the step's circulations, the Kutta
        row from T to B_1 carrying the trailing-edge circulations, the wake lines and the line
        along B_1 with Gamma_prev."""
        cat = lambda *c: torch.stack(c, 2).reshape(3, -1).to(self.dt_t)
        segs = [(cat(g["c00"], g["c01"], g["c11"], g["c10"]), cat(g["c01"], g["c11"], g["c10"], g["c00"]),
                 self.gamma.repeat_interleave(4).to(self.dt_t))]
        if self.bounds:
            lo, hi = self.span_lo, self.span_hi
            B1, Tt = self.bounds[0], T.to(self.dt_t)
            k00, k01, k11, k10 = Tt[:, lo], Tt[:, hi], B1[:, hi], B1[:, lo]
            segs.append((cat(k00, k01, k11, k10), cat(k01, k11, k10, k00),
                         self.gamma[self.te_d.long()].repeat_interleave(4).to(self.dt_t)))
            segs.append(self.lines(self.gprev))
        return [torch.cat([sg[i] for sg in segs], -1).contiguous() for i in range(3)]

    def step(self):
        main = torch.cuda.current_stream(self.dev)
        side = self.side or main
        side2 = self.side2 or main
        if self.np:
            # The particles' contributions to the solve and to the first stage depend only on
            # the particles at the start of the step: their self-interaction (the largest part
            # of the step) starts first, on the second stream; their velocities at the
            # collocation and boundary points follow on the third once the points are known.
            # The blade solve runs beside them on the main stream, which joins each result
            # before adding the segments' shares.
            P = (self.xp[:, :self.np], self.gp[:, :self.np], self.sp[:self.np])
            side.wait_stream(main)
            with torch.cuda.stream(side):
                vpm_eval_velocity_stretching(*P, u_out=self.uq[:, :self.np], dgamma_out=self.dq[:, :self.np])
        g, T = self._geometry(self.psi)
        T_t = T.to(self.dt_t)
        col_t = g["colloc"].to(self.dt_t)
        pts = torch.cat([T_t] + self.bounds, 1).contiguous()  # boundary points: the new line first
        u = torch.zeros((3, col_t.shape[1]), dtype=self.dt_t, device=self.dev)
        up = torch.zeros((3, pts.shape[1]), dtype=self.dt_t, device=self.dev)
        if self.np:
            side2.wait_stream(main)
            with torch.cuda.stream(side2):
                vpm_eval_velocity_stretching(*P, col_t, u_out=u)
                ev_col = side2.record_event()
                vpm_eval_velocity_stretching(*P, pts, u_out=up)
                ev_pts = side2.record_event()
        if self.bounds:
            B1 = self.bounds[0].to(torch.float64)
            lo, hi = self.span_lo, self.span_hi
            r00, r01 = T[:, lo].contiguous(), T[:, hi].contiguous()
            r11, r10 = B1[:, hi].contiguous(), B1[:, lo].contiguous()
            vpm_aic_update(self.A0, g["colloc"], g["normal"], r00, r01, r11, r10, self.ring_of_col, self.rc,
                           self.vn, out=self.A)
        else:
            self.A.copy_(self.A0)
        ipiv, _ = vpm_lu_factor(self.A)
        wl = self.lines(self.gprev)
        if self.np:
            main.wait_event(ev_col)
        if wl is not None:
            vpm_eval_segments(wl[0], wl[1], wl[2], col_t, self.rc, self.vn, u_out=u, accumulate=True)
        rhs = vpm_neumann_rhs(g["colloc"], g["normal"], u, self.v_inf, (0.0, 0.0, self.omega))
        gam = vpm_lu_solve(self.A, ipiv, rhs)
        self.gamma = gam
        had_wake = bool(self.bounds)
        self.bounds.insert(0, T_t.clone())
        self.sheds.insert(0, None)
        if had_wake:
            tr, sh = vpm_wake_shed(gam.to(self.dt_t), self.te_d, self.gprev, self.nb, self.ns)
            self.rows.insert(0, tr)
            self.sheds[1] = sh
        # three RK3 stages for the boundary points and the particles
        nbp = T.shape[1]
        qp = torch.zeros_like(pts)
        xq, gq = self.xp[:, :self.np], self.gp[:, :self.np]
        uq, dq = self.uq[:, :self.np], self.dq[:, :self.np]
        qx, qg = self.qx[:, :self.np], self.qg[:, :self.np]
        for k in range(3):
            if k:
                g, T = self._geometry(self.psi + RK3_C[k] * self.omega * self.dt)
                up = torch.zeros_like(pts)
                if self.np:
                    P = (xq, gq, self.sp[:self.np])
                    side.wait_stream(main)
                    with torch.cuda.stream(side):
                        vpm_eval_velocity_stretching(*P, u_out=uq, dgamma_out=dq)
                    side2.wait_stream(main)
                    with torch.cuda.stream(side2):
                        vpm_eval_velocity_stretching(*P, pts, u_out=up)
                        ev_pts = side2.record_event()
            segs = self.vortex_system(g, T)
            if self.np:
                main.wait_event(ev_pts)
            vpm_eval_segments(segs[0], segs[1], segs[2], pts, self.rc, self.vn, u_out=up, accumulate=True)
            if self.np:
                main.wait_stream(side)
                vpm_eval_segments_gradient(segs[0], segs[1], segs[2], xq, self.rc, self.vn, gamma_tgt=gq,
                                           want_grad=False, u_out=uq, dgamma_out=dq, accumulate=True)
                vpm_rk3_advect(k, xq, qx, uq, self.dt, self.v_inf, gamma=gq, qg=qg, dgamma=dq)
            vpm_rk3_advect(k, pts, qp, up, self.dt, self.v_inf)
            self.bounds = [pts[:, i * nbp:(i + 1) * nbp] for i in range(len(self.bounds))]
        self.bounds = [b.contiguous() for b in self.bounds]
        if len(self.rows) > self.n_rows:
            r = len(self.rows) - 1
            sa, sb = self._span(self.bounds[r + 1])
            a = torch.cat([self.bounds[r], sa], 1).contiguous()
            b = torch.cat([self.bounds[r + 1], sb], 1).contiguous()
            dg = torch.cat([self.rows[r], self.sheds[r + 1]]).contiguous()
            tip = torch.cat([self.tip_row, self.tip_shed + 0]).contiguous()
            room = self.cap - self.np
            x, gg, s, cnt = vpm_wake_convert(a, b, dg, tip, self.n_tip, self.sig, room, n_max=self.n_max,
                                             x_out=self.xp[:, self.np:], gamma_out=self.gp[:, self.np:],
                                             sigma_out=self.sp[self.np:])
            m = int(cnt.item())
            if m > room:
                raise RuntimeError(f"particle capacity {self.cap} exceeded")
            self.np += m
            del self.rows[r]
            del self.bounds[r + 1]
            del self.sheds[r + 1]
        self.psi += self.omega * self.dt
        return gam

    def particles(self):
        return self.xp[:, :self.np], self.gp[:, :self.np], self.sp[:self.np]

    def add_particles(self, x, g, s):
        """Append particles (x, gamma of shape (3, m), sigma (m,)), e.g. an existing wake."""
        m = x.shape[1]
        if self.np + m > self.cap:
            raise RuntimeError(f"particle capacity {self.cap} exceeded")
        self.xp[:, self.np:self.np + m].copy_(x)
        self.gp[:, self.np:self.np + m].copy_(g)
        self.sp[self.np:self.np + m].copy_(s)
        self.np += m
