"""Seeded synthetic inputs shaped like the paper's rotor wakes.

This module only draws inputs; it holds none of the method's arithmetic and serves both
the GPU library's callers and the FP64 oracle.  The paper's rotors (Caradonna-Tung
hover, AH-1G forward flight, side-by-side rotors; Sec. IV) and their measured data are
not available, so these sets stand in for them: helical tip vortices that carry most of
the particles, an inboard vortex sheet, a flat vortex-ring lattice on each blade with a
near-wake ring block behind the trailing edge, and blade control points at 3/4-chord
(Sec. II.A).  Everything is in SI units with rotor radius R = 1 m.

Values are drawn in float64.  Callers that run the FP32 path round them once with
:func:`to_f32` and hand the rounded values (promoted back to float64) to the oracle, so
that input rounding is not counted as kernel error.

Particle strengths follow the conversion rule of Eq. 6 with one particle per element:
Gamma_i = (circulation) x (element length) x (unit tangent).
"""
import math

import numpy as np

SEED = 2511_11430
R = 1.0

# Rotor operating point of the hover case (Sec. III, tip Mach 0.439), speed of sound 340.3 m/s.
TIP_MACH = 0.439
SOUND_SPEED = 340.3
OMEGA = TIP_MACH * SOUND_SPEED / R          # rad/s
DPSI_DEG = 5.0                               # azimuth step (Sec. III.D recommendation)
DT = math.radians(DPSI_DEG) / OMEGA          # s


# Viscous term (Sec. II.B): kinematic viscosity of air at sea level (the standard atmosphere
# behind a = 340.3 m/s), Vreman constant C_V = 0.07 as in the paper.
NU_AIR = 1.46e-5                              # m^2/s
C_V = 0.07


def particle_volume(sigma):
    """Particle volumes for the diffusion term: the paper takes sigma as the largest distance
    to the neighbouring particles, so each particle stands for about a cube of side sigma."""
    return np.asarray(sigma, dtype=np.float64) ** 3


def eddy_viscosity_field(n, seed, scale=1e-4):
    """Seeded synthetic per-particle eddy viscosity nu_t ~ U(0, scale) (m^2/s) for diffusion
    checks that must not depend on a computed gradient."""
    return _rng(90, seed).uniform(0.0, scale, n)


def to_f32(a):
    """Round float64 values once to float32 and return them promoted back to float64."""
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def _rng(*key):
    return np.random.default_rng([SEED, *key])


def _helix_tip(n, psi_b, revs, contraction, lam=0.27, pitch=0.05, mu=0.0):
    """Tip-vortex particles evenly spaced in wake age phi in [0, 2 pi revs).

    Radius R (1 - c + c e^{-lam phi}) for contraction c; azimuth psi_b - phi; descent
    pitch*R per revolution; convection mu R phi along +x (forward flight).
    Returns positions (3, n), arc spacing (n,), unit tangent (3, n)."""
    dphi = 2 * math.pi * revs / n
    phi = (np.arange(n) + 0.5) * dphi
    return _helix_points(np.full(n, R), phi, psi_b, dphi, contraction, lam, pitch, mu)


def _helix_points(r0, phi, psi_b, dphi, contraction, lam=0.27, pitch=0.05, mu=0.0):
    rad = r0 * (1.0 - contraction + contraction * np.exp(-lam * phi))
    drad = r0 * (-contraction * lam * np.exp(-lam * phi))
    az = psi_b - phi
    x = np.stack([rad * np.cos(az) + mu * R * phi, rad * np.sin(az), -pitch * R * phi / (2 * math.pi)])
    dx = np.stack([drad * np.cos(az) + rad * np.sin(az) + mu * R,
                   drad * np.sin(az) - rad * np.cos(az),
                   np.full_like(phi, -pitch * R / (2 * math.pi))])
    speed = np.linalg.norm(dx, axis=0)
    return x, speed * dphi, dx / speed


def hover_wake(n, n_blades, sigma, revs, rng, gamma_tip=0.5, sheet_dgamma=0.05, tip_frac=0.7):
    """Contracting helical hover wake (1.0R -> 0.78R, pitch 0.05R/rev): tip_frac of the
    particles on the n_blades tip helices, the rest an inboard sheet (blade radius
    U(0.2R, 0.95R), age U(0, 2 pi revs), circulation jump N(0, sheet_dgamma)), ordered
    by blade then age.  Returns dict(x, gamma, sigma)."""
    contraction = 0.22
    n_tip = int(tip_frac * n) // n_blades
    n_sheet_total = n - n_tip * n_blades
    xs, gs = [], []
    dphi_tip = 2 * math.pi * revs / max(n_tip, 1)
    sheet_counts = [n_sheet_total // n_blades + (1 if b < n_sheet_total % n_blades else 0)
                    for b in range(n_blades)]
    for b in range(n_blades):
        psi_b = 2 * math.pi * b / n_blades
        x, dl, t = _helix_tip(n_tip, psi_b, revs, contraction)
        xs.append(x)
        gs.append(gamma_tip * dl * t)
        m = sheet_counts[b]
        r0 = rng.uniform(0.2 * R, 0.95 * R, m)
        phi = np.sort(rng.uniform(0.0, 2 * math.pi * revs, m))
        dgam = rng.normal(0.0, sheet_dgamma, m)
        x, dl, t = _helix_points(r0, phi, psi_b, dphi_tip, contraction)
        xs.append(x)
        gs.append(dgam * dl * t)
    x = np.concatenate(xs, axis=1)
    g = np.concatenate(gs, axis=1)
    return {"x": np.ascontiguousarray(x), "gamma": np.ascontiguousarray(g),
            "sigma": np.full(x.shape[1], float(sigma))}


def _blade_frames(n_blades, collective_deg):
    th = math.radians(collective_deg)
    frames = []
    for b in range(n_blades):
        psi = 2 * math.pi * b / n_blades
        er = np.array([math.cos(psi), math.sin(psi), 0.0])
        epsi = np.array([-math.sin(psi), math.cos(psi), 0.0])
        chord_dir = -math.cos(th) * epsi - math.sin(th) * np.array([0.0, 0.0, 1.0])  # LE -> TE
        frames.append((psi, er, chord_dir))
    return frames


def lattice(n_blades=2, n_chord=8, n_span=32, chord=R / 6, r_root=0.2 * R, collective_deg=8.0,
            wake_rows=8, dpsi_deg=DPSI_DEG, rng=None):
    """Flat vortex-ring lattice on each blade (rings shifted a quarter panel chord aft,
    Sec. II.A) plus a near-wake ring block of wake_rows rows behind the trailing edge.

    Every ring contributes its 4 edges as separate straight segments with the ring's
    circulation ~ N(0.5, 0.1) m^2/s.  Returns dict(a, b, gamma) with a, b of shape (3, S)."""
    rng = rng if rng is not None else _rng(2, 1)
    cp = chord / n_chord
    rs = np.linspace(r_root, R, n_span + 1)
    A, B, G = [], [], []

    def ring(c00, c01, c11, c10, gam):
        for p, q in ((c00, c01), (c01, c11), (c11, c10), (c10, c00)):
            A.append(p)
            B.append(q)
            G.append(gam)

    for psi, er, cdir in _blade_frames(n_blades, collective_deg):
        te_z = None
        for i in range(n_chord):
            xi0 = i * cp + cp / 4
            xi1 = (i + 1) * cp + cp / 4
            for k in range(n_span):
                gam = rng.normal(0.5, 0.1)
                p = lambda xi, r: r * er + xi * cdir
                ring(p(xi0, rs[k]), p(xi0, rs[k + 1]), p(xi1, rs[k + 1]), p(xi1, rs[k]), gam)
        te_z = (chord + cp / 4) * cdir[2]
        for m in range(wake_rows):
            a0 = psi - math.radians(dpsi_deg) * m
            a1 = psi - math.radians(dpsi_deg) * (m + 1)
            z0 = te_z - 0.05 * R * (math.radians(dpsi_deg) * m) / (2 * math.pi)
            z1 = te_z - 0.05 * R * (math.radians(dpsi_deg) * (m + 1)) / (2 * math.pi)
            for k in range(n_span):
                gam = rng.normal(0.5, 0.1)
                w = lambda az, z, r: np.array([r * math.cos(az), r * math.sin(az), z])
                ring(w(a0, z0, rs[k]), w(a0, z0, rs[k + 1]), w(a1, z1, rs[k + 1]), w(a1, z1, rs[k]), gam)
    a = np.ascontiguousarray(np.array(A).T)
    b = np.ascontiguousarray(np.array(B).T)
    return {"a": a, "b": b, "gamma": np.array(G, dtype=np.float64)}


def blade_rings(n_blades=2, n_chord=8, n_span=32, chord=R / 6, r_root=0.2 * R, collective_deg=8.0):
    """Blade vortex-ring lattice for the Neumann solve (Sec. II.A): rings a quarter panel
    chord aft of the panels, collocation points at the centre of each panel's 3/4-chord line,
    unit normals e_r x e_chord.  Panel p = (blade * n_chord + i) * n_span + k (i chordwise,
    k spanwise).  Returns dict(c00, c01, c11, c10, colloc, normal) of shape (3, n_panels),
    te (the panels of the last chordwise row, blade-major) and the geometry parameters."""
    cp = chord / n_chord
    rs = np.linspace(r_root, R, n_span + 1)
    corners = {k: [] for k in ("c00", "c01", "c11", "c10")}
    colloc, normal, te = [], [], []
    for b, (psi, er, cdir) in enumerate(_blade_frames(n_blades, collective_deg)):
        nrm = np.cross(er, cdir)
        nrm = nrm / np.linalg.norm(nrm)
        for i in range(n_chord):
            xi0 = i * cp + cp / 4
            xi1 = (i + 1) * cp + cp / 4
            for k in range(n_span):
                p = lambda xi, r: r * er + xi * cdir
                corners["c00"].append(p(xi0, rs[k]))
                corners["c01"].append(p(xi0, rs[k + 1]))
                corners["c11"].append(p(xi1, rs[k + 1]))
                corners["c10"].append(p(xi1, rs[k]))
                colloc.append(p(i * cp + 0.75 * cp, 0.5 * (rs[k] + rs[k + 1])))
                normal.append(nrm)
                if i == n_chord - 1:
                    te.append((b * n_chord + i) * n_span + k)
    out = {k: np.ascontiguousarray(np.array(v).T) for k, v in corners.items()}
    out.update({"colloc": np.ascontiguousarray(np.array(colloc).T),
                "normal": np.ascontiguousarray(np.array(normal).T), "te": np.array(te, dtype=np.int64),
                "n_blades": n_blades, "n_chord": n_chord, "n_span": n_span})
    return out


def control_points(n_blades=2, n_chord=8, n_span=32, chord=R / 6, r_root=0.2 * R, collective_deg=8.0,
                   panels=(4,)):
    """Collocation points at the 3/4-chord of the given chordwise panels, strip centres
    (Sec. II.A).  Returns (3, n_blades * len(panels) * n_span)."""
    cp = chord / n_chord
    rs = np.linspace(r_root, R, n_span + 1)
    rc = 0.5 * (rs[:-1] + rs[1:])
    pts = []
    for psi, er, cdir in _blade_frames(n_blades, collective_deg):
        for i in panels:
            xi = i * cp + 0.75 * cp
            for r in rc:
                pts.append(r * er + xi * cdir)
    return np.ascontiguousarray(np.array(pts).T)


# ------------------------------------------------------------------ the five workloads
def config1(n=4096):
    """Uniform cube: x ~ U[-1,1]^3 m, Gamma ~ N(0, 1e-3) m^3/s, sigma = 0.05 m."""
    rng = _rng(1)
    x = rng.uniform(-1.0, 1.0, (3, n))
    g = rng.normal(0.0, 1e-3, (3, n))
    return {"x": x, "gamma": g, "sigma": np.full(n, 0.05), "name": f"uniform cube N_p={n}"}


def config2(n=65536):
    """Hover wake: 2-blade contracting helices (10 revs) + inboard sheet, sigma = 0.02R,
    the 2x8x32 lattice with its near-wake block (4096 segments, r_c = 0.02R, n = 2) and
    64 control points."""
    rng = _rng(2)
    w = hover_wake(n, 2, 0.02 * R, 10, rng)
    lat = lattice(rng=_rng(2, 1))
    w.update({"seg_a": lat["a"], "seg_b": lat["b"], "seg_gamma": lat["gamma"],
              "core_radius": 0.02 * R, "vatistas_n": 2, "ctrl": control_points(panels=(4,)),
              "name": f"hover wake N_p={n} + 2x8x32 lattice"})
    return w


def forward_flight_wake(n, rng, n_blades=4, revs=20, mu=0.15, tip_frac=0.7):
    """Skewed (trochoidal) 4-blade wake, no contraction; sigma log-uniform in
    [0.01R, 0.05R]; |Gamma| log-uniform in [1e-6, 1e-3] m^3/s along the local tangent."""
    n_tip = int(tip_frac * n) // n_blades
    n_sheet_total = n - n_tip * n_blades
    xs, ts = [], []
    dphi = 2 * math.pi * revs / n_tip
    for b in range(n_blades):
        psi_b = 2 * math.pi * b / n_blades
        x, _, t = _helix_tip(n_tip, psi_b, revs, 0.0, mu=mu)
        xs.append(x)
        ts.append(t)
        m = n_sheet_total // n_blades + (1 if b < n_sheet_total % n_blades else 0)
        r0 = rng.uniform(0.2 * R, 0.95 * R, m)
        phi = np.sort(rng.uniform(0.0, 2 * math.pi * revs, m))
        x, _, t = _helix_points(r0, phi, psi_b, dphi, 0.0, mu=mu)
        xs.append(x)
        ts.append(t)
    x = np.concatenate(xs, axis=1)
    t = np.concatenate(ts, axis=1)
    mag = np.exp(rng.uniform(math.log(1e-6), math.log(1e-3), n))
    sig = np.exp(rng.uniform(math.log(0.01 * R), math.log(0.05 * R), n))
    return {"x": np.ascontiguousarray(x), "gamma": np.ascontiguousarray(mag * t), "sigma": sig}


def config3(n=1 << 20, n_sample=4096):
    """Forward-flight skewed wake (advance ratio 0.15, 20 revs, 4 blades) and the seeded
    sample of targets on which it is checked."""
    rng = _rng(3)
    w = forward_flight_wake(n, rng)
    w["sample"] = np.sort(_rng(3, 1).choice(n, size=min(n_sample, n), replace=False)).astype(np.int64)
    # the 4 blades' bound rings (4 x 8 x 32 rings, 4096 segments) and 4 x 32 control points
    lat = lattice(n_blades=4, wake_rows=0, rng=_rng(3, 2))
    w.update({"seg_a": lat["a"], "seg_b": lat["b"], "seg_gamma": lat["gamma"], "core_radius": 0.02 * R,
              "vatistas_n": 2, "ctrl": control_points(n_blades=4, panels=(4,))})
    w["name"] = f"forward-flight skewed wake N_p={n}, 4 blades, mu=0.15"
    return w


def config4(n=262144, n_steps=10):
    """Differentiation workload: hover wake of config 2's law at n particles (4x the
    density at the default n), 10 RK3 steps of dPsi = 5 deg, loss on 128 control points
    (3/4-chord of chordwise panels 2 and 6 of 8, 32 strips, 2 blades)."""
    rng = _rng(4)
    w = hover_wake(n, 2, 0.02 * R, 10, rng)
    w.update({"ctrl": control_points(panels=(1, 5)), "n_steps": n_steps, "dt": DT,
              "name": f"hover wake N_p={n}, {n_steps} RK3 steps"})
    return w


def program_direction(n, k, gamma_scale):
    """Seeded direction (x_dot, gamma_dot) in the space of a program's initial state:
    x_dot ~ N(0, 1e-3) m, gamma_dot ~ N(0, gamma_scale) m^3/s per component."""
    rng = _rng(4, 100 + k)
    return rng.normal(0.0, 1e-3, (3, n)), rng.normal(0.0, gamma_scale, (3, n))


def config5(n_wakes=64, n_min=2048, n_max=200000, scale=1.0):
    """64 independent helical wakes, N_w log-uniform in [n_min, n_max], 2-4 blades,
    sigma_w ~ U(0.01R, 0.05R) per wake.  ``scale`` shrinks every N_w (parity tests)."""
    out = []
    for w in range(n_wakes):
        rng = _rng(5, w)
        nw = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        nw = max(16, int(round(nw * scale)))
        nb = int(rng.integers(2, 5))
        sig = rng.uniform(0.01 * R, 0.05 * R)
        wake = hover_wake(nw, nb, sig, 10, rng)
        wake["n_blades"] = nb
        out.append(wake)
    return out
