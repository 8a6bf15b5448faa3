"""Arbitrary-precision brute force for tiny inputs — TEST INFRASTRUCTURE ONLY.

An independent route to the same quantities as ``oracle.cpp``, used to pin it:

* Particle sums go through the vector potential instead of the kernel weights.  The
  Gaussian blob of Eq. 3 (Sec. II.B) has the textbook potential
  ``G_sigma(s) = erf(s / (sqrt(2) sigma)) / (4 pi s)`` (it solves
  ``lap G = -zeta_sigma``), so the field of Eq. 2 has vector potential
  ``psi(x) = sum_j Gamma_j G_sigma_j(|x - x_j|)`` and velocity ``u = curl psi``.
  Gradients and Hessians of ``G`` are taken by mpmath's numerical differentiation at
  high precision; the velocity gradient ``J = grad u`` then gives the stretching of
  Eq. 5, ``J^T Gamma_i`` (transposed scheme) or ``J Gamma_i`` (classical).
* Straight segments go through adaptive quadrature of the Biot-Savart line integral.

Nothing here uses q(rho), the series or the closed-form kernel weights.
"""
import mpmath as mp


def _potential(s, sigma):
    if s == 0:
        return 1 / (4 * mp.pi) * mp.sqrt(2 / mp.pi) / sigma
    return mp.erf(s / (mp.sqrt(2) * sigma)) / (4 * mp.pi * s)


def kernel_weights(s, sigma, dps=40):
    """g(s), h(s) = g'/s, k(s) = h'/s from the potential: the velocity of a unit blob is
    grad G x Gamma = g Gamma x r, hence g = -G'(s)/s."""
    with mp.workdps(dps):
        s, sigma = mp.mpf(s), mp.mpf(sigma)
        G = lambda t: _potential(t, sigma)
        g = lambda t: -mp.diff(G, t) / t
        h = lambda t: mp.diff(g, t) / t
        k = lambda t: mp.diff(h, t) / t
        return float(g(s)), float(h(s)), float(k(s))


def particle_sums(x, gam, sig, scheme=0, sigma_rule=0, dps=30, want_grad=False):
    """Self evaluation (self pair excluded) of u_i and dGamma_i/dt for a tiny set.

    x, gam: sequences of 3-vectors (n of them); sig: n core sizes.  Returns lists of
    3-tuples of floats (u, dgamma), and with want_grad also the velocity gradients
    J[k][l] = du_k/dx_l (3x3 nested tuples) as a third list."""
    n = len(x)
    with mp.workdps(dps):
        X = [[mp.mpf(float(c)) for c in p] for p in x]
        Gm = [[mp.mpf(float(c)) for c in p] for p in gam]
        S = [mp.mpf(float(c)) for c in sig]
        us, ds, js = [], [], []
        for i in range(n):
            grad_sum = [[mp.mpf(0)] * 3 for _ in range(n)]
            u = [mp.mpf(0)] * 3
            J = [[mp.mpf(0)] * 3 for _ in range(3)]
            for j in range(n):
                if j == i:
                    continue
                sj = S[j] if sigma_rule == 0 else mp.sqrt((S[i] ** 2 + S[j] ** 2) / 2)
                xj = X[j]

                def phi(a, b, c, xj=xj, sj=sj):
                    return _potential(mp.sqrt((a - xj[0]) ** 2 + (b - xj[1]) ** 2 + (c - xj[2]) ** 2), sj)

                pt = X[i]
                grad = []
                for l in range(3):
                    o = [0, 0, 0]
                    o[l] = 1
                    grad.append(mp.diff(phi, pt, tuple(o)))
                hess = [[None] * 3 for _ in range(3)]
                for l in range(3):
                    for a in range(l, 3):
                        o = [0, 0, 0]
                        o[l] += 1
                        o[a] += 1
                        hess[l][a] = hess[a][l] = mp.diff(phi, pt, tuple(o))
                Gj = Gm[j]
                # u = grad(phi) x Gamma_j
                u[0] += grad[1] * Gj[2] - grad[2] * Gj[1]
                u[1] += grad[2] * Gj[0] - grad[0] * Gj[2]
                u[2] += grad[0] * Gj[1] - grad[1] * Gj[0]
                # J_kl = d/dx_l of (grad phi x Gamma_j)_k
                for l in range(3):
                    dg = hess[l]
                    J[0][l] += dg[1] * Gj[2] - dg[2] * Gj[1]
                    J[1][l] += dg[2] * Gj[0] - dg[0] * Gj[2]
                    J[2][l] += dg[0] * Gj[1] - dg[1] * Gj[0]
            Gi = Gm[i]
            if scheme == 0:
                d = [sum(J[k][l] * Gi[k] for k in range(3)) for l in range(3)]
            else:
                d = [sum(J[l][k] * Gi[k] for k in range(3)) for l in range(3)]
            us.append(tuple(float(c) for c in u))
            ds.append(tuple(float(c) for c in d))
            js.append(tuple(tuple(float(c) for c in row) for row in J))
        return (us, ds, js) if want_grad else (us, ds)


def segment_velocity_singular(a, b, gam, p, dps=30):
    """Biot-Savart of a straight filament a->b with circulation gam at point p, by
    quadrature of (Gamma/4pi) int dl x (p - l) / |p - l|^3 (no core)."""
    with mp.workdps(dps):
        A = [mp.mpf(float(c)) for c in a]
        B = [mp.mpf(float(c)) for c in b]
        P = [mp.mpf(float(c)) for c in p]
        dl = [B[k] - A[k] for k in range(3)]
        out = []
        for comp in range(3):
            def f(t, comp=comp):
                r = [P[k] - (A[k] + t * dl[k]) for k in range(3)]
                c = [dl[1] * r[2] - dl[2] * r[1], dl[2] * r[0] - dl[0] * r[2], dl[0] * r[1] - dl[1] * r[0]]
                return c[comp] / (r[0] ** 2 + r[1] ** 2 + r[2] ** 2) ** mp.mpf(1.5)
            out.append(float(mp.mpf(gam) / (4 * mp.pi) * mp.quad(f, [0, mp.mpf(1) / 2, 1])))
        return out
