"""Coefficients of the FP32 in-core weights in device_math.h (run by hand; prints C++).

For 1 <= rho <= 7 the FP32 kernels write q(rho) = erf(rho/sqrt2) - c0 rho exp(-rho^2/2) as
    q = 1 - E (F + c0 rho),   E = exp(-rho^2/2),   F = erfcx(rho/sqrt2) = exp(rho^2/2) erfc(rho/sqrt2),
which needs one exponential (shared with the gradient weight) instead of erf and exp.  F is
smooth and bounded there; it is fitted as a polynomial in w = 1/(1 + p rho), the variable of
Hastings' rational approximations of erfc (Abramowitz & Stegun 7.1.26), with p and the degree
chosen here and the coefficients from a Lawson-weighted least-squares (minimax) fit of the
relative error of F.  p is fixed to an FP32 value first, and the error is reported for the
coefficients rounded to FP32 as the kernels hold them.

    python paper_2511_11430_amd/csrc/gen_core_fit.py
"""
import numpy as np
from scipy.special import erfcx

RHO_LO, RHO_HI = 1.0, 7.0   # the FP32 closed-form range (series below 1, point vortex beyond 7)
DEGREE = 7


def lawson(p, d, rho, f, iters=400):
    w = 1.0 / (1.0 + p * rho)
    V = np.vander(w, d + 1, increasing=True) / f[:, None]   # relative-error rows
    wt = np.ones_like(w)
    best = (None, np.inf)
    for _ in range(iters):
        c, *_ = np.linalg.lstsq(V * wt[:, None], wt, rcond=None)
        err = V @ c - 1.0
        m = np.abs(err).max()
        if m < best[1]:
            best = (c, m)
        wt = wt * np.sqrt(np.abs(err)) + 1e-300
        wt /= wt.mean()
    return best


def main():
    rho = np.linspace(RHO_LO, RHO_HI, 30001)
    f = erfcx(rho / np.sqrt(2.0))
    scan = [(lawson(float(np.float32(p)), DEGREE, rho, f, 150)[1], float(np.float32(p)))
            for p in np.linspace(0.2, 0.5, 31)]
    _, p = min(scan)
    c, _ = lawson(p, DEGREE, rho, f)
    c32 = np.array([np.float32(v) for v in c], dtype=np.float64)
    w = 1.0 / (1.0 + p * rho)
    err = np.abs(np.polyval(c32[::-1], w) / f - 1.0).max()
    print(f"// p = {str(np.float32(p))}, degree {DEGREE}: max relative error of F on [{RHO_LO}, {RHO_HI}] "
          f"{err:.2e} (FP64 evaluation of the FP32 coefficients)")
    print(f"constexpr float kErfcxP = {str(np.float32(p))}f;")
    print("constexpr float kErfcxC[%d] = {%s};" % (DEGREE + 1, ", ".join(f"{str(np.float32(v))}f" for v in c32)))


if __name__ == "__main__":
    main()
