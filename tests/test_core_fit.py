"""The FP32 kernels' closed form of the in-core weight q(rho) for 1 <= rho < 7 (device_math.h,
closed_q): q = 1 - E (F + c0 rho), E = exp(-rho^2/2), F = erfcx(rho/sqrt2) as a polynomial in
w = 1/(1 + p rho).  Checks the constants compiled into the kernels against scipy's erfcx and
erf, and an FP32 emulation of the kernels' instruction sequence against the FP64 closed form
of Eq. 3's blob (q = erf(rho/sqrt2) - c0 rho exp(-rho^2/2))."""
import pathlib
import re

import numpy as np
from scipy.special import erf, erfcx

HDR = pathlib.Path(__file__).resolve().parents[1] / "paper_2511_11430_amd" / "csrc" / "device_math.h"
C0 = np.sqrt(2.0 / np.pi)


def _constants():
    text = HDR.read_text()
    p = float(re.search(r"constexpr float kErfcxP = ([0-9.eE+-]+)f;", text).group(1))
    body = re.search(r"constexpr float kErfcxC\[8\] = \{([^}]*)\};", text, re.S).group(1)
    c = [float(v.strip().rstrip("f")) for v in body.split(",")]
    assert len(c) == 8
    return np.float32(p), np.array(c, dtype=np.float32)


def test_erfcx_fit_of_the_kernels():
    p, c = _constants()
    rho = np.linspace(1.0, 7.0, 20001)
    w = 1.0 / (1.0 + float(p) * rho)
    f = np.polyval(c.astype(np.float64)[::-1], w)
    err = np.abs(f / erfcx(rho / np.sqrt(2.0)) - 1.0).max()
    assert err < 2e-8, err


def test_fp32_sequence_against_the_closed_form():
    p, c = _constants()
    f32 = np.float32
    rho64 = np.linspace(1.0, 7.0, 200001)
    t = (rho64 * rho64).astype(f32)                      # the kernels' t = s^2 / sigma^2
    tt = t.astype(np.float64)
    rho = np.sqrt(tt).astype(f32)                        # v_sqrt_f32, ~correctly rounded
    e = np.exp2((t * f32(-0.72134752044448170368)).astype(np.float64)).astype(f32)
    w = (1.0 / (f32(p) * rho + f32(1)).astype(np.float64)).astype(f32)
    fw = c[7]
    for k in range(6, -1, -1):
        fw = (fw * w + c[k]).astype(f32)
    q = (f32(1) - e.astype(np.float64) * (f32(C0) * rho + fw).astype(np.float64)).astype(f32)
    rt = np.sqrt(tt)
    q_ref = erf(rt / np.sqrt(2.0)) - C0 * rt * np.exp(-tt / 2.0)
    rel = np.abs(q.astype(np.float64) / q_ref - 1.0)
    # cancellation near rho = 1 (q ~ 0.2 against 1 - E (F + c0 rho)); a few ulps beyond rho = 2
    assert rel[rt < 2.0].max() < 2e-6, rel[rt < 2.0].max()
    assert rel[rt >= 2.0].max() < 5e-7, rel[rt >= 2.0].max()
