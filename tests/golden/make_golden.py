"""Writes tests/golden/brute_n8.json: 30-digit potential-route values (oracle/brute_mp.py)
for a fixed 8-particle set, both stretching schemes and both core-size rules.

Run from the repository root: ``python tests/golden/make_golden.py``.  It calls only
``oracle/``; the stored values are the expected results of the particle sums of
Eqs. 2-5 (Sec. II.B) for this input."""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
from oracle import brute_mp  # noqa: E402


def main():
    rng = np.random.default_rng([2511_11430, 99])
    n = 8
    x = rng.uniform(-0.08, 0.08, (3, n))
    g = rng.normal(0, 1e-3, (3, n))
    s = rng.uniform(0.02, 0.05, n)
    out = {"source": "oracle/brute_mp.py particle_sums at 30 digits", "x": x.tolist(),
           "gamma": g.tolist(), "sigma": s.tolist(), "cases": []}
    for scheme in (0, 1):
        for rule in (0, 1):
            u, d = brute_mp.particle_sums(x.T, g.T, s, scheme=scheme, sigma_rule=rule)
            out["cases"].append({"scheme": scheme, "sigma_rule": rule,
                                 "u": np.array(u).T.tolist(), "dgamma": np.array(d).T.tolist()})
    with open(os.path.join(os.path.dirname(__file__), "brute_n8.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
