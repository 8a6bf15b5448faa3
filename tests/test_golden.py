"""The oracle against stored 30-digit potential-route values (tests/golden/brute_n8.json,
written by tests/golden/make_golden.py from oracle/brute_mp.py)."""
import json
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "brute_n8.json")


@pytest.mark.parametrize("case", range(4))
def test_oracle_matches_golden(case):
    with open(GOLDEN) as f:
        data = json.load(f)
    c = data["cases"][case]
    x, g, s = (np.array(data[k]) for k in ("x", "gamma", "sigma"))
    u, d = oracle.eval_pairs(x, g, s, scheme=c["scheme"], sigma_rule=c["sigma_rule"])
    ub, db = np.array(c["u"]), np.array(c["dgamma"])
    assert np.linalg.norm(u - ub) <= 1e-14 * np.linalg.norm(ub)
    assert np.linalg.norm(d - db) <= 1e-14 * np.linalg.norm(db)
