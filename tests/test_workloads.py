"""Seeded input generators: shapes, counts, determinism and the stated laws."""
import math

import numpy as np

from paper_2511_11430_amd import workloads as W


def test_config1_shape_and_seed():
    a, b = W.config1(), W.config1()
    assert a["x"].shape == (3, 4096) and np.array_equal(a["x"], b["x"])
    assert np.all(np.abs(a["x"]) <= 1.0) and np.all(a["sigma"] == 0.05)


def test_config2_parts():
    c = W.config2(n=4096)
    assert c["x"].shape == (3, 4096)
    assert c["seg_a"].shape == (3, 4096) and c["seg_gamma"].shape == (4096,)
    assert c["ctrl"].shape == (3, 64)
    r = np.hypot(c["x"][0], c["x"][1])
    assert r.max() <= 1.0 + 1e-12 and np.all(c["sigma"] == 0.02)
    # every ring contributes four edges that close: the sum of its edge vectors vanishes
    e = (c["seg_b"] - c["seg_a"]).reshape(3, -1, 4).sum(axis=2)
    assert np.abs(e).max() < 1e-14


def test_config3_sample_and_ranges():
    c = W.config3(n=1 << 14, n_sample=256)
    assert c["x"].shape == (3, 1 << 14) and len(np.unique(c["sample"])) == 256
    assert c["sigma"].min() >= 0.01 and c["sigma"].max() <= 0.05
    mag = np.linalg.norm(c["gamma"], axis=0)
    assert mag.min() >= 1e-6 * (1 - 1e-12) and mag.max() <= 1e-3 * (1 + 1e-12)


def test_config4_time_step():
    c = W.config4(n=4096)
    # 5 deg of rotation at tip Mach 0.439 on a 1 m rotor
    assert math.isclose(c["dt"], math.radians(5) / (0.439 * 340.3), rel_tol=1e-12)
    assert c["ctrl"].shape == (3, 128)


def test_config5_sizes():
    ws = W.config5()
    ns = [w["x"].shape[1] for w in ws]
    assert len(ws) == 64 and min(ns) >= 2048 and max(ns) <= 200000
    assert 2.0e6 < sum(ns) < 4.0e6
