"""Writes tests/golden/program_tangents_16384.json: the loss of the differentiation
workload's RK3 program (hover wake at 16,384 particles, 10 steps of 5 deg, loss on 128
blade control points; Sec. II.B) and its directional derivatives along two seeded
directions, from the FP64 oracle's dual-number tangents, for the exact program and for the
program whose evaluations read the state rounded to FP32 (the storage model of the GPU's
mixed program).  Inputs: the workload rounded once to FP32 (so the FP64 and the mixed GPU
programs take the same numbers).

Run from the repository root: ``python tests/golden/make_program_tangents.py`` (about 7
minutes on 8 cores).  It calls only ``oracle/`` and the input generator."""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle  # noqa: E402
from paper_2511_11430_amd import workloads as W  # noqa: E402

N = 16384


def inputs():
    c = W.config4(n=N)
    x, g, s, y = (W.to_f32(c[k]) for k in ("x", "gamma", "sigma", "ctrl"))
    return x, g, s, y, c["n_steps"], c["dt"]


def main():
    x, g, s, y, steps, dt = inputs()
    gs = float(np.sqrt(np.mean(g * g)))
    out = {"source": "oracle.rk3_program_jvp (FP64 dual numbers)", "n": N, "n_steps": steps, "dt": dt,
           "gamma_scale": gs, "directions": []}
    for k in range(2):
        xd, gd = W.program_direction(N, k, gs)
        rec = {"k": k}
        for name, storage in (("f64", oracle.STORE_F64), ("f32_eval", oracle.STORE_F32_EVAL)):
            t = time.time()
            L, dL = oracle.rk3_program_jvp(x, g, s, xd, gd, steps, dt, y, storage=storage)
            rec[name] = {"loss": L, "dloss": dL}
            print(f"direction {k} {name}: L {L:.17g} dL {dL:.17g} ({time.time() - t:.0f} s)", flush=True)
        out["directions"].append(rec)
    with open(os.path.join(os.path.dirname(__file__), "program_tangents_16384.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
