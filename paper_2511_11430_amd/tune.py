"""Kernel-shape tuner for the FP32C particle kernel (targets per lane x workgroup size).

For each size bucket of single-set launches, and for the batched persistent launch of 64
uneven wakes, the library's own tuner (``vpm_autotune``) times every shape variant with HIP
events on wake-shaped inputs and records the fastest in its plan; all timings are written
to a JSON cache keyed by the GPU architecture and a hash of the kernel sources.  The
binding applies a matching cache (``vpm_set_plan``) when it first loads the library.

Usage (on the GPU):  python -m paper_2511_11430_amd.tune [--out PATH] [--quick]
"""
import argparse
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "tune_cache.json")
SINGLE_SIZES = [8192, 32768, 131072, 262144, 1048576]


def source_hash():
    h = hashlib.sha256()
    # the sources of the kernels being timed (the pair kernels and their device math)
    for f in ("pair_forward.hip", "device_math.h"):
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def tune(out=DEFAULT_CACHE, quick=False, log=print):
    """Runs the library's tuner (vpm_autotune: HIP-event timings of every shape on the
    caller's stream, the fastest recorded in the plan) on forward-flight wakes of each size
    bucket and on the 64 uneven wakes of the batched launch, then writes the timings and
    choices to the JSON cache."""
    import numpy as np
    import torch

    from . import vpm_autotune
    from . import workloads as W

    dev = torch.device("cuda:0")
    f32 = lambda a: torch.tensor(np.ascontiguousarray(W.to_f32(a)), dtype=torch.float32, device=dev)
    plans = []
    sizes = SINGLE_SIZES[:3] if quick else SINGLE_SIZES
    for i, n in enumerate(sizes):
        c = W.config3(n=n)
        x, g, s = f32(c["x"]), f32(c["gamma"]), f32(c["sigma"])
        best, ms = vpm_autotune(x, g, s, reps=2 if n >= 262144 else 3)
        for v, t in enumerate(ms, 1):
            log(f"single N={n} variant {v}: {t:.3f} ms")
        lo = sizes[i - 1] + 1 if i > 0 else 0
        hi = sizes[i + 1] - 1 if i + 1 < len(sizes) else 1 << 31
        plans.append({"batched": 0, "n_lo": lo, "n_hi": hi, "variant": best,
                      "ms": {str(v): t for v, t in enumerate(ms, 1)}, "n": n})
        del x, g, s
    # batched persistent launch over the 64 uneven wakes
    wakes = W.config5(scale=0.25 if quick else 1.0)
    off = [0]
    for w in wakes:
        off.append(off[-1] + w["x"].shape[1])
    cat = lambda k: np.concatenate([W.to_f32(w[k]) for w in wakes], axis=-1)
    xw = torch.tensor(cat("x"), dtype=torch.float32, device=dev)
    gw = torch.tensor(cat("gamma"), dtype=torch.float32, device=dev)
    sw = torch.tensor(cat("sigma"), dtype=torch.float32, device=dev)
    best, ms = vpm_autotune(xw, gw, sw, src_off=off, reps=2)
    for v, t in enumerate(ms, 1):
        log(f"batched {len(wakes)} wakes ({off[-1]} particles) variant {v}: {t:.3f} ms")
    plans.append({"batched": 1, "n_lo": 0, "n_hi": 1 << 31, "variant": best,
                  "ms": {str(v): t for v, t in enumerate(ms, 1)}, "n": off[-1]})
    props = torch.cuda.get_device_properties(0)
    cache = {"arch": getattr(props, "gcnArchName", "gfx950").split(":")[0], "device": props.name,
             "hip": torch.version.hip, "source_hash": source_hash(), "created": time.strftime("%Y-%m-%d %H:%M:%S"),
             "plans": plans}
    with open(out, "w") as f:
        json.dump(cache, f, indent=1)
    apply_cache(out)
    return cache


def apply_cache(path=None):
    """Apply a tuning cache to the loaded library if it matches the kernel sources; returns the
    number of plans applied (0 if none or stale)."""
    from . import F32C, _lib
    path = path or os.environ.get("VPM_TUNE_CACHE", DEFAULT_CACHE)
    try:
        with open(path) as f:
            cache = json.load(f)
    except (OSError, ValueError):
        return 0
    if cache.get("source_hash") != source_hash():
        return 0
    lib = _lib.load()
    n = 0
    for p in cache.get("plans", []):
        if lib.vpm_set_plan(F32C, int(p["batched"]), int(p["n_lo"]), int(p["n_hi"]), int(p["variant"])) == 0:
            n += 1
    return n


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_CACHE)
    ap.add_argument("--quick", action="store_true")
    args = ap.parse_args()
    cache = tune(args.out, args.quick, log=lambda m: print(m, flush=True))
    print(json.dumps({p["n"]: p["variant"] for p in cache["plans"]}), flush=True)


if __name__ == "__main__":
    sys.exit(main())
