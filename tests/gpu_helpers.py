"""Shared helpers of the GPU parity tests (inputs to device, error metrics)."""
import numpy as np

TOL = {"f64": 1e-12, "f32c": 1e-5}


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def per_target(a, b):
    """Largest error of one target's 3-vector, relative to the RMS magnitude of the reference
    over all targets: no single target may exceed the gate that rel-L2 applies on average."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    rms = np.sqrt(np.mean(np.sum(b * b, axis=0)))
    err = np.sqrt(np.sum((a - b) ** 2, axis=0))
    return float(err.max() / rms) if rms > 0 else float(err.max())


def torch_dtype(kind):
    import torch
    return torch.float64 if kind == "f64" else torch.float32


def prepare(arrays, kind):
    """Round inputs once for the FP32 path; the oracle then sees the rounded values."""
    from paper_2511_11430_amd import workloads as W
    if kind == "f32c":
        return [W.to_f32(a) for a in arrays]
    return [np.asarray(a, dtype=np.float64) for a in arrays]


def dev(a, kind):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch_dtype(kind), device="cuda")


def host(t):
    return t.detach().cpu().double().numpy()


def say(msg):
    print(msg, flush=True)
