"""GPU parity of the hand-written adjoint: the pair vector-Jacobian product against full
Jacobians the FP64 oracle builds column by column with dual-number tangents (one tile, and
entry by entry on 4096 particles over many far and near tiles), the RK3 program gradient
against the oracle's program tangents (2 steps on a compact set; the differentiation
workload's 10 steps at 16,384 particles from stored oracle values), and central finite
differences (h = 1e-6, FP64) of the program at 16,384 and at the full 262,144 particles."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
import paper_2511_11430_amd as vpm
from paper_2511_11430_amd import autograd as AG
from paper_2511_11430_amd import workloads as W

from gpu_helpers import TOL, dev, host, per_target, prepare, rel_l2, say

pytestmark = pytest.mark.gpu
KINDS = ["f64", "f32c"]


def _set(n, seed, spread=0.08):
    rng = np.random.default_rng([777, seed])
    x = rng.uniform(-spread, spread, (3, n))
    g = rng.normal(0, 1e-3, (3, n))
    s = rng.uniform(0.02, 0.05, n)
    return x, g, s


def _oracle_vjp_self(x, g, s, ub, sb, rule, scheme=0):
    """w^T J built column by column from oracle tangents (self evaluation)."""
    n = x.shape[1]
    out = np.zeros((2, 3, n))
    for part in range(2):
        for c in range(3):
            for i in range(n):
                xd, gd = np.zeros_like(x), np.zeros_like(g)
                (xd if part == 0 else gd)[c, i] = 1.0
                _, _, ud, dd = oracle.eval_pairs_jvp(x, g, s, xd, gd, scheme=scheme, sigma_rule=rule)
                out[part, c, i] = (ub * ud).sum() + (sb * dd).sum()
    return out[0], out[1]


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("rule", [0, 1])
@pytest.mark.parametrize("scheme", [0, 1])
def test_pair_vjp_equals_oracle_jacobian(kind, rule, scheme, gpu):
    """Both stretching schemes (transposed, and classical composed from the transposed adjoint
    with the target strength and its seed exchanged) and both core rules."""
    x, g, s = prepare(_set(40, 1 + rule), kind)
    rng = np.random.default_rng(5)
    ub, sb = prepare([rng.normal(size=x.shape), rng.normal(size=x.shape) * 1e3], kind)
    say(f"pair vjp {kind} rule={rule} scheme={scheme}")
    xb, gb, _, _ = vpm.vpm_backward(dev(x, kind), dev(g, kind), dev(s, kind), dev(ub, kind), dev(sb, kind),
                                    sigma_rule=rule, scheme=scheme)
    rx, rg = _oracle_vjp_self(x, g, s, ub, sb, rule, scheme)
    assert rel_l2(host(xb), rx) <= TOL[kind]
    assert rel_l2(host(gb), rg) <= TOL[kind]


@pytest.mark.parametrize("kind", KINDS)
def test_classical_vjp_for_separate_targets(kind, gpu):
    """Classical scheme with distinct source and target sets: the gradients of both sets
    against oracle tangents."""
    x, g, s = prepare(_set(30, 7), kind)
    y, gy, sy = prepare(_set(20, 8), kind)
    rng = np.random.default_rng(12)
    ub, sb = prepare([rng.normal(size=y.shape), rng.normal(size=y.shape) * 1e3], kind)
    xb, gb, yb, gyb = vpm.vpm_backward(dev(x, kind), dev(g, kind), dev(s, kind), dev(ub, kind), dev(sb, kind),
                                       dev(y, kind), dev(gy, kind), dev(sy, kind), want_target_grads=True, scheme=1)
    refs = {k: np.zeros((3, n)) for k, n in (("x", 30), ("g", 30), ("y", 20), ("gy", 20))}
    for c in range(3):
        for key, n in (("x", 30), ("g", 30), ("y", 20), ("gy", 20)):
            for i in range(n):
                z = lambda m: np.zeros((3, m))
                xd, gd, yd, gyd = z(30), z(30), z(20), z(20)
                {"x": xd, "g": gd, "y": yd, "gy": gyd}[key][c, i] = 1.0
                _, _, ud, dd = oracle.eval_pairs_jvp(x, g, s, xd, gd, scheme=1, x_tgt=y, gam_tgt=gy, sig_tgt=sy,
                                                     x_tgt_dot=yd, gam_tgt_dot=gyd)
                refs[key][c, i] = (ub * ud).sum() + (sb * dd).sum()
    for got, key in ((xb, "x"), (gb, "g"), (yb, "y"), (gyb, "gy")):
        assert rel_l2(host(got), refs[key]) <= TOL[kind], key


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("scheme", [0, 1])
def test_batched_vjp_equals_per_set_calls(kind, scheme, gpu):
    """Twelve uneven hover wakes in one call (the persistent queue for the transposed scheme,
    set after set for the classical one): the same bits as one call per wake, and each wake's
    gradient against the oracle on sampled entries."""
    import torch
    wakes = W.config5(n_wakes=12, scale=0.02)
    parts = [prepare([w["x"], w["gamma"], w["sigma"]], kind) for w in wakes]
    off = [0]
    for x, _, _ in parts:
        off.append(off[-1] + x.shape[1])
    rng = np.random.default_rng([21, scheme])
    ubs = [prepare([rng.normal(size=p[0].shape), rng.normal(size=p[0].shape) * 1e3], kind) for p in parts]
    cat = lambda i: dev(np.concatenate([p[i] for p in parts], -1), kind)
    X, G, S = cat(0), cat(1), cat(2)
    UB = dev(np.concatenate([u[0] for u in ubs], -1), kind)
    SB = dev(np.concatenate([u[1] for u in ubs], -1), kind)
    say(f"batched vjp {kind} scheme={scheme}: {len(parts)} wakes, {off[-1]} particles")
    xb, gb, _, _ = vpm.vpm_backward(X, G, S, UB, SB, src_off=off, scheme=scheme)
    for w, (x, g, s) in enumerate(parts):
        sl = slice(off[w], off[w + 1])
        xw, gw, _, _ = vpm.vpm_backward(dev(x, kind), dev(g, kind), dev(s, kind), dev(ubs[w][0], kind),
                                        dev(ubs[w][1], kind), scheme=scheme)
        assert torch.equal(xb[:, sl], xw) and torch.equal(gb[:, sl], gw), w
        if w % 4 == 0:
            idx = np.sort(np.random.default_rng(w).choice(x.shape[1], min(8, x.shape[1]), replace=False))
            rx, rg = _oracle_vjp_columns(x, g, s, ubs[w][0], ubs[w][1], 0, idx, scheme)
            assert rel_l2(host(xw)[:, idx], rx) <= TOL[kind] and rel_l2(host(gw)[:, idx], rg) <= TOL[kind]


def _oracle_vjp_columns(x, g, s, ub, sb, rule, idx, scheme=0):
    """Entries of w^T J for the particles idx (all six components), each the oracle's
    dual-number tangent along a unit vector.  Only pairs that contain the particle carry a
    tangent, so each column sums two evaluations: the particle as the one source of every
    other target, and as the one target of every other source."""
    n = x.shape[1]
    out = np.zeros((2, 3, idx.size))
    for col, k in enumerate(idx):
        one = slice(k, k + 1)
        excl_a = np.full(n, -1, dtype=np.int64)
        excl_a[k] = 0
        for part in range(2):
            for c in range(3):
                e = np.zeros((3, 1))
                e[c, 0] = 1.0
                z = np.zeros((3, 1))
                xd, gd = (e, z) if part == 0 else (z, e)
                _, _, ua, da = oracle.eval_pairs_jvp(x[:, one], g[:, one], s[one], xd, gd, scheme=scheme,
                                                     sigma_rule=rule, x_tgt=x, gam_tgt=g, sig_tgt=s, excl=excl_a)
                _, _, ut, dtg = oracle.eval_pairs_jvp(x, g, s, np.zeros_like(x), np.zeros_like(g), scheme=scheme,
                                                      sigma_rule=rule, x_tgt=x[:, one], gam_tgt=g[:, one],
                                                      sig_tgt=s[one], x_tgt_dot=xd, gam_tgt_dot=gd,
                                                      excl=np.array([k]))
                out[part, c, col] = ((ub * ua).sum() + (sb * da).sum() + (ub[:, one] * ut).sum()
                                     + (sb[:, one] * dtg).sum())
    return out[0], out[1]


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("rule,scheme", [(0, 0), (1, 0), (0, 1)])
def test_pair_vjp_entries_on_many_tiles(kind, rule, scheme, gpu):
    """4096 particles of the forward-flight wake (cores log-uniform in [0.01R, 0.05R]): 16
    tiles of the adjoint kernel, far tiles (box-culled, no core test) and near ones.  The
    gradient of 64 particles spread over the set, all six components (384 entries), against
    oracle tangent columns, entry by entry."""
    c = W.config3(n=4096)
    x, g, s = prepare([c["x"], c["gamma"], c["sigma"]], kind)
    rng = np.random.default_rng([6, rule])
    ub, sb = prepare([rng.normal(size=x.shape), rng.normal(size=x.shape) * 1e3], kind)
    idx = np.sort(rng.choice(x.shape[1], 64, replace=False))
    say(f"pair vjp entries {kind} rule={rule} scheme={scheme}")
    xb, gb, _, _ = vpm.vpm_backward(dev(x, kind), dev(g, kind), dev(s, kind), dev(ub, kind), dev(sb, kind),
                                    sigma_rule=rule, scheme=scheme)
    rx, rg = _oracle_vjp_columns(x, g, s, ub, sb, rule, idx, scheme)
    hx, hg = host(xb)[:, idx], host(gb)[:, idx]
    errs = rel_l2(hx, rx), rel_l2(hg, rg), per_target(hx, rx), per_target(hg, rg)
    say(f"  rel-L2 x_bar {errs[0]:.2e} gamma_bar {errs[1]:.2e}; worst particle {errs[2]:.2e} {errs[3]:.2e}")
    assert max(errs) <= TOL[kind]


@pytest.mark.parametrize("kind", KINDS)
def test_velocity_only_vjp_for_sources_and_targets(kind, gpu):
    x, g, s = prepare(_set(50, 3), kind)
    y = prepare([np.random.default_rng(8).uniform(-0.1, 0.1, (3, 12))], kind)[0]
    ub = prepare([np.random.default_rng(9).normal(size=y.shape)], kind)[0]
    xb, gb, yb, _ = vpm.vpm_backward(dev(x, kind), dev(g, kind), dev(s, kind), dev(ub, kind), None,
                                     dev(y, kind), None, None, want_target_grads=True)
    n = x.shape[1]
    rx, rg, ry = np.zeros_like(x), np.zeros_like(g), np.zeros_like(y)
    for c in range(3):
        for i in range(n):
            for part, ref in ((0, rx), (1, rg)):
                xd, gd = np.zeros_like(x), np.zeros_like(g)
                (xd if part == 0 else gd)[c, i] = 1.0
                _, _, ud, _ = oracle.eval_pairs_jvp(x, g, s, xd, gd, x_tgt=y)
                ref[c, i] = (ub * ud).sum()
        for i in range(y.shape[1]):
            yd = np.zeros_like(y)
            yd[c, i] = 1.0
            _, _, ud, _ = oracle.eval_pairs_jvp(x, g, s, np.zeros_like(x), np.zeros_like(g), x_tgt=y, x_tgt_dot=yd)
            ry[c, i] = (ub * ud).sum()
    assert rel_l2(host(xb), rx) <= TOL[kind]
    assert rel_l2(host(gb), rg) <= TOL[kind]
    assert rel_l2(host(yb), ry) <= TOL[kind]


@pytest.mark.parametrize("kind", KINDS)
def test_vjp_dot_product_on_hover_wake(kind, gpu):
    """<vjp(w), v> = <w, jvp(v)> on 4096 hover-wake particles (oracle tangent)."""
    c = W.config4(n=4096)
    x, g, s = prepare([c["x"], c["gamma"], c["sigma"]], kind)
    rng = np.random.default_rng(3)
    ub, sb = rng.normal(size=x.shape), rng.normal(size=x.shape) * 1e3
    xd, gd = rng.normal(size=x.shape) * 1e-3, rng.normal(size=x.shape) * 1e-6
    ub, sb = prepare([ub, sb], kind)
    xb, gb, _, _ = vpm.vpm_backward(dev(x, kind), dev(g, kind), dev(s, kind), dev(ub, kind), dev(sb, kind))
    _, _, ud, dd = oracle.eval_pairs_jvp(x, g, s, xd, gd)
    lhs = (host(xb) * xd).sum() + (host(gb) * gd).sum()
    rhs = (ub * ud).sum() + (sb * dd).sum()
    assert abs(lhs - rhs) <= (1e-11 if kind == "f64" else 1e-5) * abs(rhs)


def _program_inputs(n, kind, seed=2):
    rng = np.random.default_rng([55, seed])
    c = W.config4(n=n)
    # a compact piece of the hover wake: the first n particles of one tip helix, and two
    # control points near it, so the loss sees near-field interactions
    x, g, s = c["x"], c["gamma"], c["sigma"]
    y = x[:, :2] + np.array([[0.0], [0.0], [-0.03]]) + rng.normal(scale=0.005, size=(3, 2))
    return prepare([x, g, s, y], kind)


STORAGE = {"f64": oracle.STORE_F64, "mixed": oracle.STORE_F32_EVAL, "f32c": oracle.STORE_F32}


@pytest.mark.parametrize("kind", KINDS + ["mixed"])
def test_rk3_program_gradient_vs_oracle_tangents(kind, gpu):
    """kind 'mixed': FP64 state and registers, FP32-compensated pair sums; 'f32c': FP32 state.

    A compact piece of a tip helix (0.5 mm spacing, cores of 20 mm) and two control points
    30 mm away, 2 steps.  Each GPU program is compared with the oracle program under its own
    storage model (evaluations read the state rounded to FP32 and return FP32 results; for
    f32c the state and registers are FP32 too) to the adjoint gate of 1e-6, so the kernels'
    error is measured alone.  The storage model's own distance from the exact program (FP32
    positions near 1 m carry 6e-8 m of rounding, 1e-4 of the particle spacing) is printed:
    that is the cost of FP32 evaluation inputs on this near-field case, not kernel error."""
    n, steps = 36, 2
    ek = "f32c" if kind != "f64" else "f64"
    sk = "f64" if kind != "f32c" else "f32c"
    x, g, s, y = _program_inputs(n, ek)
    dt = 2e-4
    say(f"RK3 program gradient {kind}")
    X, G = dev(x, sk).requires_grad_(True), dev(g, sk).requires_grad_(True)
    L = AG.rk3_program_loss(X, G, dev(s, ek), steps, dt, dev(y, ek))
    L.backward()
    st = STORAGE[kind]
    Lo = oracle.rk3_program(x, g, s, steps, dt, y, storage=st)[3]
    L_exact = oracle.rk3_program(x, g, s, steps, dt, y)[3]
    el = abs(L.item() - Lo) / abs(Lo)
    say(f"  loss rel err {el:.2e} against the storage model; the model against the exact program "
        f"{abs(Lo - L_exact) / abs(L_exact):.2e}")
    assert el <= (1e-12 if kind == "f64" else 1e-6)
    ref = np.zeros((2, 3, n))
    ref_exact = np.zeros((2, 3, n))
    for part in range(2):
        for cc in range(3):
            for i in range(n):
                xd, gd = np.zeros_like(x), np.zeros_like(g)
                (xd if part == 0 else gd)[cc, i] = 1.0
                ref[part, cc, i] = oracle.rk3_program_jvp(x, g, s, xd, gd, steps, dt, y, storage=st)[1]
                if kind != "f64":
                    ref_exact[part, cc, i] = oracle.rk3_program_jvp(x, g, s, xd, gd, steps, dt, y)[1]
    tol = 1e-10 if kind == "f64" else 1e-6
    ex, eg = rel_l2(host(X.grad), ref[0]), rel_l2(host(G.grad), ref[1])
    say(f"  rel-L2 dL/dx {ex:.2e}  dL/dGamma {eg:.2e} against the storage model")
    if kind != "f64":
        say(f"  storage model against the exact program: dL/dx {rel_l2(ref[0], ref_exact[0]):.2e} "
            f"dL/dGamma {rel_l2(ref[1], ref_exact[1]):.2e}")
    assert ex <= tol and eg <= tol


def _golden_tangents():
    path = os.path.join(os.path.dirname(__file__), "golden", "program_tangents_16384.json")
    with open(path) as f:
        return json.load(f)


@pytest.mark.parametrize("kind", ["f64", "mixed"])
def test_program_tangents_at_16384(kind, gpu):
    """The differentiation workload's program (hover wake at 16,384 particles, 10 RK3 steps of
    5 deg, 128 control points) differentiated by the GPU adjoint, projected on two seeded
    directions, against the oracle's dual-number tangents stored by
    tests/golden/make_program_tangents.py: the FP64 program to 1e-10, the mixed program
    (FP64 state, FP32C sums) to the adjoint gate of 1e-6 against the exact program."""
    gold = _golden_tangents()
    n = gold["n"]
    c = W.config4(n=n)
    x, g, s, y = (W.to_f32(c[k]) for k in ("x", "gamma", "sigma", "ctrl"))
    assert c["n_steps"] == gold["n_steps"] and c["dt"] == gold["dt"]
    ek = "f64" if kind == "f64" else "f32c"
    X, G = dev(x, "f64").requires_grad_(True), dev(g, "f64").requires_grad_(True)
    L = AG.rk3_program_loss(X, G, dev(s, ek), c["n_steps"], c["dt"], dev(y, ek))
    L.backward()
    gx, gg = host(X.grad), host(G.grad)
    for rec in gold["directions"]:
        xd, gd = W.program_direction(n, rec["k"], gold["gamma_scale"])
        dl = float((gx * xd).sum() + (gg * gd).sum())
        ref = rec["f64"]
        el = abs(L.item() - ref["loss"]) / abs(ref["loss"])
        ed = abs(dl - ref["dloss"]) / abs(ref["dloss"])
        em = abs(dl - rec["f32_eval"]["dloss"]) / abs(rec["f32_eval"]["dloss"])
        say(f"{kind} direction {rec['k']}: loss {el:.2e}, dL {ed:.2e} against the exact program "
            f"({em:.2e} against the FP32-evaluation model)")
        if kind == "f64":
            assert el <= 1e-12 and ed <= 1e-10
        else:
            assert el <= 1e-6 and ed <= 1e-6


def test_rk3_program_gradient_vs_central_differences(gpu):
    """FP64 GPU program on 16384 hover-wake particles, 10 RK3 steps of 5 deg: the adjoint
    gradient against central differences (h = 1e-6) of the same program, 64 random particles."""
    c = W.config4(n=16384)
    x, g, s = (np.asarray(c[k], dtype=np.float64) for k in ("x", "gamma", "sigma"))
    y = c["ctrl"]
    steps, dt = c["n_steps"], c["dt"]
    X, G = dev(x, "f64").requires_grad_(True), dev(g, "f64").requires_grad_(True)
    S, Y = dev(s, "f64"), dev(y, "f64")
    L = AG.rk3_program_loss(X, G, S, steps, dt, Y)
    L.backward()
    gx, gg = host(X.grad), host(G.grad)
    rng = np.random.default_rng(64)
    idx = rng.choice(x.shape[1], 64, replace=False)
    h = 1e-6
    fd, ad = [], []
    X0, G0 = dev(x, "f64"), dev(g, "f64")
    for i in idx:
        for part in range(2):
            for cc in range(3):
                base = X0 if part == 0 else G0
                step = h  # absolute, SI units, for x (m) and Gamma (m^3/s) alike
                e = torch.zeros_like(base)
                e[cc, i] = step
                xp, gp = (X0 + e, G0) if part == 0 else (X0, G0 + e)
                xm, gm = (X0 - e, G0) if part == 0 else (X0, G0 - e)
                Lp = AG.rk3_forward(xp, gp, S, steps, dt, Y)[3].item()
                Lm = AG.rk3_forward(xm, gm, S, steps, dt, Y)[3].item()
                fd.append((Lp - Lm) / (2 * step))
                ad.append((gx if part == 0 else gg)[cc, i])
    fd, ad = np.array(fd), np.array(ad)
    err = np.linalg.norm(fd - ad) / np.linalg.norm(fd)
    say(f"FD check: rel-L2 {err:.2e} over {len(fd)} components")
    assert err <= 1e-6


@pytest.fixture(scope="module")
def full_size_fp64_program(gpu):
    """FP64 program of the differentiation workload at full size and its adjoint gradient."""
    c = W.config4()
    x, g, s, y = (W.to_f32(c[k]) for k in ("x", "gamma", "sigma", "ctrl"))
    X, G = dev(x, "f64").requires_grad_(True), dev(g, "f64").requires_grad_(True)
    S, Y = dev(s, "f64"), dev(y, "f64")
    L = AG.rk3_program_loss(X, G, S, c["n_steps"], c["dt"], Y)
    L.backward()
    out = dict(x=dev(x, "f64"), g=dev(g, "f64"), S=S, Y=Y, steps=c["n_steps"], dt=c["dt"], gx=host(X.grad),
               gg=host(G.grad))
    del X, G, L
    torch.cuda.empty_cache()
    return out


@pytest.mark.parametrize("chunk", range(4))
def test_full_size_program_gradient_vs_central_differences(chunk, full_size_fp64_program):
    """Differentiation workload at full size (262,144 particles, 10 RK3 steps, 128 control
    points), FP64 GPU program: 64 seeded particles, each perturbed along its own random
    6-vector (position and strength, h = 1e-6 in SI units), central differences of the
    program's loss against the adjoint gradient projected on that vector; 16 particles per
    chunk (two 2.5 s programs each)."""
    P = full_size_fp64_program
    n = P["x"].shape[1]
    rng = np.random.default_rng(262144)
    idx = rng.choice(n, 64, replace=False)
    dirs = rng.normal(size=(64, 2, 3))
    h = 1e-6
    fd, ad = [], []
    for j in range(16 * chunk, 16 * chunk + 16):
        i = int(idx[j])
        v = torch.tensor(dirs[j], dtype=torch.float64, device="cuda")
        L = []
        for sgn in (1.0, -1.0):
            xp, gp = P["x"].clone(), P["g"].clone()
            xp[:, i] += sgn * h * v[0]
            gp[:, i] += sgn * h * v[1]
            L.append(AG.rk3_forward(xp, gp, P["S"], P["steps"], P["dt"], P["Y"])[3].item())
        fd.append((L[0] - L[1]) / (2 * h))
        ad.append(float(P["gx"][:, i] @ dirs[j][0] + P["gg"][:, i] @ dirs[j][1]))
    fd, ad = np.array(fd), np.array(ad)
    err = np.linalg.norm(fd - ad) / np.linalg.norm(fd)
    worst = np.abs(fd - ad).max() / np.sqrt(np.mean(fd * fd))
    say(f"full-size FD chunk {chunk}: rel-L2 {err:.2e}, worst particle {worst:.2e}")
    assert err <= 1e-6 and worst <= 1e-6


def test_mixed_program_gradient_matches_fp64_at_full_size(gpu):
    """Differentiation workload at full size (262144 hover-wake particles, 10 RK3 steps of
    5 deg, 128 control points): the mixed program's gradient (FP64 state, FP32-compensated
    pair sums) against the FP64 GPU program's gradient, itself pinned to the oracle above."""
    c = W.config4()
    x, g, s, y = (W.to_f32(c[k]) for k in ("x", "gamma", "sigma", "ctrl"))
    grads = {}
    for kind in ("f64", "mixed"):
        ek = "f64" if kind == "f64" else "f32c"
        X, G = dev(x, "f64").requires_grad_(True), dev(g, "f64").requires_grad_(True)
        L = AG.rk3_program_loss(X, G, dev(s, ek), c["n_steps"], c["dt"], dev(y, ek))
        L.backward()
        grads[kind] = (host(X.grad), host(G.grad), L.item())
        del X, G, L
        torch.cuda.empty_cache()
    ex = rel_l2(grads["mixed"][0], grads["f64"][0])
    eg = rel_l2(grads["mixed"][1], grads["f64"][1])
    el = abs(grads["mixed"][2] - grads["f64"][2]) / abs(grads["f64"][2])
    say(f"full-size program: loss rel {el:.2e}, dL/dx rel-L2 {ex:.2e}, dL/dGamma rel-L2 {eg:.2e}")
    assert el <= 1e-6 and ex <= 1e-6 and eg <= 1e-6


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("rule", [0, 1])
def test_vjp_dot_product_varied_cores(kind, rule, gpu):
    """Forward-flight wake (cores log-uniform in [0.01R, 0.05R]) at 8192 particles: the
    adjoint's dot product against oracle tangents, source and symmetric core rules."""
    c = W.config3(n=8192)
    x, g, s = prepare([c["x"], c["gamma"], c["sigma"]], kind)
    rng = np.random.default_rng([4, rule])
    ub, sb = prepare([rng.normal(size=x.shape), rng.normal(size=x.shape) * 1e3], kind)
    xd, gd = rng.normal(size=x.shape) * 1e-3, rng.normal(size=x.shape) * 1e-6
    xb, gb, _, _ = vpm.vpm_backward(dev(x, kind), dev(g, kind), dev(s, kind), dev(ub, kind), dev(sb, kind),
                                    sigma_rule=rule)
    _, _, ud, dd = oracle.eval_pairs_jvp(x, g, s, xd, gd, sigma_rule=rule)
    lhs = (host(xb) * xd).sum() + (host(gb) * gd).sum()
    rhs = (ub * ud).sum() + (sb * dd).sum()
    assert abs(lhs - rhs) <= (1e-11 if kind == "f64" else 1e-5) * abs(rhs)


@pytest.mark.parametrize("kind", ["f64", "mixed"])
def test_checkpointed_and_recomputed_gradients_are_the_same_bits(kind, gpu):
    """The program's gradient from its stage checkpoints and from stage inputs recomputed from
    the initial state (no checkpoints kept) are bitwise equal: the checkpoints hold exactly the
    states the backward pass needs."""
    c = W.config4(n=4096, n_steps=3)
    x, g, s, y = (W.to_f32(c[k]) for k in ("x", "gamma", "sigma", "ctrl"))
    ek = "f64" if kind == "f64" else "f32c"
    S, Y = dev(s, ek), dev(y, ek)
    X, G = dev(x, "f64").requires_grad_(True), dev(g, "f64").requires_grad_(True)
    L = AG.rk3_program_loss(X, G, S, c["n_steps"], c["dt"], Y)
    L.backward()
    L2, xb, gb = AG.rk3_gradient_recompute(dev(x, "f64"), dev(g, "f64"), S, c["n_steps"], c["dt"], Y)
    assert torch.equal(L.detach(), L2)
    assert torch.equal(X.grad, xb) and torch.equal(G.grad, gb)
