"""GPU parity of the forward particle sums (Eqs. 2-5) and the segment velocity (Sec. II.A)
against the FP64 oracle: element-wise at sizes the oracle finishes in seconds (several tiles
plus a ragged tail), and on sampled outputs at the benchmark's full sizes and launch shape."""
import numpy as np
import pytest

import oracle
import paper_2511_11430_amd as vpm
from paper_2511_11430_amd import workloads as W

from gpu_helpers import TOL, dev, host, per_target, prepare, rel_l2, say

pytestmark = pytest.mark.gpu
KINDS = ["f64", "f32c"]


def _random_set(n, seed, spread=0.3):
    rng = np.random.default_rng([4242, seed])
    x = rng.uniform(-spread, spread, (3, n))
    g = rng.normal(0, 1e-3, (3, n))
    s = rng.uniform(0.02, 0.06, n)
    return x, g, s


@pytest.mark.parametrize("kind", KINDS)
def test_config1_uniform_cube(kind, gpu):
    c = W.config1()
    x, g, s = prepare([c["x"], c["gamma"], c["sigma"]], kind)
    say(f"config1 {kind} N={x.shape[1]}")
    u, d = vpm.vpm_eval_velocity_stretching(dev_(x, kind), dev_(g, kind), dev_(s, kind))
    uo, do = oracle.eval_pairs(x, g, s)
    assert rel_l2(host(u), uo) <= TOL[kind]
    assert rel_l2(host(d), do) <= TOL[kind]


def dev_(a, kind):
    return dev(a, kind)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("n", [1, 2, 37, 300, 1537])
@pytest.mark.parametrize("scheme,rule", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_ragged_sizes_schemes_rules(kind, n, scheme, rule, gpu):
    x, g, s = prepare(_random_set(n, n), kind)
    say(f"ragged {kind} n={n} scheme={scheme} rule={rule}")
    u, d = vpm.vpm_eval_velocity_stretching(dev_(x, kind), dev_(g, kind), dev_(s, kind), scheme=scheme,
                                            sigma_rule=rule)
    uo, do = oracle.eval_pairs(x, g, s, scheme=scheme, sigma_rule=rule)
    if n == 1:
        assert np.all(host(u) == 0) and np.all(host(d) == 0)
        return
    assert rel_l2(host(u), uo) <= TOL[kind]
    assert rel_l2(host(d), do) <= TOL[kind]


@pytest.mark.parametrize("variant", range(1, 9))
def test_every_fp32_kernel_shape(variant, gpu):
    x, g, s = prepare(_random_set(2111, 5), "f32c")
    say(f"variant {variant}")
    u, d = vpm.vpm_eval_velocity_stretching(dev_(x, "f32c"), dev_(g, "f32c"), dev_(s, "f32c"), variant=variant)
    uo, do = oracle.eval_pairs(x, g, s)
    assert rel_l2(host(u), uo) <= TOL["f32c"]
    assert rel_l2(host(d), do) <= TOL["f32c"]


@pytest.mark.parametrize("kind", KINDS)
def test_empty_and_coincident(kind, gpu):
    import torch
    e = torch.zeros((3, 0), dtype=torch.float64 if kind == "f64" else torch.float32, device="cuda")
    u, d = vpm.vpm_eval_velocity_stretching(e, e, e[0])
    assert u.shape == (3, 0)
    # two distinct particles at one point: no velocity, stretching g(0) Gamma_i x Gamma_j
    x = np.zeros((3, 2))
    g = np.array([[1e-3, 0.0], [0.0, 2e-3], [0.0, 0.0]])
    s = np.full(2, 0.04)
    u, d = vpm.vpm_eval_velocity_stretching(dev_(x, kind), dev_(g, kind), dev_(s, kind))
    uo, do = oracle.eval_pairs(x, g, s)
    assert np.all(host(u) == 0)
    assert rel_l2(host(d), do) <= TOL[kind]


@pytest.mark.parametrize("kind", KINDS)
def test_accumulate_and_velocity_only(kind, gpu):
    x, g, s = prepare(_random_set(700, 9), kind)
    X, G, S = dev_(x, kind), dev_(g, kind), dev_(s, kind)
    u, d = vpm.vpm_eval_velocity_stretching(X, G, S)
    u2, d2 = vpm.vpm_eval_velocity_stretching(X, G, S, u_out=u.clone(), dgamma_out=d.clone(), accumulate=True)
    uo, do = oracle.eval_pairs(x, g, s)
    assert rel_l2(host(u2), 2 * uo) <= TOL[kind]
    assert rel_l2(host(d2), 2 * do) <= TOL[kind]
    uv, dv = vpm.vpm_eval_velocity_stretching(X, G, S, velocity_only=True)
    assert dv is None and rel_l2(host(uv), uo) <= TOL[kind]


@pytest.mark.parametrize("kind", KINDS)
def test_control_points_and_sampled_targets(kind, gpu):
    c = W.config2(n=6000)
    x, g, s, y = prepare([c["x"], c["gamma"], c["sigma"], c["ctrl"]], kind)
    X, G, S = dev_(x, kind), dev_(g, kind), dev_(s, kind)
    # blade control points: velocity only (source-core rule)
    uc, dc = vpm.vpm_eval_velocity_stretching(X, G, S, dev_(y, kind))
    assert dc is None
    uco, _ = oracle.eval_pairs(x, g, s, x_tgt=y)
    assert rel_l2(host(uc), uco) <= TOL[kind]
    # a subset of the particles as explicit targets, each skipping itself
    import torch
    idx = np.sort(np.random.default_rng(3).choice(x.shape[1], 300, replace=False))
    ex = torch.tensor(idx, dtype=torch.int32, device="cuda")
    ut, dt_ = vpm.vpm_eval_velocity_stretching(X, G, S, dev_(x[:, idx], kind), dev_(g[:, idx], kind),
                                               dev_(s[idx], kind), tgt_exclude=ex)
    uo, do = oracle.eval_pairs(x, g, s, x_tgt=x[:, idx], gam_tgt=g[:, idx], excl=idx)
    assert rel_l2(host(ut), uo) <= TOL[kind]
    assert rel_l2(host(dt_), do) <= TOL[kind]


def _sampled_parity(c, kind, idx, rule=0):
    """Self evaluation of the whole set on the GPU, checked on the targets idx against the
    oracle: rel-L2 and the worst single target (both within the gate)."""
    x, g, s = prepare([c["x"], c["gamma"], c["sigma"]], kind)
    say(f"full-size self evaluation {kind} N={x.shape[1]} rule={rule}, {idx.size} sampled targets")
    u, d = vpm.vpm_eval_velocity_stretching(dev_(x, kind), dev_(g, kind), dev_(s, kind), sigma_rule=rule)
    uo, do = oracle.eval_pairs(x, g, s, x_tgt=x[:, idx], gam_tgt=g[:, idx], sig_tgt=s[idx], excl=idx,
                               sigma_rule=rule)
    U, D = host(u)[:, idx], host(d)[:, idx]
    out = rel_l2(U, uo), rel_l2(D, do), per_target(U, uo), per_target(D, do)
    say(f"  rel-L2 u {out[0]:.3e} dgamma {out[1]:.3e}; worst target u {out[2]:.3e} dgamma {out[3]:.3e}")
    return out


@pytest.mark.parametrize("kind", KINDS)
def test_config2_full_size_sampled(kind, gpu):
    idx = np.sort(np.random.default_rng(21).choice(65536, 512, replace=False))
    errs = _sampled_parity(W.config2(), kind, idx)
    assert max(errs) <= TOL[kind]


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("rule", [0, 1])
def test_config3_full_size_sampled(kind, rule, gpu):
    """The 1M forward-flight wake in the benchmark's launch, on all 4096 seeded sample
    targets, with the source and the symmetric core rule."""
    c = W.config3()
    assert c["sample"].size == 4096
    errs = _sampled_parity(c, kind, c["sample"], rule)
    assert max(errs) <= TOL[kind]


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("rc,vn", [(0.02, 2), (0.0, 2), (0.02, 1), (0.03, 3)])
def test_segments(kind, rc, vn, gpu):
    c = W.config2(n=3000)
    a, b, gs, x = prepare([c["seg_a"], c["seg_b"], c["seg_gamma"], c["x"]], kind)
    say(f"segments {kind} rc={rc} n={vn}")
    u = vpm.vpm_eval_segments(dev_(a, kind), dev_(b, kind), dev_(gs, kind), dev_(x, kind), rc, vn)
    uo = oracle.segments(a, b, gs, x, rc, vn)
    assert rel_l2(host(u), uo) <= TOL[kind]


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("n_tgt", [1, 65, 8192, 8193])
def test_segments_on_either_side_of_the_few_target_kernel(kind, n_tgt, gpu):
    """Up to 8192 targets take a wavefront per target, beyond one lane per target: both
    against the oracle, accumulating onto a given field."""
    c = W.config2(n=8193)
    a, b, gs, x = prepare([c["seg_a"], c["seg_b"], c["seg_gamma"], c["x"]], kind)
    x = np.ascontiguousarray(x[:, :n_tgt])
    uo = oracle.segments(a, b, gs, x, 0.02, 2)
    # a field of the same size to accumulate onto
    base = (np.random.default_rng(n_tgt).normal(size=(3, n_tgt)) * uo.std()).astype(x.dtype)
    say(f"segments {kind} n_tgt={n_tgt}")
    u = dev_(base, kind)
    vpm.vpm_eval_segments(dev_(a, kind), dev_(b, kind), dev_(gs, kind), dev_(x, kind), 0.02, 2, u_out=u,
                          accumulate=True)
    assert rel_l2(host(u), base.astype(np.float64) + uo) <= TOL[kind]


@pytest.mark.parametrize("kind", KINDS)
def test_segments_full_size_on_particles_and_control_points(kind, gpu):
    c = W.config2()
    a, b, gs, x, y = prepare([c["seg_a"], c["seg_b"], c["seg_gamma"], c["x"], c["ctrl"]], kind)
    u = vpm.vpm_eval_segments(dev_(a, kind), dev_(b, kind), dev_(gs, kind), dev_(x, kind), 0.02, 2)
    idx = np.sort(np.random.default_rng(5).choice(x.shape[1], 2048, replace=False))
    uo = oracle.segments(a, b, gs, x[:, idx], 0.02, 2)
    assert rel_l2(host(u)[:, idx], uo) <= TOL[kind]
    uc = vpm.vpm_eval_segments(dev_(a, kind), dev_(b, kind), dev_(gs, kind), dev_(y, kind), 0.02, 2)
    assert rel_l2(host(uc), oracle.segments(a, b, gs, y, 0.02, 2)) <= TOL[kind]


@pytest.mark.parametrize("kind", KINDS)
def test_batched_persistent_matches_single_launches(kind, gpu):
    import torch
    wakes = W.config5(scale=0.02)
    xs = [prepare([w["x"], w["gamma"], w["sigma"]], kind) for w in wakes]
    off = [0]
    for x, _, _ in xs:
        off.append(off[-1] + x.shape[1])
    X = dev_(np.concatenate([x for x, _, _ in xs], 1), kind)
    G = dev_(np.concatenate([g for _, g, _ in xs], 1), kind)
    S = dev_(np.concatenate([s for _, _, s in xs], 0), kind)
    say(f"batched {kind}: {len(wakes)} wakes, {off[-1]} particles")
    u, d = vpm.vpm_eval_velocity_stretching(X, G, S, src_off=off)
    torch.cuda.synchronize()
    U, D = host(u), host(d)
    for w in (0, 7, 31, 63):
        lo, hi = off[w], off[w + 1]
        u1, d1 = vpm.vpm_eval_velocity_stretching(X[:, lo:hi].contiguous(), G[:, lo:hi].contiguous(),
                                                  S[lo:hi].contiguous())
        # same kernel shape and summation order: equal to rounding of the per-target epilogue
        tight = 1e-14 if kind == "f64" else 1e-6
        assert rel_l2(U[:, lo:hi], host(u1)) <= tight and rel_l2(D[:, lo:hi], host(d1)) <= tight
        x, g, s = xs[w]
        idx = np.arange(0, x.shape[1], max(1, x.shape[1] // 64))
        uo, do = oracle.eval_pairs(x, g, s, x_tgt=x[:, idx], gam_tgt=g[:, idx], excl=idx)
        assert rel_l2(U[:, lo:hi][:, idx], uo) <= TOL[kind]
        assert rel_l2(D[:, lo:hi][:, idx], do) <= TOL[kind]


@pytest.mark.parametrize("kind", KINDS)
def test_diagnostics(kind, gpu):
    x, g, s = prepare(_random_set(3000, 12), kind)
    X, G, S = dev_(x, kind), dev_(g, kind), dev_(s, kind)
    u, d = vpm.vpm_eval_velocity_stretching(X, G, S, sigma_rule=1)
    out = vpm.vpm_diagnostics(X, G, u, d).cpu().numpy()
    ref = oracle.diagnostics(x, g, host(u), host(d))
    # Sums are compared against the scale of their terms (several of them cancel to ~0).
    U, D = host(u), host(d)
    scales = {"sum_gamma": np.abs(g).sum(), "sum_dgamma": np.abs(D).sum(),
              "impulse": np.abs(x).max() * np.abs(g).sum(),
              "impulse_rate": np.abs(U).max() * np.abs(g).sum() + np.abs(x).max() * np.abs(D).sum()}
    for k, sl in (("sum_gamma", slice(0, 3)), ("sum_dgamma", slice(3, 6)), ("impulse", slice(6, 9)),
                  ("impulse_rate", slice(9, 12))):
        assert np.abs(out[sl] - ref[k]).max() <= 1e-14 * scales[k], k
    assert out[12] == 0
    # transposed scheme with symmetric cores conserves total vorticity on the GPU too
    _, do = oracle.eval_pairs(x, g, s, sigma_rule=1)
    scale = np.abs(do).sum()
    assert np.abs(out[3:6]).max() <= (1e-13 if kind == "f64" else 1e-6) * scale


@pytest.mark.parametrize("kind", KINDS)
def test_source_split_for_small_target_sets(kind, gpu):
    """Few targets, many sources: the sources are split into chunks whose FP64 partials are
    added in order; same result as the unsplit launch (no workspace) and the oracle."""
    import torch
    x, g, s = prepare(_random_set(40000, 17, spread=0.5), kind)
    X, G, S = dev_(x, kind), dev_(g, kind), dev_(s, kind)
    idx = np.arange(0, 40000, 400)
    ex = torch.tensor(idx, dtype=torch.int32, device="cuda")
    xt, gt, st = dev_(x[:, idx], kind), dev_(g[:, idx], kind), dev_(s[idx], kind)
    need = vpm.vpm_workspace_size(vpm.F64 if kind == "f64" else vpm.F32C, [0, 40000], [0, len(idx)],
                                  self_eval=False)
    assert need > 0
    u1, d1 = vpm.vpm_eval_velocity_stretching(X, G, S, xt, gt, st, tgt_exclude=ex)
    ws0 = torch.empty(0, dtype=torch.uint8, device="cuda")
    u0, d0 = vpm.vpm_eval_velocity_stretching(X, G, S, xt, gt, st, tgt_exclude=ex, workspace=ws0)
    uo, do = oracle.eval_pairs(x, g, s, x_tgt=x[:, idx], gam_tgt=g[:, idx], excl=idx)
    assert rel_l2(host(u1), uo) <= TOL[kind] and rel_l2(host(d1), do) <= TOL[kind]
    assert rel_l2(host(u0), uo) <= TOL[kind] and rel_l2(host(d0), do) <= TOL[kind]
    # velocity-only control points take the same split path
    uc, _ = vpm.vpm_eval_velocity_stretching(X, G, S, xt)
    uco, _ = oracle.eval_pairs(x, g, s, x_tgt=x[:, idx])
    assert rel_l2(host(uc), uco) <= TOL[kind]


@pytest.mark.parametrize("kind", KINDS)
def test_permutation_invariance(kind, gpu):
    """Shuffling the particles changes every tile and the summation order; results agree to
    rounding (also a guard against LDS races: a missing barrier would not reproduce)."""
    import torch
    c = W.config2(n=20000)
    x, g, s = prepare([c["x"], c["gamma"], c["sigma"]], kind)
    perm = np.random.default_rng(9).permutation(x.shape[1])
    u1, d1 = vpm.vpm_eval_velocity_stretching(dev_(x, kind), dev_(g, kind), dev_(s, kind))
    u2, d2 = vpm.vpm_eval_velocity_stretching(dev_(x[:, perm], kind), dev_(g[:, perm], kind), dev_(s[perm], kind))
    tight = 1e-13 if kind == "f64" else 1e-6  # measured 1.6e-7 (u), 2.2e-7 (dgamma)
    eu, ed = rel_l2(host(u2), host(u1)[:, perm]), rel_l2(host(d2), host(d1)[:, perm])
    say(f"permutation {kind}: rel-L2 u {eu:.2e} dgamma {ed:.2e}")
    assert eu <= tight and ed <= tight
    # and twice the same launch is bitwise identical (no order-dependent reduction)
    u3, d3 = vpm.vpm_eval_velocity_stretching(dev_(x, kind), dev_(g, kind), dev_(s, kind))
    assert torch.equal(u1, u3) and torch.equal(d1, d3)


@pytest.mark.parametrize("kind", KINDS)
def test_batched_full_size_sampled(kind, gpu):
    """All 64 wakes at full size (2.77M particles) in one persistent launch; 48 sampled
    targets per wake against the oracle."""
    wakes = W.config5()
    parts = [prepare([w["x"], w["gamma"], w["sigma"]], kind) for w in wakes]
    off = [0]
    for x, _, _ in parts:
        off.append(off[-1] + x.shape[1])
    X = dev_(np.concatenate([p[0] for p in parts], 1), kind)
    G = dev_(np.concatenate([p[1] for p in parts], 1), kind)
    S = dev_(np.concatenate([p[2] for p in parts], 0), kind)
    say(f"batched full size {kind}: {off[-1]} particles")
    u, d = vpm.vpm_eval_velocity_stretching(X, G, S, src_off=off)
    U, D = host(u), host(d)
    del X, G, S, u, d
    worst = 0.0
    for w, (x, g, s) in enumerate(parts):
        idx = np.sort(np.random.default_rng([31, w]).choice(x.shape[1], 48, replace=False))
        uo, do = oracle.eval_pairs(x, g, s, x_tgt=x[:, idx], gam_tgt=g[:, idx], excl=idx)
        lo = off[w]
        eu, ed = rel_l2(U[:, lo + idx], uo), rel_l2(D[:, lo + idx], do)
        pu, pd = per_target(U[:, lo + idx], uo), per_target(D[:, lo + idx], do)
        worst = max(worst, eu, ed, pu, pd)
        assert max(eu, ed, pu, pd) <= TOL[kind], (w, eu, ed, pu, pd)
    say(f"  worst per-wake rel-L2 or single-target error {worst:.2e}")


@pytest.mark.parametrize("kind", KINDS)
def test_validate_inputs_flags_bad_particles(kind, gpu):
    """Failure detection from the host side: planted bad values are counted on the GPU."""
    x, g, s = prepare(_random_set(1000, 3), kind)
    s = s.copy()
    x = x.copy()
    s[[5, 17]] = [0.0, -1.0]
    s[40] = np.nan
    x[1, 99] = np.inf
    out = vpm.vpm_validate_inputs(dev_(x, kind), dev_(g, kind), dev_(s, kind)).cpu().numpy()
    assert out[0] == 3 and out[1] == 1
    assert not vpm.vpm_check_inputs(dev_(x, kind), dev_(g, kind), dev_(s, kind))  # VPM_ERR_INPUT
    x2, g2, s2 = prepare(_random_set(1000, 3), kind)
    out = vpm.vpm_validate_inputs(dev_(x2, kind), dev_(g2, kind), dev_(s2, kind)).cpu().numpy()
    assert out[0] == 0 and out[1] == 0
    assert vpm.vpm_check_inputs(dev_(x2, kind), dev_(g2, kind), dev_(s2, kind))


def test_autotune_times_every_shape_and_sets_the_plan(gpu):
    """The library's tuner on an 8192-particle forward-flight wake and on six uneven wakes:
    every shape timed, the fastest recorded in the plan (the tuning cache is re-applied after)."""
    from paper_2511_11430_amd import tune
    c = W.config3(n=8192)
    x, g, s = (dev_(W.to_f32(c[k]), "f32c") for k in ("x", "gamma", "sigma"))
    try:
        best, ms = vpm.vpm_autotune(x, g, s, reps=2)
        say(f"autotune 8192: variant {best}, ms {['%.3f' % t for t in ms]}")
        assert len(ms) == vpm.vpm_variant_count() and all(t > 0 for t in ms)
        assert best == 1 + int(np.argmin(ms))
        assert vpm._lib.load().vpm_get_plan(vpm.F32C, 0, 8192) == best
        wakes = W.config5(n_wakes=6, scale=0.05)
        off = [0]
        for w in wakes:
            off.append(off[-1] + w["x"].shape[1])
        cat = lambda k: dev_(np.concatenate([W.to_f32(w[k]) for w in wakes], -1), "f32c")
        best_b, ms_b = vpm.vpm_autotune(cat("x"), cat("gamma"), cat("sigma"), src_off=off, reps=2)
        assert best_b == 1 + int(np.argmin(ms_b))
        assert vpm._lib.load().vpm_get_plan(vpm.F32C, 1, off[-1]) == best_b
    finally:
        for b in (0, 1):
            vpm._lib.load().vpm_set_plan(vpm.F32C, b, 0, 1 << 31, 0)
        tune.apply_cache()


@pytest.mark.parametrize("form", [0, 1, 2, 3, 4])
def test_fma_chain_calibration_kernel(form, gpu):
    """The calibration kernel reports the FMA instruction count it issues and computes the
    chains it claims: each lane's result is the sum of its 8 chains, checked on the host (FP64
    emulation of the FP32 steps, each rounded to FP32, for a short chain)."""
    import ctypes
    import torch
    lanes, fmas = 256, 8
    out = torch.empty(lanes, dtype=torch.float32, device="cuda")
    n = ctypes.c_int64()
    lib = vpm._lib.load()
    assert lib.vpm_fma_chain(lanes, fmas, form, ctypes.c_void_p(out.data_ptr()), ctypes.byref(n), None) == 0
    torch.cuda.synchronize()
    assert n.value == (lanes // 64) * (8, 8, 8, 16, 24)[form] * fmas
    assert lib.vpm_fma_chain(lanes, fmas, 5, ctypes.c_void_p(out.data_ptr()), None, None) == vpm.ENUM_ERROR
    if form >= 3:  # matrix forms: the count above and a finite result
        assert np.all(np.isfinite(host(out)))
        return
    s, t = np.float32(0.999), np.float32(1e-3)
    f32 = np.float32
    got = host(out)
    for lane in (0, 5, 63, 200):
        b = np.frombuffer((np.frombuffer(s.tobytes(), np.int32) + (lane & 7)).tobytes(), np.float32)[0]
        d = f32(t * f32(1 + (lane & 3)))
        a = [f32(lane + k) for k in range(8)]
        for _ in range(fmas):
            for k in range(8):
                if form == 0:
                    a[k] = f32(float(b) * float(d) + float(a[k]))
                elif form == 1:
                    a[k] = f32(float(a[k]) * float(s) + float(t))
                else:
                    a[k] = f32(float(a[k]) * float(b) + float(d))
        acc = a[0]
        for k in range(1, 8):
            acc = f32(acc + a[k])
        assert got[lane] == acc, (lane, got[lane], acc)
