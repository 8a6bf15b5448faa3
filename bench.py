#!/usr/bin/env python3
"""Benchmark of the vortex-particle hot path on one MI355X.

One step = one right-hand-side pass of the forward hot path over the forward-flight
wake (N_p = 1,048,576 particles, 4 blades, advance ratio 0.15, 20 revolutions):
  1. FP32-compensated particle velocity + transposed stretching, all pairs (Eqs. 2-5),
  2. velocity of the 4x8x32 bound-ring lattice (4096 Vatistas-cored segments) on every
     particle (Sec. II.A), accumulated into u,
  3. velocity of the particles and the lattice at the 128 blade control points,
  4. one low-storage RK3 stage update of (x, Gamma) (Sec. II.B),
  5. FP64 invariant diagnostics (total vorticity, impulse, non-finite count).
``value`` is particle-pair interactions per second of the whole step (N_p^2 / step time).

Also measured (same JSON line): the plain FP64 GPU path on the same particles (speedup),
the backward/forward time ratio of the 10-step differentiated program on the 262,144-particle
hover wake (and of one adjoint call), the batched
persistent launch of 64 uneven wakes vs 64 separate launches, the dominant kernel's
roofline position, the error against the FP64 oracle on seeded sample targets, and the
oracle's own throughput on the host cores (cpu_baseline).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--quick]
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK_TFLOPS = 157.3     # MI355X published FP32 vector peak (256 CU x 2.4 GHz x 256 FLOP/clk)
FLOP_PER_PAIR_VS = 45               # velocity + transposed stretching, point-vortex branch
# gradient mode, point-vortex branch: r 3, s^2 5, rsqrt 1, s^-3 and s^-5 3, v = Gamma_j x r 9,
# u += G v 6, A += G Gamma_j 6, Hn v 3, H += (Hn v) r^T 18
FLOP_PER_PAIR_GRAD = 54
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_pair_fwd_f32c_forward_flight_1M.json")
COUNTER_FILE = os.path.join(ROOT, "profiles", "counters_pair_fwd_f32c_forward_flight_1M.json")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("pair_forward.hip", "device_math.h"):
        with open(os.path.join(ROOT, "paper_2511_11430_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(variant):
    """HBM bytes per launch from committed rocprofv3 --pmc counters, if they were taken on the
    same kernel source and kernel shape; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_source_hash() or t.get("variant") != variant:
        return None
    return t.get("bytes_per_launch")


def load_counters(variant):
    """FP32 instruction counters of the pair kernel (rocprofv3 --pmc, calibrated against the
    FMA-chain kernel) from the committed summary, if taken on the same kernel source and shape."""
    try:
        with open(COUNTER_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_source_hash() or t.get("variant") != variant:
        return None
    d = t["derived"]
    keys = ("counter_tflops", "counter_flop_per_pair", "valu_instructions_per_pair", "fp32_fma_per_pair",
            "fp32_mul_per_pair", "fp32_add_per_pair", "fp32_trans_per_pair", "valu_issue_per_cu_clock",
            "clock_ghz")
    out = {k: round(d[k], 4) for k in keys}
    out["source"] = os.path.relpath(COUNTER_FILE, ROOT)
    return out


def fma_chain_run(vpm, torch, stream, form):
    """Best of five timings (ms) and FP32 rate (TFLOP/s) of the library's calibration kernel on
    this GPU, packed FP32 instructions disabled.  form 0: independent FMA chains in the
    accumulating form with register operands, the VALU FMA rate that the pair kernel's
    arithmetic competes with; 1: one operand in a scalar register; 2: three register operands
    (VOP3 encoding); 3: FP32 matrix FMAs (16x16x4); 4: forms 0 and 3 interleaved (the same
    work as 0 and 3 together)."""
    import ctypes
    lanes, fmas = 1 << 22, 2048
    out = torch.empty(lanes, dtype=torch.float32, device="cuda")
    n = ctypes.c_int64()
    lib = vpm._lib.load()
    call = lambda: lib.vpm_fma_chain(lanes, fmas, form, ctypes.c_void_p(out.data_ptr()), ctypes.byref(n),
                                     ctypes.c_void_p(stream.cuda_stream))
    assert call() == 0
    torch.cuda.synchronize()
    best = None
    for _ in range(5):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        call()
        b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        best = ms if best is None else min(best, ms)
    return best, 2.0 * 64 * n.value / (best * 1e-3) / 1e12


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quick", action="store_true", help="skip the FP64, viscous, adjoint and batching legs")
    ap.add_argument("--n", type=int, default=1 << 20, help="particles (default: the full 1,048,576)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain 256 MiB device copy (calibrates rocprofv3 FETCH/WRITE_SIZE)")
    ap.add_argument("--calib-fma", action="store_true",
                    help="also run the library's FMA-chain kernel with a known FP32 FMA instruction count "
                         "(calibrates rocprofv3's SQ_INSTS_VALU_* counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(sharding over GPUs is described, not implemented)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2511_11430_amd as vpm
    from paper_2511_11430_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()

    # ------------------------------------------------------------------ inputs (resident in HBM)
    log("generating the forward-flight wake")
    c = W.config3(n=args.n)
    f32 = lambda a: torch.tensor(np.ascontiguousarray(W.to_f32(a)), dtype=torch.float32, device=dev)
    x0, g0, s = f32(c["x"]), f32(c["gamma"]), f32(c["sigma"])
    sa, sb, sg = f32(c["seg_a"]), f32(c["seg_b"]), f32(c["seg_gamma"])
    ctrl = f32(c["ctrl"])
    N, S, M = x0.shape[1], sa.shape[1], ctrl.shape[1]
    rc, vn = c["core_radius"], c["vatistas_n"]
    x, g = x0.clone(), g0.clone()
    u = torch.empty_like(x)
    dg = torch.empty_like(x)
    qx, qg = torch.zeros_like(x), torch.zeros_like(x)
    uc = torch.empty((3, M), dtype=torch.float32, device=dev)
    diag = torch.empty(13, dtype=torch.float64, device=dev)
    diag_ws = torch.empty(vpm._lib.load().vpm_diagnostics_workspace_size(), dtype=torch.uint8, device=dev)
    # source-split partials of the small control-point target set, allocated once
    ctrl_ws = torch.empty(max(1, vpm.vpm_workspace_size(vpm.F32C, [0, N], [0, M], self_eval=False)),
                          dtype=torch.uint8, device=dev)
    dt = W.DT

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]

    def step(i, timed):
        # particle self-interaction (the dominant kernel), events on its own stream
        if timed:
            ev[i][0].record(stream)
        vpm.vpm_eval_velocity_stretching(x, g, s, u_out=u, dgamma_out=dg)
        if timed:
            ev[i][1].record(stream)
        vpm.vpm_eval_segments(sa, sb, sg, x, rc, vn, u_out=u, accumulate=True)
        vpm.vpm_eval_velocity_stretching(x, g, s, ctrl, u_out=uc, workspace=ctrl_ws)
        vpm.vpm_eval_segments(sa, sb, sg, ctrl, rc, vn, u_out=uc, accumulate=True)
        vpm.vpm_rk3_stage(i % 3, dt, x, g, qx, qg, u, dg)
        vpm.vpm_diagnostics(x, g, u, dg, out=diag, workspace=diag_ws)

    log(f"warmup {args.warmup} step(s), N_p={N}")
    for i in range(args.warmup):
        step(i, False)
    torch.cuda.synchronize()
    x.copy_(x0)
    g.copy_(g0)
    qx.zero_()
    qg.zero_()
    torch.cuda.synchronize()
    log(f"timing {args.steps} step(s)")
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(i, True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    kernel_ms = [a.elapsed_time(b) for a, b in ev]
    k_ms = float(np.mean(kernel_ms))
    pairs = float(N) * float(N)
    value = pairs / (ms_per_step * 1e-3) / 1e9
    achieved = FLOP_PER_PAIR_VS * pairs / (k_ms * 1e-3) / 1e12
    log(f"step {ms_per_step:.1f} ms, pair kernel {k_ms:.1f} ms, {value:.1f} Gpair/s")
    plan = vpm.vpm_get_plan(0, N)
    tpl, wg = vpm.vpm_variant_info(plan)
    pair_kernel = f"k_pair_fwd<float, {tpl} target(s)/lane, {wg} lanes, transposed, source rule> (shape {plan})"
    if args.calib_fma:
        import ctypes
        lanes, fmas = 1 << 20, 1024
        out = torch.empty(lanes, dtype=torch.float32, device=dev)
        n_fma = ctypes.c_int64()
        st_ = vpm._lib.load().vpm_fma_chain(lanes, fmas, 0, ctypes.c_void_p(out.data_ptr()), ctypes.byref(n_fma),
                                            ctypes.c_void_p(stream.cuda_stream))
        torch.cuda.synchronize()
        log(f"calibration k_fma_chain: status {st_}, {n_fma.value} FP32 FMA wavefront instructions "
            f"({lanes} lanes x 8 chains x {fmas})")
        del out
    if args.calib_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    nonfinite = int(diag[12].item())
    t_acc, fma_tf = fma_chain_run(vpm, torch, stream, 0)
    _, fma_tf_s = fma_chain_run(vpm, torch, stream, 1)
    _, fma_tf_3 = fma_chain_run(vpm, torch, stream, 2)
    t_mfma, mfma_tf = fma_chain_run(vpm, torch, stream, 3)
    t_both, _ = fma_chain_run(vpm, torch, stream, 4)
    log(f"FMA chains: {fma_tf:.1f} TFLOP/s (accumulating, register operands), {fma_tf_3:.1f} (three register "
        f"operands), {fma_tf_s:.1f} (scalar operand), {mfma_tf:.1f} (FP32 MFMA); MFMA and VALU interleaved "
        f"{t_both:.3f} ms vs {t_acc:.3f} + {t_mfma:.3f} ms apart; pair kernel {achieved:.1f} TFLOP/s algorithmic")

    result = {
        "metric": "Gpair-interactions/s FP32-comp vs FP64 GPU at 1e-5 relL2; adjoint/fwd time",
        "value": round(value, 2), "unit": "Gpair/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": c["name"] + " + 4x8x32 bound-ring lattice (4096 segments) + 128 control points",
                   "n_particles": N, "n_segments": S, "n_control_points": M, "scheme": "transposed",
                   "sigma_rule": "source", "step": "particle RHS + segments + control points + RK3 stage + "
                                                   "FP64 diagnostics"},
        "roofline": {"bound": "alu", "achieved": round(achieved, 2), "peak": FP32_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
                     "traffic": load_traffic(plan), "kernel": pair_kernel, "kernel_ms": round(k_ms, 3),
                     "flop_per_pair": FLOP_PER_PAIR_VS, "counters": load_counters(plan),
                     "fma_chain_tflops": {"accumulating_register_operands": round(fma_tf, 2),
                                          "three_register_operands": round(fma_tf_3, 2),
                                          "scalar_operand": round(fma_tf_s, 2),
                                          "fp32_mfma_16x16x4": round(mfma_tf, 2),
                                          "mfma_and_valu_interleaved_ms": round(t_both, 3),
                                          "mfma_and_valu_apart_ms": [round(t_acc, 3), round(t_mfma, 3)]},
                     "frac_of_fma_chain": round(achieved / fma_tf, 4)},
        "nonfinite": nonfinite,
        "env": {"gpu": torch.cuda.get_device_name(0),
                "arch": getattr(torch.cuda.get_device_properties(0), "gcnArchName", None),
                "compute_units": torch.cuda.get_device_properties(0).multi_processor_count,
                "rocm": torch.version.hip, "torch": torch.__version__,
                "kernel_ms_min": round(float(np.min(kernel_ms)), 3),
                "kernel_ms_median": round(float(np.median(kernel_ms)), 3)},
    }

    def timed_once(fn, reps=1):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    # ------------------------------------------------------------------ accuracy + CPU baseline
    import oracle
    xs_h, gs_h, ss_h = (W.to_f32(c[k]) for k in ("x", "gamma", "sigma"))
    x.copy_(x0)
    g.copy_(g0)
    vpm.vpm_eval_velocity_stretching(x, g, s, u_out=u, dgamma_out=dg)
    U, D = u.cpu().double().numpy(), dg.cpu().double().numpy()
    threads = len(os.sched_getaffinity(0))
    sample = c["sample"]
    # all seeded sample targets (4096 at the full size); --no-cpu-baseline keeps 64
    m = 64 if args.no_cpu_baseline else len(sample)
    idx = sample[:m]
    log(f"oracle on {m} sample targets x {N} sources, {threads} threads")
    t = time.perf_counter()
    uo, do = oracle.eval_pairs(xs_h, gs_h, ss_h, x_tgt=xs_h[:, idx], gam_tgt=gs_h[:, idx], excl=idx,
                               nthreads=threads)
    t_or = time.perf_counter() - t
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))

    def worst(a, b):
        """largest single-target error, relative to the RMS magnitude of the reference"""
        return float(np.sqrt(((a - b) ** 2).sum(0)).max() / np.sqrt((b * b).sum(0).mean()))

    result["accuracy"] = {"rel_l2_u": rel(U[:, idx], uo), "rel_l2_dgamma": rel(D[:, idx], do),
                          "worst_target_u": worst(U[:, idx], uo), "worst_target_dgamma": worst(D[:, idx], do),
                          "sample_targets": m, "gate": 1e-5, "against": "FP64 oracle"}
    # the symmetric core rule on the same wake: time and accuracy on the same sample targets
    if not args.quick:
        us, ds_ = torch.empty_like(u), torch.empty_like(dg)
        sym_ms = timed_once(lambda: vpm.vpm_eval_velocity_stretching(x, g, s, u_out=us, dgamma_out=ds_,
                                                                     sigma_rule=vpm.SIGMA_SYMMETRIC))
        uso, dso = oracle.eval_pairs(xs_h, gs_h, ss_h, x_tgt=xs_h[:, idx], gam_tgt=gs_h[:, idx], excl=idx,
                                     sig_tgt=ss_h[idx], sigma_rule=oracle.SIGMA_SYMMETRIC, nthreads=threads)
        US, DS = us.cpu().double().numpy(), ds_.cpu().double().numpy()
        result["symmetric_rule"] = {"kernel_ms": round(sym_ms, 3), "gpair_s": round(pairs / (sym_ms * 1e-3) / 1e9, 2),
                                    "rel_l2_u": rel(US[:, idx], uso), "rel_l2_dgamma": rel(DS[:, idx], dso),
                                    "worst_target_u": worst(US[:, idx], uso),
                                    "worst_target_dgamma": worst(DS[:, idx], dso), "sample_targets": m}
        del us, ds_
    if not args.no_cpu_baseline:
        # one core, 4 sample targets
        t = time.perf_counter()
        oracle.eval_pairs(xs_h, gs_h, ss_h, x_tgt=xs_h[:, sample[:4]], gam_tgt=gs_h[:, sample[:4]], excl=sample[:4],
                          nthreads=1)
        t1 = time.perf_counter() - t
        cpu_model = ""
        try:
            with open("/proc/cpuinfo") as f:
                cpu_model = next(ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name"))
        except (OSError, StopIteration):
            pass
        result["cpu_baseline"] = {"value": round(m * N / t_or / 1e9, 4), "unit": "Gpair/s", "cores": threads,
                                  "kind": "oracle",
                                  "sample": f"{m} seeded targets x {N} sources of the same wake, FP64 direct sums "
                                            f"({t_or:.1f} s)", "cpu": cpu_model,
                                  "single_core_gpair_s": round(4 * N / t1 / 1e9, 4)}

    if not args.quick:
        # ------------------------------------------------------------------ Cartesian FMM (Sec. II.B)
        # the same 1M wake and sums through the FMM: depth 6 (leaf width 6.5 sigma_max), three
        # orders (18: within 1e-5 of the direct sums for u and dGamma/dt); error against the
        # direct FP32C sums above and the oracle's sample
        fmm_legs = []
        for lev, order in ((6, 8), (6, 12), (6, 18)):
            fws = torch.empty(vpm.vpm_fmm_workspace_size(N, lev, order, torch.float32), dtype=torch.uint8,
                              device=dev)
            uf, df = torch.empty_like(x), torch.empty_like(x)
            fmm_ms = timed_once(lambda: vpm.vpm_fmm_eval(x0, g0, s, lev, order, u_out=uf, dgamma_out=df,
                                                         workspace=fws), reps=3)
            UF, DF = uf.cpu().double().numpy(), df.cpu().double().numpy()
            fmm_legs.append({"level": lev, "order": order, "ms": round(fmm_ms, 3),
                             "speedup_over_direct": round(k_ms / fmm_ms, 2),
                             "direct_equivalent_gpair_s": round(pairs / (fmm_ms * 1e-3) / 1e9, 1),
                             "rel_l2_u_vs_direct": rel(UF, U), "rel_l2_dgamma_vs_direct": rel(DF, D),
                             "rel_l2_u_vs_oracle": rel(UF[:, idx], uo), "rel_l2_dgamma_vs_oracle": rel(DF[:, idx], do)})
            log(f"fmm level {lev} order {order}: {fmm_ms:.1f} ms")
            del fws, uf, df
        result["fmm"] = {"workload": f"forward-flight skewed wake N_p={N} (self evaluation, FP32C near field, "
                                     f"FP64 expansions)", "legs": fmm_legs}

        # ------------------------------------------------------------------ FP64 GPU path
        x64, g64, s64 = (torch.tensor(np.ascontiguousarray(W.to_f32(c[k])), dtype=torch.float64, device=dev)
                         for k in ("x", "gamma", "sigma"))
        u64, d64 = torch.empty_like(x64), torch.empty_like(x64)
        vpm.vpm_eval_velocity_stretching(x64, g64, s64, u_out=u64, dgamma_out=d64)
        torch.cuda.synchronize()
        f64_runs = []
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            vpm.vpm_eval_velocity_stretching(x64, g64, s64, u_out=u64, dgamma_out=d64)
            e1.record(stream)
            torch.cuda.synchronize()
            f64_runs.append(e0.elapsed_time(e1))
        f64_ms = float(np.median(f64_runs))
        U64, D64 = u64.cpu().numpy(), d64.cpu().numpy()
        result["fp64"] = {"kernel_ms": round(f64_ms, 2), "kernel_ms_min": round(float(np.min(f64_runs)), 2),
                          "reps": len(f64_runs), "gpair_s": round(pairs / (f64_ms * 1e-3) / 1e9, 2),
                          "speedup_f32c_over_f64": round(f64_ms / k_ms, 3),
                          "rel_l2_u": rel(U64[:, idx], uo), "rel_l2_dgamma": rel(D64[:, idx], do),
                          "worst_target_u": worst(U64[:, idx], uo), "worst_target_dgamma": worst(D64[:, idx], do),
                          "gate": 1e-12}
        del x64, g64, s64, u64, d64

        # ------------------------------------------------------------------ viscous term (Eq. 5)
        # gradient-mode pair kernel (u, stretching and du/dx in one pass), Vreman eddy
        # viscosity, PSE diffusion with it, on the same 1M wake (FP32C)
        x.copy_(x0)
        g.copy_(g0)
        Jv = torch.empty((9, N), dtype=torch.float32, device=dev)
        nut = torch.empty(N, dtype=torch.float32, device=dev)
        vol = f32(W.particle_volume(c["sigma"]))
        dv = torch.empty_like(x)
        pse_ws = torch.empty(vpm._lib.load().vpm_diffusion_workspace_size(vpm.F32C, 1, vpm._offsets([0, N])),
                             dtype=torch.uint8, device=dev)

        grad_ms = timed_once(lambda: vpm.vpm_eval_velocity_gradient(x, g, s, u_out=u, dgamma_out=dg, grad_out=Jv))
        vre_ms = timed_once(lambda: vpm.vpm_sgs_vreman(Jv, s, W.C_V, nu_t_out=nut), reps=5)
        pse_ms = timed_once(lambda: vpm.vpm_eval_diffusion(x, g, s, vol, W.NU_AIR, nut, dgamma_out=dv,
                                                          workspace=pse_ws), reps=3)
        result["viscous"] = {
            "workload": c["name"], "nu": W.NU_AIR, "c_v": W.C_V, "volume": "sigma^3",
            "gradient_kernel_ms": round(grad_ms, 3), "stretching_kernel_ms": round(k_ms, 3),
            "gradient_over_stretching": round(grad_ms / k_ms, 3),
            "gradient_tflops": round(FLOP_PER_PAIR_GRAD * pairs / (grad_ms * 1e-3) / 1e12, 2),
            "flop_per_pair_gradient": FLOP_PER_PAIR_GRAD,
            "vreman_ms": round(vre_ms, 4), "pse_ms": round(pse_ms, 3),
            "rhs_with_viscous_ms": round(grad_ms + vre_ms + pse_ms, 3)}
        # the same right-hand side with the FMM's velocity, stretching and gradient (depth 6,
        # order 12), against the direct gradient
        fws = torch.empty(vpm.vpm_fmm_workspace_size(N, 6, 12, torch.float32), dtype=torch.uint8, device=dev)
        uf, df = torch.empty_like(x), torch.empty_like(x)
        Jf = torch.empty((9, N), dtype=torch.float32, device=dev)
        fg_ms = timed_once(lambda: vpm.vpm_fmm_eval(x, g, s, 6, 12, u_out=uf, dgamma_out=df, grad_out=Jf,
                                                    workspace=fws), reps=3)
        nut_f = torch.empty_like(nut)
        vpm.vpm_sgs_vreman(Jf, s, W.C_V, nu_t_out=nut_f)
        Jh, Jfh = Jv.cpu().double().numpy(), Jf.cpu().double().numpy()
        result["viscous"].update({
            "fmm_gradient_ms": round(fg_ms, 3), "fmm_level": 6, "fmm_order": 12,
            "fmm_rel_l2_J_vs_direct": rel(Jfh, Jh),
            "fmm_rel_l2_nu_t_vs_direct": rel(nut_f.cpu().double().numpy(), nut.cpu().double().numpy()),
            "rhs_with_viscous_fmm_ms": round(fg_ms + vre_ms + pse_ms, 3)})
        log(f"viscous RHS: direct gradient {grad_ms:.1f} ms, FMM gradient {fg_ms:.1f} ms")
        del fws, uf, df, Jf, nut_f
        del Jv, nut, vol, dv, pse_ws

        # ------------------------------------------------------------------ closed solver step
        # hover lattice (2 x 8 x 32 rings) turning in its own 65,536-particle wake (FP32C wake,
        # FP64 blade solve): influence update + LU + solve, shedding, three RK3 stages of the
        # wake (velocities and stretching at each), conversion of the oldest row (Eqs. 6-8)
        from paper_2511_11430_amd.solver import Step
        c2 = W.config2()
        geom = W.blade_rings()
        st = Step(geom, omega=W.OMEGA, v_inf=(0.0, 0.0, 0.0), dt=W.DT, core_radius=c2["core_radius"], vatistas_n=2,
                  sigma_p=0.02 * W.R, n_tip=2, n_rows=8, dtype=torch.float32, capacity=1 << 18, device=dev)
        st.add_particles(f32(c2["x"]), f32(c2["gamma"]), f32(c2["sigma"]))
        for _ in range(10):  # build up the line rows so that every timed step converts one
            st.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n_steps = 3
        for _ in range(n_steps):
            st.step()
        torch.cuda.synchronize()
        step_ms = (time.perf_counter() - t0) * 1e3 / n_steps
        result["solver_step"] = {"workload": "hover lattice 2x8x32 rings in a 65,536-particle wake, 8 line rows",
                                 "ms_per_step": round(step_ms, 3), "particles_after": int(st.np),
                                 "panels": int(geom["colloc"].shape[1])}
        del st

        # ------------------------------------------------------------------ adjoint / forward
        c4 = W.config4()
        xa, ga, sa4 = (torch.tensor(np.ascontiguousarray(W.to_f32(c4[k])), dtype=torch.float32, device=dev)
                       for k in ("x", "gamma", "sigma"))
        ua, da = torch.empty_like(xa), torch.empty_like(xa)
        ub, db = torch.randn_like(xa), torch.randn_like(xa)
        xb, gb = torch.zeros_like(xa), torch.zeros_like(xa)

        def timed(fn, reps=3):
            fn()
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(reps):
                fn()
            b.record(stream)
            torch.cuda.synchronize()
            return a.elapsed_time(b) / reps

        fwd_ms = timed(lambda: vpm.vpm_eval_velocity_stretching(xa, ga, sa4, u_out=ua, dgamma_out=da))
        bwd_ms = timed(lambda: vpm.vpm_backward(xa, ga, sa4, ub, db, x_src_bar=xb, gamma_src_bar=gb))
        # the blade lattice acting on the same particles (4096 segments, r_c = 0.02 R): its
        # velocity and stretching, and their adjoint
        c2l = W.config2(n=16)
        la, lb, lg = (torch.tensor(np.ascontiguousarray(W.to_f32(c2l[k])), dtype=torch.float32, device=dev)
                      for k in ("seg_a", "seg_b", "seg_gamma"))
        lrc = float(c2l["core_radius"])
        seg_fwd_ms = timed(lambda: vpm.vpm_eval_segments_gradient(la, lb, lg, xa, lrc, 2, gamma_tgt=ga, want_grad=False,
                                                                  u_out=ua, dgamma_out=da, accumulate=True))
        seg_bwd_ms = timed(lambda: vpm.vpm_segments_backward(la, lb, lg, xa, lrc, 2, ub, db, gamma_tgt=ga,
                                                             x_bar=xb, gamma_bar=gb))
        # the differentiation workload's whole program: 10 RK3 steps (30 stages) on the
        # 262,144-particle hover wake and the loss on 128 control points, forward with every
        # stage's input kept in HBM, then the backward pass over the checkpoints
        from paper_2511_11430_amd import autograd as AG
        y4 = torch.tensor(np.ascontiguousarray(W.to_f32(c4["ctrl"])), dtype=torch.float32, device=dev)
        programs = {}
        for kind, sdt in (("mixed", torch.float64), ("f32c", torch.float32)):
            X4, G4 = xa.to(sdt), ga.to(sdt)

            def run_fwd(ck):
                return AG.rk3_forward(X4, G4, sa4, c4["n_steps"], c4["dt"], y4, checkpoints=ck)

            run_fwd(None)
            torch.cuda.synchronize()
            t0p = time.perf_counter()
            run_fwd(None)
            torch.cuda.synchronize()
            plain_ms = (time.perf_counter() - t0p) * 1e3
            ck = []
            t0p = time.perf_counter()
            _, _, ucp, lossp, fin = run_fwd(ck)
            torch.cuda.synchronize()
            pf_ms = (time.perf_counter() - t0p) * 1e3
            t0p = time.perf_counter()
            AG.rk3_backward(ck, fin, sa4, ucp, y4, c4["dt"], sdt)
            torch.cuda.synchronize()
            pb_ms = (time.perf_counter() - t0p) * 1e3
            ck_mb = sum(a.numel() * a.element_size() + b.numel() * b.element_size() for a, b in ck) / 2 ** 20
            programs[kind] = {"state": "FP64 state, FP32C sums" if kind == "mixed" else "FP32 state, FP32C sums",
                              "forward_ms": round(plain_ms, 1), "forward_with_checkpoints_ms": round(pf_ms, 1),
                              "backward_ms": round(pb_ms, 1), "bwd_over_fwd": round(pb_ms / pf_ms, 3),
                              "checkpoints_mib": round(ck_mb, 1), "stages": len(ck)}
            log(f"program {kind}: forward {pf_ms:.0f} ms, backward {pb_ms:.0f} ms")
            del ck, fin, ucp, X4, G4
        result["adjoint"] = {"workload": c4["name"] + ", 128 control points",
                             "program": programs, "program_bwd_over_fwd": programs["mixed"]["bwd_over_fwd"],
                             "target": 3.0,
                             "single_call": {"what": "one vpm_backward against one forward evaluation",
                                             "fwd_ms": round(fwd_ms, 3), "bwd_ms": round(bwd_ms, 3),
                                             "bwd_over_fwd": round(bwd_ms / fwd_ms, 3)},
                             "lattice": {"n_segments": int(la.shape[1]), "fwd_ms": round(seg_fwd_ms, 3),
                                         "bwd_ms": round(seg_bwd_ms, 3),
                                         "bwd_over_fwd": round(seg_bwd_ms / seg_fwd_ms, 3)}}
        del xa, ga, sa4, ua, da, ub, db, xb, gb, la, lb, lg, y4

        # ------------------------------------------------------------------ batched persistent
        wakes = W.config5()
        off = [0]
        for w in wakes:
            off.append(off[-1] + w["x"].shape[1])
        cat = lambda k: np.concatenate([W.to_f32(w[k]) for w in wakes], axis=-1)
        xw = torch.tensor(cat("x"), dtype=torch.float32, device=dev)
        gw = torch.tensor(cat("gamma"), dtype=torch.float32, device=dev)
        sw = torch.tensor(cat("sigma"), dtype=torch.float32, device=dev)
        uw, dw = torch.empty_like(xw), torch.empty_like(xw)
        ws = torch.empty(vpm.vpm_workspace_size(vpm.F32C, off), dtype=torch.uint8, device=dev)
        views = [(xw[:, a:b], gw[:, a:b], sw[a:b], uw[:, a:b], dw[:, a:b]) for a, b in zip(off[:-1], off[1:])]

        def separate():
            for xv, gv, sv, uv, dv in views:
                vpm.vpm_eval_velocity_stretching(xv, gv, sv, u_out=uv, dgamma_out=dv)

        t_batched = timed(lambda: vpm.vpm_eval_velocity_stretching(xw, gw, sw, u_out=uw, dgamma_out=dw,
                                                                    src_off=off, workspace=ws), reps=2)
        t_sep = timed(separate, reps=2)
        sq = float(sum((b - a) ** 2 for a, b in zip(off[:-1], off[1:])))
        # per-wake error of the persistent launch on 256 seeded targets per wake
        UW, DW = uw.cpu().double().numpy(), dw.cpu().double().numpy()
        worst_u = worst_d = 0.0
        for wi, w in enumerate(wakes):
            a0, b0 = off[wi], off[wi + 1]
            xw_h, gw_h, sw_h = (W.to_f32(w[k]) for k in ("x", "gamma", "sigma"))
            it = np.sort(np.random.default_rng([5, wi]).choice(b0 - a0, min(256, b0 - a0), replace=False))
            uo_w, do_w = oracle.eval_pairs(xw_h, gw_h, sw_h, x_tgt=xw_h[:, it], gam_tgt=gw_h[:, it], excl=it,
                                           nthreads=threads)
            worst_u = max(worst_u, rel(UW[:, a0:b0][:, it], uo_w))
            worst_d = max(worst_d, rel(DW[:, a0:b0][:, it], do_w))
        result["batched"] = {"n_wakes": len(wakes), "n_particles": off[-1], "sum_n_sq": sq,
                             "persistent_ms": round(t_batched, 3), "separate_ms": round(t_sep, 3),
                             "gpair_s": round(sq / (t_batched * 1e-3) / 1e9, 2),
                             "speedup": round(t_sep / t_batched, 3),
                             "max_wake_rel_l2_u": worst_u, "max_wake_rel_l2_dgamma": worst_d,
                             "targets_per_wake": 256}
        del xw, gw, sw, uw, dw, ws, views

        # ------------------------------------------------------------------ C1: FP64, 4096 particles
        c1 = W.config1()
        x1, g1, s1 = (torch.tensor(c1[k], dtype=torch.float64, device=dev) for k in ("x", "gamma", "sigma"))
        u1, d1 = torch.empty_like(x1), torch.empty_like(x1)
        c1_ms = timed_once(lambda: vpm.vpm_eval_velocity_stretching(x1, g1, s1, u_out=u1, dgamma_out=d1), reps=10)
        t = time.perf_counter()
        uo1, do1 = oracle.eval_pairs(c1["x"], c1["gamma"], c1["sigma"], nthreads=threads)
        or1 = time.perf_counter() - t
        n1 = c1["x"].shape[1]
        result["c1_fp64"] = {"workload": c1["name"], "gpu_ms": round(c1_ms, 4), "oracle_s": round(or1, 3),
                             "gpu_gpair_s": round(n1 * n1 / (c1_ms * 1e-3) / 1e9, 2),
                             "oracle_gpair_s": round(n1 * n1 / or1 / 1e9, 4), "oracle_cores": threads,
                             "rel_l2_u": rel(u1.cpu().numpy(), uo1), "rel_l2_dgamma": rel(d1.cpu().numpy(), do1),
                             "gate": 1e-12}

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
