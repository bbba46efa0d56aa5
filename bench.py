#!/usr/bin/env python3
"""Throughput of the SMC / ChEES-HMC hot path on one MI355X.

Workload (synthetic, seeded): Bayesian logistic regression, N = 10000 rows,
d = 100 standardised N(0,1) features, beta* ~ N(0, 0.25 I), prior N(0, I);
J = 8192 particles, 50 SMC iterations (warm-up adaptation for the first 25),
at most 64 leapfrog steps per jittered trajectory, 1-d Halton jitter,
systematic resampling at J_eff < J/2, FP32 trajectories.

A step is one SMC iteration (smc_step + chees_adapt) over all particles.
`value` = particle-gradient evaluations per second = sum_j n_j over the timed
steps / wall time (stream-synchronised on both sides).  Prints one JSON line.
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

N_ROWS, DIM, PARTICLES, ITERS, NMAX = 10000, 100, 8192, 50, 64
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_BF16_MFMA_TFLOPS = 2500.0
METRIC = "particle-gradient evals/s and ESS/s vs plain FP32 GPU at matched posterior error"
KERNEL_SRCS = [os.path.join(ROOT, "paper_2504_02627_amd", "csrc", f)
               for f in ("smc_kernels.hip", "smc_internal.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "leapfrog_traffic.json")


def kernel_hash():
    h = hashlib.sha256()
    for p in KERNEL_SRCS:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def workload_params():
    from paper_2504_02627_amd import synth
    eps0 = synth.default_step_size(N_ROWS, DIM)
    return dict(step_size=eps0, traj_length=eps0 * NMAX / 2, max_leapfrog=NMAX,
                num_warmup=ITERS // 2, seed=2, jitter="halton1d", resampling="systematic")


def traffic_for_current_kernel():
    """HBM bytes per leapfrog launch from the committed rocprofv3 counter runs,
    valid only for the kernel source they were taken on."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha256_16") != kernel_hash():
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(X, y, params, seconds):
    """The oracle, as it stands, on a bounded sample of the same workload."""
    import numpy as np
    from threadpoolctl import threadpool_info
    from oracle import philox, smc as O
    Js = 512
    t = O.LogisticRegression(X.astype(np.float64), y.astype(np.float64))
    th0 = philox.normals_np(params["seed"], Js, 0, philox.STREAM_INIT, DIM)
    o = O.OracleSMC(t, Js, theta0=th0, **params)
    evals, iters = 0, 0
    t0 = time.perf_counter()
    while True:
        st = o.step()
        o.adapt()
        evals += st["grad_evals"]
        iters += 1
        if time.perf_counter() - t0 >= seconds or iters >= ITERS:
            break
    dt = time.perf_counter() - t0
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    return {"value": evals / dt, "unit": "particle-gradient evals/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"{Js} particles of the same workload, first {iters} SMC iterations "
                      f"({evals} particle-gradient evals in {dt:.1f} s, FP64 numpy, "
                      f"{threads} BLAS threads)"}


def _steps(s, n):
    for _ in range(n):
        s.step(stats=False)
        s.adapt(stats=False)


def _moments(s):
    import torch
    theta, logw, _ = s.state()
    w = torch.softmax(logw, 0)
    th = theta.double()
    mean = (w[:, None] * th).sum(0)
    var = (w[:, None] * (th - mean) ** 2).sum(0)
    return mean.cpu().numpy(), var.cpu().numpy()


def run_form(Xd, yd, params, precision, args):
    """One form of the sampler on the workload.

    Pass 1 (the timed region of `value`): warm-up, then the timed iterations
    replayed from the captured iteration graph (smc_run), with no per-kernel
    instrumentation.  Pass 2: the same with eager smc_step + chees_adapt calls.
    Pass 3: the same seed from scratch -- the run is deterministic, so it
    repeats exactly the same kernels -- eager, with HIP events around every
    leapfrog, reduction and log-likelihood launch on the sampler's stream, for
    the per-kernel averages.  Replicates with other seeds give the
    spread of the final posterior moments (untimed)."""
    import torch
    from paper_2504_02627_amd import chees

    def timed(seed, instrument, graph):
        s = chees.Sampler(Xd, yd, PARTICLES, precision=precision, **dict(params, seed=seed))
        if graph:
            s.run(args.warmup)          # the first call captures the iteration graph
        else:
            _steps(s, args.warmup)
        torch.cuda.synchronize()
        c0 = s.counters()
        if instrument:
            s.set_timing(True)
            s.timing()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if graph:
            s.run(args.steps)
        else:
            _steps(s, args.steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        tm = s.timing() if instrument else None
        c1 = s.counters()
        return s, t1 - t0, c1["grad_evals"] - c0["grad_evals"], c1["ess_sum"] - c0["ess_sum"], tm

    s, T, evals, ess_sum, _ = timed(params["seed"], False, not args.eager)
    print(f"[bench] {precision}: timed {args.steps} steps in {T:.3f} s", file=sys.stderr, flush=True)
    moments = [_moments(s)]
    s.close()
    s1, T1, evals1, _, _ = timed(params["seed"], False, args.eager)
    s1.close()
    s2, T2, evals2, _, tm = timed(params["seed"], True, False)
    s2.close()
    if evals2 != evals or evals1 != evals:
        raise RuntimeError("the replayed passes did not repeat the timed run")
    for r in range(1, args.replicates):
        sr = chees.Sampler(Xd, yd, PARTICLES, precision=precision,
                           **dict(params, seed=params["seed"] + 1000 * r))
        sr.run(args.warmup + args.steps)
        moments.append(_moments(sr))
        sr.close()
    print(f"[bench] {precision}: instrumented pass {T2:.3f} s, {len(moments)} replicates",
          file=sys.stderr, flush=True)
    return {"evals": evals, "ess_sum": ess_sum, "seconds": T, "timing": tm,
            "other_mode_seconds": T1, "instrumented_seconds": T2, "moments": moments}


def long_reference(Xd, yd, params, precision, iters, pool):
    """Posterior moments from one long run (seed 7777, twice the particles): the
    weighted means and variances averaged over the last `pool` of `iters` SMC
    iterations."""
    import numpy as np
    from paper_2504_02627_amd import chees
    s = chees.Sampler(Xd, yd, 2 * PARTICLES, precision=precision, **dict(params, seed=7777))
    ms, vs = [], []
    for k in range(iters):
        s.step(stats=False)
        s.adapt(stats=False)
        if k >= iters - pool:
            m, v = _moments(s)
            ms.append(m)
            vs.append(v)
    s.close()
    return np.mean(ms, 0), np.mean(vs, 0)


def moment_match(ref, a, b, ta, tb):
    """Posterior error of the two forms at the end of the workload, over R
    replicate seeds each, against the long-run reference moments `ref`:
    RMS over dimensions and replicates of (mean - ref_mean) / ref_sd (bias and
    spread together), the same for the variances relative to ref_var, the
    per-dimension two-sample z of the forms' replicate-averaged means, and the
    efficiency at matched error (T_a err_a^2) / (T_b err_b^2)."""
    import numpy as np
    rm, rv = ref
    sd = np.sqrt(rv)
    ma = np.array([m for m, _ in a]); mb = np.array([m for m, _ in b])
    va = np.array([v for _, v in a]); vb = np.array([v for _, v in b])
    R = len(a)
    ea = float(np.sqrt(np.mean(((ma - rm) / sd) ** 2)))
    eb = float(np.sqrt(np.mean(((mb - rm) / sd) ** 2)))
    out = {"replicates": R, "reference": "FP32 form, 2J particles, seed 7777, moments averaged "
                                         "over the last third of a long run",
           "mean_error_rms_ref_sd": [ea, eb],
           "var_error_rms_rel": [float(np.sqrt(np.mean((va / rv - 1) ** 2))),
                                 float(np.sqrt(np.mean((vb / rv - 1) ** 2)))],
           "efficiency_at_matched_error_vs_f32": float((ta * ea ** 2) / (tb * eb ** 2))}
    if R >= 2:
        sa, sb = ma.std(0, ddof=1), mb.std(0, ddof=1)
        z = np.abs(ma.mean(0) - mb.mean(0)) / np.sqrt(sa ** 2 / R + sb ** 2 / R)
        out.update({"max_abs_z_between_forms": float(z.max()),
                    "frac_dims_within_3se_between_forms": float(np.mean(z <= 3.0))})
    return out


def run_workload(Xs, ys, J, params, iters, burn):
    """One sampler over `iters` SMC iterations (captured-graph replay for the
    wall time, then the same seed again eagerly with per-kernel events).
    Returns throughput, ESS figures after `burn` iterations and kernel times."""
    import torch
    from paper_2504_02627_amd import chees
    s = chees.Sampler(Xs, ys, J, **params)
    s.run(1)
    torch.cuda.synchronize()
    c0 = s.counters()
    t0 = time.perf_counter()
    s.run(iters - 1)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    c1 = s.counters()
    s.close()
    s = chees.Sampler(Xs, ys, J, **params)
    s.set_timing(True)
    ess_post, ge_post = 0.0, 0
    for k in range(iters):
        st = s.step()
        s.adapt(stats=False)
        if k >= burn:
            ess_post += st["ess"]
            ge_post += st["grad_evals"] + J * s.B
    tm = s.timing()
    s.close()
    evals = c1["grad_evals"] - c0["grad_evals"]
    return {"ms_per_iteration": 1e3 * T / (iters - 1), "evals_per_s": evals / T,
            "ess_per_s": (c1["ess_sum"] - c0["ess_sum"]) / T,
            "ess_per_grad_eval_after_burn_in": ess_post / max(1, ge_post),
            "kernel_ms_per_iteration": {k[:-3]: round(v / iters, 4) for k, v in tm.items()
                                        if k.endswith("_ms")},
            "leapfrog_launches": tm["leapfrog_launches"]}


def other_workloads(args):
    """The batched form, the precision form on the small model and the flow
    preconditioner on the Toeplitz model, with their comparison forms."""
    import numpy as np
    import torch
    from paper_2504_02627_amd import synth
    dev = torch.device("cuda:0")
    out = {}
    # batched form: 64 posteriors, N ~ U[500, 20000], d ~ U[10, 200], J = 1024 each
    data = synth.batched_logistic(64)
    Xs = [torch.from_numpy(X).to(dev) for X, _, _ in data]
    ys = [torch.from_numpy(y).to(dev) for _, y, _ in data]
    eps = min(synth.default_step_size(X.shape[0], X.shape[1]) for X, _, _ in data)
    p = dict(step_size=eps, traj_length=eps * 32, max_leapfrog=64, num_warmup=25, seed=4)
    r = run_workload(Xs, ys, 1024, p, args.other_iters, args.other_iters // 2)
    r["workload"] = ("64 logistic posteriors, N_b ~ U[500, 20000], d_b ~ U[10, 200], J = 1024 "
                     "each, FP32 trajectories, one context")
    r["leapfrog_kernel_note"] = ("achieved TFLOP/s not reported: the flop count per launch "
                                 "mixes posteriors of different N_b d_b")
    out["batched_64_posteriors"] = r
    print("[bench] batched form done", file=sys.stderr, flush=True)
    # precision form on the small model: N = 200, d = 5, J = 16384
    X, y, _ = synth.small_logistic()
    Xd, yd = torch.from_numpy(X).to(dev), torch.from_numpy(y).to(dev)
    e5 = synth.default_step_size(200, 5)
    p = dict(step_size=e5, traj_length=e5 * 32, max_leapfrog=64, num_warmup=10, seed=1,
             adapt_step_size=True)
    out["small_model_J16384"] = {
        prec: run_workload(Xd if prec == "f32" else Xd.to(torch.bfloat16), yd, 16384,
                           dict(p, precision=prec), 20, 10)
        for prec in ("f32", "bf16")}
    # the same with one leapfrog launch per step instead of whole trajectories
    os.environ["CHEES_SMC_PER_STEP"] = "1"
    try:
        out["small_model_J16384"]["f32_per_step_launches"] = run_workload(
            Xd, yd, 16384, dict(p, precision="f32"), 20, 10)
    finally:
        del os.environ["CHEES_SMC_PER_STEP"]
    out["small_model_J16384"]["workload"] = ("logistic N=200, d=5, J=16384, 20 iterations; bf16: "
                                             "X stored in bfloat16; whole trajectories in one "
                                             "launch unless named per-step")
    # the small model at J = 256 (latency-bound: 16 waves)
    out["small_model_J256"] = run_workload(Xd, yd, 256, dict(p, precision="f32"), 20, 10)
    out["small_model_J256"]["workload"] = "logistic N=200, d=5, J=256, 20 iterations, FP32"
    print("[bench] small model done", file=sys.stderr, flush=True)
    # flow preconditioner on the Toeplitz model: N = 5000, d = 100, J = 4096
    X, y, _ = synth.toeplitz_logistic()
    Xd, yd = torch.from_numpy(X).to(dev), torch.from_numpy(y).to(dev)
    e0 = synth.default_step_size(5000, 100)
    base = dict(max_leapfrog=64, num_warmup=25, seed=3, adapt_step_size=True)
    forms = {
        "unit_mass": dict(step_size=e0, traj_length=e0 * 32),
        "diagonal_mass": dict(step_size=0.05, traj_length=1.6, precond="diag"),
        "flow_base_only": dict(step_size=0.3, traj_length=2.4, precond="flow", flow_layers=0),
        "flow_4x128_trained": dict(step_size=0.3, traj_length=2.4, precond="flow", flow_layers=4,
                                   flow_train_steps=10, flow_lr=2e-5),
    }
    fl = {}
    for name, f in forms.items():
        fl[name] = run_workload(Xd, yd, 4096, dict(base, **f), 50, 25)
    fl["workload"] = ("logistic N=5000, d=100, rows ~ N(0, S), S_ij = 0.95^|i-j|, J=4096, "
                      "50 iterations (25 warm-up), FP32 likelihood")
    out["toeplitz_flow"] = fl
    print("[bench] flow forms done", file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=ITERS - 5)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-bf16", action="store_true", help="skip the BF16 precision form")
    ap.add_argument("--no-other", action="store_true",
                    help="skip the batched, small-model and flow workloads")
    ap.add_argument("--other-iters", type=int, default=50)
    ap.add_argument("--eager", action="store_true",
                    help="time eager step/adapt calls for `value` (default: graph replay)")
    ap.add_argument("--ref-iters", type=int, default=300,
                    help="iterations of the long reference runs (last third pooled)")
    ap.add_argument("--replicates", type=int, default=10,
                    help="seeds per form for the posterior-error comparison")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain device copy of known size (counter scaling)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        if int(os.environ.get("RANK", "0")) == 0:
            print(f"bench.py measures one GPU only: the sampler runs on a single MI355X "
                  f"(asked for --gpus {args.gpus}, WORLD_SIZE {world}); particles would "
                  f"shard across GPUs with a few FP64 all-reduces per iteration and a "
                  f"particle exchange at resampling; only the single-GPU path is implemented.",
                  file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2504_02627_amd import chees, synth

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        n = 256 << 20
        a = torch.ones(n // 4, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "launches": 3}))
        return

    X, y, _ = synth.large_logistic()
    params = workload_params()
    Xd = torch.from_numpy(X).to(dev)
    yd = torch.from_numpy(y).to(dev)

    f32 = run_form(Xd, yd, params, "f32", args)
    flops = 4.0 * N_ROWS * DIM * f32["evals"]
    tm = f32["timing"]
    lf_s = tm["leapfrog_ms"] / 1e3
    achieved = flops / lf_s / 1e12 if lf_s > 0 else 0.0
    launches = max(1, tm["leapfrog_launches"])
    traffic = traffic_for_current_kernel()
    roofline = {"bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK_FP32_MFMA_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_MFMA_TFLOPS, 4),
                "traffic": traffic,
                "kernel": "k_lf_partial<7>: fused leapfrog step (drift, X theta'^T -> sigmoid -> "
                          "R X on v_mfma_f32_16x16x4f32) over a data-row split",
                "algorithmic_flops_per_launch": flops / launches,
                "avg_launch_ms": tm["leapfrog_ms"] / launches, "launches": tm["leapfrog_launches"],
                "flop_unit": "4 N d per particle-gradient evaluation",
                "timing_pass": "HIP events on the sampler stream, same-seed replay of the timed steps "
                               f"({1e3 * f32['instrumented_seconds'] / args.steps:.3f} ms/step with events)",
                "other_kernels_ms_per_step": {
                    "k_lf_reduce": tm["reduce_ms"] / args.steps,
                    "k_loglik": tm["loglik_ms"] / args.steps}}
    T = f32["seconds"]
    out = {
        "metric": METRIC, "value": f32["evals"] / T, "unit": "particle-gradient evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * T / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"logistic regression N={N_ROWS} d={DIM}, J={PARTICLES} particles, "
                               f"{ITERS} SMC iterations (warm-up {args.warmup} + timed {args.steps}), "
                               f"<= {NMAX} leapfrog steps, 1-d Halton jitter, systematic resampling",
                   "particles": PARTICLES, "rows": N_ROWS, "dim": DIM, "max_leapfrog": NMAX,
                   "parallelism": "single GPU"},
        "ms_per_step_other_mode": 1e3 * f32["other_mode_seconds"] / args.steps,
        "launch_mode": "eager smc_step + chees_adapt" if args.eager else
                       "captured iteration graph (smc_run); other mode = eager calls",
        "ess_per_s": f32["ess_sum"] / T,
        "ess_per_grad_eval": f32["ess_sum"] / (f32["evals"] + PARTICLES * args.steps),
        "roofline": roofline,
    }
    if not args.no_bf16:
        bf = run_form(Xd, yd, params, "bf16", args)
        tb = bf["timing"]
        fl_b = 4.0 * N_ROWS * DIM * bf["evals"]
        ach_b = fl_b / (tb["leapfrog_ms"] / 1e3) / 1e12 if tb["leapfrog_ms"] > 0 else 0.0
        print("[bench] long-run reference moments ...", file=sys.stderr, flush=True)
        ref = long_reference(Xd, yd, params, "f32", args.ref_iters, args.ref_iters // 3)
        ref_b = long_reference(Xd, yd, params, "bf16", args.ref_iters, args.ref_iters // 3)
        z = moment_match(ref, f32["moments"], bf["moments"], T, bf["seconds"])
        z["bf16_long_run_vs_reference_mean_rms_sd"] = float(
            np.sqrt(np.mean((ref_b[0] - ref[0]) ** 2 / ref[1])))
        z["bf16_long_run_vs_reference_var_rms_rel"] = float(
            np.sqrt(np.mean((ref_b[1] / ref[1] - 1) ** 2)))
        out["forms"] = {"bf16": {
            "what": "same workload and target: X held in FP32 for the energies (compensated "
                    "FP32 sums, weights exact for the FP32-data posterior) and in bfloat16 for "
                    "the trajectory gradients on v_mfma_f32_16x16x32_bf16 (FP32 accumulation); "
                    "LSE/ESS/evidence FP64",
            "value": bf["evals"] / bf["seconds"], "unit": "particle-gradient evals/s",
            "ms_per_step": 1e3 * bf["seconds"] / args.steps,
            "ess_per_s": bf["ess_sum"] / bf["seconds"],
            "speedup_vs_f32_evals": (bf["evals"] / bf["seconds"]) / (f32["evals"] / T),
            "speedup_vs_f32_ess_per_s": (bf["ess_sum"] / bf["seconds"]) / (f32["ess_sum"] / T),
            "leapfrog_kernel": {"achieved": round(ach_b, 2), "peak": PEAK_BF16_MFMA_TFLOPS,
                                "unit": "TFLOP/s", "frac": round(ach_b / PEAK_BF16_MFMA_TFLOPS, 4),
                                "avg_launch_ms": tb["leapfrog_ms"] / max(1, tb["leapfrog_launches"])},
            "other_kernels_ms_per_step": {"k_lf_reduce": tb["reduce_ms"] / args.steps,
                                          "k_loglik": tb["loglik_ms"] / args.steps},
            "instrumented_ms_per_step": 1e3 * bf["instrumented_seconds"] / args.steps,
            "ms_per_step_other_mode": 1e3 * bf["other_mode_seconds"] / args.steps,
            "posterior_vs_f32": z,
        }}
    if not args.no_other:
        out["other_workloads"] = other_workloads(args)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(X, y, params, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
