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


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=ITERS - 5)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain device copy of known size (counter scaling)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        if int(os.environ.get("RANK", "0")) == 0:
            print(f"bench.py measures one GPU only: the sampler runs on a single MI355X "
                  f"(asked for --gpus {args.gpus}, WORLD_SIZE {world}); see DESIGN.md for "
                  f"how the path would shard.", file=sys.stderr)
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
    s = chees.Sampler(Xd, yd, PARTICLES, **params)
    print(f"[bench] init done: N={N_ROWS} d={DIM} J={PARTICLES}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        s.step(stats=False)
        s.adapt(stats=False)
    torch.cuda.synchronize()
    c0 = s.counters()
    s.set_timing(True)
    s.timing()
    print(f"[bench] warm-up done ({args.warmup} steps)", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s.step(stats=False)
        s.adapt(stats=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tm = s.timing()
    c1 = s.counters()
    T = t1 - t0
    evals = c1["grad_evals"] - c0["grad_evals"]
    ess_sum = c1["ess_sum"] - c0["ess_sum"]
    print(f"[bench] timed {args.steps} steps in {T:.3f} s", file=sys.stderr, flush=True)

    flops = 4.0 * N_ROWS * DIM * evals
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
                "other_kernels_ms_per_step": {
                    "k_lf_reduce": tm["reduce_ms"] / args.steps,
                    "k_loglik": tm["loglik_ms"] / args.steps}}
    out = {
        "metric": METRIC, "value": evals / T, "unit": "particle-gradient evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * T / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"logistic regression N={N_ROWS} d={DIM}, J={PARTICLES} particles, "
                               f"{ITERS} SMC iterations (warm-up {args.warmup} + timed {args.steps}), "
                               f"<= {NMAX} leapfrog steps, 1-d Halton jitter, systematic resampling",
                   "particles": PARTICLES, "rows": N_ROWS, "dim": DIM, "max_leapfrog": NMAX,
                   "parallelism": "single GPU"},
        "ess_per_s": ess_sum / T,
        "ess_per_grad_eval": ess_sum / (evals + PARTICLES * args.steps),
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(X, y, params, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
