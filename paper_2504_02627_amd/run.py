"""Run the sampler on one of the synthetic workloads and log every iteration
as a JSON line (device library only).

Per iteration: J_eff after the move and the one that decided resampling, the
resampling flag, mean acceptance, mean and largest n_j, gradient evaluations,
L and eps used, the ChEES estimate and its gradient, log Z_hat, and the wall
time of the iteration (step + adaptation, synchronised).  A checkpoint of the
final state can be written (smc_save; the run's schedule beside it in FILE.json)
and a run resumed from one (smc_load), keeping the interrupted run's schedule.

Workloads (seeded, see synth.py): small (N = 200, d = 5), large (N = 10000,
d = 100), toeplitz (N = 5000, d = 100, rows correlated 0.95^|i-j|), batched
(64 posteriors of mixed sizes).

Usage: python -m paper_2504_02627_amd.run --workload small --iterations 50
           [--particles J] [--precision f32|bf16] [--jitter halton1d ...]
           [--precond none|diag|flow] [--step-size EPS] [--traj-length L]
           [--adapt-step-size none|adam|dual_averaging] [--flow-layers K]
           [--flow-train-steps S] [--flow-lr LR] [--jsonl FILE] [--save FILE]
           [--resume FILE]
"""

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

DEFAULT_J = {"small": 16384, "large": 8192, "toeplitz": 4096, "batched": 1024}


def problem(name):
    """(list of X, list of y) as numpy arrays."""
    from paper_2504_02627_amd import synth
    if name == "small":
        data = [synth.small_logistic()]
    elif name == "large":
        data = [synth.large_logistic()]
    elif name == "toeplitz":
        data = [synth.toeplitz_logistic()]
    elif name == "batched":
        data = synth.batched_logistic(64)
    else:
        raise ValueError(name)
    return [X for X, _, _ in data], [y for _, y, _ in data]


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--workload", default="small", choices=sorted(DEFAULT_J))
    ap.add_argument("--iterations", type=int, default=50)
    ap.add_argument("--particles", type=int, default=0)
    ap.add_argument("--precision", default="f32", choices=["f32", "bf16"])
    ap.add_argument("--jitter", default="halton1d")
    ap.add_argument("--precond", default="none", choices=["none", "diag", "flow"])
    ap.add_argument("--max-leapfrog", type=int, default=64)
    ap.add_argument("--step-size", type=float, default=0.0,
                    help="initial eps (default: the workload's conservative step size)")
    ap.add_argument("--traj-length", type=float, default=0.0,
                    help="initial L (default: eps * max_leapfrog / 2)")
    ap.add_argument("--adapt-step-size", default="none", choices=["none", "adam", "dual_averaging"])
    ap.add_argument("--flow-layers", type=int, default=4)
    ap.add_argument("--flow-train-steps", type=int, default=10)
    ap.add_argument("--flow-lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--jsonl", default=None, help="write the per-iteration records here")
    ap.add_argument("--save", default=None, help="write a checkpoint of the final state")
    ap.add_argument("--resume", default=None, help="start from a checkpoint")
    a = ap.parse_args(argv)

    import torch
    from paper_2504_02627_amd import chees, synth
    dev = torch.device("cuda:0")
    Xs, ys = problem(a.workload)
    J = a.particles or DEFAULT_J[a.workload]
    eps = a.step_size or min(synth.default_step_size(X.shape[0], X.shape[1]) for X in Xs)
    L = a.traj_length or eps * a.max_leapfrog / 2
    Xd = [torch.from_numpy(X).to(dev) for X in Xs]
    if a.precision == "bf16":
        Xd = [X.to(torch.bfloat16) for X in Xd]
    yd = [torch.from_numpy(y).to(dev) for y in ys]
    # the schedule of the whole run (warm-up boundary, jitter columns K) comes
    # from the checkpoint's own record when resuming, so that a resumed run
    # continues the interrupted one rather than starting another schedule
    sched = dict(num_warmup=a.iterations // 2, num_iterations=a.iterations, jitter=a.jitter)
    if a.resume:
        with open(a.resume + ".json") as f:
            rec = json.load(f)
        if rec["jitter"] != a.jitter:
            raise SystemExit(f"--resume: the checkpoint ran jitter {rec['jitter']}, not {a.jitter}")
        sched.update(num_warmup=rec["num_warmup"], num_iterations=rec["num_iterations"])
    s = chees.Sampler(Xd if len(Xd) > 1 else Xd[0], yd if len(yd) > 1 else yd[0], J,
                      step_size=eps, traj_length=L, max_leapfrog=a.max_leapfrog,
                      precision=a.precision, precond=a.precond,
                      adapt_step_size=a.adapt_step_size, flow_layers=a.flow_layers,
                      flow_train_steps=a.flow_train_steps, flow_lr=a.flow_lr, seed=a.seed,
                      **sched)
    if a.resume:
        with open(a.resume, "rb") as f:
            s.load(f.read())
    out = open(a.jsonl, "w") if a.jsonl else sys.stdout
    for _ in range(a.iterations):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = s.step()
        s.adapt(stats=False)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0)
        n = s.trace()["n"].cpu().numpy()[:J]     # posterior 0
        rec = dict(iteration=st["iteration"], ess=st["ess"], ess_before=st["ess_before"],
                   resampled=bool(st["resampled"]), mean_accept=st["mean_accept"],
                   n_mean=float(n.mean()), n_max=int(n.max()), grad_evals=st["grad_evals"],
                   L=st["L"], eps=st["eps"], chees=st["chees"], chees_grad=st["chees_grad"],
                   log_z=st["log_z"], wall_ms=ms)
        out.write(json.dumps(rec) + "\n")
        out.flush()
    if a.save:
        with open(a.save, "wb") as f:
            f.write(s.save())
        with open(a.save + ".json", "w") as f:
            json.dump(sched, f)
    if out is not sys.stdout:
        out.close()
    s.close()


if __name__ == "__main__":
    main()
