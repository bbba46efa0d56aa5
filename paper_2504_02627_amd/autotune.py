"""Autotuner of the leapfrog launch shape (smc_params.lf_items, lf_split_cap).

For one workload (posterior sizes, particle count, precision, n_max) it runs
the sampler's captured iteration graph under each candidate setting, times a
few iterations after a short warm-up, and keeps the fastest.  The choice is
stored in a JSON cache keyed by the workload's signature; Sampler(...,
tune="cache") reads it and passes the setting to smc_init.  The settings only
move data-row boundaries between work items, so a tuned run differs from the
default one by the order of the partial-gradient sums (see
tests/test_gpu_tuning.py).

Usage (on the GPU):
    python -m paper_2504_02627_amd.autotune --workload large --precision bf16
    python -m paper_2504_02627_amd.autotune --all
"""

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tune_cache.json")

# candidate grid: work items per resident work-group slot and the cap on the
# data-row splits of one particle tile in one step
ITEMS = (128, 256, 512)
SPLIT_CAPS = (8, 16, 32, 64)


def signature(dims, rows, J, precision, max_leapfrog):
    """Key of a workload: the sizes that decide the launch plan."""
    return json.dumps({"rows": [int(n) for n in rows], "dims": [int(d) for d in dims], "J": int(J),
                       "precision": precision, "max_leapfrog": int(max_leapfrog)},
                      sort_keys=True, separators=(",", ":"))


def load_cache(path=CACHE):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def lookup(dims, rows, J, precision, max_leapfrog, path=CACHE):
    """The cached setting (dict of smc_params fields) for this workload, or {}."""
    e = load_cache(path).get(signature(dims, rows, J, precision, max_leapfrog))
    return dict(e["best"]) if e else {}


def _time_setting(Xs, ys, J, params, warm, iters):
    import torch
    from paper_2504_02627_amd import chees
    s = chees.Sampler(Xs, ys, J, **params)
    s.run(warm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.run(iters)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / iters
    s.close()
    return ms


def tune(Xs, ys, J, params, warm=3, iters=8, items=ITEMS, caps=SPLIT_CAPS, path=CACHE, log=print):
    """Time every (lf_items, lf_split_cap) candidate on this workload and store
    the fastest in the cache.  Xs, ys: device tensors (lists for a batched
    context); params: the sampler's parameters (seed, step size, ...)."""
    Xl = Xs if isinstance(Xs, (list, tuple)) else [Xs]
    key = signature([X.shape[1] for X in Xl], [X.shape[0] for X in Xl], J,
                    params.get("precision", "f32"), params.get("max_leapfrog", 64))
    results = []
    for it in items:
        for cap in caps:
            p = dict(params, lf_items=it, lf_split_cap=cap)
            ms = _time_setting(Xs, ys, J, p, warm, iters)
            results.append({"lf_items": it, "lf_split_cap": cap, "ms_per_iteration": round(ms, 4)})
            log(f"[autotune] items {it:4d} split cap {cap:2d}: {ms:.3f} ms per iteration")
    default_ms = _time_setting(Xs, ys, J, dict(params, lf_items=0, lf_split_cap=0), warm, iters)
    best = min(results, key=lambda r: r["ms_per_iteration"])
    cache = load_cache(path)
    cache[key] = {"best": {"lf_items": best["lf_items"], "lf_split_cap": best["lf_split_cap"]},
                  "ms_per_iteration": best["ms_per_iteration"],
                  "default_ms_per_iteration": round(default_ms, 4),
                  "candidates": results, "warmup": warm, "timed_iterations": iters}
    with open(path, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    log(f"[autotune] best {best} (default {default_ms:.3f} ms) -> {path}")
    return cache[key]


def workload(name):
    """(Xs, ys, J, params) of the named benchmark workload on cuda:0."""
    import torch
    from paper_2504_02627_amd import synth
    dev = torch.device("cuda:0")
    if name == "large":
        X, y, _ = synth.large_logistic()
        eps = synth.default_step_size(10000, 100)
        return (torch.from_numpy(X).to(dev), torch.from_numpy(y).to(dev), 8192,
                dict(step_size=eps, traj_length=eps * 32, max_leapfrog=64, num_warmup=25, seed=2))
    if name == "batched":
        data = synth.batched_logistic(64)
        eps = min(synth.default_step_size(X.shape[0], X.shape[1]) for X, _, _ in data)
        return ([torch.from_numpy(X).to(dev) for X, _, _ in data],
                [torch.from_numpy(y).to(dev) for _, y, _ in data], 1024,
                dict(step_size=eps, traj_length=eps * 32, max_leapfrog=64, num_warmup=25, seed=4))
    if name == "toeplitz":
        X, y, _ = synth.toeplitz_logistic()
        eps = synth.default_step_size(5000, 100)
        return (torch.from_numpy(X).to(dev), torch.from_numpy(y).to(dev), 4096,
                dict(step_size=eps, traj_length=eps * 32, max_leapfrog=64, num_warmup=25, seed=3))
    raise ValueError(name)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--workload", choices=["large", "batched", "toeplitz"], default="large")
    ap.add_argument("--precision", choices=["f32", "bf16"], default="f32")
    ap.add_argument("--all", action="store_true", help="large and batched, FP32 and BF16")
    ap.add_argument("--cache", default=CACHE)
    a = ap.parse_args(argv)
    jobs = ([(w, p) for w in ("large", "batched") for p in ("f32", "bf16")] if a.all
            else [(a.workload, a.precision)])
    for w, p in jobs:
        Xs, ys, J, params = workload(w)
        print(f"[autotune] {w} {p}", flush=True)
        tune(Xs, ys, J, dict(params, precision=p), path=a.cache,
             log=lambda m: print(m, flush=True))


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(HERE))
    main()
