"""Jitter-generator study on the synthetic targets (the protocol of Sec. IV,
reported like Table 1), on the device library.

Protocol: J = 1000 particles, K = 200 iterations of which the first 100 are
warm-up (ChEES adaptation), initial draw N(0, I), L0 = 5, step sizes 0.1
(Gaussian), 0.001 (ill-conditioned Gaussian) and 0.01 (banana), at most 500
leapfrog steps, 10 runs per cell.  Per cell it reports, averaged over the
runs and over all iterations (and, separately, over the iterations after the
warm-up),
  * grad/N: gradient evaluations per particle and iteration, counted like the
    paper (the n_j leapfrog gradients plus one), and
  * ESS/grad: (J_eff / J) / (grad/N), the effective sample fraction after the
    move per gradient evaluation of a particle.
The Adam learning rate of the ChEES adaptation is not given in the paper;
--adam-lr sets it (library default 0.025).

Usage: python -m paper_2504_02627_amd.rng_study [--runs R] [--iters K] [--out FILE]
"""

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

SCHEMES = ["none", "uniform", "haltonNd", "haltonNd_inv", "halton1d", "primes", "primes_inv",
           "golden", "equidistant", "equidistant_offset", "sobol1d", "sobolNd", "sobolNd_inv"]
TARGETS = ["gaussian", "illcond", "banana"]
STEP = {"gaussian": 0.1, "illcond": 0.001, "banana": 0.01}


def target_spec(name):
    import torch
    from paper_2504_02627_amd import synth
    dev = torch.device("cuda:0")
    if name == "banana":
        return dict(kind="banana", dim=2, banana=synth.BANANA)
    mu, P, _ = synth.gaussian5() if name == "gaussian" else synth.ill_conditioned_gaussian()
    return dict(kind="gaussian", dim=len(mu), mean=torch.from_numpy(mu).to(dev),
                precision=torch.from_numpy(P).to(dev))


def one_run(spec, eps, scheme, seed, J, K, burn, nmax, L0, lr):
    from paper_2504_02627_amd import chees
    s = chees.Sampler(None, None, J, target=spec, step_size=eps, traj_length=L0,
                      max_leapfrog=nmax, num_warmup=burn, jitter=scheme, num_iterations=K,
                      seed=seed, adam_lr=lr)
    gpn, epg = [], []
    for _ in range(K):
        st = s.step()
        s.adapt(stats=False)
        g = (st["grad_evals"] + J) / J       # n_j + 1 per particle
        gpn.append(g)
        epg.append((st["ess"] / J) / g)
    gpn, epg = np.array(gpn), np.array(epg)
    return gpn.mean(), epg.mean(), gpn[burn:].mean(), epg[burn:].mean()


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--runs", type=int, default=10)
    ap.add_argument("--iters", type=int, default=200)
    ap.add_argument("--burn", type=int, default=100)
    ap.add_argument("--particles", type=int, default=1000)
    ap.add_argument("--max-leapfrog", type=int, default=500)
    ap.add_argument("--traj-length", type=float, default=5.0)
    ap.add_argument("--targets", default=",".join(TARGETS))
    ap.add_argument("--schemes", default=",".join(SCHEMES))
    ap.add_argument("--adam-lr", type=float, default=0.025)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    table = {}
    t0 = time.time()
    for tname in a.targets.split(","):
        spec = target_spec(tname)
        for scheme in a.schemes.split(","):
            res = np.array([one_run(spec, STEP[tname], scheme, 1000 + r, a.particles, a.iters,
                                    a.burn, a.max_leapfrog, a.traj_length, a.adam_lr)
                            for r in range(a.runs)])
            g, e, gb, eb = (float(v) for v in res.mean(axis=0))
            table.setdefault(tname, {})[scheme] = {
                "grad_per_N": round(g, 3), "ess_per_grad": e,
                "grad_per_N_after_warmup": round(gb, 3), "ess_per_grad_after_warmup": eb}
            print(f"[rng-study] {tname:9s} {scheme:19s} grad/N {g:8.2f} ESS/grad {e:.3e} | "
                  f"after warm-up {gb:8.2f} {eb:.3e}  ({time.time() - t0:.0f} s)", flush=True)
    out = {"protocol": dict(particles=a.particles, iterations=a.iters, warmup=a.burn,
                            runs=a.runs, traj_length0=a.traj_length, adam_lr=a.adam_lr,
                            max_leapfrog=a.max_leapfrog, step_size=STEP),
           "table": table}
    text = json.dumps(out)
    if a.out:
        with open(a.out, "w") as f:
            f.write(text + "\n")
    print(text)


if __name__ == "__main__":
    main()
