"""End-to-end statistical parity: the sampler's final weighted posterior mean
and variance per dimension (eq. realised_estimates) and its evidence estimate,
over R replicate seeds, against brute-force quadrature of the same posterior
(oracle/quadrature.py).  Bar: the replicate average within 3 Monte Carlo
standard errors (sd over replicates / sqrt R) of the reference; for the
evidence, the average of Z_hat / Z (an unbiased estimator) within 3 SE of 1.

Workload: logistic regression N = 200, d = 5 (the small logistic workload),
20 SMC iterations from the prior, 10 of them adapting L (and the step size),
1-d Halton jitter, systematic resampling at J_eff < J/2."""

import math

import numpy as np
import pytest

from oracle import quadrature as Q, smc as O
from paper_2504_02627_amd import synth
from tests._gpu_common import log, to_dev

pytestmark = pytest.mark.gpu

R = 16


def _replicates(Xdev, y, J, precision, iters=20, **extra):
    from paper_2504_02627_amd import chees
    import torch
    N, d = Xdev.shape
    eps = synth.default_step_size(N, d)
    means, vars_, logz = [], [], []
    for r in range(R):
        kw = dict(step_size=eps, traj_length=eps * 32, max_leapfrog=64, num_warmup=iters // 2,
                  adapt_step_size=True, seed=100 + r)
        kw.update(extra)
        s = chees.Sampler(Xdev, to_dev(y), J, precision=precision, **kw)
        for _ in range(iters):
            s.step(stats=False)
            s.adapt(stats=False)
        theta, logw, _ = s.state()
        w = torch.softmax(logw, 0)
        th = theta.double()
        m = (w[:, None] * th).sum(0)
        means.append(m.cpu().numpy())
        vars_.append((w[:, None] * (th - m) ** 2).sum(0).cpu().numpy())
        logz.append(s.log_evidence())
        s.close()
    return np.array(means), np.array(vars_), np.array(logz)


def _check(name, means, vars_, logz, ref):
    lz, mu, C = ref
    var = np.diag(C)
    zm = (means.mean(0) - mu) / (means.std(0, ddof=1) / math.sqrt(R))
    zv = (vars_.mean(0) - var) / (vars_.std(0, ddof=1) / math.sqrt(R))
    ratio = np.exp(logz - lz)
    zz = (ratio.mean() - 1.0) / (ratio.std(ddof=1) / math.sqrt(R))
    log(f"[statistical] {name}: z(mean) {np.round(zm, 2)}  z(var) {np.round(zv, 2)}  "
        f"z(Z/Z) {zz:.2f}  mean log Z_hat - log Z {np.mean(logz) - lz:.4f} "
        f"(sd {np.std(logz, ddof=1):.4f})")
    rel_m = np.max(np.abs(means.mean(0) - mu) / np.sqrt(var))
    log(f"  max |mean error| / posterior sd {rel_m:.3e}; max rel var error "
        f"{np.max(np.abs(vars_.mean(0) / var - 1)):.3e}")
    assert np.all(np.abs(zm) <= 3) and np.all(np.abs(zv) <= 3) and abs(zz) <= 3


def test_fp32_small_logistic_matches_quadrature():
    # J = 16384.  With a few hundred or thousand particles the first (prior ->
    # posterior) importance step is degenerate enough that after 20 iterations
    # the population still leans toward the prior by a few MC standard errors,
    # and Z_hat / Z is heavy-tailed; the oracle does the same (next test)
    X, y, _ = synth.small_logistic()
    ref = Q.logistic_reference(X.astype(np.float64), y.astype(np.float64), K=12)
    m, v, lz = _replicates(to_dev(X), y, 16384, "f32")
    _check("f32 J=16384", m, v, lz, ref)


def test_fp32_small_logistic_j256_same_distribution_as_oracle():
    """At J = 256 (the oracle's own configuration) the device and the FP64
    oracle are run on the same seeds -- the same initial draws, momenta,
    jitter and resampling uniforms -- and their replicate results compared
    pairwise: the mean of the paired differences of log Z_hat and of each
    posterior mean and variance lies within 3 SE of 0."""
    import torch
    from paper_2504_02627_amd import chees
    X, y, _ = synth.small_logistic()
    N, d = X.shape
    J, iters = 256, 20
    eps = synth.default_step_size(N, d)
    params = dict(step_size=eps, traj_length=eps * 32, max_leapfrog=64, num_warmup=iters // 2,
                  adapt_step_size=True)
    t = O.LogisticRegression(X.astype(np.float64), y.astype(np.float64))
    dl, dm, dv = [], [], []
    for r in range(R):
        s = chees.Sampler(to_dev(X), to_dev(y), J, seed=100 + r, **params)
        o = O.OracleSMC(t, J, seed=100 + r, **params)
        for _ in range(iters):
            s.step(stats=False)
            s.adapt(stats=False)
            o.step()
            o.adapt()
        theta, logw, _ = s.state()
        w = torch.softmax(logw, 0).cpu().numpy()
        th = theta.double().cpu().numpy()
        m = w @ th
        wo = np.exp(o.logw - np.max(o.logw))
        wo /= wo.sum()
        mo = wo @ o.theta
        dl.append(s.log_evidence() - o.log_evidence())
        dm.append(m - mo)
        dv.append(w @ (th - m) ** 2 - wo @ (o.theta - mo) ** 2)
        s.close()
    for name, x in (("log Z", np.array(dl)[:, None]), ("mean", np.array(dm)), ("var", np.array(dv))):
        se = x.std(0, ddof=1) / math.sqrt(R)
        z = np.where(se > 0, x.mean(0) / np.where(se > 0, se, 1), 0.0)
        log(f"[statistical] J=256 device - oracle, {name}: mean diff {np.round(x.mean(0), 5)} "
            f"z {np.round(z, 2)}")
        assert np.all(np.abs(z) <= 3)


def test_bf16_trajectories_small_logistic_matches_quadrature():
    # precision form with X held in FP32 for the energies: same posterior
    X, y, _ = synth.small_logistic()
    ref = Q.logistic_reference(X.astype(np.float64), y.astype(np.float64), K=12)
    m, v, lz = _replicates(to_dev(X), y, 16384, "bf16")
    _check("bf16 trajectories, FP32 energies, J=16384", m, v, lz, ref)


def test_bf16_stored_x_matches_quadrature_of_rounded_data():
    # X stored in bfloat16: the target is the posterior of the rounded data;
    # its distance from the FP32-data posterior is reported
    import torch
    X, y, _ = synth.small_logistic()
    Xb = O.bf16_round(X)
    ref_b = Q.logistic_reference(Xb, y.astype(np.float64), K=12)
    ref = Q.logistic_reference(X.astype(np.float64), y.astype(np.float64), K=12)
    log(f"  rounded-data posterior vs FP32-data posterior: max |d mean| / sd "
        f"{np.max(np.abs(ref_b[1] - ref[1]) / np.sqrt(np.diag(ref[2]))):.3e}, "
        f"d log Z {ref_b[0] - ref[0]:.3e}")
    m, v, lz = _replicates(to_dev(X).to(torch.bfloat16), y, 16384, "bf16")
    _check("bf16 stored X, J=16384", m, v, lz, ref_b)


@pytest.mark.parametrize("precond", ["flow", "diag"])
def test_preconditioned_small_logistic_matches_quadrature(precond):
    # latent-space trajectories under the fitted flow (or the diagonal mass);
    # the weights use the exact latent target, so the weighted population is
    # the posterior's.  100 iterations: started in standardised units, these
    # forms leave the collapsed population of the first resampling more
    # slowly than the unit-mass form (about 0.02 posterior sd of lean toward
    # the prior remains after 20 iterations, below 0.005 after 60), and at
    # J = 16384 with 16 replicates one Monte Carlo SE is about 0.002 sd
    X, y, _ = synth.small_logistic()
    ref = Q.logistic_reference(X.astype(np.float64), y.astype(np.float64), K=12)
    extra = dict(flow_layers=2, flow_train_steps=5, flow_lr=5e-3) if precond == "flow" else {}
    m, v, lz = _replicates(to_dev(X), y, 16384, "f32", iters=100, precond=precond,
                           step_size=0.3, traj_length=1.5, max_leapfrog=16, **extra)
    _check(f"{precond}, J=16384, 100 iterations", m, v, lz, ref)
