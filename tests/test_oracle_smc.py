"""End-to-end pins for the oracle's SMC sampler (Alg. smc_BNN with the
ChEES-HMC proposal): Gaussian targets with known moments and evidence, and a
2-d logistic regression whose evidence is computed by brute-force quadrature."""

import math
import os

import numpy as np
import pytest

from oracle import philox, smc as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    with open(os.path.join(GOLDEN, "philox_kat.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        assert philox.philox4x32_10(v[0:4], v[4:6]) == tuple(v[6:10])
        got = philox.philox4x32_10_np(*[np.array([x], dtype=np.uint64) for x in v[0:4]], v[4:6])
        assert tuple(int(g[0]) for g in got) == tuple(v[6:10])


def test_philox_normals_moments():
    z = philox.normals_np(9, 4000, 1, philox.STREAM_MOMENTUM, 10).ravel()
    assert abs(z.mean()) < 4 / math.sqrt(z.size)
    assert abs(z.var() - 1) < 4 * math.sqrt(2 / z.size)


def _run(target, J, K, seed, **kw):
    s = O.OracleSMC(target, J, seed=seed, **kw)
    for _ in range(K):
        s.step()
        s.adapt()
    return s


def test_gaussian_5d_moments():
    # Sec. IV Gaussian: mu = [-4,-2,0,2,4], Sigma = diag(1, 1.5, 2, 2.5, 3) (variances), eps = 0.1, L0 = 5.
    mu = np.array([-4.0, -2.0, 0.0, 2.0, 4.0])
    var = np.array([1.0, 1.5, 2.0, 2.5, 3.0])
    t = O.Gaussian(mu, np.diag(var))
    means, vars_ = [], []
    for seed in range(4):
        s = _run(t, 500, 30, seed, step_size=0.1, traj_length=5.0, num_warmup=15, max_leapfrog=100)
        m, v = s.moments()
        means.append(m)
        vars_.append(v)
    means, vars_ = np.array(means), np.array(vars_)
    # per-run standard error of a weighted mean is about sqrt(var / ESS); ESS >= 250
    assert np.all(np.abs(means.mean(0) - mu) < 4 * np.sqrt(var / (4 * 250)) + 0.02)
    assert np.all(np.abs(vars_.mean(0) / var - 1) < 0.15)


def test_gaussian_evidence_is_scale():
    # pi = c N(mu, Sigma): the evidence is c exactly; E[Z_hat] = c.
    mu = np.array([0.5, -0.3, 0.2])
    t = O.Gaussian(mu, np.diag([0.6, 1.0, 1.4]), log_scale=2.3)
    z = []
    for seed in range(8):
        s = _run(t, 400, 6, seed, step_size=0.1, traj_length=1.0, num_warmup=3)
        z.append(math.exp(s.log_evidence() - 2.3))
    z = np.array(z)
    assert abs(z.mean() - 1.0) < 3 * z.std(ddof=1) / math.sqrt(len(z)) + 0.02


def test_logistic_2d_evidence_against_quadrature():
    rng = np.random.default_rng(21)
    X = rng.standard_normal((15, 2))
    y = (rng.random(15) < 1 / (1 + np.exp(-X @ np.array([1.0, -0.5])))).astype(float)
    t = O.LogisticRegression(X, y)
    g = np.linspace(-7, 7, 701)
    T1, T2 = np.meshgrid(g, g, indexing="ij")
    lp, _ = t.log_and_grad(np.stack([T1.ravel(), T2.ravel()], 1))
    logZ = math.log(np.sum(np.exp(lp)) * (g[1] - g[0]) ** 2)
    z = []
    for seed in range(8):
        s = _run(t, 500, 5, seed, step_size=0.15, traj_length=1.0, num_warmup=3)
        z.append(math.exp(s.log_evidence() - logZ))
    z = np.array(z)
    assert abs(z.mean() - 1.0) < 3 * z.std(ddof=1) / math.sqrt(len(z)) + 0.02


def test_mh_mode_keeps_weights_and_targets_posterior():
    mu = np.array([1.0, -1.0])
    t = O.Gaussian(mu, np.diag([0.5, 2.0]))
    s = O.OracleSMC(t, 400, seed=3, mh_accept=True, step_size=0.2, traj_length=1.5, num_warmup=5)
    s.step()
    lw_after_first = s.logw.copy()
    for _ in range(15):
        s.step()
        np.testing.assert_array_equal(s.logw, lw_after_first)
        s.adapt()
    m, v = s.moments()
    # weights untouched after the first resampling, so the population itself targets pi
    np.testing.assert_allclose(m, mu, atol=0.25)


def test_injected_randomness_is_used():
    t = O.Gaussian(np.zeros(2), np.eye(2))
    J = 16
    s1 = O.OracleSMC(t, J, seed=1, num_warmup=2, step_size=0.2)
    s2 = O.OracleSMC(t, J, seed=1, num_warmup=2, step_size=0.2)
    xi = philox.normals_np(1, J, 1, philox.STREAM_MOMENTUM, 2)
    a = s1.step()
    b = s2.step(momenta=xi)
    np.testing.assert_array_equal(s1.theta, s2.theta)
    assert a["resampled"] == b["resampled"]


def test_degenerate_weights_raise():
    t = O.Gaussian(np.zeros(1), np.eye(1))
    s = O.OracleSMC(t, 4, seed=0, num_warmup=2)
    s.logw[:] = -np.inf
    with pytest.raises(FloatingPointError):
        s.step()
