"""Pins of the diagonal-mass reading (oracle.smc.diag_mass): the weighted
population variance against numpy's own variance and weighted covariance, the
collapsed-population floor, and the adapted mass on a Gaussian target."""

import math

import numpy as np
import pytest

from oracle import smc as O


def _reg(var, n):
    return (n / (n + 5.0)) * var + 1e-3 * (5.0 / (n + 5.0))


def test_uniform_weights_give_population_variance():
    rng = np.random.default_rng(0)
    th = rng.standard_normal((500, 7)) * np.arange(1, 8)
    lw = np.full(500, -math.log(500))
    got = O.diag_mass(th, lw, 500.0)
    np.testing.assert_allclose(got, _reg(np.var(th, axis=0), 500.0).astype(np.float32), rtol=0, atol=0)


def test_weighted_variance_matches_numpy_weighted_covariance():
    rng = np.random.default_rng(1)
    th = rng.standard_normal((300, 4)) + 2.0
    lw = rng.standard_normal(300) * 2.0 - 40.0
    W = np.exp(lw - lw.max())
    W /= W.sum()
    n = 1.0 / np.sum(W * W)
    ref = np.diag(np.cov(th.T, aweights=W, bias=True))
    np.testing.assert_allclose(O.diag_mass(th, lw, n), _reg(ref, n), rtol=1e-6)


def test_collapsed_population_is_floored():
    th = np.tile(np.array([[1.5, -2.0, 0.25]]), (64, 1))
    lw = np.full(64, -math.log(64))
    got = O.diag_mass(th, lw, 1.0)
    np.testing.assert_allclose(got, np.full(3, 1e-3 * 5.0 / 6.0), rtol=1e-7)
    # one particle carries all the weight: its spread is zero whatever the others
    rng = np.random.default_rng(2)
    th2 = rng.standard_normal((10, 3))
    lw2 = np.full(10, -np.inf)
    lw2[4] = 0.0
    np.testing.assert_allclose(O.diag_mass(th2, lw2, 1.0), np.full(3, 1e-3 * 5.0 / 6.0), rtol=1e-7)


def test_diag_mass_keeps_a_target_population_on_target():
    # N(mu, diag(s^2)) with very different scales.  A population drawn from the
    # target with equal weights stays properly weighted under moves with the
    # adapted mass (the weights stay exact for any fixed M), so at every
    # iteration the mass is the target variance and the weighted moments are
    # the target's, up to Monte Carlo error
    s2 = np.array([0.01, 1.0, 25.0])
    mu = np.array([1.0, -1.0, 3.0])
    J = 4000
    t = O.Gaussian(mu, np.diag(s2))
    rng = np.random.default_rng(3)
    o = O.OracleSMC(t, J, step_size=0.4, traj_length=2.0, max_leapfrog=16, num_warmup=3,
                    precond="diag", seed=7)
    o.set_state(mu + rng.standard_normal((J, 3)) * np.sqrt(s2), np.full(J, -math.log(J)))
    for _ in range(6):
        st = o.step()
        o.adapt()
        assert np.all(np.abs(st["minv"] / s2 - 1) < 0.12), st["minv"]
    m, v = o.moments()
    ess = O.ess(o.logw)
    assert np.all(np.abs(m - mu) <= 5 * np.sqrt(s2 / ess)), (m, ess)
    assert np.all(np.abs(v / s2 - 1) < 0.12), v
