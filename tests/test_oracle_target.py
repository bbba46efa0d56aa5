"""Pins for the oracle's targets: log pi and grad log pi (Sec. II problem
statement; Sec. IV targets).  Each check is independent of the oracle's own
formula: finite differences, closed forms at special points, quadrature."""

import math

import numpy as np
import pytest

from oracle import smc as O


def _fd_grad(f, theta, h=1e-6):
    g = np.zeros_like(theta)
    for i in range(theta.size):
        e = np.zeros_like(theta)
        e[i] = h
        g[i] = (f(theta + e) - f(theta - e)) / (2 * h)
    return g


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_logistic_gradient_matches_finite_differences(seed):
    rng = np.random.default_rng(seed)
    N, d = 7, 3
    X = rng.standard_normal((N, d))
    y = (rng.random(N) < 0.5).astype(float)
    t = O.LogisticRegression(X, y, prior_var=1.7)
    theta = rng.standard_normal(d)
    _, g = t.log_and_grad(theta)
    fd = _fd_grad(lambda th: t.log_and_grad(th)[0][0], theta)
    np.testing.assert_allclose(g[0], fd, rtol=1e-7, atol=1e-7)


def test_logistic_at_zero_closed_form():
    # theta = 0: z = 0, sigmoid = 1/2, log(1 + e^0) = log 2 for every row.
    rng = np.random.default_rng(5)
    N, d, s2 = 11, 4, 2.5
    X = rng.standard_normal((N, d))
    y = (rng.random(N) < 0.4).astype(float)
    t = O.LogisticRegression(X, y, prior_var=s2)
    lp, g = t.log_and_grad(np.zeros(d))
    assert lp[0] == pytest.approx(-N * math.log(2.0) - 0.5 * d * math.log(2 * math.pi * s2), rel=1e-15)
    np.testing.assert_allclose(g[0], X.T @ (y - 0.5), rtol=1e-15, atol=1e-15)


@pytest.mark.parametrize("theta", [-3.0, -0.4, 0.0, 0.9, 2.2])
def test_logistic_one_row_one_feature(theta):
    # N = d = 1, x = 2, y = 1: log pi = -log(1 + e^{-2 theta}) - theta^2/2 - log(2 pi)/2,
    # grad = 2 e^{-2 theta}/(1 + e^{-2 theta}) - theta.
    t = O.LogisticRegression(np.array([[2.0]]), np.array([1.0]), prior_var=1.0)
    lp, g = t.log_and_grad(np.array([theta]))
    e = math.exp(-2 * theta)
    assert lp[0] == pytest.approx(-math.log1p(e) - 0.5 * theta ** 2 - 0.5 * math.log(2 * math.pi), rel=1e-13)
    assert g[0, 0] == pytest.approx(2 * e / (1 + e) - theta, rel=1e-13, abs=1e-15)


def test_logistic_evidence_matches_quadrature_identity():
    # log pi integrates to the evidence: exp(log pi) over a fine grid equals
    # the sum over grid of likelihood * prior; check against the likelihood alone
    # times the N(0,1) prior density written out by hand.
    rng = np.random.default_rng(3)
    X = rng.standard_normal((5, 1))
    y = np.array([1.0, 0.0, 1.0, 1.0, 0.0])
    t = O.LogisticRegression(X, y)
    grid = np.linspace(-8, 8, 4001)[:, None]
    lp, _ = t.log_and_grad(grid)
    like = np.prod(np.where(y == 1, 1 / (1 + np.exp(-grid * X[:, 0])), 1 / (1 + np.exp(grid * X[:, 0]))), axis=1)
    prior = np.exp(-0.5 * grid[:, 0] ** 2) / math.sqrt(2 * math.pi)
    np.testing.assert_allclose(np.exp(lp), like * prior, rtol=1e-12)


def test_gaussian_normalised_and_gradient():
    mu = np.array([-4.0, -2.0, 0.0, 2.0, 4.0])
    cov = np.diag([1.0, 1.5, 2.0, 2.5, 3.0])
    t = O.Gaussian(mu, cov, log_scale=0.7)
    rng = np.random.default_rng(0)
    th = rng.standard_normal(5)
    fd = _fd_grad(lambda v: t.log_and_grad(v)[0][0], th)
    np.testing.assert_allclose(t.log_and_grad(th)[1][0], fd, rtol=1e-7, atol=1e-8)
    # product of 1-d normal densities, written out, times e^0.7
    ref = sum(-0.5 * (th[i] - mu[i]) ** 2 / cov[i, i] - 0.5 * math.log(2 * math.pi * cov[i, i]) for i in range(5)) + 0.7
    assert t.log_and_grad(th)[0][0] == pytest.approx(ref, rel=1e-13)


def test_banana_normalised_moments_by_quadrature():
    t = O.Banana()
    g1 = np.linspace(-60, 60, 1201)
    g2 = np.linspace(-40, 120, 1601)
    T1, T2 = np.meshgrid(g1, g2, indexing="ij")
    lp, _ = t.log_and_grad(np.stack([T1.ravel(), T2.ravel()], axis=1))
    w = np.exp(lp) * (g1[1] - g1[0]) * (g2[1] - g2[0])
    assert w.sum() == pytest.approx(1.0, abs=2e-3)
    e2 = np.sum(w * T2.ravel())
    v2 = np.sum(w * T2.ravel() ** 2) - e2 ** 2
    # theta1 ~ N(0, 100): E[theta2] = 0.03 (E theta1^2 - 100) = 0,
    # Var theta2 = 1 + 0.03^2 Var(theta1^2) = 1 + 0.0009 * 2 * 100^2 = 19
    assert e2 == pytest.approx(0.0, abs=2e-2)
    assert v2 == pytest.approx(19.0, rel=2e-2)
    th = np.array([3.0, -1.5])
    fd = _fd_grad(lambda v: t.log_and_grad(v)[0][0], th)
    np.testing.assert_allclose(t.log_and_grad(th)[1][0], fd, rtol=1e-7)
