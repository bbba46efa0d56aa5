"""Pins of the quadrature reference (oracle/quadrature.py) used by the
end-to-end statistical tests: exactness on Gaussian integrands, the
closed-form evidence of conjugate Bayesian linear regression, and
one-dimensional logistic posteriors against scipy's adaptive quadrature."""

import math

import numpy as np
import pytest
from scipy import integrate

from oracle import quadrature as Q


def _gauss_logpdf(th, mu, S):
    d = len(mu)
    L = np.linalg.cholesky(S)
    r = np.linalg.solve(L, (th - mu).T).T
    return -0.5 * np.sum(r * r, 1) - np.sum(np.log(np.diag(L))) - 0.5 * d * math.log(2 * math.pi)


def test_gaussian_target_is_integrated_exactly():
    rng = np.random.default_rng(0)
    d = 3
    A = rng.standard_normal((d, d))
    S = A @ A.T + 0.5 * np.eye(d)
    mu = rng.standard_normal(d)
    logc = 2.75
    logZ, m, C = Q.gauss_hermite(lambda t: logc + _gauss_logpdf(t, mu, S), mu, S, K=4)
    assert logZ == pytest.approx(logc, abs=1e-12)
    np.testing.assert_allclose(m, mu, rtol=0, atol=1e-12)
    np.testing.assert_allclose(C, S, rtol=0, atol=1e-12)


def test_conjugate_linear_regression_evidence():
    # y = X theta + e, e ~ N(0, s2 I), theta ~ N(0, I):  p(y) = N(y; 0, s2 I + X X^T)
    rng = np.random.default_rng(1)
    N, d, s2 = 30, 2, 0.7
    X = rng.standard_normal((N, d))
    y = X @ np.array([0.4, -1.1]) + math.sqrt(s2) * rng.standard_normal(N)

    def logpi(th):
        r = y[None, :] - th @ X.T
        return (-0.5 * np.sum(r * r, 1) / s2 - 0.5 * N * math.log(2 * math.pi * s2)
                - 0.5 * np.sum(th * th, 1) - 0.5 * d * math.log(2 * math.pi))

    def lgh(th):
        g = X.T @ (y - X @ th) / s2 - th
        H = -X.T @ X / s2 - np.eye(d)
        return None, g, H

    m, S = Q.laplace(lgh, d)
    logZ, mean, cov = Q.gauss_hermite(logpi, m, S, K=3)
    Sy = s2 * np.eye(N) + X @ X.T
    sign, logdet = np.linalg.slogdet(Sy)
    exact = -0.5 * y @ np.linalg.solve(Sy, y) - 0.5 * logdet - 0.5 * N * math.log(2 * math.pi)
    assert logZ == pytest.approx(exact, abs=1e-10)
    post_cov = np.linalg.inv(X.T @ X / s2 + np.eye(d))
    np.testing.assert_allclose(mean, post_cov @ X.T @ y / s2, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(cov, post_cov, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("seed", [3, 4])
def test_one_dimensional_logistic_against_adaptive_quadrature(seed):
    rng = np.random.default_rng(seed)
    N = 40
    x = rng.standard_normal((N, 1))
    y = (rng.random(N) < 1 / (1 + np.exp(-0.8 * x[:, 0]))).astype(np.float64)
    logZ, mean, cov = Q.logistic_reference(x, y, prior_var=1.0, K=40)

    def dens(t):
        z = t * x[:, 0]
        return math.exp(np.sum(y * z - np.logaddexp(0.0, z)) - 0.5 * t * t - 0.5 * math.log(2 * math.pi))

    Z = integrate.quad(dens, -12, 12, epsabs=0, epsrel=1e-13, limit=400)[0]
    m1 = integrate.quad(lambda t: t * dens(t), -12, 12, epsabs=0, epsrel=1e-13, limit=400)[0] / Z
    m2 = integrate.quad(lambda t: t * t * dens(t), -12, 12, epsabs=0, epsrel=1e-13, limit=400)[0] / Z
    assert logZ == pytest.approx(math.log(Z), abs=1e-9)
    assert mean[0] == pytest.approx(m1, abs=1e-9)
    assert cov[0, 0] == pytest.approx(m2 - m1 * m1, rel=1e-8)
