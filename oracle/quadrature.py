"""Reference posterior moments and evidence by brute-force quadrature.

TEST INFRASTRUCTURE ONLY (like the rest of oracle/): the end-to-end statistical
tests compare the sampler's final weighted moments (eq. realised_estimates,
Sec. III) and its evidence estimate against these values.

For a low-dimensional target pi(theta) = p(x|theta) q0(theta) (Sec. II) the
normalising constant Z and the moments are integrals over R^d.  They are
computed on a tensor-product Gauss--Hermite grid centred on the mode m with
the Laplace covariance S = (-Hessian)^-1:  theta = m + C u, C C^T = S,
  int f(theta) pi(theta) dtheta
    = |C| int f(m + C u) pi(m + C u) e^{|u|^2/2} e^{-|u|^2/2} du,
and the probabilists' Gauss--Hermite rule integrates g(u) e^{-|u|^2/2}.  The
rule is exact for polynomial g of degree < 2K per axis, so it is exact for a
Gaussian pi (g is then constant or polynomial); for a posterior close to
Gaussian it converges quickly in K.  Plain numpy, FP64, evaluated in chunks.
"""

import math

import numpy as np
from numpy.polynomial.hermite_e import hermegauss


def laplace(log_and_grad_hess, d, iters=50):
    """Mode and Laplace covariance by Newton's method from theta = 0.
    log_and_grad_hess(theta) -> (log pi, gradient, Hessian) for one theta."""
    th = np.zeros(d)
    for _ in range(iters):
        _, g, H = log_and_grad_hess(th)
        step = np.linalg.solve(H, g)
        th = th - step
        if np.max(np.abs(step)) < 1e-14 * (1 + np.max(np.abs(th))):
            break
    _, _, H = log_and_grad_hess(th)
    return th, np.linalg.inv(-H)


def gauss_hermite(logpi, mode, cov, K, chunk=1 << 16):
    """log Z, posterior mean and covariance of exp(logpi) by a K^d-point
    tensor Gauss--Hermite rule around (mode, cov).
    logpi(thetas (M, d)) -> (M,) unnormalised log density."""
    d = len(mode)
    x, w = hermegauss(K)                        # weight e^{-x^2/2}
    C = np.linalg.cholesky(cov)
    logdetC = float(np.sum(np.log(np.diag(C))))
    grids = np.stack(np.meshgrid(*([np.arange(K)] * d), indexing="ij"), -1).reshape(-1, d)
    M = grids.shape[0]
    # log of the integrand weights, accumulated with a running log-sum-exp
    logs, s1, s2 = [], None, None
    vals = []
    for a in range(0, M, chunk):
        idx = grids[a:a + chunk]
        u = x[idx]
        lw = np.sum(np.log(w[idx]), 1) + 0.5 * np.sum(u * u, 1)
        th = mode + u @ C.T
        vals.append((th, lw + logpi(th)))
    mx = max(float(np.max(v)) for _, v in vals)
    Zs, S1, S2 = 0.0, np.zeros(d), np.zeros((d, d))
    for th, lv in vals:
        e = np.exp(lv - mx)
        Zs += float(np.sum(e))
        S1 += e @ th
        S2 += (th * e[:, None]).T @ th
    logZ = mx + math.log(Zs) + logdetC
    mean = S1 / Zs
    cov_post = S2 / Zs - np.outer(mean, mean)
    return logZ, mean, cov_post


def logistic_reference(X, y, prior_var=1.0, K=20):
    """(log Z, mean, covariance) of the Bayesian logistic regression posterior
    pi(theta) = prod_n sigma(x_n theta)^y_n (1 - sigma(x_n theta))^(1 - y_n)
    N(theta; 0, prior_var I) (Sec. V workload), Z including the prior's
    normalisation."""
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    d = X.shape[1]

    def logpi(th):
        z = th @ X.T
        ll = np.sum(y * z - np.logaddexp(0.0, z), axis=1)
        return ll - 0.5 * np.sum(th * th, 1) / prior_var - 0.5 * d * math.log(2 * math.pi * prior_var)

    def lgh(th):
        z = X @ th
        s = 1.0 / (1.0 + np.exp(-z))
        g = X.T @ (y - s) - th / prior_var
        H = -(X.T * (s * (1 - s))) @ X - np.eye(d) / prior_var
        return None, g, H

    m, S = laplace(lgh, d)
    return gauss_hermite(logpi, m, S, K)
