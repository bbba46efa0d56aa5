"""Seeded synthetic workloads (inputs only).

This module draws data sets and nothing else: it holds none of the sampler's
arithmetic.  Both the device path and the oracle consume its arrays.  The
recipes stand in for the paper's logistic-regression experiment (Sec. IV,
German Credit, whose data are not used here) with the same model: Bernoulli
likelihood with a sigmoid link and an N(0, I) prior.

Every generator returns float32 X (row-major N x d) and float32 y in {0, 1};
the oracle takes the same float32 values promoted to float64.
"""

import numpy as np


def _labels(rng, X, beta):
    z = X.astype(np.float64) @ beta
    prob = 1.0 / (1.0 + np.exp(-z))
    return (rng.random(X.shape[0]) < prob).astype(np.float32)


def logistic_iid(N, d, seed, beta_var=1.0, standardise=False):
    """X ~ N(0,1) iid (optionally column-standardised), beta* ~ N(0, beta_var I),
    y ~ Bernoulli(sigmoid(X beta*))."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((N, d))
    if standardise:
        X = (X - X.mean(axis=0)) / X.std(axis=0)
    X = X.astype(np.float32)
    beta = rng.standard_normal(d) * np.sqrt(beta_var)
    return X, _labels(rng, X, beta), beta


def logistic_toeplitz(N, d, seed, rho=0.95, beta_var=0.25):
    """Rows x_n ~ N(0, S) with S_ij = rho^|i-j| (an ill-conditioned posterior)."""
    rng = np.random.default_rng(seed)
    idx = np.arange(d)
    S = rho ** np.abs(idx[:, None] - idx[None, :])
    Lc = np.linalg.cholesky(S)
    X = (rng.standard_normal((N, d)) @ Lc.T).astype(np.float32)
    beta = rng.standard_normal(d) * np.sqrt(beta_var)
    return X, _labels(rng, X, beta), beta


def batched_sizes(B, seed, n_range=(500, 20000), d_range=(10, 200)):
    rng = np.random.default_rng(seed)
    Ns = rng.integers(n_range[0], n_range[1] + 1, size=B)
    ds = rng.integers(d_range[0], d_range[1] + 1, size=B)
    return [int(v) for v in Ns], [int(v) for v in ds]


# Workloads (seed = 1000 + workload number).
def small_logistic():
    """N=200, d=5, X ~ N(0,1) iid, beta* ~ N(0, I)."""
    return logistic_iid(200, 5, 1001, beta_var=1.0)


def large_logistic():
    """N=10000, d=100, X standardised N(0,1), beta* ~ N(0, 0.25 I)."""
    return logistic_iid(10000, 100, 1002, beta_var=0.25, standardise=True)


def toeplitz_logistic():
    """N=5000, d=100, Toeplitz(0.95) rows, beta* ~ N(0, 0.25 I)."""
    return logistic_toeplitz(5000, 100, 1005)


def batched_logistic(B=64):
    """B posteriors, N_b ~ U{500..20000}, d_b ~ U{10..200}, X ~ N(0,1), beta* ~ N(0, 0.25 I)."""
    Ns, ds = batched_sizes(B, 1004)
    out = []
    for b, (n, d) in enumerate(zip(Ns, ds)):
        X, y, beta = logistic_iid(n, d, 1004 * 1000 + b, beta_var=0.25)
        out.append((X, y, beta))
    return out


def default_step_size(N, d):
    """A Fisher-scale starting step size d^(-1/4) / sqrt(1 + N/4) (the logistic
    curvature is at most N/4 per unit-variance feature)."""
    return float(d) ** -0.25 / np.sqrt(1.0 + N / 4.0)


# ---------------------------------------------------------------------------
# Synthetic targets of Sec. IV (parameters only; the densities themselves are
# evaluated by the device library and by the oracle, each on its own).
# ---------------------------------------------------------------------------

def gaussian5():
    """Sec. IV Gaussian, D = 5: mu = [-4, -2, 0, 2, 4], Sigma = diag(1, 1.5, 2,
    2.5, 3).  Returns float32 (mu, precision) and the float64 covariance."""
    mu = np.array([-4.0, -2.0, 0.0, 2.0, 4.0])
    var = np.array([1.0, 1.5, 2.0, 2.5, 3.0])
    return mu.astype(np.float32), np.diag(1.0 / var).astype(np.float32), np.diag(var)


def ill_conditioned_gaussian(d=100, seed=14):
    """Sec. IV ill-conditioned Gaussian: Sigma = Q diag(lambda) Q^T with Q
    Haar-distributed on O(d) (QR of a Gaussian matrix with the signs of R's
    diagonal folded into Q) and lambda_i ~ Gamma(shape 0.5, scale 1); mu = 0.
    The default seed gives condition number 1.27e5 (the paper quotes about
    1.3e5).  Returns float32 (mu, precision) and the float64 covariance."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((d, d))
    Q, R = np.linalg.qr(A)
    Q = Q * np.sign(np.diag(R))
    lam = rng.gamma(0.5, 1.0, size=d)
    cov = (Q * lam) @ Q.T
    prec = (Q / lam) @ Q.T
    prec = 0.5 * (prec + prec.T)
    return np.zeros(d, dtype=np.float32), prec.astype(np.float32), 0.5 * (cov + cov.T)


BANANA = (10.0, 0.03, 100.0)  # Sec. IV Rosenbrock: s1, b, c
FUNNEL = (10, 3.0)            # Neal's funnel: dimension, standard deviation of v
