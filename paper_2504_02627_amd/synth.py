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
