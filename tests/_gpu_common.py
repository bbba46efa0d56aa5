"""Shared helpers of the GPU tests: build device problems from the seeded
generators and run the oracle on the same inputs.  Nothing here computes any
of the sampler's arithmetic: that lives in oracle/ (expected values) and in the
library (device values)."""

import sys

import numpy as np

from oracle import smc as O


def dev():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev())


def rel_rows(a, b):
    """max over rows of ||a_j - b_j||_inf / max(||b_j||_inf, 1e-30)."""
    num = np.max(np.abs(a - b), axis=1)
    den = np.maximum(np.max(np.abs(b), axis=1), 1e-30)
    return float(np.max(num / den))


def oracle_for(X32, y32, J, theta0_32, **params):
    t = O.LogisticRegression(X32.astype(np.float64), y32.astype(np.float64),
                             prior_var=params.pop("prior_var", 1.0))
    return O.OracleSMC(t, J, theta0=theta0_32.astype(np.float64), **params)
