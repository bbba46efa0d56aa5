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


def rel_each(a, b):
    """Per row: ||a_j - b_j||_inf / max(||b_j||_inf, 1e-30)."""
    num = np.max(np.abs(a - b), axis=1)
    den = np.maximum(np.max(np.abs(b), axis=1), 1e-30)
    return num / den


# BF16 trajectories against the BF16-emulating oracle.  Both sides round the
# residuals and the positions to bfloat16, but each takes the rounding decision
# from its own value: the device from binary32 (summed in an order that depends
# on the launch plan), the oracle from binary64.  Where the two straddle a
# rounding midpoint the operands differ by one bfloat16 unit and the leapfrog
# carries the difference to the end point.  Such flips are rare: most
# particles agree at the binary32 level and a few carry a flip.  Measured at
# full size (N = 10000, d = 100, 608 particles, two iterations): medians 4e-7
# (positions) and 2e-6 (momenta), 75th percentiles at most 1e-5, maxima 1.2e-3
# and 5.5e-3; two valid emulations of the form, deciding in binary32 and in
# binary64, differ from each other by as much.  A rounding mistake moves the
# median instead: truncation in place of round-to-nearest gives medians of
# 8e-4 to 6e-3, no rounding at all 6e-4 to 6e-3.  Bars: median 1e-5, 75th
# percentile 1e-4, every particle 5e-3 (positions) and 2e-2 (momenta).
BF16_MEDIAN_BAR = 1e-5
BF16_Q75_BAR = 1e-4
BF16_MAX_BAR = {"theta": 5e-3, "z": 5e-3, "p": 2e-2}


def check_bf16_trajectories(errs):
    """errs: {"theta"|"z"|"p": per-particle relative errors against the
    BF16-emulating oracle}.  Asserts the bars above; returns a summary."""
    out = []
    for k, e in errs.items():
        e = np.asarray(e, dtype=np.float64)
        q50, q75, mx = np.quantile(e, 0.5), np.quantile(e, 0.75), e.max()
        out.append(f"{k}: median {q50:.1e} q75 {q75:.1e} max {mx:.1e}")
        assert q50 <= BF16_MEDIAN_BAR and q75 <= BF16_Q75_BAR and mx <= BF16_MAX_BAR[k], out[-1]
    return "; ".join(out)
