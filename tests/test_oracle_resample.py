"""Pins for the oracle's resampling (Sec. III: resample with probability
wtilde; systematic and multinomial schemes).  Checked by brute force on tiny
inputs, by known properties of systematic resampling and by comparison with
the floating-point textbook form."""

import itertools
import math

import numpy as np
import pytest

from oracle import smc as O


def _brute_systematic(w, u):
    """Textbook systematic resampling with exact rationals from the float
    weights: point i sits at (i + u)/J on [0, 1); its ancestor is the particle
    whose cumulative-weight interval [C_{j-1}, C_j) contains it."""
    from fractions import Fraction
    W = [Fraction(v) for v in w]
    T = sum(W)
    C = list(itertools.accumulate(W))
    J = len(w)
    out = []
    for i in range(J):
        x = (i + Fraction(u)) / J * T
        out.append(next(j for j in range(J) if C[j] > x))
    return out


@pytest.mark.parametrize("seed", range(6))
def test_systematic_matches_brute_force_on_dyadic_weights(seed):
    # weights that are multiples of 2^-40 of the maximum are quantised exactly,
    # so the integer scheme must equal the exact-rational textbook scheme.
    rng = np.random.default_rng(seed)
    J = int(rng.integers(1, 8))
    w = rng.integers(0, 9, size=J).astype(float)
    w[rng.integers(J)] = 8.0
    for u in np.linspace(0.0, 1.0, 41, endpoint=False) + 1.0 / 97:
        got = O.resample_indices(w, u)
        assert list(got) == _brute_systematic(w / 8.0, O.uniform_to_u32(u) / 2 ** 32)


@pytest.mark.parametrize("seed", range(5))
def test_systematic_properties(seed):
    rng = np.random.default_rng(seed + 10)
    J = 200
    w = rng.gamma(0.3, size=J)
    w[rng.random(J) < 0.2] = 0.0
    u = rng.random()
    a = O.resample_indices(w, u)
    assert a.shape == (J,)
    assert np.all(np.diff(a) >= 0)
    counts = np.bincount(a, minlength=J)
    assert counts.sum() == J
    assert np.all(counts[w == 0.0] == 0)
    q = np.array(O.quantise_weights(w / w.max()), dtype=float)
    q /= q.sum()
    assert np.all(counts >= np.floor(J * q) - 0) and np.all(counts <= np.ceil(J * q))


def test_systematic_uniform_weights_identity():
    for J in (1, 2, 7, 64, 1000):
        for u in (0.0, 0.3, 0.999999):
            np.testing.assert_array_equal(O.resample_indices(np.ones(J), u), np.arange(J))


def test_systematic_unbiased_over_offset():
    # E_u[count_j] = J w_j: average the counts over a fine grid of offsets.
    rng = np.random.default_rng(7)
    J = 9
    w = rng.integers(1, 50, size=J).astype(float)
    M = 2048
    tot = np.zeros(J)
    for m in range(M):
        tot += np.bincount(O.resample_indices(w, (m + 0.5) / M), minlength=J)
    np.testing.assert_allclose(tot / M, J * w / w.sum(), atol=J / M + 1e-12)


def test_systematic_matches_float_textbook_form():
    rng = np.random.default_rng(11)
    for _ in range(20):
        J = 500
        lw = rng.standard_normal(J) * 2
        w = np.exp(lw - lw.max())
        u = rng.random()
        cdf = np.cumsum(w / w.sum())
        ref = np.searchsorted(cdf, (np.arange(J) + u) / J, side="right")
        got = O.resample_from_logw(lw, u)
        # identical except where a point falls within rounding of a boundary
        assert np.mean(got == np.minimum(ref, J - 1)) > 0.995


def test_multinomial_chi_square():
    rng = np.random.default_rng(3)
    J = 6
    w = np.array([1.0, 2.0, 3.0, 0.5, 0.0, 3.5])
    p = w / w.sum()
    counts = np.zeros(J)
    for _ in range(400):
        counts += np.bincount(O.resample_indices(w, rng.random(J), scheme="multinomial"), minlength=J)
    n = counts.sum()
    assert counts[4] == 0
    nz = p > 0
    chi2 = np.sum((counts[nz] - n * p[nz]) ** 2 / (n * p[nz]))
    assert chi2 < 20.5  # 5 degrees of freedom, p ~ 0.001


def test_zero_weights_raise():
    with pytest.raises(ValueError):
        O.resample_indices(np.zeros(4), 0.5)
    with pytest.raises(ValueError):
        O.resample_from_logw(np.full(4, -np.inf), 0.5)


def test_uniform_to_u32():
    assert O.uniform_to_u32(0.0) == 0
    assert O.uniform_to_u32((123 + 0.5) / 2 ** 32) == 123
    assert O.uniform_to_u32(math.nextafter(1.0, 0.0)) == 2 ** 32 - 1
