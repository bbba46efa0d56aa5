"""Pins for the oracle's jitter (Sec. III-B-1), step counts (Alg. smc_ChEES)
and weight arithmetic (Sec. III, eqs. normalise_smc2 and ess_smc)."""

import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import smc as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _halton_golden():
    rows = []
    with open(os.path.join(GOLDEN, "halton_textbook.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                b, i, num, den = (int(v) for v in line.split())
                rows.append((b, i, Fraction(num, den)))
    return rows


def test_radical_inverse_textbook_values_bit_exact():
    rows = _halton_golden()
    assert len(rows) >= 20
    for b, i, frac in rows:
        assert O.radical_inverse(i, b) == float(frac)  # bit-exact


def test_radical_inverse_large_index_is_exact_ratio():
    # phi_2(i) is k / 2^m exactly; reconstruct by bit reversal with integers.
    for i in [1, 12345, 2 ** 20 + 7, 2 ** 31 - 1, 3 * 2 ** 40 + 5]:
        m = i.bit_length()
        rev = int(bin(i)[2:][::-1], 2)
        assert O.radical_inverse(i, 2) == rev / 2 ** m


def test_halton_1d_stratifies_each_iteration_for_power_of_two_J():
    J = 256
    for k in (1, 2, 7):
        h = np.sort(O.halton_1d(k, J))
        # one point in each interval [i/J, (i+1)/J)
        np.testing.assert_array_equal(np.floor(h * J), np.arange(J))


def test_halton_nd_uses_kth_prime():
    assert [O.nth_prime(k) for k in range(1, 8)] == [2, 3, 5, 7, 11, 13, 17]
    np.testing.assert_array_equal(O.halton_nd(2, 4), [1 / 3, 2 / 3, 1 / 9, 4 / 9])


def test_step_counts_clamp_and_ceil():
    l, n = O.step_counts(np.array([1e-9, 0.25, 0.5, 0.999, 1.0]), 2.0, 0.1, 15)
    np.testing.assert_array_equal(n, [1, 5, 10, 15, 15])
    np.testing.assert_array_equal(l, [2e-9, 0.5, 1.0, 1.998, 2.0])


def test_ess_identities():
    J = 37
    assert O.ess(np.full(J, -3.2)) == pytest.approx(J, rel=1e-15)
    lw = np.full(J, -np.inf)
    lw[5] = 1.0
    assert O.ess(lw) == 1.0
    lw[[1, 9, 30]] = 1.0
    assert O.ess(lw) == pytest.approx(4.0, rel=1e-15)
    rng = np.random.default_rng(0)
    lw = rng.standard_normal(J) * 3
    w = np.exp(lw) / np.sum(np.exp(lw))
    assert O.ess(lw) == pytest.approx(1.0 / np.sum(w * w), rel=1e-12)
    assert O.ess(lw + 1234.5) == pytest.approx(O.ess(lw), rel=1e-12)
    np.testing.assert_allclose(O.normalise(lw + 700.0), w, rtol=1e-12)
    assert 1.0 <= O.ess(lw) <= J


def test_log_sum_exp_matches_direct_sum():
    rng = np.random.default_rng(1)
    lw = rng.standard_normal(50)
    m, S, S2 = O.log_sum_exp(lw)
    assert m + math.log(S) == pytest.approx(math.log(sum(math.exp(v) for v in lw)), rel=1e-14)
    assert O.log_sum_exp(np.full(4, -np.inf))[1] == 0.0


def test_realised_estimates():
    theta = np.array([[1.0, 2.0], [3.0, 6.0]])
    lw = np.log(np.array([0.25, 0.75]))
    mean, var = O.realised_mean_var(theta, lw)
    np.testing.assert_allclose(mean, [2.5, 5.0])
    np.testing.assert_allclose(var, [0.75, 3.0])
