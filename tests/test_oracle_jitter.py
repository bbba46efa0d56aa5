"""Pins of the oracle's jitter generators (Sec. III-B-1) against values and
properties the definitions fix independently of the code: hand-computed
radical inverses, closed forms of j sqrt(p) mod 1 and of the golden-ratio
sequence, the three-distance theorem, permutation and uniformity properties.
"""

import math

import numpy as np
import pytest
from scipy import stats

from oracle import philox, smc as O


# --- N-d inverse Halton ---------------------------------------------------------

def test_inverse_halton_first_column_uses_last_base():
    # K = 3: iteration 1 takes column 3, base P_3 = 5; by hand
    # phi_5(1..6) = 1/5, 2/5, 3/5, 4/5, 0/5 + 1/25, 1/5 + 1/25
    h = O.halton_nd_inverse(1, 3, 6)
    np.testing.assert_allclose(h, [0.2, 0.4, 0.6, 0.8, 0.04, 0.24], rtol=0, atol=1e-16)
    # iteration 3 of 3 takes column 1, base 2: 1/2, 1/4, 3/4, 1/8, 5/8, 3/8
    h = O.halton_nd_inverse(3, 3, 6)
    np.testing.assert_array_equal(h, [0.5, 0.25, 0.75, 0.125, 0.625, 0.375])
    # iteration 2 of 3: the middle column, base 3: 1/3, 2/3, 1/9, 4/9, 7/9, 2/9
    h = O.halton_nd_inverse(2, 3, 6)
    np.testing.assert_allclose(h, [1 / 3, 2 / 3, 1 / 9, 4 / 9, 7 / 9, 2 / 9], rtol=0, atol=1e-16)


def test_inverse_halton_wraps_after_K():
    # reading: a run longer than K starts over from column K
    np.testing.assert_array_equal(O.halton_nd_inverse(4, 3, 10), O.halton_nd_inverse(1, 3, 10))
    np.testing.assert_array_equal(O.halton_nd_inverse(6, 3, 10), O.halton_nd_inverse(3, 3, 10))


def test_inverse_halton_column_is_stratified():
    # radical inverse in base b: the first b^m points hit every cell [i/b^m, (i+1)/b^m) once
    # (they are (0, ..) shifted by one index: j = 1..b^m gives the cells 1..b^m - 1 and 0)
    K, b = 4, 7  # iteration 1 of 4 uses P_4 = 7
    h = O.halton_nd_inverse(1, K, b ** 2)
    cells = np.floor(h * b ** 2 + 1e-9).astype(int)  # h = i / 49 exactly up to rounding
    assert sorted(cells.tolist()) == list(range(b ** 2))


# --- N-d primes -------------------------------------------------------------------

def test_primes_closed_forms():
    h1 = O.primes_nd(1, 3)   # P_1 = 2
    np.testing.assert_allclose(h1, [math.sqrt(2) - 1, 2 * math.sqrt(2) - 2, 3 * math.sqrt(2) - 4],
                               rtol=0, atol=4e-16)
    h2 = O.primes_nd(2, 2)   # P_2 = 3
    np.testing.assert_allclose(h2, [math.sqrt(3) - 1, 2 * math.sqrt(3) - 3], rtol=0, atol=4e-16)
    h5 = O.primes_nd(5, 1)   # P_5 = 11
    assert h5[0] == pytest.approx(math.sqrt(11) - 3, abs=4e-16)


def _gaps(points):
    p = np.sort(np.mod(points, 1.0))
    g = np.diff(np.concatenate([p, [p[0] + 1.0]]))
    return g


def _distinct(values, tol):
    v = np.sort(values)
    out = [v[0]]
    for x in v[1:]:
        if x - out[-1] > tol:
            out.append(x)
    return out


@pytest.mark.parametrize("k", [1, 2, 3, 7])
def test_primes_three_distance(k):
    # three-distance theorem: {j alpha}, j = 1..n, alpha irrational, cut the
    # circle into gaps of at most three lengths
    h = O.primes_nd(k, 500)
    assert len(_distinct(_gaps(h), 1e-9)) <= 3
    assert np.all((h > 0) & (h < 1))


def test_primes_inverse_reverses_columns():
    K = 4
    np.testing.assert_array_equal(O.primes_nd_inverse(1, K, 20), O.primes_nd(4, 20))
    np.testing.assert_array_equal(O.primes_nd_inverse(4, K, 20), O.primes_nd(1, 20))


# --- 1-d golden ratio ---------------------------------------------------------------

def test_golden_closed_forms():
    g = (math.sqrt(5) - 1) / 2
    K = 5
    h = O.golden_1d(1, K, 3)   # indices 1, 6, 11
    np.testing.assert_allclose(h, [g, 6 * g - 3, 11 * g - 6], rtol=0, atol=1e-14)
    h = O.golden_1d(2, K, 1)   # index 2: 2 g - 1 = g^3 (from g^2 = 1 - g)
    assert h[0] == pytest.approx(g ** 3, abs=1e-15)


def test_golden_three_distance_and_order():
    # all J K values of the matrix are the first J K points of the sequence
    J, K = 40, 25
    allh = np.concatenate([O.golden_1d(k, K, J) for k in range(1, K + 1)])
    gaps = _gaps(allh)
    d = _distinct(gaps, 1e-9)
    assert len(d) <= 3
    # for the golden ratio the two largest gap lengths are in ratio 1/g
    d = sorted(d)
    assert d[-1] / d[-2] == pytest.approx((1 + math.sqrt(5)) / 2, rel=1e-6)


# --- uniform -------------------------------------------------------------------------

def test_uniform_jitter_distribution():
    J = 20000
    h = O.uniform_jitter(11, 3, J)
    assert np.all((h > 0) & (h < 1))
    assert stats.kstest(h, "uniform").pvalue > 1e-3
    h2 = O.uniform_jitter(11, 4, J)
    assert abs(np.corrcoef(h, h2)[0, 1]) < 0.05
    # the stream's first word, (x + 1/2) / 2^32
    w = philox.philox4x32_10((0, 5, 3, philox.STREAM_JITTER), philox.seed_key(11))[0]
    assert h[5] == (w + 0.5) / 2 ** 32


# --- equidistant ----------------------------------------------------------------------

@pytest.mark.parametrize("J", [1, 2, 3, 4, 5, 16, 17, 100, 257, 1000])
def test_shuffle_is_a_permutation(J):
    for k in (1, 2, 9):
        pi = O.shuffle(5, k, J)
        assert sorted(pi.tolist()) == list(range(J))
        h = O.equidistant(5, k, J)
        np.testing.assert_array_equal(np.sort(h), np.arange(1, J + 1) / J)


def test_shuffle_changes_with_iteration_and_posterior():
    J = 200
    a, b, c = O.shuffle(5, 1, J), O.shuffle(5, 2, J), O.shuffle(5, 1, J, b=1)
    assert not np.array_equal(a, b) and not np.array_equal(a, c)
    # not the identity and not a rotation
    assert np.mean(a == np.arange(J)) < 0.1
    assert len(set(((a - np.arange(J)) % J).tolist())) > J // 4


def test_shuffle_positions_uniform():
    # over many iterations particle 0's position is uniform on {0..J-1}
    J, Kn = 6, 3000
    pos = np.array([O.shuffle(17, k, J)[0] for k in range(1, Kn + 1)])
    counts = np.bincount(pos, minlength=J)
    assert stats.chisquare(counts).pvalue > 1e-3


def test_offset_equidistant():
    J = 3000
    h0 = O.equidistant(3, 2, J)
    h = O.equidistant_offset(3, 2, J)
    off = h - h0
    assert np.all((off > 0) & (off < 0.1 + 1e-15))
    assert stats.kstest(off / 0.1, "uniform").pvalue > 1e-3


# --- the sampler's dispatch ------------------------------------------------------------

@pytest.mark.parametrize("kind", ["uniform", "haltonNd_inv", "primes", "primes_inv", "golden",
                                  "equidistant", "equidistant_offset"])
def test_sampler_uses_scheme(kind):
    from paper_2504_02627_amd import synth
    X, y, _ = synth.logistic_iid(50, 3, 1)
    t = O.LogisticRegression(X.astype(np.float64), y.astype(np.float64))
    J = 64
    o = O.OracleSMC(t, J, theta0=np.zeros((J, 3)), jitter=kind, num_iterations=4, seed=9,
                    step_size=0.05, traj_length=0.5, max_leapfrog=16, num_warmup=2)
    h = o.jitter(2)
    assert h.shape == (J,) and np.all(h > 0) and np.all(h < 1.1)
    # distinct schemes give distinct columns
    o2 = O.OracleSMC(t, J, theta0=np.zeros((J, 3)), jitter="halton1d", seed=9,
                     step_size=0.05, traj_length=0.5, max_leapfrog=16, num_warmup=2)
    assert not np.array_equal(h, o2.jitter(2))


# --- Sobol ------------------------------------------------------------------------------

def test_sobol_first_dimension_by_hand():
    # nu_b = 2^-b: x_i is the base-2 radical inverse of the Gray code of i;
    # Gray codes of 1..8 are 1, 3, 2, 6, 7, 5, 4, 12
    np.testing.assert_array_equal(O.sobol_1d(1, 8), [1 / 2, 3 / 4, 1 / 4, 3 / 8, 7 / 8, 5 / 8,
                                                     1 / 8, 3 / 16])
    # iteration 2 of J = 4 continues the sequence at index 5
    np.testing.assert_array_equal(O.sobol_1d(2, 4), [7 / 8, 5 / 8, 1 / 8, 3 / 16])


def test_sobol_direction_integers_by_hand():
    # x + 1 (mask 3), m_1 = 1: m_i = 2 m_(i-1) ^ m_(i-1) -> 1, 3, 5, 15, 17
    assert O.sobol_direction_integers(3, [1], 5) == [1, 3, 5, 15, 17]
    # x^2 + x + 1 (mask 7), m = 1, 3: m_3 = 2 m_2 ^ 4 m_1 ^ m_1 = 6 ^ 4 ^ 1 = 3,
    # m_4 = 2 m_3 ^ 4 m_2 ^ m_2 = 6 ^ 12 ^ 3 = 9
    assert O.sobol_direction_integers(7, [1, 3], 4) == [1, 3, 3, 9]
    rows = O.joe_kuo_rows(3)
    assert rows[1][0] == 3 and rows[2][0] == 7 and rows[2][1][:2] == [1, 3]
    # dimension 2: nu = 1/2, 3/4, 5/8; points by hand
    np.testing.assert_array_equal(O.sobol_nd(2, 4, rows), [1 / 2, 1 / 4, 3 / 4, 3 / 8])
    # dimension 3: nu = 1/2, 3/4, 3/8
    np.testing.assert_array_equal(O.sobol_nd(3, 4, rows), [1 / 2, 1 / 4, 3 / 4, 5 / 8])


def test_sobol_matches_scipy():
    # the library generator the paper names, unscrambled, 32-bit: its points
    # 1..2^10 - 1 in every one of the first 200 dimensions, and its first
    # dimension continued past one block
    K = 200
    rows = O.joe_kuo_rows(K)
    ref = stats.qmc.Sobol(d=K, scramble=False, bits=32).random_base2(10)[1:]
    for k in (1, 2, 3, 4, 17, 64, 123, 200):
        np.testing.assert_array_equal(O.sobol_nd(k, 1023, rows), ref[:, k - 1])
    g = stats.qmc.Sobol(d=1, scramble=False, bits=32)
    g.fast_forward(1 + 2 * 300)                    # iteration 3 of J = 300
    np.testing.assert_array_equal(O.sobol_1d(3, 300), g.random(300)[:, 0])


def test_sobol_every_dimension_is_a_net():
    # any valid direction numbers (m_i odd, m_i < 2^i) make the first 2^m
    # points of each dimension, the point 0 included, hit every cell of width
    # 2^-m once; dimensions 1 and 2 together form a (0, m, 2)-net
    m = 8
    rows = O.joe_kuo_rows(60)
    for k in range(1, 61):
        x = np.concatenate([[0.0], O.sobol_nd(k, 2 ** m - 1, rows)])
        assert sorted((x * 2 ** m).astype(int).tolist()) == list(range(2 ** m))
    x1 = np.concatenate([[0.0], O.sobol_nd(1, 2 ** m - 1, rows)])
    x2 = np.concatenate([[0.0], O.sobol_nd(2, 2 ** m - 1, rows)])
    for a in range(m + 1):                         # boxes 2^-a x 2^-(m-a)
        cells = set(zip((x1 * 2 ** a).astype(int).tolist(), (x2 * 2 ** (m - a)).astype(int).tolist()))
        assert len(cells) == 2 ** m


def test_sobol_inverse_reverses_columns():
    rows = O.joe_kuo_rows(5)
    np.testing.assert_array_equal(O.sobol_nd_inverse(1, 5, 40, rows), O.sobol_nd(5, 40, rows))
    np.testing.assert_array_equal(O.sobol_nd_inverse(5, 5, 40, rows), O.sobol_nd(1, 40, rows))
    np.testing.assert_array_equal(O.sobol_nd_inverse(6, 5, 40, rows), O.sobol_nd(5, 40, rows))
