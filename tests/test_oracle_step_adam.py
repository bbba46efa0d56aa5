"""Pins of the oracle's optional step-size adaptation by Adam on log eps
toward a harmonic-mean acceptance (not in the paper, whose step size is fixed;
Sec. II-A gives the acceptance probability it acts on, Alg. smc_ChEES the
warm-up branch it runs in).  Closed forms: the harmonic mean of a few values
and its floor; Adam's bias-corrected step under a constant gradient,
lr g / (|g| + eps_A) at every step; the direction of the move; L left alone
when sum alpha = 0; nothing moves after the freeze at k = M_w."""

import math

import numpy as np
import pytest

from oracle import smc as O

LR, EPS_A, TARGET = 0.025, 1e-8, 0.651


def test_harmonic_mean_values():
    assert O.harmonic_mean([1.0, 0.5]) == 2.0 / 3.0          # 2 / (1 + 2)
    assert O.harmonic_mean([0.25, 0.25, 0.25]) == 0.25
    # below the arithmetic mean whenever the values differ
    assert O.harmonic_mean([1.0, 0.2]) == pytest.approx(2.0 / 6.0, rel=1e-15)
    assert O.harmonic_mean([1.0, 0.2]) < 0.6


def test_harmonic_mean_floor():
    # alpha = 0 is replaced by the floor, so one zero pulls the mean to ~J floor
    assert O.harmonic_mean([0.0]) == 1e-20
    assert O.harmonic_mean([0.0, 1.0]) == pytest.approx(2.0 / (1e20 + 1.0), rel=1e-15)
    assert O.harmonic_mean([0.0, 1.0], floor=0.5) == pytest.approx(2.0 / 3.0, rel=1e-15)


def _oracle(eps0=0.2, L0=1.0, Mw=10):
    t = O.Gaussian(np.zeros(2), np.eye(2))
    return O.OracleSMC(t, 4, theta0=np.zeros((4, 2)), step_size=eps0, traj_length=L0,
                       num_warmup=Mw, adapt_step_size="adam", target_accept=TARGET,
                       adam_lr=LR, adam_eps=EPS_A)


def _adapt(o, k, alpha, ghat=0.0):
    alpha = np.asarray(alpha, dtype=np.float64)
    o.k = k
    o.last = dict(sum_alpha=float(np.sum(alpha)), ghat=ghat, alpha=alpha)
    return o.adapt()


@pytest.mark.parametrize("c", [0.9, 0.3])
def test_first_step_is_bias_corrected_signed_lr(c):
    # all alpha = c: harmonic mean c, gap g = c - target; Adam's first step is
    # m_hat / (sqrt(v_hat) + eps_A) = g / (|g| + eps_A)
    o = _oracle()
    _adapt(o, 1, [c] * 4)
    g = c - TARGET
    assert math.log(o.eps) - math.log(0.2) == pytest.approx(LR * g / (abs(g) + EPS_A), rel=1e-12)


def test_constant_gap_moves_lr_per_step():
    # a constant gradient keeps m_hat = g and v_hat = g^2 exactly (up to
    # rounding), so m steps move log eps by m lr g / (|g| + eps_A)
    o = _oracle(Mw=50)
    m = 20
    for k in range(1, m + 1):
        _adapt(o, k, [0.95] * 4)
    g = 0.95 - TARGET
    assert math.log(o.eps) - math.log(0.2) == pytest.approx(m * LR * g / (abs(g) + EPS_A),
                                                           rel=1e-9)


def test_harmonic_not_arithmetic_mean_decides_direction():
    # harmonic mean 0.571 < target 0.651 < arithmetic mean 0.7: eps must shrink
    o = _oracle()
    _adapt(o, 1, [1.0, 0.4, 1.0, 0.4])
    assert o.eps < 0.2
    hm = 2.0 / 3.5
    assert math.log(o.eps) - math.log(0.2) == pytest.approx(
        LR * (hm - TARGET) / (abs(hm - TARGET) + EPS_A), rel=1e-12)
    # acceptance above the target grows eps
    o2 = _oracle()
    _adapt(o2, 1, [0.99] * 4)
    assert o2.eps > 0.2


def test_zero_acceptance_leaves_L_and_shrinks_eps():
    # sum alpha = 0 skips the ChEES update of L (whatever g_hat says) but the
    # step size still sees the floored harmonic mean and moves down by ~lr
    o = _oracle(L0=1.5)
    r = _adapt(o, 1, [0.0] * 4, ghat=7.0)
    assert r["L"] == 1.5 and o.L == 1.5
    assert r["Lbar"] == pytest.approx(0.1 * 1.5, rel=1e-15)
    g = 1e-20 - TARGET
    assert math.log(o.eps) - math.log(0.2) == pytest.approx(LR * g / (abs(g) + EPS_A), rel=1e-12)


def test_L_and_eps_adapt_together_then_freeze():
    # both Adams run in the same warm-up step; at k = M_w, L <- L_bar and eps
    # keeps its last value; afterwards nothing moves
    o = _oracle(Mw=3)
    for k in (1, 2):
        _adapt(o, k, [0.9] * 4, ghat=2.0)
    g = 0.9 - TARGET
    assert math.log(o.eps) - math.log(0.2) == pytest.approx(2 * LR * g / (abs(g) + EPS_A),
                                                           rel=1e-9)
    assert math.log(o.L) == pytest.approx(2 * LR * 2.0 / (2.0 + EPS_A), rel=1e-9)
    L1 = math.exp(LR * 2.0 / (2.0 + EPS_A))
    Lbar = 0.9 * (0.1 * L1) + 0.1 * o.L
    eps_w = o.eps
    _adapt(o, 3, [0.1] * 4, ghat=-5.0)
    assert o.L == pytest.approx(Lbar, rel=1e-14)
    assert o.eps == eps_w
    _adapt(o, 4, [0.1] * 4, ghat=-5.0)
    assert o.L == pytest.approx(Lbar, rel=1e-14) and o.eps == eps_w
