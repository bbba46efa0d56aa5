"""Pins for the oracle's ChEES statistics and adaptation (Sec. II-C,
Alg. smc_ChEES), against closed forms for Gaussian targets under the exact
Hamiltonian flow, Adam's first-step property and the moving average."""

import math

import numpy as np
import pytest

from oracle import smc as O


def _exact_flow(J, D, t, seed):
    # For N(0, I) and M = I, Hamilton's equations give
    # theta(t) = theta0 cos t + p0 sin t,  p(t) = -theta0 sin t + p0 cos t.
    rng = np.random.default_rng(seed)
    th0 = rng.standard_normal((J, D))
    p0 = rng.standard_normal((J, D))
    return th0, th0 * math.cos(t) + p0 * math.sin(t), -th0 * math.sin(t) + p0 * math.cos(t)


@pytest.mark.parametrize("t", [0.4, 1.0, 2.0])
def test_chees_value_closed_form(t):
    # ChEES(t) = D sin^2 t for N(0, I_D): per dimension
    # ||theta'||^2 - ||theta||^2 = sin^2 t (p^2 - theta^2) + sin 2t theta p, variance 4 sin^2 t.
    J, D = 200000, 3
    th0, th1, p1 = _exact_flow(J, D, t, 0)
    st = O.chees_statistics(th0, th1, p1, np.full(J, t), np.ones(J))
    ref = D * math.sin(t) ** 2
    # Var(a^2)/J bounds the Monte Carlo error of the 1/4 mean a^2
    se = 0.25 * math.sqrt(np.var(st["a"] ** 2) / J)
    assert abs(st["chees"] - ref) < 4 * se + 1e-3


@pytest.mark.parametrize("t", [0.4, 1.0, 2.0])
def test_chees_gradient_closed_form(t):
    # E[g] = t dChEES/dt = t D sin 2t (l = t, alpha = 1).
    J, D = 200000, 2
    th0, th1, p1 = _exact_flow(J, D, t, 1)
    st = O.chees_statistics(th0, th1, p1, np.full(J, t), np.ones(J))
    ref = t * D * math.sin(2 * t)
    se = math.sqrt(np.var(st["g"]) / J)
    assert abs(st["ghat"] - ref) < 4 * se + 2e-3


def test_chees_alpha_weighting_and_zero_alpha():
    rng = np.random.default_rng(2)
    th0, th1, p1 = rng.standard_normal((3, 10, 2))
    alpha = rng.random(10)
    st = O.chees_statistics(th0, th1, p1, np.ones(10), alpha)
    assert st["ghat"] == pytest.approx(np.dot(alpha, st["g"]) / alpha.sum(), rel=1e-14)
    st0 = O.chees_statistics(th0, th1, p1, np.ones(10), np.zeros(10))
    assert st0["ghat"] == 0.0 and st0["sum_alpha"] == 0.0
    # translating both populations leaves the statistics unchanged
    st1 = O.chees_statistics(th0 + 5.0, th1 - 2.0, p1, np.ones(10), alpha)
    assert st1["ghat"] == pytest.approx(st["ghat"], rel=1e-12)


def test_adam_first_step_is_signed_learning_rate():
    for g in (3.7, -0.002, 1e4):
        a = O.Adam(0.025, 0.9, 0.999, 1e-8)
        x1 = a.ascend(1.0, g)
        # bias correction: mhat_1 = g, vhat_1 = g^2
        assert x1 - 1.0 == pytest.approx(0.025 * g / (abs(g) + 1e-8), rel=1e-12)


def test_adam_constant_gradient_moves_lr_per_step():
    a = O.Adam(0.1, 0.9, 0.999, 1e-8)
    x = 0.0
    for _ in range(50):
        x = a.ascend(x, 2.0)
    assert x == pytest.approx(5.0, rel=1e-6)


def test_moving_average_and_freeze():
    # With ghat forced to zero (sum alpha = 0), L stays at L0 and after m updates
    # Lbar = (1 - 0.9^m) L0; at m = M_w, L <- Lbar.
    t = O.Gaussian(np.zeros(2), np.eye(2))
    s = O.OracleSMC(t, 8, theta0=np.zeros((8, 2)), num_warmup=4, traj_length=2.0, step_size=0.5)
    for m in range(1, 6):
        s.step()
        s.last["sum_alpha"] = 0.0
        s.adapt()
        if m < 4:
            assert s.L == 2.0
            assert s.Lbar == pytest.approx((1 - 0.9 ** m) * 2.0, rel=1e-15)
        else:
            assert s.L == pytest.approx((1 - 0.9 ** 3) * 2.0, rel=1e-15)


def test_adaptation_reaches_closed_form_optimum():
    # For N(0, I_D) under the exact flow, ChEES(t) = D sin^2 t.  With jitter
    # h ~ U(0, 1) the adapted L maximises E_h[sin^2(h L)], whose stationary point
    # solves tan(2L) = 2L, L* = 2.2467.  The whole loop (Alg. smc_ChEES: final
    # momentum in g_c, alpha weighting, Adam ascent on log L) must find it; using
    # the initial momentum or descending would settle elsewhere.
    t = O.Gaussian(np.zeros(10), np.eye(10))
    s = O.OracleSMC(t, 1000, seed=1, step_size=0.05, traj_length=0.8, num_warmup=100,
                    adam_lr=0.05, max_leapfrog=200)
    Ls = []
    for _ in range(60):
        s.step()
        s.adapt()
        Ls.append(s.L)
    assert 1.95 < np.mean(Ls[-20:]) < 2.55
