"""Pins of the oracle's funnel target and dual-averaging step-size adaptation
(both named as future work in Sec. VI): finite differences and the
normalisation of the funnel; the closed form of the dual-averaging recursion
under a constant acceptance, and its averaged iterate in product form."""

import math

import numpy as np
import pytest
from scipy import integrate

from oracle import smc as O


def test_funnel_gradient_finite_differences():
    t = O.Funnel(5, scale=3.0)
    rng = np.random.default_rng(0)
    th = rng.standard_normal((4, 5)) * np.array([2.0, 1, 1, 1, 1])
    _, g = t.log_and_grad(th)
    h = 1e-6
    for i in range(5):
        e = np.zeros(5)
        e[i] = h
        fd = (t.log_and_grad(th + e)[0] - t.log_and_grad(th - e)[0]) / (2 * h)
        np.testing.assert_allclose(g[:, i], fd, rtol=1e-6, atol=1e-6)


def test_funnel_is_normalised_and_v_marginal():
    t = O.Funnel(2, scale=3.0, log_scale=0.7)
    f = lambda x, v: math.exp(t.log_and_grad(np.array([[v, x]]))[0][0])
    Z, _ = integrate.dblquad(f, -20, 20, lambda v: -12 * math.exp(v / 2),
                             lambda v: 12 * math.exp(v / 2), epsabs=1e-10)
    assert Z == pytest.approx(math.exp(0.7), rel=1e-6)
    # integrating x out leaves N(v; 0, 9)
    for v in (-4.0, 0.0, 2.5):
        mv, _ = integrate.quad(lambda x: f(x, v), -12 * math.exp(v / 2), 12 * math.exp(v / 2),
                               epsabs=1e-12)
        ref = math.exp(0.7 - v * v / 18) / (3 * math.sqrt(2 * math.pi))
        assert mv == pytest.approx(ref, rel=1e-7)


def _oracle(J=8, eps0=0.2, Mw=30, delta=0.65):
    t = O.Gaussian(np.zeros(2), np.eye(2))
    return O.OracleSMC(t, J, theta0=np.zeros((J, 2)), step_size=eps0, traj_length=1.0,
                       num_warmup=Mw, adapt_step_size="dual_averaging", target_accept=delta)


def _drive(o, alphas):
    eps = []
    for m, a in enumerate(alphas, start=1):
        o.k = m
        o.last = dict(sum_alpha=float(np.sum(a)), ghat=0.0, alpha=np.asarray(a, dtype=float))
        o.adapt()
        eps.append(o.eps)
    return eps


def test_dual_averaging_on_target_acceptance():
    # alpha = delta every iteration: H_bar = 0, log eps_m = mu = log(10 eps0),
    # and the averaged iterate is mu from the first update on
    o = _oracle()
    eps = _drive(o, [np.full(8, 0.65)] * 30)
    np.testing.assert_allclose(eps, 10 * 0.2, rtol=1e-14)


def test_dual_averaging_closed_form_constant_acceptance():
    # alpha = c constant: H_bar_m = (delta - c) m / (m + t0), so
    # log eps_m = mu - sqrt(m) / gamma (delta - c) m / (m + t0)
    c, delta, eps0, Mw = 0.9, 0.65, 0.2, 30
    o = _oracle(eps0=eps0, Mw=Mw, delta=delta)
    eps = _drive(o, [np.full(8, c)] * (Mw - 1))
    mu = math.log(10 * eps0)
    for m, e in enumerate(eps, start=1):
        ref = mu - math.sqrt(m) / 0.05 * (delta - c) * m / (m + 10.0)
        assert math.log(e) == pytest.approx(ref, rel=1e-12, abs=1e-12)
    # freeze at m = M_w: the averaged iterate, written as a weighted sum
    # sum_m w_m log eps_m with w_m = m^-kappa prod_{i > m} (1 - i^-kappa)
    o.k = Mw
    o.adapt()
    logs = [math.log(e) for e in eps]
    M = Mw - 1
    wsum, tot = 0.0, 0.0
    for m in range(1, M + 1):
        w = m ** -0.75
        for i in range(m + 1, M + 1):
            w *= 1 - i ** -0.75
        tot += w * logs[m - 1]
        wsum += w
    assert wsum == pytest.approx(1.0, rel=1e-12)
    assert math.log(o.eps) == pytest.approx(tot, rel=1e-12)


def test_dual_averaging_moves_toward_target():
    # acceptance above the target raises eps, below lowers it
    o_hi, o_lo = _oracle(), _oracle()
    e_hi = _drive(o_hi, [np.full(8, 0.95)] * 5)
    e_lo = _drive(o_lo, [np.full(8, 0.2)] * 5)
    assert e_hi[-1] > 10 * 0.2 > e_lo[-1]
