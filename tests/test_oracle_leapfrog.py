"""Pins for the oracle's leapfrog integrator (Sec. II-A, eqs. LF_p1/2,
LF_theta, LF_p; Alg. LF_example) and its energy bookkeeping."""

import math

import numpy as np
import pytest

from oracle import smc as O


def _std_normal_1d():
    return O.Gaussian(np.zeros(1), np.eye(1))


@pytest.mark.parametrize("eps,n", [(0.1, 1), (0.3, 7), (0.05, 40)])
def test_harmonic_oscillator_matrix(eps, n):
    # For H = p^2/2 + q^2/2 one kick-drift-kick step is the linear map
    # [[1 - e^2/2, e], [-e (1 - e^2/4), 1 - e^2/2]] acting on (q, p).
    A = np.array([[1 - eps ** 2 / 2, eps], [-eps * (1 - eps ** 2 / 4), 1 - eps ** 2 / 2]])
    assert np.linalg.det(A) == pytest.approx(1.0, abs=1e-15)
    q0, p0 = 0.8, -1.3
    t = _std_normal_1d()
    _, g0 = t.log_and_grad(np.array([[q0]]))
    th, p, g, lp, ng = O.leapfrog(t, np.array([[q0]]), np.array([[p0]]), g0, eps, np.array([n]))
    ref = np.linalg.matrix_power(A, n) @ np.array([q0, p0])
    assert th[0, 0] == pytest.approx(ref[0], abs=1e-13)
    assert p[0, 0] == pytest.approx(ref[1], abs=1e-13)
    assert ng[0] == n
    # the shadow energy p^2/2 + (1 - e^2/4) q^2/2 is conserved exactly
    sh0 = 0.5 * p0 ** 2 + 0.5 * (1 - eps ** 2 / 4) * q0 ** 2
    sh1 = 0.5 * p[0, 0] ** 2 + 0.5 * (1 - eps ** 2 / 4) * th[0, 0] ** 2
    assert sh1 == pytest.approx(sh0, abs=1e-13)
    # Delta H = (eps^2/8) (q'^2 - q^2) follows from the shadow energy
    dh = O.delta_h(t.log_and_grad(np.array([[q0]]))[0], np.array([[p0]]), lp, p)
    assert dh[0] == pytest.approx(eps ** 2 / 8 * (th[0, 0] ** 2 - q0 ** 2), abs=1e-13)


def _logistic(seed=0, N=30, d=3):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((N, d))
    y = (rng.random(N) < 0.5).astype(float)
    return O.LogisticRegression(X, y)


def test_reversibility_on_logistic():
    t = _logistic()
    rng = np.random.default_rng(1)
    th0 = 0.3 * rng.standard_normal((4, 3))
    p0 = rng.standard_normal((4, 3))
    _, g0 = t.log_and_grad(th0)
    n = np.array([1, 5, 17, 33])
    th1, p1, g1, _, _ = O.leapfrog(t, th0, p0, g0, 0.05, n)
    th2, p2, _, _, _ = O.leapfrog(t, th1, -p1, g1, 0.05, n)
    np.testing.assert_allclose(th2, th0, atol=1e-11)
    np.testing.assert_allclose(-p2, p0, atol=1e-11)


def test_volume_preservation_finite_difference_jacobian():
    t = _logistic(seed=2, N=20, d=2)
    x0 = np.array([0.2, -0.1, 0.7, 1.1])  # (theta, p)

    def flow(x):
        th = x[None, :2]
        _, g = t.log_and_grad(th)
        a, b, _, _, _ = O.leapfrog(t, th, x[None, 2:], g, 0.08, np.array([6]))
        return np.concatenate([a[0], b[0]])

    h = 1e-6
    Jm = np.zeros((4, 4))
    for i in range(4):
        e = np.zeros(4)
        e[i] = h
        Jm[:, i] = (flow(x0 + e) - flow(x0 - e)) / (2 * h)
    assert np.linalg.det(Jm) == pytest.approx(1.0, abs=1e-7)


def test_masked_steps_leave_finished_particles_alone():
    t = _logistic()
    rng = np.random.default_rng(3)
    th0 = rng.standard_normal((3, 3)) * 0.2
    p0 = rng.standard_normal((3, 3))
    _, g0 = t.log_and_grad(th0)
    a = O.leapfrog(t, th0, p0, g0, 0.05, np.array([2, 9, 4]))
    for j, nj in enumerate([2, 9, 4]):
        b = O.leapfrog(t, th0[j:j + 1], p0[j:j + 1], g0[j:j + 1], 0.05, np.array([nj]))
        # equal up to the BLAS's blocking of the row count
        np.testing.assert_allclose(a[0][j], b[0][0], rtol=1e-13, atol=1e-15)
        np.testing.assert_allclose(a[1][j], b[1][0], rtol=1e-13, atol=1e-15)


def test_energy_error_vanishes_with_step_size():
    t = _logistic(seed=4)
    rng = np.random.default_rng(4)
    th0 = 0.2 * rng.standard_normal((1, 3))
    p0 = rng.standard_normal((1, 3))
    lp0, g0 = t.log_and_grad(th0)
    errs = []
    for eps in (0.04, 0.02, 0.01):
        n = int(round(0.4 / eps))
        _, p1, _, lp1, _ = O.leapfrog(t, th0, p0, g0, eps, np.array([n]))
        errs.append(abs(O.delta_h(lp0, p0, lp1, p1)[0]))
    # second-order integrator: halving eps divides the error by about 4
    assert errs[1] < errs[0] / 3 and errs[2] < errs[1] / 3


def test_acceptance_probability():
    dh = np.array([-1.0, 0.0, 0.5, np.inf])
    np.testing.assert_allclose(O.accept_prob(dh), [1.0, 1.0, math.exp(-0.5), 0.0])
    assert O.delta_h(np.array([np.nan]), np.zeros((1, 1)), np.array([0.0]), np.zeros((1, 1)))[0] == np.inf


def test_gradient_count_convention_no_jitter_cap():
    # No jitter (h = 1), L = 5, eps = 0.001, cap 500: every trajectory hits the
    # cap, and with the gradient taken before the loop each particle costs
    # 501 gradients per iteration -- Table I, "No Jitter" entries of 501.00.
    _, n = O.step_counts(np.ones(1000), 5.0, 0.001, 500)
    assert np.all(n == 500)
    assert float(np.mean(n + 1)) == 501.0


def test_bf16_rounding_ties_to_even_and_matches_torch():
    import torch
    cases = {1.0: 1.0, 1.0 + 2 ** -8: 1.0, 1.0 + 3 * 2 ** -8: 1.0 + 2 ** -6,
             1.0 + 2 ** -8 + 2 ** -20: 1.0 + 2 ** -7, -(1.0 + 2 ** -8 + 2 ** -20): -(1.0 + 2 ** -7),
             0.0: 0.0, 3.0e38: 226 / 128 * 2.0 ** 127}
    for x, r in cases.items():
        assert O.bf16_round(x) == pytest.approx(r, rel=1e-7)
    assert np.isnan(O.bf16_round(np.nan)) and O.bf16_round(np.inf) == np.inf
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000) * 10 ** rng.uniform(-6, 6, 20000),
                        rng.uniform(-1, 1, 20000)]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(O.bf16_round(x), ref)


def test_bf16_gradient_is_the_exact_gradient_on_bf16_grids():
    # When theta, X and the residual are already bfloat16 values, the
    # precision-form gradient equals the exact one: choose y and theta so that
    # sigmoid(X theta) = 1/2 (theta = 0) and y in {0, 1}: R = +-1/2 exactly.
    rng = np.random.default_rng(4)
    X = O.bf16_round(rng.standard_normal((40, 6)))
    y = (rng.random(40) < 0.5).astype(float)
    t = O.LogisticRegression(X, y)
    th = np.zeros((3, 6))
    np.testing.assert_allclose(t.grad_bf16(th), t.log_and_grad(th)[1], rtol=0, atol=1e-12)
    # and it differs from the exact gradient at a generic point by about 2^-8
    th = rng.standard_normal((3, 6)) * 0.3
    rel = np.abs(t.grad_bf16(th) - t.log_and_grad(th)[1]).max() / np.abs(t.log_and_grad(th)[1]).max()
    assert 1e-6 < rel < 2e-2


def test_bf16_trajectories_keep_weights_exact():
    # With any position-only force field the leapfrog map is volume preserving
    # and reversible, so the weight increment -Delta H with exact energies
    # remains the exact change-of-variables weight: reversing the BF16
    # trajectory returns to the start.
    rng = np.random.default_rng(5)
    X = rng.standard_normal((50, 3))
    y = (rng.random(50) < 0.5).astype(float)
    t = O.LogisticRegression(X, y)
    th0 = 0.2 * rng.standard_normal((4, 3))
    p0 = rng.standard_normal((4, 3))
    g0 = t.grad_bf16(th0)
    n = np.array([3, 9, 15, 21])
    th1, p1, g1, _, _ = O.leapfrog(t, th0, p0, g0, 0.05, n, traj_grad=t.grad_bf16)
    th2, p2, _, _, _ = O.leapfrog(t, th1, -p1, g1, 0.05, n, traj_grad=t.grad_bf16)
    np.testing.assert_allclose(th2, th0, atol=1e-11)
    np.testing.assert_allclose(-p2, p0, atol=1e-11)
