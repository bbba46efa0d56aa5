"""Pins of the flow oracle (oracle/flow.py): identity special case, inverse,
log-determinant against a finite-difference Jacobian, the latent gradient and
the training gradient against finite differences, Adam's first step, the
exactness of the latent leapfrog (reversibility), the identity flow reducing
the SMC iteration to the plain one, and training whitening a correlated
Gaussian population."""

import math

import numpy as np
import pytest

from oracle import flow as F, smc as O


def _random_flow(d, layers=4, width=16, seed=0, scale=0.3):
    rng = np.random.default_rng(seed)
    ps = F.init_params(d, layers, width, rng)
    for p in ps:
        p["W3"] = scale * rng.standard_normal(p["W3"].shape) / math.sqrt(width)
        p["b3"] = scale * rng.standard_normal(p["b3"].shape)
        p["b1"] = 0.1 * rng.standard_normal(p["b1"].shape)
        p["b2"] = 0.1 * rng.standard_normal(p["b2"].shape)
    m = rng.standard_normal(d)
    A = rng.standard_normal((d, d))
    S = A @ A.T / d + 0.5 * np.eye(d)
    return ps, F.Base(m, np.linalg.cholesky(S))


def test_zero_last_layer_is_the_identity():
    d = 7
    ps = F.init_params(d, 4, 16, np.random.default_rng(1))
    z = np.random.default_rng(2).standard_normal((5, d))
    q = F.interleave(d)
    # the identity couplings leave only the interleaving: theta_c = z_q(c)
    assert sorted(q) == list(range(d)) and list(q[:4]) == [0, 4, 1, 5]
    I = F.Base(np.zeros(d), np.eye(d))
    th, ld = F.forward(ps, I, z)
    assert np.array_equal(th, z[:, q]) and np.array_equal(ld, np.zeros(5))
    g = np.random.default_rng(3).standard_normal((5, d))
    gz = F.latent_grad(ps, I, z, g)
    assert np.array_equal(gz[:, q], g)


@pytest.mark.parametrize("d", [2, 5, 8])
def test_inverse_undoes_forward(d):
    ps, B = _random_flow(d, seed=d)
    z = np.random.default_rng(4).standard_normal((6, d))
    th, ld = F.forward(ps, B, z)
    z2, ldi = F.inverse(ps, B, th)
    np.testing.assert_allclose(z2, z, rtol=0, atol=1e-12)
    np.testing.assert_allclose(ldi, -ld, rtol=0, atol=1e-12)


def test_log_det_matches_finite_difference_jacobian():
    d = 5
    ps, B = _random_flow(d, seed=7)
    z = np.random.default_rng(8).standard_normal(d)
    h = 1e-6
    Jm = np.zeros((d, d))
    for i in range(d):
        e = np.zeros(d)
        e[i] = h
        Jm[:, i] = (F.forward(ps, B, z + e)[0][0] - F.forward(ps, B, z - e)[0][0]) / (2 * h)
    ld = F.forward(ps, B, z)[1][0]
    assert ld == pytest.approx(np.linalg.slogdet(Jm)[1], abs=1e-7)


def test_latent_gradient_matches_finite_differences():
    d = 6
    ps, B = _random_flow(d, seed=11)
    rng = np.random.default_rng(12)
    A = rng.standard_normal((d, d))
    t = O.Gaussian(rng.standard_normal(d), A @ A.T + np.eye(d))

    def logpz(z):
        th, ld = F.forward(ps, B, z[None])
        return t.log_and_grad(th)[0][0] + ld[0]

    z = rng.standard_normal(d)
    th, _ = F.forward(ps, B, z[None])
    g = F.latent_grad(ps, B, z[None], t.log_and_grad(th)[1])[0]
    h = 1e-6
    fd = np.array([(logpz(z + h * e) - logpz(z - h * e)) / (2 * h) for e in np.eye(d)])
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-7)


def test_training_gradient_matches_finite_differences():
    d = 5
    ps, B = _random_flow(d, layers=3, width=8, seed=21)
    rng = np.random.default_rng(22)
    theta = rng.standard_normal((40, d)) * 1.5 + 0.5
    W = rng.random(40)
    W /= W.sum()
    _, grads = F.objective_and_grad(ps, B, theta, W)
    h = 1e-6
    for l in range(3):
        for key in ("W1", "b1", "W2", "b2", "W3", "b3"):
            idx = tuple(rng.integers(0, s) for s in ps[l][key].shape)
            up = [dict(p) for p in ps]
            dn = [dict(p) for p in ps]
            up[l] = {k: v.copy() for k, v in ps[l].items()}
            dn[l] = {k: v.copy() for k, v in ps[l].items()}
            up[l][key][idx] += h
            dn[l][key][idx] -= h
            fd = (F.objective_and_grad(up, B, theta, W)[0]
                  - F.objective_and_grad(dn, B, theta, W)[0]) / (2 * h)
            assert grads[l][key][idx] == pytest.approx(fd, rel=1e-5, abs=1e-8), (l, key)


def test_adam_first_step_is_lr_times_sign():
    d = 4
    ps = F.init_params(d, 2, 8, np.random.default_rng(5))
    g = [{k: np.random.default_rng(6 + i).standard_normal(v.shape) for k, v in p.items()}
         for i, p in enumerate(ps)]
    ad = F.FlowAdam(1e-3)
    q = ad.ascend(ps, g)
    for p0, p1, gg in zip(ps, q, g):
        for k in p0:
            # lr g / (|g| + eps_A): lr sign(g) to within lr eps_A / |g|
            dev = np.abs(p1[k] - p0[k] - 1e-3 * np.sign(gg[k]))
            assert np.all(dev <= 1e-3 * 1e-8 / np.abs(gg[k]) + 1e-15)


def test_latent_leapfrog_is_reversible():
    d = 4
    ps, B = _random_flow(d, seed=31)
    rng = np.random.default_rng(32)
    t = O.Gaussian(np.zeros(d), np.diag([0.5, 1.0, 2.0, 4.0]))
    z0 = rng.standard_normal((3, d))
    p0 = rng.standard_normal((3, d))
    th0, _ = F.forward(ps, B, z0)
    g0 = F.latent_grad(ps, B, z0, t.log_and_grad(th0)[1])
    n = np.array([5, 9, 13])
    z1, p1, g1, *_ = F.leapfrog_latent(t, ps, B, z0, p0, g0, 0.05, n)
    z2, p2, *_ = F.leapfrog_latent(t, ps, B, z1, -p1, g1, 0.05, n)
    np.testing.assert_allclose(z2, z0, atol=1e-11)
    np.testing.assert_allclose(-p2, p0, atol=1e-11)


def test_identity_flow_iteration_equals_the_plain_iteration():
    """With no training and a zero last layer the latent map is theta = m +
    exp(a) z, a linear change of variables; with m = 0, a = 0 forced (through
    a population that standardises to them exactly is impractical), check the
    pure identity directly: latent leapfrog with the identity flow equals the
    plain leapfrog bit for bit."""
    d = 5
    X = np.random.default_rng(41).standard_normal((60, d))
    y = (np.random.default_rng(42).random(60) < 0.5).astype(float)
    t = O.LogisticRegression(X, y)
    ps = F.init_params(d, 4, 16, np.random.default_rng(43))
    q = F.interleave(d)
    th0 = np.random.default_rng(44).standard_normal((8, d)) * 0.3
    p0 = np.random.default_rng(45).standard_normal((8, d))
    z0 = np.empty_like(th0)
    z0[:, q] = th0
    pz0 = np.empty_like(p0)
    pz0[:, q] = p0
    lp0, g0 = t.log_and_grad(th0)
    n = np.arange(1, 9)
    I = F.Base(np.zeros(d), np.eye(d))
    zl, pl, gl, thl, gthl, lpl, ldl = F.leapfrog_latent(
        t, ps, I, z0, pz0, F.latent_grad(ps, I, z0, g0), 0.07, n)
    th, p, g, lp, _ = O.leapfrog(t, th0, p0, g0, 0.07, n)
    assert np.array_equal(thl, th) and np.array_equal(pl[:, q], p) and np.array_equal(lpl, lp)
    assert np.array_equal(zl[:, q], th) and np.array_equal(ldl, np.zeros(8))


def test_dense_base_whitens_a_correlated_population():
    # the base map alone: L L^T is the shrunk weighted covariance and the
    # standardised population has the identity covariance (up to shrinkage)
    d = 6
    rho = 0.9
    S = rho ** np.abs(np.subtract.outer(np.arange(d), np.arange(d)))
    rng = np.random.default_rng(51)
    theta = rng.standard_normal((20000, d)) @ np.linalg.cholesky(S).T * 2.0 + 1.0
    lw = np.full(20000, -math.log(20000))
    B = F.standardise(theta, lw, 20000.0)
    C = np.cov(theta.T, bias=True)
    np.testing.assert_allclose(B.L @ B.L.T, 20000 / 20005 * C + 1e-3 * 5 / 20005 * np.eye(d),
                               rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(B.Linv @ B.L, np.eye(d), atol=1e-6)
    ps = F.init_params(d, 2, 16, np.random.default_rng(0))
    z, _ = F.inverse(ps, B, theta)
    np.testing.assert_allclose(np.cov(z.T, bias=True), np.eye(d), atol=2e-3)


def test_training_captures_a_nonlinear_dependence():
    # theta_2 = theta_1^2 + noise: the dense base cannot remove the dependence
    # of z_2 on z_1^2; trained couplings shrink it and raise the likelihood
    d = 4
    rng = np.random.default_rng(52)
    t1 = rng.standard_normal(3000)
    theta = np.stack([t1, t1 ** 2 + 0.3 * rng.standard_normal(3000),
                      rng.standard_normal(3000), rng.standard_normal(3000)], 1)
    lw = np.full(3000, -math.log(3000))
    B = F.standardise(theta, lw, 3000.0)
    ps = F.init_params(d, 4, 32, np.random.default_rng(53))
    W = np.full(3000, 1 / 3000)

    def dep(z):
        q = F.interleave(d)
        return abs(np.corrcoef(z[:, q[1]], z[:, q[0]] ** 2)[0, 1])

    z0, _ = F.inverse(ps, B, theta)
    obj0, _ = F.objective_and_grad(ps, B, theta, W)
    ad = F.FlowAdam(1e-2)
    for _ in range(300):
        _, g = F.objective_and_grad(ps, B, theta, W)
        ps = ad.ascend(ps, g)
    obj1, _ = F.objective_and_grad(ps, B, theta, W)
    z1, _ = F.inverse(ps, B, theta)
    assert obj1 > obj0 + 0.5, (obj0, obj1)
    assert dep(z1) < 0.5 * dep(z0), (dep(z0), dep(z1))


def test_flow_smc_keeps_gaussian_population_on_target():
    # a population drawn from a correlated Gaussian target with equal weights
    # stays properly weighted under flow-preconditioned moves (exact weights)
    d = 4
    rng = np.random.default_rng(61)
    A = rng.standard_normal((d, d))
    S = A @ A.T / d + 0.2 * np.eye(d)
    mu = rng.standard_normal(d)
    t = O.Gaussian(mu, S)
    J = 3000
    o = O.OracleSMC(t, J, step_size=0.3, traj_length=1.2, max_leapfrog=12, num_warmup=2,
                    precond="flow", flow_layers=2, flow_width=16, flow_train_steps=5,
                    flow_lr=1e-2, seed=3)
    o.set_state(mu + rng.standard_normal((J, d)) @ np.linalg.cholesky(S).T, np.full(J, -math.log(J)))
    for _ in range(4):
        o.step()
        o.adapt()
    mm, vv = o.moments()
    ess = O.ess(o.logw)
    assert np.all(np.abs(mm - mu) <= 5 * np.sqrt(np.diag(S) / ess)), (mm, mu, ess)
    assert np.all(np.abs(vv / np.diag(S) - 1) < 0.15), vv
