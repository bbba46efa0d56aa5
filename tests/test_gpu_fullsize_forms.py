"""Full-size parity of the batched form and of the flow preconditioner, in the
launch configuration the benchmark times, against the oracle on the same
inputs and injected randomness.

Batched: the 64 posteriors of the benchmark (N_b ~ U{500..20000}, d_b ~
U{10..200}; 13 feature-tile groups, more than the four stream lanes, three of
them with d > 128), J = 1024 each, n_max = 64.  h and n for all 65536
particles bit for bit; theta' and p' of four particles of every posterior
(the longest and the shortest trajectory and two others) against the oracle's
leapfrog at 1e-5 relative (FP32) and Delta H at 1e-5 (|H0| + |H1|).  The BF16
form against the BF16-emulating oracle to the bars of check_bf16_trajectories
(over the 256 sampled particles), and its Delta H against the exact energies
of its own end points.

Flow: the Toeplitz model (N = 5000, d = 100, rows correlated 0.95^|i-j|),
J = 4096, four affine couplings of width 128 with couplings set from the host
(seeded, non-trivial), no fit.  The oracle forms its own base map from its own
initial weights; 256 sampled particles' z0 at 1e-5, z', theta', p' at 1e-5
(FP32) or to the BF16 bars, and Delta H at 1e-5 (|H0| + |H1|).

One iteration without resampling (ess_frac = 0), so every particle moves from
its injected theta_0."""

import numpy as np
import pytest

from oracle import flow as F, smc as O
from paper_2504_02627_amd import synth
from tests._gpu_common import check_bf16_trajectories, dev, log, rel_each, rel_rows, to_dev

pytestmark = pytest.mark.gpu

def _batched_case(precision):
    import torch
    from paper_2504_02627_amd import chees
    dev()
    data = synth.batched_logistic(64)
    J = 1024
    rng = np.random.default_rng(41)
    thetas = [(0.2 * rng.standard_normal((J, X.shape[1]))).astype(np.float32) for X, _, _ in data]
    xis = [rng.standard_normal((J, X.shape[1])).astype(np.float32) for X, _, _ in data]
    eps = min(synth.default_step_size(X.shape[0], X.shape[1]) for X, _, _ in data)
    params = dict(step_size=eps, traj_length=eps * 32, max_leapfrog=64, num_warmup=25, seed=4,
                  ess_frac=0.0, precision=precision)
    log(f"[fullsize batched {precision}] 64 posteriors, J={J}, eps={eps:.3g}")
    s = chees.Sampler([to_dev(X) for X, _, _ in data], [to_dev(y) for _, y, _ in data], J,
                      theta0=to_dev(np.concatenate([t.ravel() for t in thetas])), **params)
    st = s.step(momenta=to_dev(np.concatenate([x.ravel() for x in xis])))
    assert not st["resampled"]
    tr = s.trace()
    jc = tr["jcap"]
    h_all, n_all = tr["h"].cpu().numpy(), tr["n"].cpu().numpy()
    th_all, p_all = tr["theta_prop"].cpu().numpy(), tr["p_final"].cpu().numpy()
    dh_all = tr["dH"].cpu().numpy()
    s.close()
    # jitter and step counts: the oracle's definition, every particle
    h = O.halton_1d(1, J)
    _, n = O.step_counts(h, params["traj_length"], eps, 64)
    worst_t, worst_p = 0.0, 0.0
    bf_t, bf_p = [], []
    for b, (X, y, _) in enumerate(data):
        rows = slice(b * jc, b * jc + J)
        np.testing.assert_array_equal(h_all[rows], h)
        np.testing.assert_array_equal(n_all[rows], n)
        d = X.shape[1]
        t = O.LogisticRegression(X.astype(np.float64), y.astype(np.float64))
        sel = np.unique(np.r_[np.argmax(n), np.argmin(n), rng.integers(0, J, 2)])
        th0 = thetas[b].astype(np.float64)[sel]
        p0 = xis[b].astype(np.float64)[sel]
        tg = t.grad_bf16 if precision == "bf16" else None
        g0 = tg(th0) if tg else t.log_and_grad(th0)[1]
        th1, p1, _, lp1, _ = O.leapfrog(t, th0, p0, g0, eps, n[sel], traj_grad=tg)
        dth = th_all[rows][sel, :d].astype(np.float64)
        dp = p_all[rows][sel, :d].astype(np.float64)
        et, ep = rel_rows(dth, th1), rel_rows(dp, p1)
        worst_t, worst_p = max(worst_t, et), max(worst_p, ep)
        if precision == "f32":
            assert et <= 1e-5 and ep <= 1e-5, (b, X.shape, et, ep)
        else:
            bf_t.append(rel_each(dth, th1))
            bf_p.append(rel_each(dp, p1))
        # Delta H: the oracle's energies of its own end points (FP32), or of the
        # device's end points (BF16: the trajectories differ by tie roundings)
        lp0, _ = t.log_and_grad(th0)
        if precision == "bf16":
            lp1, _ = t.log_and_grad(dth)
            p1 = dp
        H0, H1 = O.hamiltonian(lp0, p0), O.hamiltonian(lp1, p1)
        err = np.abs(dh_all[rows][sel] - (H1 - H0))
        assert np.all(err <= 1e-5 * (np.abs(H0) + np.abs(H1))), (b, err)
    log(f"  all 64 posteriors: h, n exact for 65536 particles; sampled trajectories "
        f"theta' {worst_t:.2e} p' {worst_p:.2e}")
    if precision == "bf16":
        log("  " + check_bf16_trajectories({"theta": np.concatenate(bf_t), "p": np.concatenate(bf_p)}))


def test_batched_64_posteriors_full_size_f32():
    _batched_case("f32")


def test_batched_64_posteriors_full_size_bf16():
    _batched_case("bf16")


def _flow_params(d, layers, width, seed):
    """Couplings set from the host: the identity initialisation plus small
    seeded weights in the last layer (so that the couplings act)."""
    rng = np.random.default_rng(seed)
    ps = F.init_params(d, layers, width, rng)
    for q in ps:
        q["W3"] = 0.05 * rng.standard_normal(q["W3"].shape) / np.sqrt(width)
        q["b3"] = 0.02 * rng.standard_normal(q["b3"].shape)
    return ps


@pytest.mark.parametrize("precision", ["f32", "bf16"])
def test_flow_full_size_iteration(precision):
    import torch
    from paper_2504_02627_amd import chees
    dev()
    X, y, _ = synth.toeplitz_logistic()
    N, d, J, layers = 5000, 100, 4096, 4
    t = O.LogisticRegression(X.astype(np.float64), y.astype(np.float64))
    rng = np.random.default_rng(51)
    # a population spread around the posterior mode (non-degenerate weights)
    from oracle import quadrature as Q
    X64, y64 = X.astype(np.float64), y.astype(np.float64)

    def lgh(th):
        z = X64 @ th
        sg = 1.0 / (1.0 + np.exp(-z))
        return None, X64.T @ (y64 - sg) - th, -(X64.T * (sg * (1 - sg))) @ X64 - np.eye(d)

    mode, S = Q.laplace(lgh, d)
    theta0 = (mode + 0.7 * rng.standard_normal((J, d)) @ np.linalg.cholesky(S).T).astype(np.float32)
    xi = rng.standard_normal((J, d)).astype(np.float32)
    eps = 0.3
    params = dict(step_size=eps, traj_length=2.4, max_leapfrog=24, num_warmup=25, seed=3,
                  ess_frac=0.0, precond="flow", flow_layers=layers, flow_width=128,
                  flow_train_steps=0, precision=precision)
    ps = _flow_params(d, layers, 128, 52)
    log(f"[fullsize flow {precision}] Toeplitz N={N} d={d} J={J} {layers}x128")
    s = chees.Sampler(to_dev(X), to_dev(y), J, theta0=to_dev(theta0), **params)
    s.set_flow(torch.from_numpy(F.flatten(ps).astype(np.float32)).to("cuda"))
    st = s.step(momenta=to_dev(xi))
    assert not st["resampled"]
    tr = s.trace()
    # the oracle's own weights and base map of the pre-move population
    th0 = theta0.astype(np.float64)
    lp_all, g_all = t.log_and_grad(th0)
    logq0 = -0.5 * np.sum(th0 ** 2, axis=1) - 0.5 * d * np.log(2 * np.pi)
    lw0 = lp_all - logq0 - np.log(J)
    W = O.normalise(lw0)
    base = F.standardise(th0, lw0, 1.0 / np.sum(W * W))
    psb = F.bf16_params(ps)
    h = O.halton_1d(1, J)
    _, n = O.step_counts(h, params["traj_length"], eps, params["max_leapfrog"])
    np.testing.assert_array_equal(tr["n"].cpu().numpy()[:J], n)
    sel = np.unique(np.r_[np.argmax(n), np.argmin(n), rng.integers(0, J, 254)])
    z0, ldi = F.inverse(psb, base, th0[sel])
    z0_dev = tr["latent0"].cpu().numpy()[:J, :d][sel].astype(np.float64)
    ez0 = rel_rows(z0_dev, z0)
    tg = t.grad_bf16 if precision == "bf16" else None
    g0 = tg(th0[sel]) if tg else g_all[sel]
    gz0 = F.latent_grad(psb, base, z0, g0)
    z1, p1, _, th1, _, lp1, ld1 = F.leapfrog_latent(t, psb, base, z0, xi.astype(np.float64)[sel],
                                                    gz0, eps, n[sel], traj_grad=tg)
    z1_dev = tr["latent"].cpu().numpy()[:J, :d][sel].astype(np.float64)
    th1_dev = tr["theta_prop"].cpu().numpy()[:J, :d][sel].astype(np.float64)
    p1_dev = tr["p_final"].cpu().numpy()[:J, :d][sel].astype(np.float64)
    ez, et, ep = rel_rows(z1_dev, z1), rel_rows(th1_dev, th1), rel_rows(p1_dev, p1)
    log(f"  n in [{n.min()}, {n.max()}]; z0 {ez0:.2e}; traj rel err z {ez:.2e} theta {et:.2e} "
        f"p {ep:.2e}")
    assert ez0 <= 1e-5
    if precision == "f32":
        assert ez <= 1e-5 and et <= 1e-5 and ep <= 1e-5
    else:
        log("  " + check_bf16_trajectories({"z": rel_each(z1_dev, z1), "theta": rel_each(th1_dev, th1),
                                            "p": rel_each(p1_dev, p1)}))
    dh = tr["dH"].cpu().numpy()[:J][sel]
    if precision == "bf16":
        # energies of the device's own end points (the latent target's exact
        # log-density: log pi(theta') + log|det J_T(z')|)
        lp1, _ = t.log_and_grad(th1_dev)
        ld1 = tr["logdet"].cpu().numpy()[:J][sel].astype(np.float64)
        p1 = p1_dev
    H0 = O.hamiltonian(lp_all[sel] - ldi, xi.astype(np.float64)[sel])
    H1 = O.hamiltonian(lp1 + ld1, p1)
    err = np.abs(dh - (H1 - H0))
    log(f"  max |dH err| {err.max():.2e}")
    assert np.all(err <= 1e-5 * (np.abs(H0) + np.abs(H1)))
    s.close()
