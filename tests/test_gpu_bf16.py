"""Precision form: trajectory gradients with theta', X and the residual in
bfloat16 on the BF16 matrix cores (FP32 accumulation); energies for the
weights recomputed in FP32 with compensated sums; LSE, ESS and evidence in
FP64.  The oracle's BF16 mode (grad_bf16) rounds the same operands and sums
exactly.

Bars:
  * initial gradient: inside the interval spanned by the two admissible
    bfloat16 roundings of every residual that lies within rounding distance of
    a tie, widened by a worst-case FP32 summation bound;
  * energies: Delta H of the device's own end points equals the exact FP64
    Delta H at those points within 1e-5 (|H0| + |H1|) -- the weights stay exact;
  * jitter, step counts and resampling ancestors: bit-exact;
  * trajectories: against the BF16-emulating oracle to the bars of
    check_bf16_trajectories (median, 75th percentile and maximum over the
    particles: rounding-tie flips are rare but carry to the end point);
    against the exact FP64 oracle stated (logged) and bounded.
"""

import numpy as np
import pytest

from oracle import smc as O
from paper_2504_02627_amd import synth
from tests._gpu_common import check_bf16_trajectories, dev, log, rel_each, rel_rows, to_dev

pytestmark = pytest.mark.gpu


def _setup(N, d, J, seed, x_bf16=True, **kw):
    import torch
    from paper_2504_02627_amd import chees
    X, y, _ = synth.logistic_iid(N, d, seed)
    if x_bf16:
        X = O.bf16_round(X).astype(np.float32)   # data stored in bfloat16
    rng = np.random.default_rng(seed + 3)
    theta0 = (0.3 * rng.standard_normal((J, d))).astype(np.float32)
    eps = synth.default_step_size(N, d)
    params = dict(step_size=eps, traj_length=eps * 16, max_leapfrog=32, num_warmup=5, seed=seed)
    params.update(kw)
    Xd = to_dev(X).to(torch.bfloat16) if x_bf16 else to_dev(X)
    s = chees.Sampler(Xd, to_dev(y), J, theta0=to_dev(theta0), precision="bf16", **params)
    t = O.LogisticRegression(X.astype(np.float64), y.astype(np.float64))
    return X, y, theta0, params, s, t, rng


def _bf16_neighbours(r32):
    """The two bfloat16 values around each float32 value (toward zero and away)."""
    u = r32.astype(np.float32).view(np.uint32)
    t0 = (u & np.uint32(0xFFFF0000)).view(np.float32).astype(np.float64)
    t1 = ((u & np.uint32(0xFFFF0000)) + np.uint32(0x10000)).view(np.float32).astype(np.float64)
    return t0, t1


@pytest.mark.parametrize("N,d,J", [(300, 5, 200), (1000, 37, 130), (700, 100, 256)])
def test_bf16_initial_gradient_interval(N, d, J):
    X, y, theta0, params, s, t, rng = _setup(N, d, J, 11)
    log(f"[bf16 grad] N={N} d={d} J={J}")
    g_dev = s.trace()["grad"].cpu().numpy()[:J, :d].astype(np.float64)
    from scipy.special import expit
    th = theta0.astype(np.float64)
    thb, Xb = O.bf16_round(th), O.bf16_round(X)
    Z = thb @ Xb.T
    Rf = (y - expit(Z)).astype(np.float32)          # residual before the bfloat16 rounding
    R = O.bf16_round(Rf)
    # device residual differs from Rf by at most delta: FP32 accumulation of
    # the exact bf16 products (d terms) through sigmoid' <= 1/4, plus the
    # sigmoid and subtraction rounding
    delta = 0.25 * (d + 2) * 2.0 ** -24 * (np.abs(thb) @ np.abs(Xb).T) + 1e-6
    t0, t1 = _bf16_neighbours(Rf)
    near = np.abs(Rf.astype(np.float64) - 0.5 * (t0 + t1)) <= delta
    alt = np.where(R == t0, t1, t0)
    D = np.where(near, alt - R, 0.0)
    g_a = R @ Xb - th
    half_span = 0.5 * (np.abs(D) @ np.abs(Xb))
    mid = g_a + 0.5 * (D @ Xb)
    # worst-case FP32 summation of the N products and the prior term
    acc = (N + 2) * 2.0 ** -24 * (np.abs(R) @ np.abs(Xb) + half_span + np.abs(th))
    excess = np.abs(g_dev - mid) - (half_span + acc)
    log(f"  ambiguous residuals {int(near.sum())} of {near.size}; "
        f"max |g - g_bf16| {np.abs(g_dev - g_a).max():.2e}; worst margin {excess.max():.2e}")
    assert np.all(excess <= 0)


@pytest.mark.parametrize("N,d,J", [(400, 12, 256), (200, 5, 256), (150, 24, 130)])
def test_bf16_energies_exact_at_device_end_points(N, d, J):
    # the two small cases run whole trajectories in one launch
    log(f"[bf16 energies] N={N} d={d} J={J}")
    X, y, theta0, params, s, t, rng = _setup(N, d, J, 12)
    xi = rng.standard_normal((J, d)).astype(np.float32)
    u0 = rng.random(1)
    st = s.step(momenta=to_dev(xi), resample_u=to_dev(u0))
    tr = s.trace()
    # the population that moved: theta_0 (after resampling, its ancestors)
    _, lw0 = None, None
    o = O.OracleSMC(t, J, theta0=theta0.astype(np.float64), precision="bf16", **params)
    ost = o.step(momenta=xi.astype(np.float64), resample_u=float(u0[0]))
    assert st["resampled"] == int(ost["resampled"])
    anc = tr["ancestors"].cpu().numpy()[:J] if st["resampled"] else np.arange(J)
    np.testing.assert_array_equal(anc, ost["ancestors"] if ost["resampled"] else anc)
    np.testing.assert_array_equal(tr["h"].cpu().numpy()[:J], ost["h"])
    np.testing.assert_array_equal(tr["n"].cpu().numpy()[:J], ost["n"])
    th_b = theta0.astype(np.float64)[anc]
    th1 = tr["theta_prop"].cpu().numpy()[:J, :d].astype(np.float64)
    p1 = tr["p_final"].cpu().numpy()[:J, :d].astype(np.float64)
    lp0, _ = t.log_and_grad(th_b)
    lp1, _ = t.log_and_grad(th1)
    H0 = O.hamiltonian(lp0, xi.astype(np.float64))
    H1 = O.hamiltonian(lp1, p1)
    dh = tr["dH"].cpu().numpy()[:J]
    err = np.abs(dh - (H1 - H0))
    log(f"  max |dH - dH_exact(device end points)| {err.max():.2e}")
    assert np.all(err <= 1e-5 * (np.abs(H0) + np.abs(H1)))
    # trajectories: BF16 vs BF16-emulating oracle, and vs the exact oracle
    e_emul = rel_rows(th1, ost["theta_prop"])
    log("  " + check_bf16_trajectories({"theta": rel_each(th1, ost["theta_prop"]),
                                        "p": rel_each(p1, ost["p1"])}))
    ox = O.OracleSMC(t, J, theta0=theta0.astype(np.float64), **params)
    oxs = ox.step(momenta=xi.astype(np.float64), resample_u=float(u0[0]))
    e_exact = rel_rows(th1, oxs["theta_prop"])
    log(f"  trajectory rel err vs BF16-emulating oracle {e_emul:.2e}, vs exact FP64 oracle {e_exact:.2e}")
    assert e_exact <= 5e-2


def test_bf16_batched_mixed_widths_runs_and_weights_exact():
    import torch
    from paper_2504_02627_amd import chees
    shapes = [(300, 5), (800, 40), (500, 17)]
    J = 128
    data = [synth.logistic_iid(N, d, 20 + i) for i, (N, d) in enumerate(shapes)]
    Xs = [O.bf16_round(X).astype(np.float32) for X, _, _ in data]
    rng = np.random.default_rng(9)
    thetas = [(0.3 * rng.standard_normal((J, d))).astype(np.float32) for _, d in shapes]
    xis = [rng.standard_normal((J, d)).astype(np.float32) for _, d in shapes]
    eps = min(synth.default_step_size(N, d) for N, d in shapes)
    s = chees.Sampler([to_dev(X).to(torch.bfloat16) for X in Xs], [to_dev(y) for _, y, _ in data], J,
                      theta0=to_dev(np.concatenate([t_.ravel() for t_ in thetas])), precision="bf16",
                      step_size=eps, traj_length=eps * 16, max_leapfrog=32, num_warmup=5, seed=1)
    s.step(momenta=to_dev(np.concatenate([x.ravel() for x in xis])), resample_u=to_dev(np.full(3, 0.4)))
    tr = s.trace()
    jc = tr["jcap"]
    for b, ((N, d), X) in enumerate(zip(shapes, Xs)):
        t = O.LogisticRegression(X.astype(np.float64), data[b][1].astype(np.float64))
        rows = slice(b * jc, b * jc + J)
        anc = tr["ancestors"].cpu().numpy()[rows]
        th1 = tr["theta_prop"].cpu().numpy()[rows, :d].astype(np.float64)
        p1 = tr["p_final"].cpu().numpy()[rows, :d].astype(np.float64)
        H0 = O.hamiltonian(t.log_and_grad(thetas[b].astype(np.float64)[anc])[0], xis[b].astype(np.float64))
        H1 = O.hamiltonian(t.log_and_grad(th1)[0], p1)
        dh = tr["dH"].cpu().numpy()[rows]
        assert np.all(np.abs(dh - (H1 - H0)) <= 1e-5 * (np.abs(H0) + np.abs(H1))), b
