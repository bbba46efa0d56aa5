"""Flow preconditioner on the device against the flow oracle (oracle/flow.py).

* initial couplings: the Philox draws of the oracle, to binary32 rounding;
* base map m, L (weighted mean, Cholesky factor of the shrunk weighted
  covariance) of the pre-move population: to binary32 rounding;
* training: the device's FP32 Adam fit against the oracle's FP64 fit from the
  same initial parameters and population (elementwise to a tolerance that
  allows Adam's sign sensitivity on near-zero gradients, and equal objective);
* moves: from the device's own trained parameters (BF16-rounded), latent
  start z0 = T^-1(theta0), its log-determinant, the latent trajectory z',
  theta' = T(z'), p' within 1e-5 relative (per particle), and Delta H within
  1e-5 (|H0| + |H1|) -- the weights are exact for the latent target."""

import math

import numpy as np
import pytest

from oracle import flow as F, smc as O
from paper_2504_02627_amd import synth
from tests._gpu_common import log, rel_rows, to_dev

pytestmark = pytest.mark.gpu

LAYERS = 4


def _near_posterior(X, y, J, rng, spread=0.7):
    """A population around the Laplace approximation of the posterior, so that
    the initial weights are not degenerate and the fit sees a spread."""
    from oracle import quadrature as Q
    X64, y64 = X.astype(np.float64), y.astype(np.float64)
    d = X.shape[1]

    def lgh(th):
        z = X64 @ th
        sg = 1.0 / (1.0 + np.exp(-z))
        return None, X64.T @ (y64 - sg) - th, -(X64.T * (sg * (1 - sg))) @ X64 - np.eye(d)

    mode, S = Q.laplace(lgh, d)
    return (mode + spread * rng.standard_normal((J, d)) @ np.linalg.cholesky(S).T).astype(np.float32)


def _setup(N, d, J, seed, ntrain, lr, **kw):
    from paper_2504_02627_amd import chees
    X, y, _ = synth.logistic_iid(N, d, seed)
    rng = np.random.default_rng(seed + 7)
    theta0 = _near_posterior(X, y, J, rng)
    eps = kw.pop("eps", 0.3)
    params = dict(step_size=eps, traj_length=eps * 8, max_leapfrog=24, num_warmup=5, seed=seed,
                  precond="flow", flow_layers=LAYERS, flow_width=128, flow_train_steps=ntrain,
                  flow_lr=lr)
    params.update(kw)
    s = chees.Sampler(to_dev(X), to_dev(y), J, theta0=to_dev(theta0), **params)
    t = O.LogisticRegression(X.astype(np.float64), y.astype(np.float64))
    return X, y, theta0, params, s, t, rng


def test_initial_couplings_are_the_philox_draws():
    X, y, theta0, params, s, t, rng = _setup(200, 11, 130, 3, 0, 1e-3)
    prm, _, _ = s.flow()
    ref = F.flatten(F.philox_init(params["seed"], 11, LAYERS, 128))
    got = prm.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(got, ref.astype(np.float32), rtol=2e-7, atol=1e-30)


def _blocks_close(dev, ref, d, what, rtol=1e-4):
    """Elementwise per parameter block: |dev - ref| <= rtol (|ref| + max|ref| of
    the block) -- summation-order noise of FP32 sums relative to the block."""
    worst = 0.0
    for ql, qr in zip(F.unflatten(dev, d, LAYERS, 128)[0], F.unflatten(ref, d, LAYERS, 128)[0]):
        for k in ql:
            scale = np.abs(qr[k]).max() + 1e-30
            e = np.abs(ql[k] - qr[k]) / (np.abs(qr[k]) + scale)
            worst = max(worst, float(e.max()))
    log(f"  {what}: worst relative deviation {worst:.2e}")
    assert worst <= rtol


@pytest.mark.parametrize("N,d,J,seed,layers", [(500, 12, 256, 5, LAYERS), (800, 37, 130, 6, LAYERS),
                                               (500, 12, 256, 7, 0),
                                               # the base map's factorisation in LDS up to
                                               # d = 128, in global memory above
                                               (600, 128, 256, 8, 0), (600, 150, 200, 9, 0)])
def test_flow_iteration_parity(N, d, J, seed, layers):
    """Two iterations with one Adam step each (the fit is warm-started), no
    resampling, so that the weighted objective sees the population's own
    weights.  Adam normalises each coordinate of the gradient, so coordinates
    whose exact gradient vanishes (the shift of the standardised population's
    weighted mean, for one) amplify FP32 summation noise; the fit is therefore
    checked through its gradient (the device's against the oracle's, at the
    same parameters and population) and through the Adam update applied to the
    device's gradient."""
    lr = 1e-2
    X, y, theta0, params, s, t, rng = _setup(N, d, J, seed, 1, lr, ess_frac=0.0,
                                             flow_layers=layers)
    log(f"[flow] N={N} d={d} J={J} seed={seed} layers={layers}")
    P0 = s.flow()[0].cpu().numpy().astype(np.float64)
    ad = F.FlowAdam(lr)
    th_prev = theta0.astype(np.float64)
    lw_prev = s.state()[1].cpu().numpy()
    Pprev = P0
    for k in (1, 2):
        xi = rng.standard_normal((J, d)).astype(np.float32)
        st = s.step(momenta=to_dev(xi), resample_u=to_dev(rng.random(1)))
        s.adapt()
        assert not st["resampled"]
        tr = s.trace()
        prm, m_dev, L_dev, g_dev = (v.cpu().numpy().astype(np.float64) for v in s.flow(True))
        th0 = th_prev
        ref = F.standardise(th0, lw_prev, st["ess_before"])
        np.testing.assert_allclose(m_dev, ref.m, rtol=1e-6, atol=1e-7)
        np.testing.assert_allclose(L_dev, ref.L, rtol=1e-5, atol=1e-6 * np.abs(ref.L).max())
        base = F.Base(m_dev, L_dev)
        if layers:
            W = O.normalise(lw_prev)
            _, g = F.objective_and_grad(F.unflatten(Pprev, d, layers, 128)[0], base, th0, W)
            _blocks_close(g_dev, F.flatten(g), d, f"iteration {k}: fit gradient")
            P_exp = F.flatten(ad.ascend(F.unflatten(Pprev, d, layers, 128)[0],
                                        F.unflatten(g_dev, d, layers, 128)[0]))
            dP = np.abs(prm - P_exp)
            log(f"  iteration {k}: Adam update max |dP| {dP.max():.2e}")
            assert np.all(dP <= 1e-6 * (np.abs(P_exp) + lr))
        else:
            assert prm.size == 0   # the base map alone: no parameters to fit
        # moves with the device's trained couplings, BF16-rounded
        psb = F.bf16_params(F.unflatten(prm, d, layers, 128)[0])
        z0, ldi = F.inverse(psb, base, th0)
        z0_dev = tr["latent0"].cpu().numpy()[:J, :d].astype(np.float64)
        ez0 = rel_rows(z0_dev, z0)
        ld0_dev = tr["logdet0"].cpu().numpy()[:J].astype(np.float64)
        log(f"  weights ESS {st['ess_before']:.1f}; max |z0| {np.abs(z0).max():.2f}; "
            f"z0 rel err {ez0:.2e}; max |logdet0 err| {np.max(np.abs(ld0_dev + ldi)):.2e}")
        assert np.abs(z0).max() > 0.5   # a spread population, not a collapsed one
        assert ez0 <= 1e-5
        assert np.all(np.abs(ld0_dev + ldi) <= 1e-5 * (1 + np.abs(ldi)))
        lp0, g0 = t.log_and_grad(th0)
        gz0 = F.latent_grad(psb, base, z0, g0)
        n = tr["n"].cpu().numpy()[:J]
        z1, p1, gz1, th1, _, lp1, ld1 = F.leapfrog_latent(t, psb, base, z0, xi.astype(np.float64),
                                                          gz0, params["step_size"] if k == 1
                                                          else st["eps"], n)
        z1_dev = tr["latent"].cpu().numpy()[:J, :d].astype(np.float64)
        th1_dev = tr["theta_prop"].cpu().numpy()[:J, :d].astype(np.float64)
        p1_dev = tr["p_final"].cpu().numpy()[:J, :d].astype(np.float64)
        ez, et, ep = rel_rows(z1_dev, z1), rel_rows(th1_dev, th1), rel_rows(p1_dev, p1)
        log(f"  n in [{n.min()}, {n.max()}]; traj rel err z {ez:.2e} theta {et:.2e} p {ep:.2e}")
        assert ez <= 1e-5 and et <= 1e-5 and ep <= 1e-5
        H0 = O.hamiltonian(lp0 - ldi, xi.astype(np.float64))
        H1 = O.hamiltonian(lp1 + ld1, p1)
        dh = tr["dH"].cpu().numpy()[:J]
        err = np.abs(dh - (H1 - H0))
        log(f"  max |dH err| {err.max():.2e} (bar {(1e-5 * (np.abs(H0) + np.abs(H1))).min():.2e}); "
            f"ESS {st['ess']:.1f}")
        assert np.all(err <= 1e-5 * (np.abs(H0) + np.abs(H1)))
        theta, logw, _ = s.state()
        th_prev = theta.cpu().numpy().astype(np.float64)
        lw_prev = logw.cpu().numpy()
        Pprev = prm


@pytest.mark.parametrize("d", [2, 63, 64, 65, 127])
def test_base_map_at_the_register_layout_edges(d):
    """The base map alone (no couplings) at dimensions around the one-work-group
    factorisation's register layout (lane l holds columns l and l + 64 of a
    row; 16 waves of 8 rows): m and L of the pre-move population against the
    oracle's FP64 standardisation, the latent start z0 = L^-1 (theta0 - m) and
    log|det L| of one iteration."""
    N, J, seed = 300, 256, 20 + d
    X, y, theta0, params, s, t, rng = _setup(N, d, J, seed, 0, 1e-3, ess_frac=0.0,
                                             flow_layers=0)
    lw0 = s.state()[1].cpu().numpy()
    xi = rng.standard_normal((J, d)).astype(np.float32)
    st = s.step(momenta=to_dev(xi), resample_u=to_dev(np.array([0.5])))
    assert not st["resampled"]
    tr = s.trace()
    _, m_dev, L_dev = (v.cpu().numpy().astype(np.float64) for v in s.flow())
    th0 = theta0.astype(np.float64)
    ref = F.standardise(th0, lw0, st["ess_before"])
    np.testing.assert_allclose(m_dev, ref.m, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(L_dev, ref.L, rtol=1e-5, atol=1e-6 * np.abs(ref.L).max())
    z0, ldi = F.inverse([], F.Base(m_dev, L_dev), th0)
    z0_dev = tr["latent0"].cpu().numpy()[:J, :d].astype(np.float64)
    ez0 = rel_rows(z0_dev, z0)
    ld0_dev = tr["logdet0"].cpu().numpy()[:J].astype(np.float64)
    log(f"[base map d={d}] L rel err {np.max(np.abs(L_dev - ref.L)) / np.abs(ref.L).max():.2e}; "
        f"z0 rel err {ez0:.2e}; max |logdet0 err| {np.max(np.abs(ld0_dev + ldi)):.2e}")
    assert ez0 <= 1e-5
    assert np.all(np.abs(ld0_dev + ldi) <= 1e-5 * (1 + np.abs(ldi)))


def test_flow_with_no_training_and_identity_couplings_is_a_dense_mass():
    """Zero couplings (set through smc_set_flow) and no training: T(z) = m +
    L u with u_c = z_q(c).  The latent leapfrog is then the plain leapfrog in
    theta with the dense mass M^-1 = L L^T: theta += eps L p_u, p_u = L^T
    p_theta; written out here in theta and compared with the device."""
    import torch
    N, d, J = 400, 9, 256
    X, y, theta0, params, s, t, rng = _setup(N, d, J, 8, 0, 1e-3)
    n_par = len(F.flatten(F.init_params(d, LAYERS, 128, np.random.default_rng(0))))
    s.set_flow(torch.zeros(n_par, dtype=torch.float32, device="cuda"))
    xi = rng.standard_normal((J, d)).astype(np.float32)
    st = s.step(momenta=to_dev(xi), resample_u=to_dev(np.array([0.5])))
    tr = s.trace()
    _, m, L = (v.cpu().numpy().astype(np.float64) for v in s.flow())
    anc = tr["ancestors"].cpu().numpy()[:J] if st["resampled"] else np.arange(J)
    th = theta0.astype(np.float64)[anc].copy()
    _, g = t.log_and_grad(th)
    pu = xi.astype(np.float64)[:, F.interleave(d)]      # latent momentum in theta's order
    eps = params["step_size"]
    n = tr["n"].cpu().numpy()[:J]
    for k in range(int(n.max())):
        act = n > k
        pu[act] += 0.5 * eps * g[act] @ L
        th[act] += eps * pu[act] @ L.T
        _, g_new = t.log_and_grad(th[act])
        g[act] = g_new
        pu[act] += 0.5 * eps * g[act] @ L
    th1_dev = tr["theta_prop"].cpu().numpy()[:J, :d].astype(np.float64)
    e = rel_rows(th1_dev, th)
    log(f"[flow identity] theta' vs dense-mass leapfrog rel err {e:.2e}")
    assert e <= 1e-5
    np.testing.assert_allclose(tr["logdet"].cpu().numpy()[:J], np.sum(np.log(np.diag(L))),
                               rtol=1e-5)


def test_evidence_is_flagged_adaptive_after_a_fit():
    """log_evidence returns SMC_WADAPTIVE once a move used couplings fitted to
    the population it moved (the estimate is then adaptive); without a fit the
    same estimate comes back with SMC_OK.  The value is the evidence
    bookkeeping either way."""
    from paper_2504_02627_amd import chees
    N, d, J = 300, 7, 256
    lz = {}
    for ntrain in (0, 3):
        X, y, theta0, params, s, t, rng = _setup(N, d, J, 12, ntrain, 1e-3, ess_frac=0.0)
        s.log_evidence()
        assert not s.evidence_adaptive
        s.step()
        lz[ntrain] = s.log_evidence()
        rc = s.lib.log_evidence(s.ctx, None, None)
        log(f"[flow evidence] train steps {ntrain}: log Z {lz[ntrain]:.6f} status {rc}")
        assert s.evidence_adaptive == (ntrain > 0)
        assert rc == (chees.SMC_WADAPTIVE if ntrain > 0 else chees.SMC_OK)
        assert math.isfinite(lz[ntrain])
        s.close()
