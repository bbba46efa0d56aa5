"""Synthetic targets on the device (Sec. IV: Gaussian D = 5, ill-conditioned
Gaussian D = 100, banana D = 2; Sec. VI: Neal's funnel D = 10) against the
oracle's densities.

Bars: the initial weights and one iteration from the same injected inputs
(jitter and step counts bit-exact; theta', p' within the FP32 trajectory
tolerance; Delta H and the log-weights within 1e-5 (|H0| + |H1|)); the
counting convention of the no-jitter rows of Table 1 (every trajectory at the
500-step cap); moments of the targets after a run; the evidence of a scaled
Gaussian.
"""

import math

import numpy as np
import pytest

from oracle import smc as O
from paper_2504_02627_amd import synth
from tests._gpu_common import log, rel_rows, to_dev

pytestmark = pytest.mark.gpu

LOGW_TOL = 1e-5


def _target(kind):
    """(device target dict, oracle target, step size)."""
    if kind == "gauss5":
        mu, P, _ = synth.gaussian5()
        eps = 0.1
    elif kind == "illcond":
        mu, P, _ = synth.ill_conditioned_gaussian()
        eps = 0.001
    elif kind == "funnel":
        d, sv = synth.FUNNEL
        return (dict(kind="funnel", dim=d, funnel_scale=sv), O.Funnel(d, sv), 0.05)
    else:
        s1, b, c = synth.BANANA
        return (dict(kind="banana", dim=2, banana=synth.BANANA), O.Banana(s1, b, c), 0.01)
    t = dict(kind="gaussian", dim=len(mu), mean=to_dev(mu), precision=to_dev(P))
    return t, O.Gaussian(mu.astype(np.float64), prec=P.astype(np.float64)), eps


def _pair(kind, J, seed, nmax=64, **kw):
    from paper_2504_02627_amd import chees
    t, ot, eps = _target(kind)
    d = t["dim"]
    rng = np.random.default_rng(seed)
    theta0 = rng.standard_normal((J, d)).astype(np.float32)
    params = dict(step_size=eps, traj_length=eps * nmax / 2, max_leapfrog=nmax, num_warmup=5,
                  seed=seed)
    params.update(kw)
    s = chees.Sampler(None, None, J, theta0=to_dev(theta0), target=t, **params)
    o = O.OracleSMC(ot, J, theta0=theta0.astype(np.float64), **params)
    return s, o, rng, d


@pytest.mark.parametrize("kind", ["gauss5", "illcond", "banana", "funnel"])
def test_initial_weights(kind):
    J = 300
    log(f"[targets] init {kind} J={J}")
    s, o, _, d = _pair(kind, J, 3)
    _, logw, logpi = s.state()
    np.testing.assert_allclose(logpi.cpu().numpy(), o.logpi, rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(logw.cpu().numpy(), o.logw, rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("kind,traj_tol", [("gauss5", 1e-5), ("illcond", 1e-5), ("banana", 1e-5),
                                           ("funnel", 1e-5)])
def test_one_iteration(kind, traj_tol):
    J = 300
    log(f"[targets] one iteration {kind} J={J}")
    s, o, rng, d = _pair(kind, J, 5)
    xi = rng.standard_normal((J, d)).astype(np.float32)
    st = s.step(momenta=to_dev(xi))
    ost = o.step(momenta=xi.astype(np.float64))
    tr = s.trace()
    assert st["resampled"] == int(ost["resampled"])
    np.testing.assert_array_equal(tr["h"].cpu().numpy()[:J], ost["h"])
    np.testing.assert_array_equal(tr["n"].cpu().numpy()[:J], ost["n"])
    th1 = tr["theta_prop"].cpu().numpy()[:J, :d].astype(np.float64)
    p1 = tr["p_final"].cpu().numpy()[:J, :d].astype(np.float64)
    et, ep = rel_rows(th1, ost["theta_prop"]), rel_rows(p1, ost["p1"])
    log(f"  traj rel err theta {et:.2e} p {ep:.2e}")
    assert et <= traj_tol and ep <= traj_tol
    # energies from the device's own FP32 end points against the oracle's
    # density at those points: exact up to binary64 rounding
    lp_dev, _ = o.target.log_and_grad(th1)
    dh = tr["dH"].cpu().numpy()[:J]
    scale = np.abs(ost["H0"]) + np.abs(ost["H1"])
    assert np.all(np.abs(dh - ost["dh"]) <= LOGW_TOL * scale + 1e-6 * np.abs(dh))
    _, logw, logpi = s.state()
    np.testing.assert_allclose(logpi.cpu().numpy(), lp_dev, rtol=1e-10, atol=1e-9)
    err = np.abs(logw.cpu().numpy() - o.logw)
    assert np.all(err <= LOGW_TOL * scale + 1e-6 * np.abs(dh))


def test_counting_convention_no_jitter():
    # ill-conditioned Gaussian, no jitter, L = 5, eps = 0.001, cap 500: every
    # trajectory runs 500 leapfrog steps (Table 1 counts 501 gradients per
    # particle: the cap plus one)
    from paper_2504_02627_amd import chees
    t, _, _ = _target("illcond")
    J = 1000
    log("[targets] counting test J=1000 cap 500")
    s = chees.Sampler(None, None, J, target=t, step_size=0.001, traj_length=5.0,
                      max_leapfrog=500, num_warmup=100, jitter="none", seed=1)
    for _ in range(3):
        st = s.step()
        s.adapt()
        assert st["grad_evals"] == 500 * J


@pytest.mark.parametrize("kind", ["gauss5", "banana"])
def test_moments(kind):
    # the paper's protocol, shortened: J = 1000, L0 = 5, 1-d Halton, 100
    # iterations, the last 50 pooled
    from paper_2504_02627_amd import chees
    t, _, eps = _target(kind)
    J, K, burn = 1000, 100, 50
    log(f"[targets] moments {kind} J={J} K={K}")
    s = chees.Sampler(None, None, J, target=t, step_size=eps, traj_length=5.0,
                      max_leapfrog=500, num_warmup=burn, seed=11)
    means, sq = [], []
    for k in range(K):
        s.step()
        s.adapt()
        if k >= burn:
            theta, logw, _ = s.state()
            th = theta.cpu().numpy().astype(np.float64)
            w = np.exp(logw.cpu().numpy() - logw.cpu().numpy().max())
            w /= w.sum()
            means.append(w @ th)
            sq.append(w @ th ** 2)
    m = np.mean(means, axis=0)
    v = np.mean(sq, axis=0) - m ** 2
    lz = s.log_evidence()
    log(f"  mean {m}  var {v}  log Z {lz:.3f}")
    if kind == "gauss5":
        mu, _, cov = synth.gaussian5()
        sd = np.sqrt(np.diag(cov))
        assert np.all(np.abs(m - mu) < 0.1 * sd)
        assert np.all(np.abs(v / np.diag(cov) - 1) < 0.15)
    else:
        s1, b, c = synth.BANANA
        # theta_1 ~ N(0, s1^2); theta_2 = b (theta_1^2 - c) + N(0, 1):
        # E theta_2 = b (s1^2 - c) = 0, Var theta_2 = 1 + 2 b^2 s1^4
        assert abs(m[0]) < 0.15 * s1 and abs(m[1]) < 0.15 * math.sqrt(1 + 2 * b * b * s1 ** 4)
        assert abs(v[0] / s1 ** 2 - 1) < 0.2
        assert abs(v[1] / (1 + 2 * b * b * s1 ** 4) - 1) < 0.3


def test_evidence_of_a_scaled_gaussian():
    # pi = exp(2.3) N(mu, Sigma) near q0 = N(0, I), so that importance weights
    # from q0 are well behaved: log Z -> 2.3
    from paper_2504_02627_amd import chees
    d = 4
    mu = np.array([0.3, -0.2, 0.1, 0.0], dtype=np.float32)
    P = np.diag([1.25, 1.0, 0.9, 1.1]).astype(np.float32)
    t = dict(kind="gaussian", dim=d, mean=to_dev(mu), precision=to_dev(P), log_const=2.3)
    J = 8192
    log(f"[targets] evidence J={J}")
    s = chees.Sampler(None, None, J, target=t, step_size=0.1, traj_length=1.0, max_leapfrog=32,
                      num_warmup=10, seed=3)
    lz0 = s.log_evidence()
    for _ in range(20):
        s.step()
        s.adapt()
    lz = s.log_evidence()
    log(f"  log Z at init {lz0:.4f}, after 20 iterations {lz:.4f}")
    assert abs(lz0 - 2.3) < 0.03 and abs(lz - 2.3) < 0.05
