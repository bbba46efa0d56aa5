"""Batched form: several independent logistic posteriors of uneven N and d in
one context (one launch per leapfrog step and feature-tile group).  Each
posterior is compared with its own oracle run on the same inputs and injected
randomness, to the same bars as the single-posterior parity tests."""

import numpy as np
import pytest

from oracle import smc as O
from paper_2504_02627_amd import synth
from tests._gpu_common import dev, log, rel_rows, to_dev

pytestmark = pytest.mark.gpu


def _run_batched(shapes, J, seed, **kw):
    import torch
    from paper_2504_02627_amd import chees
    log(f"[batched] shapes={shapes} J={J} seed={seed}")
    rng = np.random.default_rng(seed)
    data = [synth.logistic_iid(N, d, seed * 10 + i) for i, (N, d) in enumerate(shapes)]
    thetas = [(0.3 * rng.standard_normal((J, d))).astype(np.float32) for _, d in shapes]
    xis = [rng.standard_normal((J, d)).astype(np.float32) for _, d in shapes]
    u_rs = rng.random(len(shapes))
    eps = min(synth.default_step_size(N, d) for N, d in shapes)
    params = dict(step_size=eps, traj_length=eps * 24, max_leapfrog=48, num_warmup=5, seed=seed)
    params.update(kw)
    s = chees.Sampler([to_dev(X) for X, _, _ in data], [to_dev(y) for _, y, _ in data], J,
                      theta0=to_dev(np.concatenate([t.ravel() for t in thetas])), **params)
    st = s.step(momenta=to_dev(np.concatenate([x.ravel() for x in xis])), resample_u=to_dev(u_rs))
    tr = s.trace()
    theta, logw, logpi = s.state()
    jc = tr["jcap"]
    res = []
    for b, ((X, y, _), (N, d)) in enumerate(zip(data, shapes)):
        o = O.OracleSMC(O.LogisticRegression(X.astype(np.float64), y.astype(np.float64)), J,
                        theta0=thetas[b].astype(np.float64), **params)
        ost = o.step(momenta=xis[b].astype(np.float64), resample_u=float(u_rs[b]))
        rows = slice(b * jc, b * jc + J)
        if ost["resampled"]:
            np.testing.assert_array_equal(tr["ancestors"].cpu().numpy()[rows], ost["ancestors"])
        np.testing.assert_array_equal(tr["h"].cpu().numpy()[rows], ost["h"])
        np.testing.assert_array_equal(tr["n"].cpu().numpy()[rows], ost["n"])
        th1 = tr["theta_prop"].cpu().numpy()[rows, :d].astype(np.float64)
        p1 = tr["p_final"].cpu().numpy()[rows, :d].astype(np.float64)
        et, ep = rel_rows(th1, ost["theta_prop"]), rel_rows(p1, ost["p1"])
        log(f"  posterior {b} (N={N}, d={d}): traj rel err theta {et:.2e} p {ep:.2e}")
        assert et <= 1e-5 and ep <= 1e-5
        lw = logw.cpu().numpy()[b * J:(b + 1) * J]
        scale = np.abs(ost["H0"]) + np.abs(ost["H1"])
        fin = np.isfinite(ost["dh"])
        assert np.all(np.abs(lw[fin] - o.logw[fin]) <= 1e-5 * scale[fin])
        th_b = theta[b] if isinstance(theta, list) else theta
        res.append((o, ost))
    return s, res


def test_batched_three_posteriors_mixed_widths():
    # d = 5, 37, 17: three different feature-tile groups (C2 = 1, 3, 2)
    _run_batched([(300, 5), (1000, 37), (500, 17)], 200, 3)


def test_batched_same_width_different_rows():
    # one feature-tile group, uneven rows and split counts
    _run_batched([(2000, 20), (150, 24), (777, 30), (16, 18)], 130, 4)


def test_batched_evidence_per_posterior():
    s, res = _run_batched([(300, 5), (400, 9)], 256, 5)
    per = s.log_evidence(per_posterior=True)
    for b, (o, ost) in enumerate(res):
        # same resampling decision; the evidence matches to the log-weight bar
        assert abs(per[b] - o.log_evidence()) <= 1e-5 * (abs(o.log_evidence()) + 1.0) * 10
