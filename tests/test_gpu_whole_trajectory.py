"""Whole trajectories in one launch (small data sets whose packed tiles fit in
a work group's LDS) against the per-step launches (CHEES_SMC_PER_STEP=1) on
identical inputs, and the launch counts that show which path ran.

Bars: FP32 trajectories of the two paths agree to 1e-5 relative, Delta H and
the log-weights to 1e-5 (|H0| + |H1|), the parity bars against the oracle
(the arithmetic is the same but for the order of GEMM1's K sum: the
one-launch kernel interleaves the features over the lane groups to skip the
MFMAs on the padding); the precision form's trajectories of the two paths
(FP32 MFMA on bfloat16 operands vs the BF16 MFMA; each within 5e-3 of the
BF16-emulating oracle) agree to 1e-2.  Parity against the oracle for this
path is covered by the small cases of test_gpu_parity.py and
test_gpu_bf16.py, which take it by default.
"""

import numpy as np
import pytest

from paper_2504_02627_amd import synth
from tests._gpu_common import log, rel_rows, to_dev

pytestmark = pytest.mark.gpu


def _run(N, d, J, seed, per_step, monkeypatch, precision="f32", steps=2):
    import torch
    from paper_2504_02627_amd import chees
    if per_step:
        monkeypatch.setenv("CHEES_SMC_PER_STEP", "1")
    else:
        monkeypatch.delenv("CHEES_SMC_PER_STEP", raising=False)
    X, y, _ = synth.logistic_iid(N, d, seed)
    rng = np.random.default_rng(seed + 7)
    theta0 = (rng.standard_normal((J, d)) * 0.3).astype(np.float32)
    eps = synth.default_step_size(N, d)
    s = chees.Sampler(to_dev(X), to_dev(y), J, theta0=to_dev(theta0), step_size=eps,
                      traj_length=eps * 32, max_leapfrog=64, num_warmup=5, seed=seed,
                      precision=precision)
    monkeypatch.delenv("CHEES_SMC_PER_STEP", raising=False)
    s.set_timing(True)
    out = []
    for _ in range(steps):
        xi = rng.standard_normal((J, d)).astype(np.float32)
        u = rng.random(1)
        st = s.step(momenta=to_dev(xi), resample_u=to_dev(u))
        s.adapt()
        tr = s.trace()
        _, logw, logpi = s.state()
        out.append(dict(st=st, th=tr["theta_prop"].cpu().numpy()[:J, :d].astype(np.float64),
                        p=tr["p_final"].cpu().numpy()[:J, :d].astype(np.float64),
                        dh=tr["dH"].cpu().numpy()[:J], n=tr["n"].cpu().numpy()[:J],
                        logw=logw.cpu().numpy()[:J], lp=logpi.cpu().numpy()[:J]))
    torch.cuda.synchronize()
    launches = s.timing()["leapfrog_launches"]
    s.close()
    return out, launches


@pytest.mark.parametrize("N,d,J", [(200, 5, 256), (150, 24, 200), (17, 1, 1), (1, 3, 5)])
def test_whole_trajectory_matches_per_step(N, d, J, monkeypatch):
    log(f"[traj] FP32 N={N} d={d} J={J}")
    a, la = _run(N, d, J, 3, False, monkeypatch)
    b, lb = _run(N, d, J, 3, True, monkeypatch)
    log(f"  leapfrog launches: whole {la}, per step {lb}")
    assert la == 2 and lb == 2 * 64
    for x, y_ in zip(a, b):
        np.testing.assert_array_equal(x["n"], y_["n"])
        et, ep = rel_rows(x["th"], y_["th"]), rel_rows(x["p"], y_["p"])
        log(f"  theta rel {et:.1e}  p rel {ep:.1e}")
        assert et <= 1e-5 and ep <= 1e-5
        # Delta H cancels two energies of size |log pi|: the parity bar
        # 1e-5 (|H0| + |H1|), with |H0| + |H1| >= 2 |log pi(theta')| - |Delta H|
        scale = np.maximum(2 * np.abs(x["lp"]) - np.abs(x["dh"]), 1.0)
        err = np.abs(x["dh"] - y_["dh"])
        log(f"  max |dH_a - dH_b| / scale {np.max(err / scale):.1e}")
        assert np.all(err <= 1e-5 * scale)
        assert np.all(np.abs(x["logw"] - y_["logw"]) <= 1e-5 * scale)


@pytest.mark.parametrize("N,d,J", [(200, 5, 256), (150, 24, 130)])
def test_whole_trajectory_precision_form(N, d, J, monkeypatch):
    log(f"[traj] BF16 N={N} d={d} J={J}")
    a, la = _run(N, d, J, 4, False, monkeypatch, precision="bf16", steps=1)
    b, lb = _run(N, d, J, 4, True, monkeypatch, precision="bf16", steps=1)
    assert la == 1 and lb == 64
    x, y_ = a[0], b[0]
    np.testing.assert_array_equal(x["n"], y_["n"])
    et = rel_rows(x["th"], y_["th"])
    log(f"  theta rel (FP32 MFMA on bf16 operands vs BF16 MFMA) {et:.1e}")
    assert et <= 1e-2


def test_large_data_keeps_per_step_launches(monkeypatch):
    # 400 rows x 12 features: 25 tiles, more than a work group's LDS
    a, la = _run(400, 12, 128, 5, False, monkeypatch, steps=1)
    assert la == 64
