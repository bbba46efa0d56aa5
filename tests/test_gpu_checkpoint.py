"""Checkpoint and resume (smc_save / smc_load): a run resumed from an image
continues bit-identically to the run that wrote it (counter-based randomness
keyed by the iteration), for the one-launch trajectories, the split path,
a batched context, the diagonal mass and the flow preconditioner; images of
another shape are refused, and saving between smc_step and chees_adapt is a
call-order error."""

import numpy as np
import pytest

from paper_2504_02627_amd import synth
from tests._gpu_common import log, to_dev

pytestmark = pytest.mark.gpu


def _make(shapes, J, **kw):
    from paper_2504_02627_amd import chees
    data = [synth.logistic_iid(N, d, 40 + i) for i, (N, d) in enumerate(shapes)]
    Xs = [to_dev(X) for X, _, _ in data]
    ys = [to_dev(y) for _, y, _ in data]
    N, d = shapes[0]
    eps = min(synth.default_step_size(N_, d_) for N_, d_ in shapes)
    params = dict(step_size=eps, traj_length=eps * 16, max_leapfrog=32, num_warmup=4, seed=21,
                  adapt_step_size=True)
    params.update(kw)
    return lambda: chees.Sampler(Xs if len(Xs) > 1 else Xs[0], ys if len(ys) > 1 else ys[0], J,
                                 **params)


def _host(t):
    # one tensor, or one per posterior of a batched context
    ts = t if isinstance(t, (list, tuple)) else [t]
    return np.concatenate([x.cpu().numpy().ravel() for x in ts])


def _iterate(s, k):
    out = []
    for _ in range(k):
        st = s.step()
        s.adapt()
        theta, logw, logpi = s.state()
        out.append((st["L"], st["eps"], st["resampled"], st["grad_evals"], s.log_evidence(),
                    _host(theta), _host(logw), _host(logpi)))
    return out


@pytest.mark.parametrize("case", ["whole_trajectory", "split", "batched", "diag_mass", "flow"])
def test_resume_is_bit_identical(case):
    if case == "whole_trajectory":
        make = _make([(200, 5)], 512)
    elif case == "split":
        make = _make([(1000, 37)], 300)
    elif case == "batched":
        make = _make([(300, 5), (800, 40), (500, 17)], 128)
    elif case == "diag_mass":
        make = _make([(600, 12)], 256, precond="diag")
    else:
        make = _make([(300, 8)], 256, precond="flow", flow_layers=2, flow_train_steps=3,
                     flow_lr=1e-3)
    log(f"[checkpoint] {case}")
    a = make()
    _iterate(a, 4)
    image = a.save()
    ref = _iterate(a, 3)
    a.close()
    b = make()
    _iterate(b, 1)                      # a different state, overwritten by the image
    b.load(image)
    got = _iterate(b, 3)
    b.close()
    for r, g in zip(ref, got):
        assert r[:5] == g[:5]
        for x, y in zip(r[5:], g[5:]):
            np.testing.assert_array_equal(x, y)


def test_load_refuses_another_shape_and_save_checks_call_order():
    from paper_2504_02627_amd import chees
    a = _make([(200, 5)], 512)()
    _iterate(a, 1)
    image = a.save()
    b = _make([(200, 5)], 256)()
    with pytest.raises(chees.SmcError) as e:
        b.load(image)
    assert e.value.status == chees.SMC_EINVAL
    with pytest.raises(chees.SmcError):
        b.load(image[:100])
    a.step()
    with pytest.raises(chees.SmcError) as e:
        a.save()
    assert e.value.status == chees.SMC_ESTATE
    a.adapt()
    assert len(a.save()) == len(image)
    a.close()
    b.close()


def test_runner_logs_every_iteration_and_resumes(tmp_path):
    # the command-line runner: one JSON record per iteration; a run split by
    # a checkpoint logs what the uninterrupted run logs (wall time aside)
    import json
    from paper_2504_02627_amd import run
    full, first, second = tmp_path / "full.jsonl", tmp_path / "a.jsonl", tmp_path / "b.jsonl"
    ck = tmp_path / "state.bin"
    common = ["--workload", "small", "--particles", "2048", "--iterations", "6"]
    run.main(common + ["--jsonl", str(full)])
    run.main(["--workload", "small", "--particles", "2048", "--iterations", "6", "--jsonl",
              str(first), "--save", str(ck)])
    recs = [json.loads(l) for l in open(full)]
    assert [r["iteration"] for r in recs] == list(range(1, 7))
    assert all(0 < r["ess"] <= 2048 and 1 <= r["n_max"] <= 64 for r in recs)
    assert recs == [dict(r, wall_ms=x["wall_ms"]) for r, x in
                    zip([json.loads(l) for l in open(first)], recs)]
    # the run's schedule is recorded beside the image and governs the resume
    assert json.load(open(str(ck) + ".json")) == dict(num_warmup=3, num_iterations=6,
                                                      jitter="halton1d")
    # resume from the checkpoint for the same schedule: iterations 7.. of a 6 + 6 run
    run.main(common + ["--jsonl", str(second), "--resume", str(ck)])
    more = [json.loads(l) for l in open(second)]
    assert [r["iteration"] for r in more] == list(range(7, 13))
