"""smc_run: SMC iterations replayed from a captured HIP graph give the same
results, bit for bit, as the same number of eager smc_step + chees_adapt calls
(no float atomics, fixed reductions, deterministic plan).  The graph is
replayed several times with eager work and synchronisations between the
replays, and every replay is checked."""

import numpy as np
import pytest

from paper_2504_02627_amd import synth
from tests._gpu_common import log, to_dev

pytestmark = pytest.mark.gpu


def _snap(s):
    theta, logw, logpi = s.state()
    ts = theta if not isinstance(theta, list) else theta[0]
    return (ts.cpu().numpy().copy(), logw.cpu().numpy().copy(), logpi.cpu().numpy().copy(),
            s.counters()["grad_evals"], s.log_evidence())


def _same(a, b):
    for u, v in zip(a[:3], b[:3]):
        assert np.array_equal(u.view(np.uint8), v.view(np.uint8))
    assert a[3] == b[3] and a[4] == b[4]


@pytest.mark.parametrize("precision,precond", [("f32", "none"), ("bf16", "none"), ("f32", "diag"),
                                               ("f32", "flow")])
def test_graph_replays_match_eager(precision, precond):
    import torch
    from paper_2504_02627_amd import chees
    N, d, J = 2500, 30, 1000
    X, y, _ = synth.logistic_iid(N, d, 41)
    eps = synth.default_step_size(N, d)
    kw = dict(step_size=eps, traj_length=eps * 20, max_leapfrog=40, num_warmup=4, seed=9,
              precision=precision, precond=precond, adapt_step_size=True)
    if precond == "flow":
        kw.update(step_size=0.2, traj_length=1.0, flow_layers=2, flow_train_steps=3, flow_lr=5e-3)
    log(f"[graph] {precision} {precond} N={N} d={d} J={J}")
    eager = chees.Sampler(to_dev(X), to_dev(y), J, **kw)
    graph = chees.Sampler(to_dev(X), to_dev(y), J, **kw)
    for rep, k in enumerate((1, 3, 2)):
        for _ in range(k):
            eager.step(stats=False)
            eager.adapt(stats=False)
        graph.run(k)
        torch.cuda.synchronize()
        _same(_snap(eager), _snap(graph))
        # eager work on the graph context between replays
        eager.step(stats=False)
        eager.adapt(stats=False)
        st = graph.step()
        graph.adapt()
        _same(_snap(eager), _snap(graph))
        log(f"  replay {rep}: {k} iterations identical; ESS {st['ess']:.1f}")
    eager.close()
    graph.close()


def test_run_after_unadapted_step_is_a_state_error():
    from paper_2504_02627_amd import chees
    X, y, _ = synth.small_logistic()
    s = chees.Sampler(to_dev(X), to_dev(y), 256, num_warmup=5)
    s.step(stats=False)
    with pytest.raises(chees.SmcError):
        s.run(1)
    s.adapt(stats=False)
    s.run(2)
    s.close()
