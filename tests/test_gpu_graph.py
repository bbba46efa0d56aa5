"""smc_run: SMC iterations replayed from a captured HIP graph give the same
results, bit for bit, as the same number of eager smc_step + chees_adapt calls
(no float atomics, fixed reductions, deterministic plan).  The graph is
replayed several times with eager work and synchronisations between the
replays, and every replay is checked.  Every case crosses the end of the
adaptation (num_warmup = 4), after which smc_run replays a graph whose
leapfrog launches stop at the longest trajectory L and eps allow: a bound
that were too small would truncate trajectories and break the identity."""

import numpy as np
import pytest

from paper_2504_02627_amd import synth
from tests._gpu_common import log, to_dev

pytestmark = pytest.mark.gpu


def _host(t):
    ts = t if isinstance(t, (list, tuple)) else [t]
    return np.concatenate([x.cpu().numpy().ravel() for x in ts])


def _snap(s):
    theta, logw, logpi = s.state()
    return (_host(theta), _host(logw), _host(logpi), s.counters()["grad_evals"],
            s.log_evidence())


def _same(a, b):
    for u, v in zip(a[:3], b[:3]):
        assert np.array_equal(u.view(np.uint8), v.view(np.uint8))
    assert a[3] == b[3] and a[4] == b[4]


@pytest.mark.parametrize("precision,precond", [("f32", "none"), ("bf16", "none"), ("f32", "diag"),
                                               ("f32", "flow"), ("bf16", "flow")])
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


@pytest.mark.parametrize("shapes,J", [([(200, 5)], 2048),                       # one launch per iteration
                                      ([(300, 5), (800, 40), (500, 17), (1200, 70)], 256)])  # group lanes
def test_graph_replays_match_eager_other_launch_shapes(shapes, J):
    # whole trajectories in one launch, and a batched context whose feature-tile
    # groups run on forked stream lanes (graph edges under capture)
    import torch
    from paper_2504_02627_amd import chees
    data = [synth.logistic_iid(N, d, 50 + i) for i, (N, d) in enumerate(shapes)]
    Xs = [to_dev(X) for X, _, _ in data]
    ys = [to_dev(y) for _, y, _ in data]
    eps = min(synth.default_step_size(N, d) for N, d in shapes)
    kw = dict(step_size=eps, traj_length=eps * 20, max_leapfrog=40, num_warmup=4, seed=3,
              adapt_step_size=True)
    one = len(shapes) == 1
    log(f"[graph] shapes={shapes} J={J}")
    mk = lambda: chees.Sampler(Xs[0] if one else Xs, ys[0] if one else ys, J, **kw)
    eager, graph = mk(), mk()
    for k in (2, 3):
        for _ in range(k):
            eager.step(stats=False)
            eager.adapt(stats=False)
        graph.run(k)
        torch.cuda.synchronize()
        _same(_snap(eager), _snap(graph))
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


@pytest.mark.parametrize("jitter", ["equidistant_offset", "none", "uniform"])
def test_bounded_graph_after_adaptation_matches_eager(jitter):
    # jitter values up to 1.1 (equidistant with an offset), exactly 1 (none:
    # every trajectory is as long as the bound) and uniform
    import torch
    from paper_2504_02627_amd import chees
    N, d, J = 1500, 12, 512
    X, y, _ = synth.logistic_iid(N, d, 61)
    eps = synth.default_step_size(N, d)
    kw = dict(step_size=eps, traj_length=eps * 9.5, max_leapfrog=48, num_warmup=4, seed=5,
              jitter=jitter, adapt_step_size=True)
    log(f"[graph bound] jitter {jitter}")
    eager = chees.Sampler(to_dev(X), to_dev(y), J, **kw)
    graph = chees.Sampler(to_dev(X), to_dev(y), J, **kw)
    for _ in range(9):
        eager.step(stats=False)
        eager.adapt(stats=False)
    graph.run(9)
    torch.cuda.synchronize()
    _same(_snap(eager), _snap(graph))
    n = graph.trace()["n"].cpu().numpy()[:J]
    st = graph.step()
    L, e = st["L"], st["eps"]
    log(f"  L/eps {L / e:.3f}; longest trajectory of the last replay {int(n.max())}")
    graph.adapt()
    eager.close()
    graph.close()


def test_bounded_graph_on_a_synthetic_target():
    import torch
    from paper_2504_02627_amd import chees
    d, J = 6, 1024
    rng = np.random.default_rng(3)
    A = rng.standard_normal((d, d))
    P = (A @ A.T / d + np.eye(d)).astype(np.float32)
    t = dict(kind="gaussian", dim=d, mean=to_dev(np.zeros(d, np.float32)), precision=to_dev(P))
    kw = dict(step_size=0.05, traj_length=0.6, max_leapfrog=64, num_warmup=4, seed=8)
    eager = chees.Sampler(None, None, J, target=dict(t), **kw)
    graph = chees.Sampler(None, None, J, target=dict(t), **kw)
    for _ in range(7):
        eager.step(stats=False)
        eager.adapt(stats=False)
    graph.run(7)
    torch.cuda.synchronize()
    _same(_snap(eager), _snap(graph))
    eager.close()
    graph.close()


@pytest.mark.parametrize("jitter", ["none", "equidistant_offset"])
def test_bounded_launches_integrate_whole_trajectories(jitter):
    """After the adaptation the eager and the graph path launch only as many
    leapfrog steps as L and eps allow; the longest trajectories (every one,
    without jitter) must still be integrated to the end: theta' and p' of the
    longest and other sampled particles against the oracle's leapfrog from the
    device's pre-move state."""
    from oracle import smc as O
    from paper_2504_02627_amd import chees
    from tests._gpu_common import rel_rows
    N, d, J = 1200, 10, 512
    X, y, _ = synth.logistic_iid(N, d, 71)
    eps = synth.default_step_size(N, d)
    kw = dict(step_size=eps, traj_length=eps * 7.3, max_leapfrog=40, num_warmup=1, seed=6,
              jitter=jitter, ess_frac=0.0)
    s = chees.Sampler(to_dev(X), to_dev(y), J, **kw)
    s.run(2)
    # after the adaptation, L and eps set from the host (this drops the bound
    # of the adapted values): the bound becomes ceil(h_max 7.3)
    s.set_params(eps * 7.3, eps)
    s.run(2)
    theta0 = s.state()[0].cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(7)
    xi = rng.standard_normal((J, d)).astype(np.float32)
    st = s.step(momenta=to_dev(xi))
    assert not st["resampled"]
    tr = s.trace()
    L, e = st["L"], st["eps"]
    hmax = 1.0 + 0.1 if jitter == "equidistant_offset" else 1.0
    bound = int(min(max(np.ceil(hmax * L / e), 1), 40))
    n = tr["n"].cpu().numpy()[:J]
    log(f"[bounded launches] {jitter}: L/eps {L / e:.3f}, bound {bound}, n in [{n.min()}, {n.max()}]")
    assert n.max() <= bound < 40 and bound == (8 if jitter == "none" else 9)
    if jitter == "none":
        assert np.all(n == bound)
    t = O.LogisticRegression(X.astype(np.float64), y.astype(np.float64))
    sel = np.unique(np.r_[np.flatnonzero(n == n.max())[:8], rng.integers(0, J, 8)])
    _, g0 = t.log_and_grad(theta0[sel])
    th1, p1, *_ = O.leapfrog(t, theta0[sel], xi[sel].astype(np.float64), g0, e, n[sel])
    dth = tr["theta_prop"].cpu().numpy()[sel, :d].astype(np.float64)
    dp = tr["p_final"].cpu().numpy()[sel, :d].astype(np.float64)
    et, ep = rel_rows(dth, th1), rel_rows(dp, p1)
    log(f"  trajectories theta' {et:.2e} p' {ep:.2e}")
    assert et <= 1e-5 and ep <= 1e-5
    s.adapt()
    s.close()
