"""Two runs from the same seed are bit-identical: no float atomics, fixed-order
reductions, and a stable sort of the particles by trajectory length (the tiles,
split counts and summation orders are the same on every run)."""

import numpy as np
import pytest

from paper_2504_02627_amd import synth
from tests._gpu_common import log, to_dev

pytestmark = pytest.mark.gpu


def _run(X, y, J, precision, iters, **kw):
    from paper_2504_02627_amd import chees
    s = chees.Sampler(to_dev(X), to_dev(y), J, precision=precision, **kw)
    for _ in range(iters):
        s.step(stats=False)
        s.adapt(stats=False)
    theta, logw, logpi = s.state()
    c = s.counters()
    lz = s.log_evidence()
    out = (theta.cpu().numpy(), logw.cpu().numpy(), logpi.cpu().numpy(), c["grad_evals"], lz)
    s.close()
    return out


@pytest.mark.parametrize("precision", ["f32", "bf16"])
def test_same_seed_bit_identical(precision):
    N, d, J = 3000, 40, 1500
    X, y, _ = synth.logistic_iid(N, d, 31)
    eps = synth.default_step_size(N, d)
    kw = dict(step_size=eps, traj_length=eps * 24, max_leapfrog=48, num_warmup=3, seed=5)
    log(f"[determinism] {precision} N={N} d={d} J={J}")
    a = _run(X, y, J, precision, 6, **kw)
    b = _run(X, y, J, precision, 6, **kw)
    for u, v in zip(a[:3], b[:3]):
        assert np.array_equal(u.view(np.uint8), v.view(np.uint8))
    assert a[3] == b[3] and a[4] == b[4]
