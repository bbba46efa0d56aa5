"""Jitter generators of Sec. III-B-1 on the device against the oracle's
definitions: h_jk bit-exact for every scheme over several iterations
(including iterations past K for the schemes that take K), the step counts
n_j that follow from them, per-posterior streams of a batched context, and
the Sobol schemes at the largest particle count and past the table's
dimensions.
"""

import numpy as np
import pytest

from oracle import smc as O
from paper_2504_02627_amd import synth
from tests._gpu_common import log, to_dev

pytestmark = pytest.mark.gpu

SCHEMES = ["halton1d", "none", "haltonNd", "uniform", "haltonNd_inv", "primes", "primes_inv",
           "golden", "equidistant", "equidistant_offset", "sobol1d", "sobolNd", "sobolNd_inv"]


def _oracle_h(kind, seed, k, K, J, b=0):
    if kind == "halton1d":
        return O.halton_1d(k, J)
    if kind == "none":
        return np.ones(J)
    if kind == "haltonNd":
        return O.halton_nd(k, J)
    if kind == "uniform":
        return O.uniform_jitter(seed, k, J, b)
    if kind == "haltonNd_inv":
        return O.halton_nd_inverse(k, K, J)
    if kind == "primes":
        return O.primes_nd(k, J)
    if kind == "primes_inv":
        return O.primes_nd_inverse(k, K, J)
    if kind == "golden":
        return O.golden_1d(k, K, J)
    if kind == "equidistant":
        return O.equidistant(seed, k, J, b)
    if kind == "sobol1d":
        return O.sobol_1d(k, J)
    if kind == "sobolNd":
        return O.sobol_nd(k, J)
    if kind == "sobolNd_inv":
        return O.sobol_nd_inverse(k, K, J)
    return O.equidistant_offset(seed, k, J, b)


@pytest.mark.parametrize("kind", SCHEMES)
def test_jitter_bit_exact_over_iterations(kind):
    from paper_2504_02627_amd import chees
    N, d, J, K, seed = 200, 5, 300, 2, 77   # J not a power of two, beyond one tile
    log(f"[jitter] scheme={kind} J={J} K={K}")
    X, y, _ = synth.logistic_iid(N, d, 3)
    eps = synth.default_step_size(N, d)
    s = chees.Sampler(to_dev(X), to_dev(y), J, step_size=eps, traj_length=eps * 20,
                      max_leapfrog=64, num_warmup=10, seed=seed, jitter=kind, num_iterations=K)
    for k in range(1, 5):                    # k = 3, 4 run past K
        st = s.step()
        s.adapt()
        tr = s.trace()
        h = tr["h"].cpu().numpy()[:J]
        n = tr["n"].cpu().numpy()[:J]
        ref = _oracle_h(kind, seed, k, K, J)
        np.testing.assert_array_equal(h, ref)
        _, nref = O.step_counts(ref, st["L"], st["eps"], 64)
        np.testing.assert_array_equal(n, nref)
    if kind in ("equidistant", "equidistant_offset"):
        base = O.equidistant(seed, 4, J)
        np.testing.assert_array_equal(np.sort(base), np.arange(1, J + 1) / J)


@pytest.mark.parametrize("kind", ["uniform", "equidistant", "equidistant_offset"])
def test_jitter_streams_per_posterior(kind):
    from paper_2504_02627_amd import chees
    J, seed = 130, 5
    data = [synth.logistic_iid(120, 4, 1), synth.logistic_iid(90, 7, 2)]
    Xs = [to_dev(X) for X, _, _ in data]
    ys = [to_dev(y) for _, y, _ in data]
    log(f"[jitter] batched scheme={kind} J={J}")
    s = chees.Sampler(Xs, ys, J, step_size=0.05, traj_length=1.0, max_leapfrog=32,
                      num_warmup=5, seed=seed, jitter=kind)
    s.step()
    tr = s.trace()
    jc = tr["jcap"]
    h = tr["h"].cpu().numpy()
    for b in range(2):
        np.testing.assert_array_equal(h[b * jc:b * jc + J], _oracle_h(kind, seed, 1, 0, J, b))


def test_sobol_at_full_particle_count_and_past_the_table():
    # J = 65536 (every Gray-code bit up to 2^16), and a table of 3 dimensions
    # for 5 iterations: iterations 4 and 5 reuse dimension 3
    from paper_2504_02627_amd import chees
    J = 65536
    X, y, _ = synth.logistic_iid(64, 3, 4)
    log(f"[jitter] sobolNd J={J} table of 3 dimensions")
    s = chees.Sampler(to_dev(X), to_dev(y), J, step_size=0.05, traj_length=0.5,
                      max_leapfrog=16, num_warmup=3, seed=2, jitter="sobolNd", sobol_dims=3)
    rows = O.joe_kuo_rows(3)
    for k in range(1, 6):
        s.step()
        s.adapt()
        h = s.trace()["h"].cpu().numpy()[:J]
        np.testing.assert_array_equal(h, O.sobol_nd(min(k, 3), J, rows))


@pytest.mark.parametrize("J,nmax,B", [(300, 64, 1), (16384, 64, 1), (65536, 255, 1), (1000, 300, 1),
                                      (130, 32, 2), (3000, 64, 3)])
def test_particle_order_is_a_stable_sort_by_steps(J, nmax, B):
    # the order in which the trajectory kernels take the particles: every row
    # once, n_j non-increasing, index order within equal n_j; active counts
    # #{j: n_j > s}.  n_max = 300 takes the single-group sort, the others the
    # multi-group one (up to 64 groups of 1024 particles).
    from paper_2504_02627_amd import chees
    log(f"[order] J={J} nmax={nmax} B={B}")
    data = [synth.logistic_iid(120, 4, 1 + b) for b in range(B)]
    Xs = [to_dev(X) for X, _, _ in data]
    ys = [to_dev(y) for _, y, _ in data]
    s = chees.Sampler(Xs, ys, J, step_size=0.05, traj_length=0.05 * nmax / 2, max_leapfrog=nmax,
                      num_warmup=5, seed=9, jitter="uniform")
    for _ in range(2):
        st = s.step()
        s.adapt()
        tr = s.trace()
        jc = tr["jcap"]
        n_all = tr["n"].cpu().numpy()
        order = tr["order"].cpu().numpy()
        act = tr["active"].cpu().numpy().reshape(B, nmax + 1)
        for b in range(B):
            n = n_all[b * jc:(b + 1) * jc]
            o = order[b * jc:(b + 1) * jc]
            ref = np.array(sorted(range(jc), key=lambda j: (-n[j], j)))
            np.testing.assert_array_equal(o, ref)
            np.testing.assert_array_equal(act[b], [(n > k).sum() for k in range(nmax)] + [0])
        assert st["grad_evals"] == int(n_all[:jc].sum())
