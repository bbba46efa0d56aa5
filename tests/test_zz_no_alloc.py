"""The no-allocation resampling entry point (resample_indices_noalloc, for
callers that cannot allocate device memory) against resample_indices with a
caller workspace, through the C ABI: bit-identical ancestors on two calls in a
row, the second with a smaller input, for both schemes; sizes past the static
scratch are refused before any launch."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _case(J, seed, scheme):
    import torch
    rng = np.random.default_rng(seed)
    w = rng.exponential(size=J) * (rng.random(J) < 0.7)
    w[rng.integers(J)] = 1.0  # not all zero
    u = rng.random(J if scheme == "multinomial" else 1)
    dev = torch.device("cuda:0")
    return (torch.from_numpy(w).to(dev), torch.from_numpy(u).to(dev))


@pytest.mark.parametrize("scheme", ["systematic", "multinomial"])
def test_noalloc_matches_workspace_entry_point(scheme):
    import torch
    from paper_2504_02627_amd import chees
    lib = chees.load()
    assert lib.resample_noalloc_max() == 1 << 20
    # the largest size first, then a smaller one: the static array keeps the
    # previous call's contents, which must not leak into the second result
    for J, seed in ((1 << 20, 1), (3001, 2), (1, 3)):
        w, u = _case(J, seed, scheme)
        ref = chees.resample_indices(w, u, scheme)
        anc = torch.full((J,), -7, dtype=torch.int32, device=w.device)
        chees.resample_indices_noalloc(w, u, anc, scheme)
        assert torch.equal(anc, ref), (scheme, J)


def test_noalloc_refuses_oversize_and_degenerate():
    import torch
    from paper_2504_02627_amd import chees
    lib = chees.load()
    dev = torch.device("cuda:0")
    J = (1 << 20) + 1
    w = torch.ones(J, dtype=torch.float64, device=dev)
    u = torch.full((1,), 0.5, dtype=torch.float64, device=dev)
    anc = torch.zeros(J, dtype=torch.int32, device=dev)
    with pytest.raises(chees.SmcError) as e:
        chees.resample_indices_noalloc(w, u, anc)
    assert e.value.status == chees.SMC_EINVAL
    z = torch.zeros(16, dtype=torch.float64, device=dev)
    with pytest.raises(chees.SmcError) as e:
        chees.resample_indices_noalloc(z, u, anc[:16])
    assert e.value.status == chees.SMC_EDEGENERATE
    # and the entry point still works after the refusals
    w, u = _case(5000, 4, "systematic")
    anc = torch.zeros(5000, dtype=torch.int32, device=dev)
    chees.resample_indices_noalloc(w, u, anc)
    assert torch.equal(anc, chees.resample_indices(w, u))
    assert lib.resample_noalloc_max() == 1 << 20
