"""The C-ABI library loads and exports every function include/chees_smc.h
declares.  No compute call is made (no GPU needed)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "chees_smc.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(", src, flags=re.M)
    return sorted(set(names))


def _lib():
    from paper_2504_02627_amd import build, chees
    if not os.path.exists(chees.LIB_PATH):
        build.build()
    return chees.load()


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("smc_init", "smc_step", "chees_adapt", "resample", "log_evidence",
                     "resample_indices", "smc_workspace_bytes", "smc_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = _lib()
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_struct_sizes_match_c_layout():
    from paper_2504_02627_amd import chees
    # natural alignment: these sizes follow from the field lists of the header
    # ... flow_lr, num_iterations (+pad), sobol_table, sobol_dims (+pad)
    # ... sobol_dims, lf_items, lf_split_cap (+pad)
    assert ctypes.sizeof(chees.Params) == (4 * 8 + 8 * 8 + 4 + 4 + 8 + 8 + 3 * 4 + 4 + 8 + 4 + 4
                                           + 8 + 4 + 2 * 4 + 4)
    assert ctypes.sizeof(chees.Stats) == 8 * 8 + 4 + 4 + 8
    assert ctypes.sizeof(chees.Inject) == 3 * 8
    # num_posteriors (+pad), n_rows, dims, X, y, x_dtype (+pad), prior_var,
    # target (+pad), mean, precision, log_const, banana s1/b/c, funnel_scale
    assert ctypes.sizeof(chees.Problem) == 8 + 4 * 8 + 8 + 8 + 8 + 2 * 8 + 8 + 3 * 8 + 8


def test_workspace_query_validates_without_gpu():
    from paper_2504_02627_amd import chees
    lib = _lib()
    n = (ctypes.c_int32 * 1)(200)
    d = (ctypes.c_int32 * 1)(5)
    X = (ctypes.c_void_p * 1)(0x1000)
    y = (ctypes.c_void_p * 1)(0x2000)
    prob = chees.Problem(1, n, d, X, y, chees.SMC_F32, 1.0)
    par = chees.make_params(256, max_leapfrog=64)
    assert lib.smc_workspace_bytes(ctypes.byref(prob), ctypes.byref(par)) > 0
    bad = chees.make_params(0)
    assert lib.smc_workspace_bytes(ctypes.byref(prob), ctypes.byref(bad)) == 0
    d[0] = 209
    assert lib.smc_workspace_bytes(ctypes.byref(prob), ctypes.byref(par)) == 0
    assert lib.resample_workspace_bytes(0) == 0 and lib.resample_workspace_bytes(1000) >= 8000


def test_binding_refuses_to_run_without_library(tmp_path, monkeypatch):
    from paper_2504_02627_amd import chees
    monkeypatch.setattr(chees, "_LIB", None)
    monkeypatch.setattr(chees, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError):
        chees.load()


def test_flow_parameter_count_matches_the_oracle_layout():
    import numpy as np
    from oracle import flow as F
    lib = _lib()
    for d, L in ((100, 4), (5, 2), (2, 1), (208, 8), (37, 3)):
        ps = F.init_params(d, L, 128, np.random.default_rng(0))
        assert lib.smc_flow_param_count(d, L, 128) == len(F.flatten(ps))
    assert lib.smc_flow_param_count(1, 4, 128) == 0
    assert lib.smc_flow_param_count(100, 9, 128) == 0
    assert lib.smc_flow_param_count(100, 4, 64) == 0


def test_sobol_table_is_validated_without_gpu():
    from paper_2504_02627_amd import chees
    lib = _lib()
    n = (ctypes.c_int32 * 1)(200)
    d = (ctypes.c_int32 * 1)(5)
    X = (ctypes.c_void_p * 1)(0x1000)
    y = (ctypes.c_void_p * 1)(0x2000)
    prob = chees.Problem(1, n, d, X, y, chees.SMC_F32, 1.0)
    par = chees.make_params(256, jitter="sobolNd", num_iterations=50)
    assert par.sobol_dims == 1024 and lib.smc_workspace_bytes(ctypes.byref(prob), ctypes.byref(par)) > 0
    tab = par._sobol
    assert tab[1, 0] == 3 and tab[2, 0] == 7 and list(tab[2, 1:3]) == [1, 3]
    tab[2, 2] = 2                                      # m_2 even: not a direction integer
    assert lib.smc_workspace_bytes(ctypes.byref(prob), ctypes.byref(par)) == 0
    tab[2, 2] = 5                                      # m_2 >= 2^2
    assert lib.smc_workspace_bytes(ctypes.byref(prob), ctypes.byref(par)) == 0
    tab[2, 2] = 3
    tab[4, 0] = 6                                      # polynomial without constant term
    assert lib.smc_workspace_bytes(ctypes.byref(prob), ctypes.byref(par)) == 0
    inv = chees.make_params(256, jitter="sobolNd_inv", num_iterations=50)
    assert lib.smc_workspace_bytes(ctypes.byref(prob), ctypes.byref(inv)) > 0
    inv.num_iterations = 2000                          # more columns than table rows
    assert lib.smc_workspace_bytes(ctypes.byref(prob), ctypes.byref(inv)) == 0
    inv.num_iterations = 50
    inv.sobol_table = None
    assert lib.smc_workspace_bytes(ctypes.byref(prob), ctypes.byref(inv)) == 0
    assert lib.smc_workspace_bytes(ctypes.byref(prob), ctypes.byref(
        chees.make_params(256, jitter="sobol1d"))) > 0


def test_noalloc_resampling_validates_without_gpu():
    # sizes past the static scratch and bad arguments are refused before any
    # device call
    lib = _lib()
    assert lib.resample_noalloc_max() == 1 << 20
    fake = ctypes.c_void_p(0x1000)
    assert lib.resample_indices_noalloc(fake, (1 << 20) + 1, fake, 0, fake, None) == -1
    assert lib.resample_indices_noalloc(None, 16, fake, 0, fake, None) == -1
    assert lib.resample_indices_noalloc(fake, 0, fake, 0, fake, None) == -1
    assert lib.resample_indices_noalloc(fake, 16, fake, 2, fake, None) == -1


def test_launch_tuning_is_validated():
    from paper_2504_02627_amd import chees
    lib = _lib()
    n = (ctypes.c_int32 * 1)(200)
    d = (ctypes.c_int32 * 1)(5)
    X = (ctypes.c_void_p * 1)(0x1000)
    y = (ctypes.c_void_p * 1)(0x2000)
    prob = chees.Problem(1, n, d, X, y, 0, 1.0)
    for bad in (dict(lf_split_cap=65), dict(lf_split_cap=-1), dict(lf_items=4097), dict(lf_items=-3)):
        par = chees.make_params(256, **bad)
        assert lib.smc_workspace_bytes(ctypes.byref(prob), ctypes.byref(par)) == 0, bad
    for good in (dict(lf_split_cap=1), dict(lf_items=4096, lf_split_cap=64)):
        par = chees.make_params(256, **good)
        assert lib.smc_workspace_bytes(ctypes.byref(prob), ctypes.byref(par)) > 0, good
