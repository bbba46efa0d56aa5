"""The benchmark's matched-error test (bench.matched) on synthetic replicate
moments: with standard errors estimated from 8 seeds and 4 reference runs, a
correct sampler is declared beyond "3 SE" in about the normal's 0.27 % of
dimensions (up to Welch's approximation) and passes nearly always, and a
biased one fails.  The null distribution is drawn here, independently of the
benchmark."""

import numpy as np
from scipy import stats

import bench


def _case(rng, d, R, Rref, bias=None):
    mu = rng.standard_normal(d)
    v = 0.5 + rng.random(d)
    sd_form = 0.01 * (0.5 + rng.random(d))
    sd_ref = 0.01 * (0.5 + rng.random(d))
    fm = mu + sd_form * rng.standard_normal((R, d))
    fv = v + sd_form * rng.standard_normal((R, d))
    if bias is not None:
        fm = fm + bias * sd_form
    refm = mu + sd_ref * rng.standard_normal((Rref, d))
    refv = v + sd_ref * rng.standard_normal((Rref, d))
    se = lambda a: a.std(0, ddof=1) / np.sqrt(len(a))
    ref = dict(mean=refm.mean(0), var=refv.mean(0), se_mean=se(refm), se_var=se(refv), runs=Rref)
    rep = dict(final_mean=fm, final_var=fv, ms_per_iteration=1.0, evals_per_s=1.0, ess_per_s=1.0,
               ess_per_grad_eval_after_burn_in=1.0)
    return bench.matched(ref, rep, "synthetic")


def test_correct_sampler_exceeds_at_the_normal_rate_and_passes():
    rng = np.random.default_rng(5)
    d, R, Rref, trials = 100, 8, 4, 300
    beyond, beyond_normal, fails = 0, 0, 0
    for _ in range(trials):
        out = _case(rng, d, R, Rref)
        beyond += out["mean_dims_beyond_3se"] + out["var_dims_beyond_3se"]
        beyond_normal += out["mean_dims_beyond_3_normal"] + out["var_dims_beyond_3_normal"]
        fails += not out["pass_3se"]
    rate = beyond / (2 * d * trials)
    p = 2 * stats.norm.sf(3.0)
    # Welch's degrees of freedom are an approximation (3 for the reference
    # alone here): the rate comes out near 0.4 %, against 0.27 % nominal
    assert rate < 2 * p, rate
    # a normal threshold on estimated SEs exceeds several times as often
    assert beyond_normal / (2 * d * trials) > 3 * p
    assert fails <= 0.03 * trials, fails


def test_biased_sampler_fails():
    rng = np.random.default_rng(6)
    d = 100
    bias = np.zeros(d)
    bias[:10] = 6.0  # six single-run SDs in ten dimensions of the means
    out = _case(rng, d, 8, 4, bias=bias)
    assert out["mean_dims_beyond_3se"] >= 3
    assert not out["pass_3se"]
