"""Random problems and parameters through the library's host-side validation
and planning (smc_workspace_bytes and the other calls that need no GPU), for
a run under AddressSanitizer / UndefinedBehaviorSanitizer.  Usage:
python tests/_host_fuzz.py LIBRARY CASES.  Mostly valid configurations (so
the planner runs on many shapes), the rest with invalid fields."""

import ctypes
import os
import random
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from paper_2504_02627_amd import chees  # noqa: E402


def case(rng, valid):
    B = rng.choice([1, 1, 1, 2, 3, 7, 64]) if valid else rng.choice([0, 1, 2])
    target = 0 if (valid and B > 1) or rng.random() < 0.7 else rng.choice([1, 2, 3, 4])
    N = [rng.randint(1, 30000) if valid else rng.choice([0, 1, 200]) for _ in range(B)]
    d = [rng.randint(1, 208) if valid else rng.choice([0, 5, 209]) for _ in range(B)]
    if target == 2:
        d = [2] * B
    n = (ctypes.c_int32 * max(B, 1))(*(N or [0]))
    dd = (ctypes.c_int32 * max(B, 1))(*(d or [0]))
    X = (ctypes.c_void_p * max(B, 1))(*([0x1000] * max(B, 1)))
    y = (ctypes.c_void_p * max(B, 1))(*([0x2000] * max(B, 1)))
    prob = chees.Problem(B, n, dd, X, y, rng.choice([0, 1]) if valid else rng.choice([0, 2]),
                         1.0 if valid else rng.choice([1.0, 0.0]))
    prob.target = target
    prob.mean, prob.precision = 0x3000, 0x4000
    prob.banana_s1, prob.banana_b, prob.banana_c = 10.0, 0.03, 100.0
    prob.funnel_scale = 3.0 if valid else rng.choice([3.0, -1.0])
    jit = rng.choice(list(chees.JITTER))
    K = rng.randint(1, 1024) if valid else rng.choice([0, 2000])
    kw = dict(max_leapfrog=rng.randint(1, 4096) if valid else rng.choice([0, 5000]),
              num_warmup=rng.randint(1, 100), jitter=jit,
              resampling=rng.choice(["systematic", "multinomial"]),
              precision=rng.choice(["f32", "bf16"]),
              precond=rng.choice(["none", "diag"] + (["flow"] if B == 1 else [])),
              flow_layers=rng.randint(0, 8) if valid else 9, flow_width=128,
              num_iterations=K, sobol_dims=K if jit.startswith("sobol") else 0)
    par = chees.make_params(rng.randint(1, 65536) if valid else rng.choice([0, 70000]), **kw)
    if not valid and getattr(par, "_sobol", None) is not None and rng.random() < 0.5:
        par._sobol[rng.randrange(len(par._sobol)), rng.randrange(19)] = rng.randrange(1 << 20)
    return prob, par


def main():
    chees.LIB_PATH = sys.argv[1]
    lib = chees.load()
    cases = int(sys.argv[2]) if len(sys.argv) > 2 else 2000
    rng = random.Random(12345)
    accepted = 0
    for i in range(cases):
        prob, par = case(rng, valid=rng.random() < 0.8)
        accepted += lib.smc_workspace_bytes(ctypes.byref(prob), ctypes.byref(par)) > 0
    for J in (0, 1, 1000, 1 << 20):
        lib.resample_workspace_bytes(J)
    for d, L, w in ((100, 4, 128), (1, 4, 128), (2, 0, 128), (208, 8, 128), (100, 9, 128)):
        lib.smc_flow_param_count(d, L, w)
    lib.smc_state_bytes(None)
    print(f"host fuzz: {cases} cases, {accepted} accepted", flush=True)


if __name__ == "__main__":
    main()
