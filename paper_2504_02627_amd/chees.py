"""Thin ctypes binding of libchees_smc.so (include/chees_smc.h).

Argument marshalling only: every step of the sampler runs in the library's
HIP kernels.  torch supplies device memory and the stream.  The binding fails
loudly when the library is missing: there is no CPU fallback.
"""

import ctypes
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libchees_smc.so")

SMC_OK, SMC_EINVAL, SMC_EDEVICE, SMC_EDEGENERATE, SMC_ESTATE, SMC_ENOMEM = 0, -1, -2, -3, -4, -5
SMC_WADAPTIVE = 1
STATUS = {0: "SMC_OK", -1: "SMC_EINVAL", -2: "SMC_EDEVICE", -3: "SMC_EDEGENERATE",
          -4: "SMC_ESTATE", -5: "SMC_ENOMEM", 1: "SMC_WADAPTIVE"}
SMC_F32, SMC_BF16 = 0, 1
JITTER = {"halton1d": 0, "none": 1, "haltonNd": 2, "uniform": 3, "haltonNd_inv": 4,
          "primes": 5, "primes_inv": 6, "golden": 7, "equidistant": 8,
          "equidistant_offset": 9, "sobol1d": 10, "sobolNd": 11, "sobolNd_inv": 12}
RESAMPLING = {"systematic": 0, "multinomial": 1}
PRECISION = {"f32": 0, "bf16": 1}
PRECOND = {"none": 0, "diag": 1, "flow": 2}
TARGET = {"logistic": 0, "gaussian": 1, "banana": 2, "funnel": 3}
ADAPT_EPS = {False: 0, True: 1, "none": 0, "adam": 1, "dual_averaging": 2}


class SmcError(RuntimeError):
    def __init__(self, status, msg=""):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Problem(ctypes.Structure):
    _fields_ = [("num_posteriors", ctypes.c_int32),
                ("n_rows", ctypes.POINTER(ctypes.c_int32)),
                ("dims", ctypes.POINTER(ctypes.c_int32)),
                ("X", ctypes.POINTER(ctypes.c_void_p)),
                ("y", ctypes.POINTER(ctypes.c_void_p)),
                ("x_dtype", ctypes.c_int32),
                ("prior_var", ctypes.c_double),
                ("target", ctypes.c_int32),
                ("mean", ctypes.c_void_p),
                ("precision", ctypes.c_void_p),
                ("log_const", ctypes.c_double),
                ("banana_s1", ctypes.c_double),
                ("banana_b", ctypes.c_double),
                ("banana_c", ctypes.c_double),
                ("funnel_scale", ctypes.c_double)]


class Params(ctypes.Structure):
    _fields_ = [("num_particles", ctypes.c_int32), ("max_leapfrog", ctypes.c_int32),
                ("num_warmup", ctypes.c_int32), ("jitter", ctypes.c_int32),
                ("mh_accept", ctypes.c_int32), ("resampling", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("precond", ctypes.c_int32),
                ("step_size", ctypes.c_double), ("traj_length", ctypes.c_double),
                ("ess_frac", ctypes.c_double), ("adam_lr", ctypes.c_double),
                ("adam_b1", ctypes.c_double), ("adam_b2", ctypes.c_double),
                ("adam_eps", ctypes.c_double), ("avg_decay", ctypes.c_double),
                ("adapt_step_size", ctypes.c_int32), ("target_accept", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("flow_layers", ctypes.c_int32),
                ("flow_width", ctypes.c_int32), ("flow_train_steps", ctypes.c_int32),
                ("flow_lr", ctypes.c_double), ("num_iterations", ctypes.c_int32),
                ("sobol_table", ctypes.c_void_p), ("sobol_dims", ctypes.c_int32),
                ("lf_items", ctypes.c_int32), ("lf_split_cap", ctypes.c_int32)]


class Inject(ctypes.Structure):
    _fields_ = [("momenta", ctypes.c_void_p), ("mh_uniforms", ctypes.c_void_p),
                ("resample_u", ctypes.c_void_p)]


class Stats(ctypes.Structure):
    _fields_ = [("ess", ctypes.c_double), ("ess_before", ctypes.c_double),
                ("mean_accept", ctypes.c_double), ("chees", ctypes.c_double),
                ("chees_grad", ctypes.c_double), ("L", ctypes.c_double),
                ("eps", ctypes.c_double), ("log_z", ctypes.c_double),
                ("resampled", ctypes.c_int32), ("iteration", ctypes.c_int32),
                ("grad_evals", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Counters(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("grad_evals", ctypes.c_int64),
                ("ess_sum", ctypes.c_double), ("resamples", ctypes.c_int64)]


class Timing(ctypes.Structure):
    _fields_ = [("leapfrog_ms", ctypes.c_double), ("leapfrog_launches", ctypes.c_int64),
                ("loglik_ms", ctypes.c_double), ("loglik_launches", ctypes.c_int64),
                ("reduce_ms", ctypes.c_double), ("reduce_launches", ctypes.c_int64),
                ("flow_ms", ctypes.c_double), ("flow_launches", ctypes.c_int64),
                ("train_ms", ctypes.c_double), ("train_launches", ctypes.c_int64)]


class Trace(ctypes.Structure):
    _fields_ = [("h", ctypes.c_void_p), ("l", ctypes.c_void_p), ("n", ctypes.c_void_p),
                ("dH", ctypes.c_void_p), ("alpha", ctypes.c_void_p),
                ("ancestors", ctypes.c_void_p), ("p_final", ctypes.c_void_p),
                ("theta_prop", ctypes.c_void_p), ("grad", ctypes.c_void_p),
                ("minv", ctypes.c_void_p), ("latent0", ctypes.c_void_p),
                ("latent", ctypes.c_void_p), ("latent_grad", ctypes.c_void_p),
                ("logdet0", ctypes.c_void_p), ("logdet", ctypes.c_void_p),
                ("dpad", ctypes.c_int32), ("jcap", ctypes.c_int32),
                ("order", ctypes.c_void_p), ("active", ctypes.c_void_p)]


_LIB = None


def load():
    """Load libchees_smc.so; raise if it has not been built."""
    global _LIB
    if _LIB is None:
        # torch first: its HIP runtime (same soname) then serves the library too,
        # so torch's streams and pointers are valid in the library's calls
        _torch()
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2504_02627_amd.build")
        lib = ctypes.CDLL(LIB_PATH)
        vp, i32, sz, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t, ctypes.c_double
        P = ctypes.POINTER
        sig = {
            "smc_workspace_bytes": (sz, [P(Problem), P(Params)]),
            "smc_init": (i32, [P(Problem), P(Params), vp, sz, vp, vp, P(vp)]),
            "smc_step": (i32, [vp, P(Inject), P(Stats)]),
            "chees_adapt": (i32, [vp, P(Stats)]),
            "smc_run": (i32, [vp, i32]),
            "smc_flow_param_count": (sz, [i32, i32, i32]),
            "smc_get_flow": (i32, [vp, vp, vp, vp, vp]),
            "smc_set_flow": (i32, [vp, vp]),
            "resample": (i32, [vp, vp, vp]),
            "resample_workspace_bytes": (sz, [i32]),
            "resample_indices": (i32, [vp, i32, vp, i32, vp, vp, sz, vp]),
            "resample_noalloc_max": (i32, []),
            "resample_indices_noalloc": (i32, [vp, i32, vp, i32, vp, vp]),
            "log_evidence": (i32, [vp, P(dbl), P(dbl)]),
            "smc_get_state": (i32, [vp, vp, vp, vp]),
            "smc_get_trace": (i32, [vp, P(Trace)]),
            "smc_get_counters": (i32, [vp, P(Counters)]),
            "smc_set_params": (i32, [vp, dbl, dbl]),
            "smc_set_timing": (i32, [vp, i32]),
            "smc_state_bytes": (ctypes.c_size_t, [vp]),
            "smc_save": (i32, [vp, vp, ctypes.c_size_t]),
            "smc_load": (i32, [vp, vp, ctypes.c_size_t]),
            "smc_get_timing": (i32, [vp, P(Timing)]),
            "smc_destroy": (None, [vp]),
            "smc_last_error": (ctypes.c_char_p, [vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _LIB = lib
    return _LIB


def _torch():
    import torch
    return torch


def _stream_handle(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


DEFAULT_PARAMS = dict(max_leapfrog=64, num_warmup=10, jitter="halton1d", mh_accept=False,
                      resampling="systematic", precision="f32", precond="none",
                      step_size=0.1, traj_length=5.0, ess_frac=0.5, adam_lr=0.025,
                      adam_b1=0.9, adam_b2=0.999, adam_eps=1e-8, avg_decay=0.9,
                      adapt_step_size=False, target_accept=0.651, seed=0,
                      flow_layers=4, flow_width=128, flow_train_steps=10, flow_lr=1e-3,
                      num_iterations=0, sobol_dims=0, lf_items=0, lf_split_cap=0)


SOBOL_MAX_DIMS = 21201


def sobol_table(dims):
    """The first `dims` rows of Joe and Kuo's Sobol direction-number table in
    the layout smc_params.sobol_table takes (polynomial mask, m_1..m_18 per
    row), read from the copy the scipy package ships (a numpy archive of
    integers, loaded without pickle)."""
    import numpy as np
    import scipy.stats
    path = os.path.join(os.path.dirname(scipy.stats.__file__), "_sobol_direction_numbers.npz")
    with np.load(path) as z:
        poly, vinit = z["poly"][:dims], z["vinit"][:dims]
    tab = np.zeros((dims, 19), dtype=np.uint32)
    tab[:, 0] = poly
    tab[:, 1:] = vinit
    return np.ascontiguousarray(tab)


def make_params(num_particles, **kw):
    p = dict(DEFAULT_PARAMS)
    unknown = set(kw) - set(p)
    if unknown:
        raise TypeError(f"unknown parameters {sorted(unknown)}")
    p.update(kw)
    par = Params(num_particles, p["max_leapfrog"], p["num_warmup"], JITTER[p["jitter"]],
                 int(bool(p["mh_accept"])), RESAMPLING[p["resampling"]],
                 PRECISION[p["precision"]], PRECOND[p["precond"]], p["step_size"],
                 p["traj_length"], p["ess_frac"], p["adam_lr"], p["adam_b1"], p["adam_b2"],
                 p["adam_eps"], p["avg_decay"], ADAPT_EPS[p["adapt_step_size"]],
                 p["target_accept"], p["seed"], p["flow_layers"], p["flow_width"],
                 p["flow_train_steps"], p["flow_lr"], p["num_iterations"])
    if p["jitter"] in ("sobolNd", "sobolNd_inv"):
        # one dimension per iteration: sobol_dims if given, else K of them
        # (1024 when K is not given either)
        dims = int(p["sobol_dims"]) or min(max(int(p["num_iterations"]), 1024), SOBOL_MAX_DIMS)
        par._sobol = sobol_table(dims)      # kept alive with the struct
        par.sobol_table = par._sobol.ctypes.data
        par.sobol_dims = dims
    par.lf_items, par.lf_split_cap = int(p["lf_items"]), int(p["lf_split_cap"])
    return par


def make_problem(Xs, ys, prior_var=1.0):
    torch = _torch()
    B = len(Xs)
    dt = SMC_BF16 if Xs[0].dtype == torch.bfloat16 else SMC_F32
    for X, y in zip(Xs, ys):
        if not (X.is_cuda and y.is_cuda):
            raise ValueError("X and y must be device tensors")
        if X.dim() != 2 or not X.is_contiguous() or y.dtype != torch.float32:
            raise ValueError("X: contiguous 2-d; y: float32")
        if (X.dtype == torch.bfloat16) != (dt == SMC_BF16) or X.dtype not in (torch.float32, torch.bfloat16):
            raise ValueError("X dtype: float32 or bfloat16, the same for all posteriors")
    keep = dict(
        n=(ctypes.c_int32 * B)(*[X.shape[0] for X in Xs]),
        d=(ctypes.c_int32 * B)(*[X.shape[1] for X in Xs]),
        X=(ctypes.c_void_p * B)(*[X.data_ptr() for X in Xs]),
        y=(ctypes.c_void_p * B)(*[y.data_ptr() for y in ys]),
    )
    prob = Problem(B, keep["n"], keep["d"], keep["X"], keep["y"], dt, prior_var)
    return prob, keep


def make_target_problem(kind, dim, mean=None, precision=None, log_const=0.0,
                        banana=(10.0, 0.03, 100.0), funnel_scale=3.0, prior_var=1.0):
    """Problem for a synthetic target: "gaussian" (device float32 mean [d] and
    precision [d, d]), "banana" (d = 2; s1, b, c) or "funnel" (d >= 2; the
    standard deviation of v)."""
    keep = dict(d=(ctypes.c_int32 * 1)(int(dim)))
    prob = Problem(1, None, keep["d"], None, None, SMC_F32, prior_var)
    prob.target = TARGET[kind]
    prob.log_const = float(log_const)
    if kind == "gaussian":
        for t, shape in ((mean, (dim,)), (precision, (dim, dim))):
            if t is None or not t.is_cuda or tuple(t.shape) != shape or not t.is_contiguous() \
                    or t.dtype != _torch().float32:
                raise ValueError("gaussian target: float32 contiguous device mean [d] and precision [d, d]")
        keep["mean"], keep["precision"] = mean, precision
        prob.mean, prob.precision = mean.data_ptr(), precision.data_ptr()
    elif kind == "banana":
        prob.banana_s1, prob.banana_b, prob.banana_c = (float(v) for v in banana)
    elif kind == "funnel":
        prob.funnel_scale = float(funnel_scale)
    else:
        raise ValueError(kind)
    return prob, keep


class Sampler:
    """One SMC/ChEES-HMC sampler context over B posteriors (include/chees_smc.h)."""

    def __init__(self, Xs, ys, num_particles, prior_var=1.0, theta0=None, stream=None,
                 target=None, tune=None, **params):
        """target: None (logistic regression on Xs, ys) or a dict with "kind"
        ("gaussian" / "banana"), "dim" and the arguments of make_target_problem;
        Xs and ys are then unused.  tune="cache": take the launch setting
        (lf_items, lf_split_cap) the autotuner stored for this workload, unless
        given explicitly."""
        torch = _torch()
        self.lib = load()
        self.J = int(num_particles)
        self.stream = stream
        if target is None:
            if not isinstance(Xs, (list, tuple)):
                Xs, ys = [Xs], [ys]
            self.Xs, self.ys = list(Xs), list(ys)
            self.B = len(Xs)
            self.dims = [int(X.shape[1]) for X in Xs]
            self.device = Xs[0].device
            self.prob, self._keep = make_problem(self.Xs, self.ys, prior_var)
        else:
            t = dict(target)
            kind, dim = t.pop("kind"), int(t.pop("dim"))
            self.Xs, self.ys, self.B, self.dims = [], [], 1, [dim]
            self.device = t["mean"].device if kind == "gaussian" else torch.device("cuda:0")
            self.prob, self._keep = make_target_problem(kind, dim, prior_var=prior_var, **t)
        if tune == "cache" and target is None:
            from paper_2504_02627_amd import autotune
            best = autotune.lookup(self.dims, [X.shape[0] for X in self.Xs], self.J,
                                   params.get("precision", "f32"), params.get("max_leapfrog", 64))
            params = dict(best, **params)
        elif tune not in (None, "cache"):
            raise ValueError("tune: None or 'cache'")
        self.tuned = {k: params.get(k, 0) for k in ("lf_items", "lf_split_cap")}
        self.evidence_adaptive = False
        self.params = make_params(self.J, **params)
        nbytes = self.lib.smc_workspace_bytes(ctypes.byref(self.prob), ctypes.byref(self.params))
        if nbytes == 0:
            raise SmcError(SMC_EINVAL, "invalid problem or parameters")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        self._ws_ptr = self.workspace.data_ptr() + off
        self._theta0 = theta0
        if theta0 is not None:
            self._check_inject(theta0, sum(self.J * d for d in self.dims), torch.float32, "theta0")
        ctx = ctypes.c_void_p()
        rc = self.lib.smc_init(ctypes.byref(self.prob), ctypes.byref(self.params),
                               ctypes.c_void_p(self._ws_ptr), nbytes, _stream_handle(stream),
                               _ptr(theta0), ctypes.byref(ctx))
        if rc != SMC_OK:
            raise SmcError(rc, "smc_init")
        self.ctx = ctx

    def _check(self, rc, what):
        if rc != SMC_OK:
            raise SmcError(rc, f"{what}: {self.lib.smc_last_error(self.ctx).decode()}")

    def _check_inject(self, t, n, dtype, what):
        torch = _torch()
        if t is None:
            return
        if not t.is_cuda or t.dtype != dtype or not t.is_contiguous() or t.numel() < n:
            raise ValueError(f"{what}: contiguous {dtype} device tensor with >= {n} elements")

    def step(self, momenta=None, mh_uniforms=None, resample_u=None, stats=True):
        torch = _torch()
        sched = self.params.resampling
        self._check_inject(momenta, sum(self.J * d for d in self.dims), torch.float32, "momenta")
        self._check_inject(mh_uniforms, self.B * self.J, torch.float64, "mh_uniforms")
        self._check_inject(resample_u, self.B * (self.J if sched == 1 else 1), torch.float64,
                           "resample_u")
        inj = Inject(_ptr(momenta).value, _ptr(mh_uniforms).value, _ptr(resample_u).value)
        self._inj_keep = (momenta, mh_uniforms, resample_u)
        st = Stats() if stats else None
        rc = self.lib.smc_step(self.ctx, ctypes.byref(inj),
                               ctypes.byref(st) if st is not None else None)
        self._check(rc, "smc_step")
        return st.as_dict() if st is not None else None

    def adapt(self, stats=True):
        st = Stats() if stats else None
        rc = self.lib.chees_adapt(self.ctx, ctypes.byref(st) if st is not None else None)
        self._check(rc, "chees_adapt")
        return st.as_dict() if st is not None else None

    def run(self, iterations):
        """`iterations` x (step + adapt) by replaying a captured HIP graph of one
        iteration (library randomness only); no host synchronisation."""
        self._check(self.lib.smc_run(self.ctx, int(iterations)), "smc_run")

    def resample(self, u=None, return_ancestors=False):
        torch = _torch()
        anc = torch.empty(self.B * self.J, dtype=torch.int32, device=self.device) if return_ancestors else None
        self._check_inject(u, self.B * (self.J if self.params.resampling == 1 else 1), torch.float64, "u")
        self._check(self.lib.resample(self.ctx, _ptr(u), _ptr(anc)), "resample")
        return anc

    def log_evidence(self, per_posterior=False):
        """log Z_hat of posterior 0 (or the list over posteriors).  Sets
        evidence_adaptive: True when a flow move used couplings fitted to the
        population it moved, so that the estimate is adaptive and biased."""
        lz = ctypes.c_double()
        per = (ctypes.c_double * self.B)()
        rc = self.lib.log_evidence(self.ctx, ctypes.byref(lz), per)
        self.evidence_adaptive = rc == SMC_WADAPTIVE
        if rc != SMC_WADAPTIVE:
            self._check(rc, "log_evidence")
        return list(per) if per_posterior else lz.value

    def state(self):
        torch = _torch()
        tot = sum(self.J * d for d in self.dims)
        theta = torch.empty(tot, dtype=torch.float32, device=self.device)
        logw = torch.empty(self.B * self.J, dtype=torch.float64, device=self.device)
        logpi = torch.empty(self.B * self.J, dtype=torch.float64, device=self.device)
        self._check(self.lib.smc_get_state(self.ctx, _ptr(theta), _ptr(logw), _ptr(logpi)), "smc_get_state")
        out, o = [], 0
        for d in self.dims:
            out.append(theta[o:o + self.J * d].view(self.J, d))
            o += self.J * d
        return (out if self.B > 1 else out[0]), logw, logpi

    def trace(self):
        """Per-particle views of the last step, copied into torch tensors (rows b*jcap + j)."""
        torch = _torch()
        t = Trace()
        self._check(self.lib.smc_get_trace(self.ctx, ctypes.byref(t)), "smc_get_trace")
        rows = self.B * t.jcap

        def view(ptr, n, dtype, elem):
            # device-to-device copy through a torch tensor of the same size
            out = torch.empty(n, dtype=dtype, device=self.device)
            nbytes = n * elem
            _memcpy_d2d(out.data_ptr(), ptr, nbytes, self.stream)
            return out

        res = dict(
            h=view(t.h, rows, torch.float64, 8), l=view(t.l, rows, torch.float64, 8),
            n=view(t.n, rows, torch.int32, 4), dH=view(t.dH, rows, torch.float64, 8),
            alpha=view(t.alpha, rows, torch.float64, 8),
            ancestors=view(t.ancestors, rows, torch.int32, 4),
            p_final=view(t.p_final, rows * t.dpad, torch.float32, 4).view(rows, t.dpad),
            theta_prop=view(t.theta_prop, rows * t.dpad, torch.float32, 4).view(rows, t.dpad),
            grad=view(t.grad, rows * t.dpad, torch.float32, 4).view(rows, t.dpad),
            minv=view(t.minv, self.B * t.dpad, torch.float32, 4).view(self.B, t.dpad),
            order=view(t.order, rows, torch.int32, 4),
            active=view(t.active, self.B * (self.params.max_leapfrog + 1), torch.int32, 4),
            jcap=t.jcap, dpad=t.dpad)
        if t.latent:
            res.update(
                latent0=view(t.latent0, rows * t.dpad, torch.float32, 4).view(rows, t.dpad),
                latent=view(t.latent, rows * t.dpad, torch.float32, 4).view(rows, t.dpad),
                latent_grad=view(t.latent_grad, rows * t.dpad, torch.float32, 4).view(rows, t.dpad),
                logdet0=view(t.logdet0, rows, torch.float32, 4),
                logdet=view(t.logdet, rows, torch.float32, 4))
        return res

    def flow(self, with_grad=False):
        """(FP32 coupling parameters as one flat vector, m, L[, gradient of the
        last Adam step]) of the flow preconditioner (include/chees_smc.h gives
        the layout)."""
        torch = _torch()
        d = self.dims[0]
        n = self.lib.smc_flow_param_count(d, self.params.flow_layers, self.params.flow_width)
        prm = torch.empty(n, dtype=torch.float32, device=self.device)
        m = torch.empty(d, dtype=torch.float32, device=self.device)
        L = torch.empty((d, d), dtype=torch.float32, device=self.device)
        g = torch.empty(n, dtype=torch.float32, device=self.device) if with_grad else None
        self._check(self.lib.smc_get_flow(self.ctx, _ptr(prm), _ptr(m), _ptr(L), _ptr(g)),
                    "smc_get_flow")
        return (prm, m, L, g) if with_grad else (prm, m, L)

    def set_flow(self, params):
        """Replace the coupling parameters (flat FP32 device vector)."""
        torch = _torch()
        n = self.lib.smc_flow_param_count(self.dims[0], self.params.flow_layers,
                                          self.params.flow_width)
        self._check_inject(params, n, torch.float32, "flow parameters")
        self._flow_keep = params
        self._check(self.lib.smc_set_flow(self.ctx, _ptr(params)), "smc_set_flow")

    def counters(self):
        c = Counters()
        self._check(self.lib.smc_get_counters(self.ctx, ctypes.byref(c)), "smc_get_counters")
        return {k: getattr(c, k) for k, _ in c._fields_}

    def set_timing(self, enable=True):
        self._check(self.lib.smc_set_timing(self.ctx, int(bool(enable))), "smc_set_timing")

    def timing(self):
        t = Timing()
        self._check(self.lib.smc_get_timing(self.ctx, ctypes.byref(t)), "smc_get_timing")
        return {k: getattr(t, k) for k, _ in t._fields_}

    def save(self):
        """Checkpoint of the state after the last completed iteration (bytes)."""
        n = self.lib.smc_state_bytes(self.ctx)
        buf = ctypes.create_string_buffer(n)
        self._check(self.lib.smc_save(self.ctx, buf, n), "smc_save")
        return buf.raw

    def load(self, image):
        """Restore a checkpoint from save() of a sampler built the same way."""
        buf = ctypes.create_string_buffer(bytes(image), len(image))
        self._check(self.lib.smc_load(self.ctx, buf, len(image)), "smc_load")

    def set_params(self, L, eps):
        self._check(self.lib.smc_set_params(self.ctx, float(L), float(eps)), "smc_set_params")

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.smc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_HIP = None


def _memcpy_d2d(dst, src, nbytes, stream):
    """hipMemcpyAsync device-to-device on the sampler's stream, then wait."""
    global _HIP
    if _HIP is None:
        _HIP = ctypes.CDLL("libamdhip64.so")
        _HIP.hipMemcpyAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                        ctypes.c_int, ctypes.c_void_p]
        _HIP.hipMemcpyAsync.restype = ctypes.c_int
        _HIP.hipStreamSynchronize.argtypes = [ctypes.c_void_p]
        _HIP.hipStreamSynchronize.restype = ctypes.c_int
    h = _stream_handle(stream)
    if _HIP.hipMemcpyAsync(ctypes.c_void_p(dst), ctypes.c_void_p(src), nbytes, 3, h) != 0:
        raise SmcError(SMC_EDEVICE, "hipMemcpyAsync")
    if _HIP.hipStreamSynchronize(h) != 0:
        raise SmcError(SMC_EDEVICE, "hipStreamSynchronize")


def resample_indices(w, u, scheme="systematic", stream=None):
    """Stateless resampling (see resample_indices in include/chees_smc.h)."""
    torch = _torch()
    lib = load()
    J = int(w.numel())
    if w.dtype != torch.float64 or u.dtype != torch.float64 or not (w.is_cuda and u.is_cuda):
        raise ValueError("w and u: float64 device tensors")
    need = 1 if scheme == "systematic" else J
    if u.numel() < need:
        raise ValueError(f"u needs {need} values")
    anc = torch.empty(J, dtype=torch.int32, device=w.device)
    nb = lib.resample_workspace_bytes(J)
    if nb == 0:
        raise SmcError(SMC_EINVAL, "J out of range")
    ws = torch.empty(nb, dtype=torch.uint8, device=w.device)
    rc = lib.resample_indices(_ptr(w), J, _ptr(u), RESAMPLING[scheme], _ptr(anc), _ptr(ws), nb,
                              _stream_handle(stream))
    if rc != SMC_OK:
        raise SmcError(rc, "resample_indices")
    return anc


def resample_indices_noalloc(w, u, anc, scheme="systematic", stream=None):
    """Stateless resampling into the caller's int32 device tensor `anc` with
    the library's static scratch: no device allocation by this call (see
    resample_indices_noalloc in include/chees_smc.h)."""
    torch = _torch()
    lib = load()
    J = int(w.numel())
    if w.dtype != torch.float64 or u.dtype != torch.float64 or not (w.is_cuda and u.is_cuda):
        raise ValueError("w and u: float64 device tensors")
    if anc.dtype != torch.int32 or not anc.is_cuda or anc.numel() < J:
        raise ValueError(f"anc: int32 device tensor of at least {J} values")
    need = 1 if scheme == "systematic" else J
    if u.numel() < need:
        raise ValueError(f"u needs {need} values")
    rc = lib.resample_indices_noalloc(_ptr(w), J, _ptr(u), RESAMPLING[scheme], _ptr(anc),
                                      _stream_handle(stream))
    if rc != SMC_OK:
        raise SmcError(rc, "resample_indices_noalloc")
    return anc


def initial_step_size(N, d):
    """A Fisher-scale starting step size d^(-1/4) / sqrt(1 + N/4)."""
    return float(d) ** -0.25 / math.sqrt(1.0 + N / 4.0)
