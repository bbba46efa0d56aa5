"""Affine-coupling flow preconditioner for the SMC/ChEES-HMC sampler: FP64 oracle.

TEST INFRASTRUCTURE ONLY (like the rest of oracle/): tests, the smoke check
and the benchmark's CPU leg may call it; the device library never does.

The paper has no flow; this is the preconditioned form of the sampler.  Its
exactness rests on the change-of-variables L-kernel of Sec. III-A: the
leapfrog map in the latent space is a volume-preserving bijection for any
position-only force, and the latent target below is the exact pushforward, so
the weight increment -Delta H_z is exact whatever the flow.

Flow T: z -> theta (fixed within an SMC iteration):
  x = z;  for l = 0 .. L-1 (affine coupling l):
      C_l / T_l = conditioning / transformed halves (even l: transform the
      first floor(d/2) coordinates given the rest; odd l: the other way round)
      h1 = tanh(W1 x_C + b1);  h2 = tanh(W2 h1 + b2);  o = W3 h2 + b3
      s = tanh(o[:d_T]);  t = o[d_T:]
      x_T <- x_T * exp(s) + t;         log|det| += sum s
  theta = m + L u,  u_c = x_q(c);      log|det| += sum_c log L_cc
  (q: even coordinates of theta first, then the odd ones)
Latent target: log pi_z(z) = log pi(T(z)) + log|det J_T(z)|.

Per iteration (readings, all build choices): m and L standardise the weighted
pre-move population: m its weighted mean, L the Cholesky factor of its
weighted covariance shrunk toward 1e-3 I as n/(n + 5) C + 1e-3 5/(n + 5) I
(n the effective sample size; the dense counterpart of oracle.smc.diag_mass),
so that the identity couplings give HMC with the dense mass M^-1 = L L^T.
The fit runs only on iterations that did not resample.
The inverse base map uses L^-1.  m, L and L^-1 are held in binary32 as on the
device, the log-determinant sum_c log L_cc in binary32 from the binary64
factor.  The couplings are warm-started and
trained for a few Adam steps on the weighted maximum-likelihood objective
  l(phi) = sum_j W_j [ log N(T^-1(theta_j); 0, I) + log|det J_{T^-1}(theta_j)| ]
(ascent), W the normalised weights.  A zero last layer (W3 = 0, b3 = 0) makes
every coupling the identity.  Moves use the weights rounded to bfloat16.
"""

import math

import numpy as np


def halves(d):
    da = d // 2
    return np.arange(da), np.arange(da, d)


def interleave(d):
    """Position q(c) of coordinate c of theta in the coupling state x: the even
    coordinates first, then the odd ones, so that the contiguous halves of x
    split neighbouring coordinates of theta (coupling layers then condition
    each coordinate on its neighbours)."""
    c = np.arange(d)
    ne = (d + 1) // 2
    return np.where(c % 2 == 0, c // 2, ne + c // 2)


def layer_sets(l, d):
    A, B = halves(d)
    return (A, B) if l % 2 == 0 else (B, A)   # (transformed, conditioning)


def init_params(d, layers, width, rng):
    """Coupling parameters: W1, W2 ~ N(0, 1/fan_in), biases 0, W3 = b3 = 0."""
    ps = []
    for l in range(layers):
        T, C = layer_sets(l, d)
        ps.append(dict(
            W1=rng.standard_normal((width, len(C))) / math.sqrt(max(len(C), 1)),
            b1=np.zeros(width),
            W2=rng.standard_normal((width, width)) / math.sqrt(width),
            b2=np.zeros(width),
            W3=np.zeros((2 * len(T), width)), b3=np.zeros(2 * len(T))))
    return ps


def bf16_params(ps):
    from .smc import bf16_round
    return [{k: bf16_round(v) for k, v in p.items()} for p in ps]


def _mlp(p, xc):
    h1 = np.tanh(xc @ p["W1"].T + p["b1"])
    h2 = np.tanh(h1 @ p["W2"].T + p["b2"])
    o = h2 @ p["W3"].T + p["b3"]
    return h1, h2, o


class Base:
    """Affine base map theta = m + L u of the flow: m, L, L^-1 and
    log|det L| (see the module docstring for the binary32 convention)."""

    def __init__(self, m, L, Linv=None, logdet=None):
        self.m = np.asarray(m, dtype=np.float64)
        self.L = np.asarray(L, dtype=np.float64)
        self.Linv = np.linalg.inv(self.L) if Linv is None else np.asarray(Linv, dtype=np.float64)
        self.logdet = float(np.sum(np.log(np.diag(self.L)))) if logdet is None else float(logdet)

    @staticmethod
    def diagonal(m, a):
        a = np.asarray(a, dtype=np.float64)
        return Base(m, np.diag(np.exp(a)), np.diag(np.exp(-a)), float(np.sum(a)))


def forward(ps, base, z):
    """theta = T(z) and log|det J_T(z)| for a population z (J, d)."""
    z = np.atleast_2d(np.asarray(z, dtype=np.float64))
    x = z.copy()
    ld = np.zeros(len(x))
    d = x.shape[1]
    for l, p in enumerate(ps):
        T, C = layer_sets(l, d)
        _, _, o = _mlp(p, x[:, C])
        s = np.tanh(o[:, :len(T)])
        t = o[:, len(T):]
        x[:, T] = x[:, T] * np.exp(s) + t
        ld += s.sum(1)
    return base.m + x[:, interleave(d)] @ base.L.T, ld + base.logdet


def inverse(ps, base, theta):
    """z = T^-1(theta) and log|det J_{T^-1}(theta)| = -log|det J_T(z)|."""
    theta = np.atleast_2d(np.asarray(theta, dtype=np.float64))
    d = theta.shape[1]
    x = np.empty_like(theta)
    x[:, interleave(d)] = (theta - base.m) @ base.Linv.T
    ld = np.full(len(x), -base.logdet)
    for l in reversed(range(len(ps))):
        p = ps[l]
        T, C = layer_sets(l, d)
        _, _, o = _mlp(p, x[:, C])
        s = np.tanh(o[:, :len(T)])
        t = o[:, len(T):]
        x[:, T] = (x[:, T] - t) * np.exp(-s)
        ld -= s.sum(1)
    return x, ld


def latent_grad(ps, base, z, g_theta):
    """grad_z log pi_z(z) = J_T(z)^T g_theta + grad_z log|det J_T(z)| by reverse
    accumulation through the forward map (g_theta = grad log pi at T(z))."""
    z = np.atleast_2d(np.asarray(z, dtype=np.float64))
    d = z.shape[1]
    x = z.copy()
    tape = []
    for l, p in enumerate(ps):
        T, C = layer_sets(l, d)
        h1, h2, o = _mlp(p, x[:, C])
        s = np.tanh(o[:, :len(T)])
        t = o[:, len(T):]
        xT = x[:, T].copy()
        tape.append((T, C, h1, h2, s, xT))
        x[:, T] = xT * np.exp(s) + t
    gx = np.empty((len(z), d))
    gx[:, interleave(d)] = np.asarray(g_theta, dtype=np.float64) @ base.L   # cotangent of x
    for l in reversed(range(len(ps))):
        p = ps[l]
        T, C, h1, h2, s, xT = tape[l]
        gyT = gx[:, T]
        es = np.exp(s)
        gs = gyT * xT * es + 1.0                      # + d(sum s)/ds
        go = np.concatenate([gs * (1.0 - s * s), gyT], axis=1)
        gpre2 = (go @ p["W3"]) * (1.0 - h2 * h2)
        gpre1 = (gpre2 @ p["W2"]) * (1.0 - h1 * h1)
        gxC = gx[:, C] + gpre1 @ p["W1"]
        gx = gx.copy()
        gx[:, T] = gyT * es
        gx[:, C] = gxC
    return gx


def objective_and_grad(ps, base, theta, W):
    """l(phi) = sum_j W_j [log N(z_j; 0, I) + log|det J_{T^-1}(theta_j)|] with
    z = T^-1(theta), and its gradient with respect to every coupling parameter
    (reverse accumulation through the inverse map)."""
    theta = np.atleast_2d(np.asarray(theta, dtype=np.float64))
    J, d = theta.shape
    x = np.empty_like(theta)
    x[:, interleave(d)] = (theta - base.m) @ base.Linv.T
    ld = np.full(J, -base.logdet)
    tape = {}
    for l in reversed(range(len(ps))):
        p = ps[l]
        T, C = layer_sets(l, d)
        h1, h2, o = _mlp(p, x[:, C])
        s = np.tanh(o[:, :len(T)])
        t = o[:, len(T):]
        xT = (x[:, T] - t) * np.exp(-s)
        tape[l] = (T, C, x[:, C].copy(), h1, h2, s, xT)
        x[:, T] = xT
        ld -= s.sum(1)
    z = x
    f = -0.5 * np.sum(z * z, 1) - 0.5 * d * math.log(2 * math.pi) + ld
    obj = float(W @ f)
    gx = -z * W[:, None]                              # cotangent of z (weighted)
    grads = [None] * len(ps)
    for l in range(len(ps)):                          # reverse of the inverse order
        p = ps[l]
        T, C, xC, h1, h2, s, xT = tape[l]
        gxT = gx[:, T]
        es = np.exp(-s)
        gyT = gxT * es
        gt = -gxT * es
        gs = -gxT * xT - W[:, None]                   # - d(sum s)/ds, weighted
        go = np.concatenate([gs * (1.0 - s * s), gt], axis=1)
        gpre2 = (go @ p["W3"]) * (1.0 - h2 * h2)
        gpre1 = (gpre2 @ p["W2"]) * (1.0 - h1 * h1)
        grads[l] = dict(W3=go.T @ h2, b3=go.sum(0), W2=gpre2.T @ h1, b2=gpre2.sum(0),
                        W1=gpre1.T @ xC, b1=gpre1.sum(0))
        gx = gx.copy()
        gx[:, T] = gyT
        gx[:, C] = gx[:, C] + gpre1 @ p["W1"]
    return obj, grads


class FlowAdam:
    """Adam ascent (Kingma and Ba) on every coupling parameter."""

    def __init__(self, lr, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.t = 0
        self.mom = None

    def ascend(self, ps, grads):
        if self.mom is None:
            self.mom = [{k: (np.zeros_like(v), np.zeros_like(v)) for k, v in p.items()} for p in ps]
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        out = []
        for p, g, mm in zip(ps, grads, self.mom):
            q = {}
            for k in p:
                m1, v1 = mm[k]
                m1 = self.b1 * m1 + (1 - self.b1) * g[k]
                v1 = self.b2 * v1 + (1 - self.b2) * g[k] * g[k]
                mm[k] = (m1, v1)
                q[k] = p[k] + self.lr * (m1 / c1) / (np.sqrt(v1 / c2) + self.eps)
            out.append(q)
        return out


def philox_init(seed, d, layers, width):
    """Default initial couplings drawn from the Philox streams (the device
    draws the same numbers): W1 of layer l is row u = 0..width-1 of
    normals(seed, width rows, iteration 100 + 2l, stream FLOW) / sqrt(fan_in),
    W2 the same with iteration 101 + 2l; biases, W3 and b3 are zero."""
    from . import philox
    ps = []
    for l in range(layers):
        T, C = layer_sets(l, d)
        dc = max(len(C), 1)
        W1 = philox.normals_np(seed, width, 100 + 2 * l, philox.STREAM_FLOW, len(C)) / math.sqrt(dc)
        W2 = philox.normals_np(seed, width, 101 + 2 * l, philox.STREAM_FLOW, width) / math.sqrt(width)
        ps.append(dict(W1=W1, b1=np.zeros(width), W2=W2, b2=np.zeros(width),
                       W3=np.zeros((2 * len(T), width)), b3=np.zeros(2 * len(T))))
    return ps


def flatten(ps, m=None, a=None):
    """Flat parameter vector: per layer W1 (width x d_C, row-major), b1, W2,
    b2, W3 (2 d_T x width), b3 (then two more vectors if given)."""
    parts = []
    for p in ps:
        for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
            parts.append(np.ravel(p[k]))
    if m is not None:
        parts += [np.ravel(m), np.ravel(a)]
    return np.concatenate(parts)


def unflatten(v, d, layers, width):
    v = np.asarray(v, dtype=np.float64)
    ps, o = [], 0
    for l in range(layers):
        T, C = layer_sets(l, d)
        shapes = dict(W1=(width, len(C)), b1=(width,), W2=(width, width), b2=(width,),
                      W3=(2 * len(T), width), b3=(2 * len(T),))
        p = {}
        for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
            n = int(np.prod(shapes[k]))
            p[k] = v[o:o + n].reshape(shapes[k])
            o += n
        ps.append(p)
    rest = v[o:]
    if len(rest) == 2 * d:
        return ps, rest[:d], rest[d:]
    return ps, None, None


def standardise(theta, logw, n_eff):
    """Base of the flow from the weighted population: m = weighted mean,
    L = Cholesky factor of n/(n+5) C + 1e-3 5/(n+5) I with C the weighted
    covariance (two passes, binary64); m, L, L^-1 held in binary32."""
    from .smc import normalise
    W = normalise(logw)
    m64 = W @ theta
    dev = theta - m64
    C = (dev * W[:, None]).T @ dev
    S = (n_eff / (n_eff + 5.0)) * C + 1e-3 * (5.0 / (n_eff + 5.0)) * np.eye(theta.shape[1])
    L64 = np.linalg.cholesky(S)
    Li64 = np.linalg.inv(L64)
    f32 = lambda v: np.asarray(v).astype(np.float32).astype(np.float64)
    return Base(f32(m64), f32(L64), f32(Li64), float(np.float32(np.sum(np.log(np.diag(L64))))))


def leapfrog_latent(target, ps, base, z, p, gz, eps, n_steps, traj_grad=None):
    """Leapfrog in the latent space (unit mass) on log pi_z, n_steps[j] steps
    for particle j, the latent gradient cached between steps.  Each step:
    p += eps/2 gz;  z += eps p;  theta = T(z);  gz = J_T^T grad log pi(theta)
    + grad log|det|;  p += eps/2 gz.  Returns z', p', gz', theta', grad_theta',
    log pi(theta') (exact), log|det J_T(z')|."""
    z = np.array(z, dtype=np.float64)
    p = np.array(p, dtype=np.float64)
    gz = np.array(gz, dtype=np.float64)
    n_steps = np.asarray(n_steps)
    J, d = z.shape
    theta, ld = forward(ps, base, z)
    gth = np.full((J, d), np.nan)
    for s in range(int(n_steps.max(initial=0))):
        act = n_steps > s
        p[act] += 0.5 * eps * gz[act]
        z[act] += eps * p[act]
        th, l1 = forward(ps, base, z[act])
        theta[act], ld[act] = th, l1
        if traj_grad is None:
            _, g = target.log_and_grad(th)
        else:
            g = traj_grad(th)
        gth[act] = g
        gz[act] = latent_grad(ps, base, z[act], g)
        p[act] += 0.5 * eps * gz[act]
    lp, _ = target.log_and_grad(theta)
    return z, p, gz, theta, gth, lp, ld
