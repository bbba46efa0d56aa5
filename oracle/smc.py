"""Plain FP64 CPU oracle of SMC with a ChEES-HMC proposal.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import or call this module.  It shares no code with the
device library and never imports it.  It is slow on purpose: every step is the
definition from the paper written out in binary64, with numpy library
primitives (matrix products, exp/log, cumulative sums) as the only building
blocks and no blocking, fusion or reordering.

Paper: Millard, Murphy, Frisch, Maskell, "Incorporating the ChEES Criterion into
Sequential Monte Carlo Samplers" (arXiv 2504.02627).  Citations below name the
section and the equation/algorithm label of that paper:

  Sec. II       problem statement pi(theta) = p(x|theta) q0(theta)
  Sec. II-A     Hamiltonian (eq. HMC_mh), leapfrog (eqs. LF_p1/2, LF_theta,
                LF_p; Alg. LF_example), acceptance (eq. HMC_accept_reject)
  Sec. II       Metropolis--Hastings rule (eqs. mh_ratio, mh_ratio_rn)
  Sec. II-C     ChEES criterion, weighted gradient, Alg. smc_ChEES
  Sec. III      SMC sampler: eqs. init_sample, init_weights, proposal,
                l_weights, ess_smc, normalise_smc2, realised_estimates;
                Alg. smc_BNN; resampling rule J_eff < J/2, reset to 1/J
  Sec. III-A    momentum change-of-variables L-kernel (eqs. proposal_momentum,
                l-kernel_momentum); no accept/reject in SMC-ChEES
  Sec. III-B    per-particle jitter; III-B-1 jitter generators (eq. halton, ...)
  Sec. V        gradient-count convention: one gradient before the leapfrog
                loop plus one per leapfrog step

Readings of passages that are silent, garbled or ambiguous are listed in the
docstring of the function that takes them.
"""

import math
from bisect import bisect_right

import numpy as np
from scipy.special import expit

from . import philox

LOG_2PI = math.log(2.0 * math.pi)


# ===========================================================================
# Targets: log pi(theta) and its gradient for a population theta (J, d)
# ===========================================================================

def bf16_round(x):
    """Round to bfloat16 (8-bit significand), to nearest, ties to even, after
    rounding to binary32: the conversion the precision form applies to its
    MFMA operands.  Returned as float64.  NaN stays NaN."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + np.uint64(0x7FFF) + ((u >> np.uint64(16)) & np.uint64(1))) >> np.uint64(16)) << np.uint64(16)
    r = (u & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, r)


class LogisticRegression:
    """Bayesian logistic regression, Sec. IV (German Credit model):
    y_n ~ Bernoulli(sigmoid(theta^T x_n)), prior q0 = N(0, prior_var I).

    pi(theta) = p(y | X, theta) q0(theta) as in the problem statement of Sec. II,
    so log pi includes the prior's normalising constant and the evidence is p(y|X).
    Reading: no intercept column (the workloads list d features only).
    """

    def __init__(self, X, y, prior_var=1.0):
        self.X = np.asarray(X, dtype=np.float64)
        self.y = np.asarray(y, dtype=np.float64)
        self.prior_var = float(prior_var)
        self.dim = self.X.shape[1]

    def loglik(self, theta):
        """sum_n [ y_n z_n - log(1 + e^{z_n}) ],  z = X theta."""
        Z = np.atleast_2d(theta) @ self.X.T
        return np.sum(self.y * Z - np.logaddexp(0.0, Z), axis=1)

    def log_prior(self, theta):
        theta = np.atleast_2d(theta)
        return (-0.5 * np.sum(theta * theta, axis=1) / self.prior_var
                - 0.5 * self.dim * math.log(2.0 * math.pi * self.prior_var))

    def log_and_grad(self, theta):
        """log pi and grad log pi = X^T (y - sigmoid(X theta)) - theta / prior_var."""
        theta = np.atleast_2d(theta)
        Z = theta @ self.X.T
        loglik = np.sum(self.y * Z - np.logaddexp(0.0, Z), axis=1)
        R = self.y - expit(Z)
        grad = R @ self.X - theta / self.prior_var
        return loglik + self.log_prior(theta), grad

    def grad_bf16(self, theta):
        """Trajectory gradient of the precision form: theta, X and the residual
        R = y - sigmoid(X theta) rounded to bfloat16 (bf16_round) before the two
        products, which are then exact and summed in binary64; the prior term
        uses theta unrounded.  Only the proposal uses it: energies stay exact."""
        theta = np.atleast_2d(theta)
        Xb = bf16_round(self.X)
        Z = bf16_round(theta) @ Xb.T
        R = bf16_round(self.y - expit(Z))
        return R @ Xb - theta / self.prior_var


class Gaussian:
    """N(mu, Sigma) target (Sec. IV, Gaussian and ill-conditioned Gaussian).

    log pi is the normalised density plus `log_scale`, so that the evidence of
    pi is exactly exp(log_scale).
    """

    def __init__(self, mu, cov=None, log_scale=0.0, prec=None):
        """Either the covariance or the precision P = Sigma^{-1} (the same
        density; given P, log det Sigma = -log det P)."""
        self.mu = np.asarray(mu, dtype=np.float64)
        if prec is not None:
            self.prec = np.atleast_2d(np.asarray(prec, dtype=np.float64))
            self.cov = np.linalg.inv(self.prec)
            sign, logdet_p = np.linalg.slogdet(self.prec)
            logdet = -logdet_p
        else:
            self.cov = np.atleast_2d(np.asarray(cov, dtype=np.float64))
            self.prec = np.linalg.inv(self.cov)
            sign, logdet = np.linalg.slogdet(self.cov)
        assert sign > 0
        self.dim = self.mu.shape[0]
        self.log_norm = -0.5 * (self.dim * LOG_2PI + logdet) + log_scale

    def log_and_grad(self, theta):
        diff = np.atleast_2d(theta) - self.mu
        pd = diff @ self.prec
        return self.log_norm - 0.5 * np.sum(pd * diff, axis=1), -pd


class Banana:
    """Rosenbrock (banana) target of Sec. IV, D = 2:
    theta_1 ~ N(0, s1^2),  theta_2 | theta_1 ~ N(b (theta_1^2 - c), 1).

    Reading: "N(0, 10)" is taken as standard deviation 10 (variance 100), which
    is what makes the offset c = 100 centre theta_2 (then E[theta_2] = 0).
    """

    def __init__(self, s1=10.0, b=0.03, c=100.0):
        self.s1, self.b, self.c = float(s1), float(b), float(c)
        self.dim = 2

    def log_and_grad(self, theta):
        theta = np.atleast_2d(theta)
        t1, t2 = theta[:, 0], theta[:, 1]
        m2 = self.b * (t1 * t1 - self.c)
        r2 = t2 - m2
        logp = (-0.5 * (t1 / self.s1) ** 2 - math.log(self.s1) - 0.5 * r2 * r2 - LOG_2PI)
        g = np.empty_like(theta)
        g[:, 0] = -t1 / self.s1 ** 2 + r2 * 2.0 * self.b * t1
        g[:, 1] = -r2
        return logp, g


class Funnel:
    """Neal's funnel (named as future work in Sec. VI), d >= 2,
    theta = (v, x_1..x_{d-1}): v ~ N(0, scale^2), x_i | v ~ N(0, e^v)."""

    def __init__(self, dim, scale=3.0, log_scale=0.0):
        self.dim, self.scale, self.log_scale = int(dim), float(scale), float(log_scale)

    def log_and_grad(self, theta):
        theta = np.atleast_2d(theta)
        v, x = theta[:, 0], theta[:, 1:]
        n = self.dim - 1
        x2 = np.sum(x * x, axis=1)
        ev = np.exp(-v)
        logp = (-0.5 * (v / self.scale) ** 2 - math.log(self.scale) - 0.5 * LOG_2PI
                - 0.5 * ev * x2 - 0.5 * n * v - 0.5 * n * LOG_2PI + self.log_scale)
        g = np.empty_like(theta)
        g[:, 0] = -v / self.scale ** 2 - 0.5 * n + 0.5 * ev * x2
        g[:, 1:] = -x * ev[:, None]
        return logp, g


# ===========================================================================
# Hamiltonian dynamics (Sec. II-A)
# ===========================================================================

def kinetic(p, minv=None):
    """Kinetic energy 1/2 p^T M^{-1} p for a diagonal mass matrix M = diag(1/minv).

    Reading: the printed Hamiltonian (Sec. II-A, second line under eq. HMC_mh)
    shows -1/2 ||p||^2; the sign is taken as +, as the Gaussian momentum density
    N(0, M) requires.  M = I in the paper; `minv` is the optional diagonal.
    """
    p = np.atleast_2d(p)
    if minv is None:
        return 0.5 * np.sum(p * p, axis=1)
    return 0.5 * np.sum(p * p * minv, axis=1)


def hamiltonian(logpi, p, minv=None):
    """H(theta, p) = -log pi(theta) + 1/2 p^T M^{-1} p  (Sec. II-A, eq. HMC_mh)."""
    return -np.asarray(logpi, dtype=np.float64) + kinetic(p, minv)


def leapfrog(target, theta, p, grad, eps, n_steps, minv=None, traj_grad=None):
    """Leapfrog integrator (eqs. LF_p1/2, LF_theta, LF_p; Alg. LF_example) run
    for n_steps[j] steps on particle j, with the gradient cached between steps.

    Each step:  p += eps/2 grad;  theta += eps M^{-1} p;  grad = grad log pi(theta);
                p += eps/2 grad.
    Reading of the gradient count (Sec. V): one evaluation per step plus one
    before the loop, which the caller already holds in `grad`.

    traj_grad: optional gradient function used for the moves (the precision
    form); log pi' is then evaluated exactly at the end point.
    Returns (theta', p', grad', logpi', n_grad) where n_grad[j] = n_steps[j].
    """
    theta = np.array(theta, dtype=np.float64)
    p = np.array(p, dtype=np.float64)
    grad = np.array(grad, dtype=np.float64)
    n_steps = np.asarray(n_steps)
    J, d = theta.shape
    mv = np.ones(d) if minv is None else np.asarray(minv, dtype=np.float64)
    logpi = np.full(J, np.nan)
    for s in range(int(n_steps.max(initial=0))):
        act = n_steps > s
        p[act] += 0.5 * eps * grad[act]
        theta[act] += eps * mv * p[act]
        if traj_grad is None:
            lp, g = target.log_and_grad(theta[act])
            logpi[act] = lp
        else:
            g = traj_grad(theta[act])
        grad[act] = g
        p[act] += 0.5 * eps * grad[act]
    redo = ~(n_steps > 0) if traj_grad is None else np.ones(J, dtype=bool)
    if np.any(redo):
        logpi[redo], _ = target.log_and_grad(theta[redo])
    return theta, p, grad, logpi, n_steps.copy()


def delta_h(logpi0, p0, logpi1, p1, minv=None):
    """Energy error Delta H = H(theta', p') - H(theta, p); non-finite -> +inf."""
    dh = hamiltonian(logpi1, p1, minv) - hamiltonian(logpi0, p0, minv)
    return np.where(np.isfinite(dh), dh, np.inf)


def accept_prob(dh):
    """alpha = min(1, exp(-Delta H))  (eq. HMC_accept_reject); +inf -> 0."""
    return np.minimum(1.0, np.exp(-dh))


# ===========================================================================
# Jitter (Sec. III-B-1) and step counts (Alg. smc_ChEES)
# ===========================================================================

def radical_inverse(i, base):
    """phi_b(i) = sum_d digit_d(i) b^{-d-1}  (eq. halton), the digits of i in base b
    mirrored about the radix point.  Computed exactly as the integer ratio
    R / b^m (m = number of digits), followed by one correctly rounded division."""
    i = int(i)
    assert i >= 0
    r, bm = 0, 1
    while i > 0:
        i, dig = divmod(i, base)
        r = r * base + dig
        bm *= base
    return r / bm  # Python int / int is correctly rounded to binary64


def halton_1d(k, J):
    """1-d Halton jitter of Sec. III-B-1: J*K numbers from base 2.

    Reading: the flattening order is not stated; iteration-major index
    (k-1) J + j with j = 1..J, k = 1..K (index starts at 1 so that h > 0).
    """
    return np.array([radical_inverse((k - 1) * J + j, 2) for j in range(1, J + 1)])


def nth_prime(n):
    """n-th prime, n >= 1, by trial division."""
    count, c = 0, 1
    while count < n:
        c += 1
        if all(c % q for q in range(2, int(c ** 0.5) + 1)):
            count += 1
    return c


def halton_nd(k, J):
    """N-d Halton jitter (eq. halton): h_jk = phi_{P_k}(j), j = 1..J.
    Reading: "base-k" is taken as the k-th prime (base 1 does not exist)."""
    b = nth_prime(k)
    return np.array([radical_inverse(j, b) for j in range(1, J + 1)])


def reversed_column(k, K):
    """Column of iteration k under the inverse schemes: the J x K matrix is
    taken in reverse order of k (Sec. III-B-1, "sorted in reverse order of
    k").  Reading: column K + 1 - k for k <= K; a run longer than K starts
    over from column K (K - ((k - 1) mod K))."""
    return K - (k - 1) % K


def halton_nd_inverse(k, K, J):
    """N-d inverse Halton: the N-d Halton matrix with its columns reversed."""
    return halton_nd(reversed_column(k, K), J)


def primes_nd(k, J):
    """N-d primes jitter (eq. primes): h_jk = j sqrt(P_k) mod 1, j = 1..J, in
    binary64 (one correctly rounded square root, one product, exact fraction).
    """
    r = math.sqrt(float(nth_prime(k)))
    x = np.arange(1, J + 1, dtype=np.float64) * r
    return x - np.floor(x)


def primes_nd_inverse(k, K, J):
    """N-d inverse primes: the N-d primes matrix with its columns reversed."""
    return primes_nd(reversed_column(k, K), J)


def golden_1d(k, K, J):
    """1-d golden-ratio jitter: h_jk = ((j - 1) K + k) (sqrt 5 - 1) / 2 mod 1,
    j = 1..J, in binary64."""
    g = (math.sqrt(5.0) - 1.0) / 2.0
    idx = np.arange(J, dtype=np.float64) * float(K) + float(k)
    x = idx * g
    return x - np.floor(x)


def uniform_jitter(seed, k, J, b=0):
    """Uniform jitter h_jk ~ U(0, 1): the Philox uniform of particle
    b J + j - 1 at iteration k on the jitter stream."""
    return np.array([philox.uniform(seed, b * J + j, k, philox.STREAM_JITTER) for j in range(J)])


def shuffle(seed, k, J, b=0):
    """The shuffle of column k of the equidistant schemes ("shuffled K times").

    Reading: a keyed pseudo-random permutation of {0, .., J-1}: a balanced
    Feistel network (Luby and Rackoff) of 4 rounds on 2 h bits, h the smallest
    half width with 4^h >= J, whose round r maps the right half R to word 0 of
    Philox block (R, 4 b + r, k, STREAM_SHUFFLE) masked to h bits, restricted
    to {0, .., J-1} by cycle walking (Black and Rogaway): apply the network
    until the value falls below J.  Returns pi with pi[j] the new position of
    particle j.
    """
    h = 1
    while 4 ** h < J:
        h += 1
    mask = (1 << h) - 1
    key = philox.seed_key(seed)

    def net(x):
        hi, lo = x >> h, x & mask
        for r in range(4):
            f = philox.philox4x32_10((lo, 4 * b + r, k, philox.STREAM_SHUFFLE), key)[0] & mask
            hi, lo = lo, hi ^ f
        return (hi << h) | lo

    pi = np.empty(J, dtype=np.int64)
    for j in range(J):
        y = net(j)
        while y >= J:
            y = net(y)
        pi[j] = y
    return pi


def equidistant(seed, k, J, b=0):
    """Equidistant jitter: the J points h = i / J, i = 1..J, shuffled per
    iteration: h_jk = (pi_k(j) + 1) / J."""
    return (shuffle(seed, k, J, b) + 1).astype(np.float64) / float(J)


def equidistant_offset(seed, k, J, b=0):
    """Offset equidistant jitter: the equidistant value plus a U(0, 0.1) draw,
    0.1 u with u the particle's uniform on the jitter stream."""
    return equidistant(seed, k, J, b) + 0.1 * uniform_jitter(seed, k, J, b)


# --- Sobol (eq. sobol) ---------------------------------------------------------

def joe_kuo_rows(dims):
    """The first `dims` rows of Joe and Kuo's direction-number table, as the
    scipy package ships it (the generator the paper names for its Sobol
    schemes): for each dimension the primitive polynomial as a bit mask with
    its leading and constant terms (1 for the first dimension) and the
    initial direction integers m_1..m_s (zero beyond the degree s)."""
    import os
    import scipy.stats
    z = np.load(os.path.join(os.path.dirname(scipy.stats.__file__), "_sobol_direction_numbers.npz"))
    return [(int(p), [int(v) for v in row]) for p, row in zip(z["poly"][:dims], z["vinit"][:dims])]


def sobol_direction_integers(poly, minit, nbits):
    """m_1..m_nbits of one dimension (Bratley and Fox; Joe and Kuo).

    For the primitive polynomial x^s + a_1 x^(s-1) + .. + a_(s-1) x + 1 the
    integers after the s given ones follow
        m_i = 2 a_1 m_(i-1) ^ 4 a_2 m_(i-2) ^ .. ^ 2^(s-1) a_(s-1) m_(i-s+1)
              ^ 2^s m_(i-s) ^ m_(i-s)            (^ is bitwise xor),
    and the direction number nu_i is m_i / 2^i.  A polynomial of degree 0
    (the first dimension) has m_i = 1 for all i: the van der Corput sequence.
    """
    s = poly.bit_length() - 1
    if s == 0:
        return [1] * nbits
    m = list(minit[:s])
    for i in range(s, nbits):          # m[i] is m_(i+1)
        v = m[i - s] ^ (m[i - s] << s)
        for t in range(1, s):
            if (poly >> (s - t)) & 1:  # a_t
                v ^= m[i - t] << t
        m.append(v)
    return m


def sobol_point(m, i, nbits):
    """x_i of one Sobol dimension (eq. sobol): the xor of the direction
    numbers nu_b over the binary digits b of i, as an exact binary fraction.

    Reading: eq. sobol writes the digits of i itself; the scipy generator the
    paper uses takes the digits of the Gray code i ^ (i >> 1), which lists
    the same points in each block of 2^m in another order.  The Gray-code
    digits are used, so that the sequence is the one the paper ran."""
    g = i ^ (i >> 1)
    x, b = 0, 0
    while g:
        if g & 1:
            x ^= m[b] << (nbits - 1 - b)
        g >>= 1
        b += 1
    return x / 2 ** nbits


def sobol_1d(k, J):
    """1-d Sobol jitter: J*K numbers from the first Sobol dimension.

    Reading: the printed definition points to eq. halton with k = 1, which
    has no base; taken as the first dimension of eq. sobol (nu_b = 2^-b),
    flattened like the 1-d Halton scheme, index (k-1) J + j, j = 1..J (the
    point 0 of the sequence is never used)."""
    m = [1] * 64
    return np.array([sobol_point(m, (k - 1) * J + j, 64) for j in range(1, J + 1)])


def sobol_nd(k, J, rows=None):
    """N-d Sobol jitter (eq. sobol): h_jk = x_j of Sobol dimension k,
    j = 1..J (the point 0 is skipped), direction numbers of Joe and Kuo."""
    poly, minit = (rows or joe_kuo_rows(k))[k - 1]
    m = sobol_direction_integers(poly, minit, 32)
    return np.array([sobol_point(m, j, 32) for j in range(1, J + 1)])


def sobol_nd_inverse(k, K, J, rows=None):
    """Inverse N-d Sobol: the N-d Sobol matrix with its columns reversed."""
    return sobol_nd(reversed_column(k, K), J, rows)


def step_counts(h, L, eps, n_max):
    """Jittered length l_j = h_j L and n_j = min(max(ceil(l_j / eps), 1), n_max)
    (Alg. smc_ChEES: l_m = h_m L_{m-1}, ceil(l_m / eps) leapfrog steps).

    The cap n_max is the maximum number of leapfrog steps the paper sets by hand
    (Sec. V); the lower clamp 1 keeps every particle moving.  Binary64, one
    multiply and one divide, so the device reproduces it bit for bit.
    """
    l = np.asarray(h, dtype=np.float64) * float(L)
    n = np.ceil(l / float(eps))
    n = np.minimum(np.maximum(n, 1.0), float(n_max))
    return l, n.astype(np.int64)


# ===========================================================================
# Weights (Sec. III)
# ===========================================================================

def log_sum_exp(logw):
    """(m, S, S2): m = max log w, S = sum exp(log w - m), S2 = sum exp(2 (log w - m))."""
    logw = np.asarray(logw, dtype=np.float64)
    finite = np.isfinite(logw)
    if not np.any(finite):
        return -np.inf, 0.0, 0.0
    m = np.max(logw[finite])
    e = np.where(finite, np.exp(logw - m), 0.0)
    return m, float(np.sum(e)), float(np.sum(e * e))


def normalise(logw):
    """Normalised weights (eq. normalise_smc2) from log-weights."""
    m, S, _ = log_sum_exp(logw)
    logw = np.asarray(logw, dtype=np.float64)
    return np.where(np.isfinite(logw), np.exp(logw - m), 0.0) / S


def ess(logw):
    """J_eff = 1 / sum_j wtilde_j^2  (eq. ess_smc) = S^2 / S2."""
    m, S, S2 = log_sum_exp(logw)
    return S * S / S2 if S > 0 else 0.0


def realised_mean_var(theta, logw):
    """Weighted mean and variance per dimension, eq. realised_estimates with
    f(theta) = theta and f(theta) = (theta - mean)^2."""
    w = normalise(logw)
    mean = w @ theta
    var = w @ (theta - mean) ** 2
    return mean, var


# ===========================================================================
# Resampling (Sec. III)
# ===========================================================================

QUANT_BITS = 40


def quantise_weights(e):
    """Fixed-point weights Q_j = floor(e_j 2^40) for e_j in [0, 1].

    Reading: the paper resamples "with probability wtilde".  Weights are taken
    at a resolution of 2^-40 of the largest weight so that the cumulative sum is
    exact integer arithmetic; a particle lighter than that is never chosen.
    """
    return [int(math.floor(float(v) * (1 << QUANT_BITS))) for v in e]


def systematic_from_quantised(Q, U):
    """Systematic resampling on integer weights Q (J values) with offset U in
    [0, 2^32): ancestor a_i = min{ j : C_j > (i + U/2^32) T / J }, i = 0..J-1,
    with C the inclusive cumulative sum and T = C_J, evaluated exactly.

    Systematic rather than the paper's multinomial: the paper names systematic
    schemes as the parallel-friendly choice (Sec. III) and the hot path uses it.
    """
    J = len(Q)
    C = []
    acc = 0
    for q in Q:
        acc += q
        C.append(acc)
    T = acc
    if T == 0:
        raise ValueError("all weights are zero")
    out = np.empty(J, dtype=np.int64)
    den = J << 32
    for i in range(J):
        t = (((i << 32) + U) * T) // den  # C_j > t  <=>  C_j * den > (i 2^32 + U) T
        out[i] = bisect_right(C, t)
    return out


def multinomial_from_quantised(Q, Us):
    """Multinomial resampling (the paper's choice, Sec. III): J independent draws,
    a_i = min{ j : C_j > (U_i / 2^32) T } with U_i in [0, 2^32)."""
    C = []
    acc = 0
    for q in Q:
        acc += q
        C.append(acc)
    T = acc
    if T == 0:
        raise ValueError("all weights are zero")
    return np.array([bisect_right(C, (int(u) * T) >> 32) for u in Us], dtype=np.int64)


def uniform_to_u32(u):
    """U = floor(u 2^32) for u in [0, 1): the offset used by the integer schemes."""
    v = int(math.floor(float(u) * 4294967296.0))
    return min(max(v, 0), 0xFFFFFFFF)


def resample_indices(w, u0, scheme="systematic"):
    """Stateless resampling from nonnegative weights w (any scale).

    e_j = w_j / max_k w_k (one correctly rounded division), then the integer
    schemes above.  `u0` is one uniform (systematic) or J uniforms (multinomial).
    """
    w = np.asarray(w, dtype=np.float64)
    mx = np.max(w)
    if not (mx > 0):
        raise ValueError("all weights are zero")
    Q = quantise_weights(w / mx)
    if scheme == "systematic":
        return systematic_from_quantised(Q, uniform_to_u32(u0))
    return multinomial_from_quantised(Q, [uniform_to_u32(u) for u in np.atleast_1d(u0)])


def resample_from_logw(logw, u0, scheme="systematic"):
    """Resampling from log-weights: e_j = exp(log w_j - max log w)."""
    logw = np.asarray(logw, dtype=np.float64)
    m, _, _ = log_sum_exp(logw)
    if not np.isfinite(m):
        raise ValueError("degenerate weights")
    e = np.where(np.isfinite(logw), np.exp(logw - m), 0.0)
    Q = quantise_weights(e)
    if scheme == "systematic":
        return systematic_from_quantised(Q, uniform_to_u32(u0))
    return multinomial_from_quantised(Q, [uniform_to_u32(u) for u in np.atleast_1d(u0)])


# ===========================================================================
# ChEES criterion and adaptation (Sec. II-C, Alg. smc_ChEES)
# ===========================================================================

def chees_statistics(theta_old, theta_new, p_new, l, alpha, minv=None):
    """Per-particle ChEES gradient terms and their alpha-weighted mean.

    theta_hat' = mean_c theta'^(c),  theta_hat = mean_c theta_{m-1}^(c)  (unweighted)
    a_c   = ||theta'^(c) - theta_hat'||^2 - ||theta_{m-1}^(c) - theta_hat||^2
    g_c   = l_c a_c (theta'^(c) - theta_hat')^T M^{-1} p'^(c)
    g_hat = sum_c alpha_c g_c / sum_c alpha_c
    ChEES = 1/4 mean_c a_c^2     (the criterion's sample estimate)

    Readings: the momentum in g_c is the final momentum p' (the derivative of
    ||theta(t) - theta_hat'||^2 along the trajectory is 2 (theta(t) - theta_hat')
    . M^{-1} p(t)); l_c is the particle's own uncapped jittered length.
    Returns dict with a, g, ghat, sum_alpha, chees.
    """
    theta_old = np.asarray(theta_old, dtype=np.float64)
    theta_new = np.asarray(theta_new, dtype=np.float64)
    p_new = np.asarray(p_new, dtype=np.float64)
    d = theta_new.shape[1]
    mv = np.ones(d) if minv is None else np.asarray(minv, dtype=np.float64)
    c_new = theta_new - theta_new.mean(axis=0)
    c_old = theta_old - theta_old.mean(axis=0)
    a = np.sum(c_new * c_new, axis=1) - np.sum(c_old * c_old, axis=1)
    g = np.asarray(l, dtype=np.float64) * a * np.sum(c_new * mv * p_new, axis=1)
    alpha = np.asarray(alpha, dtype=np.float64)
    sa = float(np.sum(alpha))
    ghat = float(np.sum(alpha * g) / sa) if sa > 0 else 0.0
    return {"a": a, "g": g, "ghat": ghat, "sum_alpha": sa, "chees": 0.25 * float(np.mean(a * a))}


class Adam:
    """Adam (Kingma and Ba, 2015) on one scalar, as an ascent step:
    t += 1; m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
    x += lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)."""

    def __init__(self, lr, b1, b2, eps):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = self.v = 0.0
        self.t = 0

    def ascend(self, x, g):
        self.t += 1
        self.m = self.b1 * self.m + (1.0 - self.b1) * g
        self.v = self.b2 * self.v + (1.0 - self.b2) * g * g
        mhat = self.m / (1.0 - self.b1 ** self.t)
        vhat = self.v / (1.0 - self.b2 ** self.t)
        return x + self.lr * mhat / (math.sqrt(vhat) + self.eps)


def harmonic_mean(alpha, floor=1e-20):
    """J / sum_j 1/max(alpha_j, floor)."""
    alpha = np.maximum(np.asarray(alpha, dtype=np.float64), floor)
    return len(alpha) / float(np.sum(1.0 / alpha))


# ===========================================================================
# The SMC sampler with the ChEES-HMC proposal (Alg. smc_BNN + Alg. smc_ChEES)
# ===========================================================================

DEFAULTS = dict(
    max_leapfrog=64, num_warmup=None, jitter="halton1d", mh_accept=False,
    resampling="systematic", step_size=0.1, traj_length=5.0, ess_frac=0.5,
    adam_lr=0.025, adam_b1=0.9, adam_b2=0.999, adam_eps=1e-8, avg_decay=0.9,
    adapt_step_size=False, target_accept=0.651, seed=0, prior_var=1.0, precision="f64",
    precond="none", flow_layers=4, flow_width=128, flow_train_steps=10, flow_lr=1e-3,
    flow_init=None, num_iterations=0,
)


def diag_mass(theta, logw, n_eff):
    """Diagonal inverse mass matrix from the weighted population (the
    diagonal-mass fallback of the preconditioned form; the paper itself uses
    M = I).  Reading: M^{-1} = diag(Var_W[theta]), the weighted population
    variance with W the normalised weights (eq. normalise_smc2), shrunk toward
    1e-3 as n/(n + 5) Var + 1e-3 * 5/(n + 5) with n the effective sample size
    of those weights (the regulariser of Stan's windowed adaptation), so that
    a collapsed population cannot give a zero mass.  Two passes in binary64;
    the result is held in binary32, as the device holds it."""
    W = normalise(logw)
    mean = W @ theta
    var = W @ ((theta - mean) ** 2)
    reg = (n_eff / (n_eff + 5.0)) * var + 1e-3 * (5.0 / (n_eff + 5.0))
    return reg.astype(np.float32).astype(np.float64)


class OracleSMC:
    """SMC sampler (Alg. smc_BNN) whose proposal is a ChEES-HMC trajectory
    (Alg. smc_ChEES), with the momentum change-of-variables L-kernel of Sec. III-A.

    Call order per iteration k = 1..K:  step(), then adapt().  Randomness comes
    from Philox streams (oracle.philox) unless injected.

    Readings (the paper is silent or ambiguous):
      * init: log w_j = log pi(theta_0^j) - log q0(theta_0^j) - log J; the extra
        -log J matches the 1/J reset after resampling and makes
        sum_j exp(log w_j) an estimate of the evidence (eq. init_weights).
      * evidence: log Z = C + LSE(log w), C accumulating LSE(log w) at every
        resampling (standard product estimator of the SMC framework, Sec. III).
      * SMC-ChEES has no accept/reject (Sec. III-A): log w += -Delta H, from the
        change-of-variables L-kernel, whose Jacobians cancel.  With
        mh_accept=True (Alg. smc_ChEES as MCMC inside SMC) the move is accepted
        iff u < alpha and the weight increment is 0 (pi-invariant kernel).
      * M_warmup defaults to K/2-style half of the run, passed in by the caller.
    """

    def __init__(self, target, num_particles, theta0=None, **params):
        P = dict(DEFAULTS)
        P.update(params)
        if P["num_warmup"] is None:
            raise ValueError("num_warmup is required")
        self.P = P
        self.target = target
        self.J = int(num_particles)
        self.d = target.dim
        self.prior_var = float(P["prior_var"])
        self.minv = None
        J, d = self.J, self.d
        # a1: theta_0 ~ q0 = N(0, prior_var I)  (eq. init_sample)
        if theta0 is None:
            theta0 = math.sqrt(self.prior_var) * philox.normals_np(P["seed"], J, 0, philox.STREAM_INIT, d)
        self.theta = np.array(theta0, dtype=np.float64).reshape(J, d)
        # precision form: BF16 trajectory gradients (target.grad_bf16), exact energies
        self.traj_grad = target.grad_bf16 if P["precision"] == "bf16" else None
        self.logpi, self.grad = target.log_and_grad(self.theta)
        if self.traj_grad is not None:
            self.grad = self.traj_grad(self.theta)
        logq0 = (-0.5 * np.sum(self.theta ** 2, axis=1) / self.prior_var
                 - 0.5 * d * math.log(2.0 * math.pi * self.prior_var))
        # eq. init_weights, with the -log J reading
        self.logw = self.logpi - logq0 - math.log(J)
        self.log_c = 0.0
        self.L = float(P["traj_length"])
        self.eps = float(P["step_size"])
        self.Lbar = 0.0
        self.adam_L = Adam(P["adam_lr"], P["adam_b1"], P["adam_b2"], P["adam_eps"])
        self.adam_eps = Adam(P["adam_lr"], P["adam_b1"], P["adam_b2"], P["adam_eps"])
        self.da_hbar, self.da_logbar = 0.0, 0.0      # dual averaging state
        self.da_mu = math.log(10.0 * self.eps)
        self.k = 0
        self.grad_evals = J  # the gradient at theta_0
        self.last = None
        if P["precond"] == "flow":
            from . import flow
            self.flow_ps = (flow.unflatten(P["flow_init"], d, P["flow_layers"], P["flow_width"])[0]
                            if P["flow_init"] is not None else
                            flow.philox_init(P["seed"], d, P["flow_layers"], P["flow_width"]))
            self.flow_adam = flow.FlowAdam(P["flow_lr"], P["adam_b1"], P["adam_b2"], P["adam_eps"])
            self.flow_base = None

    # ----- one SMC iteration -------------------------------------------------
    def jitter(self, k):
        kind = self.P["jitter"]
        if kind == "halton1d":
            return halton_1d(k, self.J)
        if kind == "none":
            return np.ones(self.J)
        if kind == "haltonNd":
            return halton_nd(k, self.J)
        K, seed = self.P["num_iterations"], self.P["seed"]
        if kind == "uniform":
            return uniform_jitter(seed, k, self.J)
        if kind == "haltonNd_inv":
            return halton_nd_inverse(k, K, self.J)
        if kind == "primes":
            return primes_nd(k, self.J)
        if kind == "primes_inv":
            return primes_nd_inverse(k, K, self.J)
        if kind == "golden":
            return golden_1d(k, K, self.J)
        if kind == "equidistant":
            return equidistant(seed, k, self.J)
        if kind == "equidistant_offset":
            return equidistant_offset(seed, k, self.J)
        if kind == "sobol1d":
            return sobol_1d(k, self.J)
        if kind == "sobolNd":
            return sobol_nd(k, self.J)
        if kind == "sobolNd_inv":
            return sobol_nd_inverse(k, K, self.J)
        raise ValueError(kind)

    def step(self, momenta=None, mh_uniforms=None, resample_u=None):
        """Alg. smc_BNN body for one k: normalise, ESS, maybe resample, move, reweight.

        momenta: (J, d) standard normals xi; the momentum is p = xi / sqrt(minv).
        """
        P, J, d = self.P, self.J, self.d
        self.k += 1
        k = self.k
        # a2: normalise and ESS (eqs. normalise_smc2, ess_smc)
        m, S, S2 = log_sum_exp(self.logw)
        if not (S > 0):
            raise FloatingPointError("degenerate weights")
        j_eff_before = S * S / S2
        resampled = j_eff_before < P["ess_frac"] * J
        ancestors = None
        if resampled:
            # a3: resample with probability wtilde, reset weights to 1/J (Sec. III)
            if P["resampling"] == "systematic":
                u0 = resample_u if resample_u is not None else philox.uniform(
                    P["seed"], 0, k, philox.STREAM_RESAMPLE)
            else:
                u0 = resample_u if resample_u is not None else philox.uniforms_np(
                    P["seed"], J, k, philox.STREAM_RESAMPLE)
            ancestors = resample_from_logw(self.logw, u0, P["resampling"])
            self.theta = self.theta[ancestors]
            self.grad = self.grad[ancestors]
            self.logpi = self.logpi[ancestors]
            self.log_c += m + math.log(S)
            self.logw = np.full(J, -math.log(J))
        if P["precond"] == "diag":
            self.minv = diag_mass(self.theta, self.logw, j_eff_before)
        flow_rec = None
        if P["precond"] == "flow":
            from . import flow
            base = flow.standardise(self.theta, self.logw, j_eff_before)
            W = normalise(self.logw)
            # reading: no fit on a resampled iteration (a resampled population
            # holds duplicates, onto which a maximum-likelihood fit collapses)
            for _ in range(0 if resampled or P["flow_layers"] == 0 else P["flow_train_steps"]):
                _, g_ = flow.objective_and_grad(self.flow_ps, base, self.theta, W)
                self.flow_ps = self.flow_adam.ascend(self.flow_ps, g_)
            self.flow_base = base
            psb = flow.bf16_params(self.flow_ps)
            z0, ldi = flow.inverse(psb, base, self.theta)
            ld0 = -ldi
            gz0 = flow.latent_grad(psb, base, z0, self.grad)
        # a4: momenta, jitter, step counts, initial energy
        if momenta is None:
            momenta = philox.normals_np(P["seed"], J, k, philox.STREAM_MOMENTUM, d)
        xi = np.asarray(momenta, dtype=np.float64).reshape(J, d)
        p0 = xi if self.minv is None else xi / np.sqrt(self.minv)
        h = self.jitter(k)
        l, n = step_counts(h, self.L, self.eps, P["max_leapfrog"])
        # a5: leapfrog trajectories
        if P["precond"] == "flow":
            # in the latent space of the flow, unit mass: log pi_z = log pi(T(z)) + log|det J_T|
            z1, p1, gz1, th1, g1, lp1, ld1 = flow.leapfrog_latent(
                self.target, psb, base, z0, p0, gz0, self.eps, n, traj_grad=self.traj_grad)
            ng = n.copy()
            flow_rec = dict(z0=z0, z1=z1, gz0=gz0, gz1=gz1, ld0=ld0, ld1=ld1, base=base,
                            params_bf16=psb)
        else:
            th1, p1, g1, lp1, ng = leapfrog(self.target, self.theta, p0, self.grad, self.eps, n,
                                            self.minv, traj_grad=self.traj_grad)
        self.grad_evals += int(np.sum(ng))
        # a6: energies, acceptance, weights
        if flow_rec is None:
            dh = delta_h(self.logpi, p0, lp1, p1, self.minv)
        else:
            dh = delta_h(self.logpi + ld0, p0, lp1 + ld1, p1)
        alpha = accept_prob(dh)
        # a7: ChEES statistics on the proposals (Alg. smc_ChEES); latent
        # coordinates under the flow
        if flow_rec is None:
            st = chees_statistics(self.theta, th1, p1, l, alpha, self.minv)
        else:
            st = chees_statistics(z0, z1, p1, l, alpha)
        theta_before, logpi_before = self.theta.copy(), self.logpi.copy()
        if P["mh_accept"]:
            u = mh_uniforms if mh_uniforms is not None else philox.uniforms_np(
                P["seed"], J, k, philox.STREAM_MH)
            acc = np.asarray(u, dtype=np.float64) < alpha
            self.theta = np.where(acc[:, None], th1, self.theta)
            self.grad = np.where(acc[:, None], g1, self.grad)
            self.logpi = np.where(acc, lp1, self.logpi)
        else:
            acc = np.ones(J, dtype=bool)
            self.theta, self.grad, self.logpi = th1, g1, lp1
            self.logw = np.where(np.isfinite(dh), self.logw - dh, -np.inf)
        m2, S2_, SS2 = log_sum_exp(self.logw)
        self.last = dict(
            k=k, resampled=bool(resampled), ancestors=ancestors, ess_before=j_eff_before,
            ess=(S2_ * S2_ / SS2) if S2_ > 0 else 0.0, h=h, l=l, n=n, p0=p0, p1=p1,
            dh=dh, alpha=alpha, accepted=acc, mean_accept=float(np.mean(alpha)),
            chees=st["chees"], ghat=st["ghat"], sum_alpha=st["sum_alpha"], a=st["a"], g=st["g"],
            grad_evals=int(np.sum(ng)), L=self.L, eps=self.eps,
            theta_before=theta_before, logpi_before=logpi_before, theta_prop=th1, logpi_prop=lp1,
            H0=hamiltonian(logpi_before, p0, self.minv), H1=hamiltonian(lp1, p1, self.minv),
            minv=None if self.minv is None else self.minv.copy(), flow=flow_rec,
        )
        if flow_rec is not None:
            self.last["H0"] = hamiltonian(logpi_before + flow_rec["ld0"], p0)
            self.last["H1"] = hamiltonian(lp1 + flow_rec["ld1"], p1)
        return self.last

    def adapt(self):
        """Warm-up adaptation after iteration m = k (Alg. smc_ChEES):
        m < M_w: Adam ascent on log L with g_hat (skipped if sum alpha = 0),
                 then Lbar <- 0.9 Lbar + 0.1 L;
        m = M_w: L <- Lbar.
        Optional step-size adaptation during warm-up (not in the paper, whose
        step size is fixed; dual averaging is named there as future work):
          adapt_step_size True / "adam": Adam on log eps toward a harmonic-mean
            acceptance of target_accept;
          "dual_averaging": Nesterov dual averaging as Hoffman and Gelman
            (2014) apply it to log eps (gamma 0.05, t0 10, kappa 0.75,
            mu = log(10 eps_0)), driven by the mean alpha of the particles at
            adaptation iteration m = k; eps <- exp(log eps_bar) at m = M_w."""
        P = self.P
        if self.last is None:
            raise RuntimeError("adapt before step")
        k, Mw = self.k, P["num_warmup"]
        if k < Mw:
            if self.last["sum_alpha"] > 0:
                self.L = math.exp(self.adam_L.ascend(math.log(self.L), self.last["ghat"]))
            self.Lbar = P["avg_decay"] * self.Lbar + (1.0 - P["avg_decay"]) * self.L
            mode = P["adapt_step_size"]
            if mode is True or mode == "adam" or mode == 1:
                hm = harmonic_mean(self.last["alpha"])
                self.eps = math.exp(self.adam_eps.ascend(math.log(self.eps), hm - P["target_accept"]))
            elif mode == "dual_averaging" or mode == 2:
                m = float(k)
                abar = float(np.mean(self.last["alpha"]))
                w = 1.0 / (m + 10.0)
                self.da_hbar = (1.0 - w) * self.da_hbar + w * (P["target_accept"] - abar)
                log_eps = self.da_mu - math.sqrt(m) / 0.05 * self.da_hbar
                mk = m ** -0.75
                self.da_logbar = mk * log_eps + (1.0 - mk) * self.da_logbar
                self.eps = math.exp(log_eps)
        elif k == Mw:
            self.L = self.Lbar
            if P["adapt_step_size"] == "dual_averaging" or P["adapt_step_size"] == 2:
                self.eps = math.exp(self.da_logbar)
        return dict(L=self.L, eps=self.eps, Lbar=self.Lbar)

    def set_state(self, theta, logw, logpi=None):
        """Replace the population (used to restart from another implementation's
        state); log pi and the gradient are recomputed at theta."""
        self.theta = np.array(theta, dtype=np.float64).reshape(self.J, self.d)
        self.logpi, self.grad = self.target.log_and_grad(self.theta)
        if self.traj_grad is not None:
            self.grad = self.traj_grad(self.theta)
        self.logw = np.array(logw, dtype=np.float64).copy()

    def log_evidence(self):
        m, S, _ = log_sum_exp(self.logw)
        return self.log_c + m + math.log(S)

    def moments(self):
        return realised_mean_var(self.theta, self.logw)
