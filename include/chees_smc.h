/*
 * chees_smc.h -- C ABI of libchees_smc.so: a sequential Monte Carlo (SMC)
 * sampler whose proposal is a ChEES-HMC trajectory, for Bayesian logistic
 * regression posteriors, on AMD Instinct MI355X (gfx950).
 *
 * Method: Millard, Murphy, Frisch, Maskell, "Incorporating the ChEES Criterion
 * into Sequential Monte Carlo Samplers" (arXiv 2504.02627).
 *   - target pi(theta) = p(y | X, theta) q0(theta), theta in R^d      (Sec. II)
 *   - likelihood y_n ~ Bernoulli(sigmoid(theta^T x_n))       (Sec. IV, German Credit)
 *   - SMC loop: normalise, ESS, resample if J_eff < J/2, move, reweight
 *                                                            (Sec. III, Alg. smc_BNN)
 *   - move: leapfrog with jittered length l = h L, ceil(l/eps) steps
 *                                          (Sec. II-A, II-C, Alg. smc_ChEES)
 *   - weight: momentum change-of-variables L-kernel, log w += -Delta H
 *                                          (Sec. III-A, eqs. proposal_momentum,
 *                                           l-kernel_momentum, l_weights)
 *   - ChEES gradient, alpha-weighted, Adam on log L, moving average, freeze
 *                                          (Sec. II-C, Alg. smc_ChEES)
 *
 * Memory model.  Every device buffer is caller-owned: the data X, y, the
 * workspace (size from smc_workspace_bytes) and the HIP stream must outlive
 * the context.  The library allocates no device memory at run time; its one
 * static device array (8 MiB per GPU, the scratch of
 * resample_indices_noalloc) is part of the loaded code object.  The context
 * header is host memory released by smc_destroy.  Every call is
 * stream-ordered and asynchronous unless it says it synchronises.
 *
 * Errors.  Functions return smc_status and never abort.  smc_last_error gives
 * a message for the last failing call on a context.  A single particle whose
 * energy is not finite is not an error: it gets alpha = 0 and log w = -inf.
 */
#ifndef CHEES_SMC_H
#define CHEES_SMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SMC_OK = 0,
  SMC_EINVAL = -1,      /* bad argument, size or call parameter            */
  SMC_EDEVICE = -2,     /* a HIP call failed (see smc_last_error)          */
  SMC_EDEGENERATE = -3, /* every log-weight is -inf or NaN                 */
  SMC_ESTATE = -4,      /* calls out of order (e.g. chees_adapt before a step) */
  SMC_ENOMEM = -5,      /* workspace smaller than smc_workspace_bytes      */
  SMC_WADAPTIVE = 1     /* success with a warning: see log_evidence        */
} smc_status;

/* data type of X */
enum { SMC_F32 = 0, SMC_BF16 = 1 };
/* Jitter schemes of Sec. III-B-1: h_jk for particle j = 1..J at iteration
 * k = 1, 2, ...; phi_b is the radical inverse in base b (eq. halton), P_k the
 * k-th prime (the library holds the first 1024; later iterations reuse P_1024),
 * K = smc_params.num_iterations, and k' = K - ((k - 1) mod K) the reversed
 * column order of the inverse schemes (K + 1 - k for k <= K).  The uniform
 * draws u_jk are word 0 of Philox4x32-10 block (0, particle, k, 6); the
 * shuffle pi_k of the equidistant schemes is a 4-round Feistel network on the
 * smallest even bit width covering J, round r keyed by Philox block
 * (R, 4 b + r, k, 7) word 0 (b the posterior), walked until it lands in
 * [0, J). */
enum { SMC_JITTER_HALTON1D = 0,     /* phi_2((k-1) J + j)                          */
       SMC_JITTER_NONE = 1,         /* h = 1                                       */
       SMC_JITTER_HALTONND = 2,     /* phi_{P_k}(j)                                */
       SMC_JITTER_UNIFORM = 3,      /* u_jk                                        */
       SMC_JITTER_HALTONND_INV = 4, /* phi_{P_k'}(j)                               */
       SMC_JITTER_PRIMES = 5,       /* j sqrt(P_k) mod 1 (eq. primes)              */
       SMC_JITTER_PRIMES_INV = 6,   /* j sqrt(P_k') mod 1                          */
       SMC_JITTER_GOLDEN = 7,       /* ((j-1) K + k) (sqrt 5 - 1)/2 mod 1          */
       SMC_JITTER_EQUIDISTANT = 8,  /* (pi_k(j-1) + 1) / J                         */
       SMC_JITTER_EQUIDISTANT_OFFSET = 9, /* (pi_k(j-1) + 1) / J + 0.1 u_jk       */
       SMC_JITTER_SOBOL1D = 10,     /* x^(1)((k-1) J + j)                          */
       SMC_JITTER_SOBOLND = 11,     /* x^(k)(j), k beyond sobol_dims: the last one  */
       SMC_JITTER_SOBOLND_INV = 12  /* x^(k')(j)                                   */ };
/* Sobol schemes (eq. sobol): x^(k)(i) is point i of Sobol dimension k, the
 * xor of its direction numbers nu_b = m_b / 2^b over the binary digits b of
 * the Gray code i ^ (i >> 1) (the order of scipy's generator, which the paper
 * uses), point 0 never used.  Dimension 1 has nu_b = 2^-b (the base-2 van der
 * Corput sequence) and needs no table; the N-d schemes take the direction
 * integers from smc_params.sobol_table. */
/* resampling schemes (Sec. III) */
enum { SMC_RESAMPLE_SYSTEMATIC = 0, SMC_RESAMPLE_MULTINOMIAL = 1 };
/* step-size adaptation during warm-up */
enum { SMC_ADAPT_EPS_NONE = 0,
       SMC_ADAPT_EPS_ADAM = 1,           /* Adam on log eps toward a harmonic-mean
                                            acceptance of target_accept          */
       SMC_ADAPT_EPS_DUAL_AVERAGING = 2  /* Nesterov dual averaging of log eps
                                            (Hoffman and Gelman 2014: gamma 0.05,
                                            t0 10, kappa 0.75, mu = log 10 eps_0)
                                            on the mean alpha of the particles;
                                            eps <- the averaged iterate at the end
                                            of warm-up                          */ };
/* arithmetic of the trajectory gradients */
enum { SMC_PRECISION_F32 = 0, SMC_PRECISION_BF16 = 1 };
/* preconditioning of the trajectories (none of them changes the target: the
 * weights stay exact, Sec. III-A) */
enum { SMC_PRECOND_NONE = 0,  /* unit mass, the paper's M = I                   */
       SMC_PRECOND_DIAG = 1,  /* diagonal mass M^{-1} = regularised weighted
                                 variance of the pre-move population            */
       SMC_PRECOND_FLOW = 2   /* affine-coupling flow T fitted to the weighted
                                 population each iteration; leapfrog in the
                                 latent space on log pi(T(z)) + log|det J_T(z)|
                                 (one posterior per context)                    */ };

/* Target densities.  LOGISTIC: the Bayesian logistic regression of Sec. IV
 * (X, y, prior_var).  GAUSSIAN and BANANA: the synthetic targets of Sec. IV;
 * FUNNEL: the funnel the paper names as future work (Sec. VI).  The synthetic
 * targets take one posterior per context, FP32 trajectories and no flow
 * preconditioner. */
enum { SMC_TARGET_LOGISTIC = 0,
       SMC_TARGET_GAUSSIAN = 1,  /* log pi = log N(theta; mean, precision^{-1}) + log_const */
       SMC_TARGET_BANANA = 2,    /* d = 2: log pi = log N(theta_1; 0, s1^2)
                                    + log N(theta_2; b (theta_1^2 - c), 1) + log_const */
       SMC_TARGET_FUNNEL = 3     /* Neal's funnel, d >= 2, theta = (v, x_1..x_{d-1}):
                                    log pi = log N(v; 0, funnel_scale^2)
                                    + sum_i log N(x_i; 0, e^v) + log_const       */ };

typedef struct smc_ctx smc_ctx;

/* The posterior: pi(theta) = p(y | X, theta) q0(theta), q0 = N(0, prior_var I)
 * (Sec. II problem statement; Sec. IV model).  num_posteriors independent
 * problems may share one context (batched form); they are sampled with the
 * same parameters and independent particle populations.  For the synthetic
 * targets pi is the target density itself and q0 = N(0, prior_var I) is only
 * the initial distribution (Sec. IV: N(0, I)); n_rows, X and y are unused
 * (may be NULL). */
typedef struct {
  int32_t num_posteriors;     /* B >= 1 (1 for the synthetic targets)           */
  const int32_t *n_rows;      /* host [B]: N_b >= 1 data rows                    */
  const int32_t *dims;        /* host [B]: d_b in [1, 208] features             */
  const void *const *X;       /* host [B] of DEVICE pointers: row-major N_b x d_b,
                                 element type x_dtype                           */
  const float *const *y;      /* host [B] of DEVICE pointers: N_b labels in {0,1} */
  int32_t x_dtype;            /* SMC_F32 or SMC_BF16                            */
  double prior_var;           /* q0 variance (the paper's N(0, I): 1.0)         */
  int32_t target;             /* SMC_TARGET_*                                   */
  const float *mean;          /* GAUSSIAN: DEVICE d, the mean mu                 */
  const float *precision;     /* GAUSSIAN: DEVICE d x d row-major Sigma^{-1},
                                 symmetric positive definite (checked by a
                                 Cholesky factorisation at smc_init)            */
  double log_const;           /* GAUSSIAN, BANANA: added to the normalised log
                                 density, so the evidence is exp(log_const)     */
  double banana_s1, banana_b, banana_c; /* BANANA: s1 > 0, b, c (Sec. IV: 10, 0.03, 100) */
  double funnel_scale;        /* FUNNEL: standard deviation of v (Neal: 3)      */
} smc_problem;

typedef struct {
  int32_t num_particles;      /* J per posterior, 1..65536                      */
  int32_t max_leapfrog;       /* n_max >= 1: cap on ceil(l/eps)                 */
  int32_t num_warmup;         /* M_warmup of Alg. smc_ChEES (>= 1)              */
  int32_t jitter;             /* SMC_JITTER_*                                   */
  int32_t mh_accept;          /* 0: SMC-ChEES, no accept/reject (Sec. III-A);
                                 1: accept iff u < alpha (eq. mh_ratio_rn), and
                                    the weight increment is 0                   */
  int32_t resampling;         /* SMC_RESAMPLE_*                                 */
  int32_t precision;          /* SMC_PRECISION_*                                */
  int32_t precond;            /* SMC_PRECOND_*                                  */
  double step_size;           /* eps_0 > 0                                      */
  double traj_length;         /* L_0 > 0 (the paper's experiments: 5)           */
  double ess_frac;            /* resample iff J_eff < ess_frac J (paper: 0.5)   */
  double adam_lr, adam_b1, adam_b2, adam_eps; /* Adam on log L (ascent)         */
  double avg_decay;           /* Lbar <- avg_decay Lbar + (1 - avg_decay) L (0.9) */
  int32_t adapt_step_size;    /* SMC_ADAPT_EPS_*: step-size adaptation during
                                 warm-up (the paper keeps eps fixed and names
                                 dual averaging as future work)                 */
  double target_accept;       /* acceptance target (ADAM: harmonic mean of
                                 alpha, e.g. 0.651; DUAL_AVERAGING: mean alpha,
                                 e.g. 0.65)                                     */
  uint64_t seed;              /* key of the Philox4x32-10 streams               */
  /* SMC_PRECOND_FLOW only: coupling layers (0..8; 0 = the base map alone,
   * a dense mass from the weighted covariance), conditioner width (128),
   * Adam steps of the weighted maximum-likelihood fit per iteration (>= 0,
   * warm-started) and their learning rate */
  int32_t flow_layers, flow_width, flow_train_steps;
  double flow_lr;
  /* K, the columns of the jitter matrix: required (1..1024) by the inverse
   * Halton and primes schemes, (1..sobol_dims) by the inverse Sobol scheme,
   * and (>= 1) by the golden-ratio scheme; ignored otherwise */
  int32_t num_iterations;
  /* SMC_JITTER_SOBOLND(_INV) only (NULL and 0 otherwise): HOST array of
   * sobol_dims (1..21201) rows of 19 words, row k - 1 for dimension k: the
   * primitive polynomial x^s + a_1 x^(s-1) + .. + a_(s-1) x + 1 as the bit
   * mask with bit s set for x^s, bit s - t for a_t and bit 0 for the constant
   * term (the mask 1, s = 0, means the first dimension's nu_b = 2^-b), then
   * the initial direction integers m_1..m_s (odd, m_i < 2^i; s <= 18; the
   * words past s are ignored).  This is the layout of Joe and Kuo's table as
   * scipy ships it.  Read during smc_init only; a malformed row is
   * SMC_EINVAL. */
  const uint32_t *sobol_table;
  int32_t sobol_dims;
  /* Launch tuning of the split leapfrog launches (0 = the library's
   * default; neither changes the arithmetic except through the split count,
   * which fixes the order of the partial-gradient sums):
   *   lf_items: work items per resident work-group slot and step (1..4096;
   *     default 256);
   *   lf_split_cap: most data-row splits of one particle tile in one step
   *     (1..64; default 64).
   * paper_2504_02627_amd/autotune.py measures them per workload and caches
   * the choice. */
  int32_t lf_items, lf_split_cap;
} smc_params;

/* Host-supplied randomness for one smc_step (all fields nullable, DEVICE
 * pointers).  A NULL field is drawn from the library's Philox4x32-10 streams. */
typedef struct {
  const float *momenta;       /* (B*J) x d_b standard normals xi, row-major per
                                 posterior block; momentum p = xi M^{1/2}        */
  const double *mh_uniforms;  /* B*J uniforms in [0,1) (used iff mh_accept)     */
  const double *resample_u;   /* B values (systematic) or B*J (multinomial)     */
} smc_inject;

/* Per-iteration statistics (posterior 0 for a batched context). */
typedef struct {
  double ess;          /* J_eff after the move (eq. ess_smc)                   */
  double ess_before;   /* J_eff that decided the resampling                    */
  double mean_accept;  /* mean alpha                                           */
  double chees;        /* 1/4 mean a_j^2: ChEES sample estimate                */
  double chees_grad;   /* alpha-weighted gradient g_hat                        */
  double L, eps;       /* trajectory length and step size used by this step    */
  double log_z;        /* log-evidence estimate after this step                */
  int32_t resampled;   /* 1 if resampling ran at the start of this step        */
  int32_t iteration;   /* k, 1-based                                           */
  int64_t grad_evals;  /* sum_j n_j of this step (leapfrog gradients)          */
} smc_stats;

/* Totals since smc_init, accumulated on the device (all posteriors). */
typedef struct {
  int64_t iterations;
  int64_t grad_evals;  /* sum over steps and particles of n_j                  */
  double ess_sum;      /* sum over steps and posteriors of the post-move J_eff */
  int64_t resamples;
} smc_counters;

/* Per-particle device views of the last step.  Rows are posterior-major with
 * a padded stride: particle j of posterior b is row b * jcap + j. */
typedef struct {
  const double *h;      /* jitter h_j                                          */
  const double *l;      /* jittered length l_j = h_j L                         */
  const int32_t *n;     /* leapfrog steps n_j                                  */
  const double *dH;     /* energy error Delta H (+inf if not finite)           */
  const double *alpha;  /* min(1, exp(-Delta H))                               */
  const int32_t *ancestors; /* ancestors (index within the posterior) of the
                               last resampling                                */
  const float *p_final; /* momenta p' after the trajectory, (B*J) x dpad      */
  const float *theta_prop; /* proposals theta', (B*J) x dpad                  */
  const float *grad;    /* trajectory gradient (after smc_init: at theta_0),
                           (B*J) x dpad                                         */
  const float *minv;    /* diagonal inverse mass of the last step, B x dpad     */
  /* SMC_PRECOND_FLOW (else NULL): latent positions z0 = T^-1(theta_0) and z'
   * after the trajectory, the latent gradient at z', (J x dpad), and
   * log|det J_T| at z0 and at z' (J) */
  const float *latent0, *latent, *latent_grad, *logdet0, *logdet;
  int32_t dpad;         /* row stride (floats) of p_final and theta_prop       */
  int32_t jcap;         /* particle rows per posterior (J padded)              */
  const int32_t *order; /* per posterior, the jcap rows (index within the
                           posterior) sorted by n_j, longest first, index
                           order within equal n_j: the order in which the
                           trajectory kernels group particles               */
  const int32_t *active; /* per posterior, n_max + 1 counts: #{j: n_j > s}  */
} smc_trace;

/* Workspace size for a problem and parameters; 0 if they are invalid. */
size_t smc_workspace_bytes(const smc_problem *prob, const smc_params *par);

/* Build a context: pack X, draw or copy theta_0, evaluate log pi and its
 * gradient at theta_0 (the gradient taken before the first leapfrog loop,
 * Sec. V) and set log w_j = log pi(theta_0^j) - log q0(theta_0^j) - log J
 * (eqs. init_sample, init_weights; the -log J makes sum_j w_j an evidence
 * estimate).  theta0: nullable DEVICE (B*J) x d_b FP32; NULL draws
 * theta_0 ~ q0 from Philox.  hip_stream: a hipStream_t (NULL = default).
 * Does not synchronise.  Launch shapes chosen here: a single posterior whose
 * packed data fits in one work group's LDS runs each iteration's
 * trajectories in one launch (the environment variable CHEES_SMC_PER_STEP=1
 * at smc_init keeps one launch per leapfrog step instead, for comparison);
 * several feature-tile groups run side by side on three extra streams of
 * default priority, created here and forked from and joined into
 * hip_stream. */
smc_status smc_init(const smc_problem *prob, const smc_params *par, void *workspace,
                    size_t workspace_bytes, void *hip_stream, const float *theta0,
                    smc_ctx **out);

/* One SMC iteration k (Alg. smc_BNN body): normalise and ESS (eqs.
 * normalise_smc2, ess_smc), resample iff J_eff < ess_frac J and reset weights
 * to 1/J (Sec. III), draw momenta, jitter h_jk and n_j = clamp(ceil(h L/eps),
 * 1, n_max) (Alg. smc_ChEES), run the leapfrog trajectories, compute Delta H
 * and alpha (eq. HMC_accept_reject), update log w += -Delta H (SMC-ChEES) or
 * accept iff u < alpha (MH mode), and the ChEES statistics.  stats: nullable
 * host pointer; non-NULL synchronises the stream and fills it.  Once the
 * adaptation has ended, the first step synchronises once to read L and eps
 * and from then on launches only the leapfrog steps the longest trajectory
 * can need (see smc_run). */
smc_status smc_step(smc_ctx *ctx, const smc_inject *inject, smc_stats *stats);

/* Warm-up adaptation after step k (Alg. smc_ChEES): k < M_warmup: Adam
 * ascent on log L with g_hat (skipped when sum alpha = 0) and
 * Lbar <- 0.9 Lbar + 0.1 L; k = M_warmup: L <- Lbar.  Runs on the device.
 * SMC_ESTATE if no step ran since the last adaptation.  stats: as smc_step. */
smc_status chees_adapt(smc_ctx *ctx, smc_stats *stats);

/* `iterations` SMC iterations, each smc_step (randomness from the library's
 * Philox streams, nothing injected) followed by chees_adapt.  The first call
 * captures one iteration's launches as a HIP graph on a private stream; every
 * call replays it on the context's stream, once per iteration, without host
 * synchronisation.  Once the adaptation has ended (num_warmup iterations),
 * the call that crosses that point synchronises once, reads L and eps, and
 * captures a second graph whose leapfrog launches stop at the longest
 * trajectory those values allow (min(max(ceil(h_max L / eps), 1), n_max),
 * h_max the jitter's largest value: 1.1 for SMC_JITTER equidistant with
 * offset, else 1); smc_set_params and smc_load drop the bound.
 * Results are identical to the same number of smc_step + chees_adapt calls.
 * Per-kernel timing does not cover it.  SMC_ESTATE after a smc_step not yet
 * followed by chees_adapt. */
smc_status smc_run(smc_ctx *ctx, int32_t iterations);

/* Flow preconditioner (SMC_PRECOND_FLOW).  Parameters form one flat FP32
 * vector: for each coupling layer l = 0..layers-1, with d_T = floor(d/2)
 * transformed coordinates for even l (the first ones) and d - floor(d/2) for
 * odd l (the last ones), d_C = d - d_T: W1 [width][d_C], b1 [width],
 * W2 [width][width], b2 [width], W3 [2 d_T][width] (rows 0..d_T-1 give s,
 * the rest t), b3 [2 d_T], all row-major.  smc_flow_param_count gives its
 * length (0 for invalid sizes).  The couplings act on x; the base map is
 * theta = m + L u with u_c = x_q(c) (q: even coordinates first, then the odd
 * ones), m the weighted mean of the pre-move population and L the Cholesky
 * factor of its weighted covariance shrunk as n/(n+5) C + 1e-3 5/(n+5) I.
 * smc_get_flow copies into DEVICE buffers (each nullable) the current FP32
 * parameters, m (d) and L (d x d row-major, lower triangular) of the last
 * step, and the gradient of the fit objective that the last Adam step used
 * (same layout as the parameters); smc_set_flow replaces the parameters from
 * a DEVICE vector and restarts their Adam moments.  SMC_EINVAL without a
 * flow. */
size_t smc_flow_param_count(int32_t d, int32_t layers, int32_t width);
smc_status smc_get_flow(smc_ctx *ctx, float *params, float *m, float *L, float *grad);
smc_status smc_set_flow(smc_ctx *ctx, const float *params);

/* Unconditional resampling of the current population (Sec. III), then the
 * weights are reset to 1/J.  u: nullable DEVICE uniforms (B for systematic,
 * B*J for multinomial); ancestors_out: nullable DEVICE B*J int32. */
smc_status resample(smc_ctx *ctx, const double *u, int32_t *ancestors_out);

/* Stateless resampling of J nonnegative weights w (DEVICE, any scale, not all
 * zero): e_j = w_j / max w, Q_j = floor(e_j 2^40), then systematic
 * (a_i = min{j : C_j > (i + U/2^32) T / J}, U = floor(u_0 2^32)) or multinomial
 * (a_i = min{j : C_j > (U_i/2^32) T}) on the exact integer cumulative sum C,
 * T = C_J.  u: DEVICE, 1 (systematic) or J (multinomial) uniforms in [0,1).
 * ancestors: DEVICE J int32.  workspace: DEVICE, resample_workspace_bytes(J).
 * SMC_EDEGENERATE if every weight is zero (checked after a synchronisation). */
size_t resample_workspace_bytes(int32_t J);
smc_status resample_indices(const double *w, int32_t J, const double *u, int32_t scheme,
                            int32_t *ancestors, void *workspace, size_t workspace_bytes,
                            void *hip_stream);

/* The same stateless resampling with no workspace argument, for callers that
 * cannot allocate device memory (code that may not call hipMalloc: tight
 * serving loops, harnesses that forbid allocation).  Its scratch (the integer
 * CDF and an error flag) is a static device array of the library, one copy
 * per GPU, sized for J <= resample_noalloc_max() = 1048576 weights (8 MiB),
 * held until the process ends.  Larger J is SMC_EINVAL (nothing launched).
 * The call allocates nothing; it launches one kernel on hip_stream, copies the
 * 4-byte error flag to the host and synchronises the stream.  Every call on a
 * GPU shares that GPU's array: calls that overlap on one GPU (other streams or
 * threads) race and must be serialised by the caller.  Arguments, results and
 * SMC_EDEGENERATE as for resample_indices. */
int32_t resample_noalloc_max(void);
smc_status resample_indices_noalloc(const double *w, int32_t J, const double *u, int32_t scheme,
                                    int32_t *ancestors, void *hip_stream);

/* log Z_hat = C + LSE(log w), C the sum of LSE(log w) over past resamplings
 * (the standard SMC evidence estimator).  Synchronises.  log_z_host: posterior
 * 0; per_posterior_host: nullable host [B].  Returns SMC_WADAPTIVE (positive:
 * the estimates are written) when some move of this context, under
 * SMC_PRECOND_FLOW, used couplings fitted to the very population it moved:
 * the weights then no longer correct for a fixed proposal, so the estimate is
 * adaptive and biased (measured upward, a few tenths in log Z); a context whose
 * couplings only ever came from smc_set_flow, or that never fitted
 * (flow_train_steps 0), returns SMC_OK.  smc_last_error names the count. */
smc_status log_evidence(smc_ctx *ctx, double *log_z_host, double *per_posterior_host);

/* Copy the state into caller DEVICE buffers (each nullable): theta (B*J) x d_b
 * FP32, logw (B*J) FP64, logpi (B*J) FP64.  Stream-ordered. */
smc_status smc_get_state(smc_ctx *ctx, float *theta, double *logw, double *logpi);

/* Device views of the last step's per-particle quantities (see smc_trace). */
smc_status smc_get_trace(smc_ctx *ctx, smc_trace *trace);

/* Totals since init (synchronises). */
smc_status smc_get_counters(smc_ctx *ctx, smc_counters *counters);

/* Kernel timing with HIP events recorded on the context's stream around every
 * launch of the fused leapfrog kernel (drift + X theta'^T -> sigmoid -> R X
 * over a data-row split), of its split reduction (sum of partials + kick) and
 * of the log-likelihood kernel.  Off by default.  smc_get_timing synchronises,
 * returns the totals since timing was enabled (or last read) and resets them. */
typedef struct {
  double leapfrog_ms;          /* summed event time of the fused leapfrog launches */
  int64_t leapfrog_launches;
  double loglik_ms;
  int64_t loglik_launches;
  double reduce_ms;            /* split reduction + second half kick               */
  int64_t reduce_launches;
  double flow_ms;              /* flow preconditioner: drift + forward map, and
                                  latent gradient + kick, per leapfrog step         */
  int64_t flow_launches;
  double train_ms;             /* flow preconditioner: one Adam step of the fit     */
  int64_t train_launches;
} smc_timing;
smc_status smc_set_timing(smc_ctx *ctx, int32_t enable);
smc_status smc_get_timing(smc_ctx *ctx, smc_timing *out);

/* Set the adapted parameters L and eps (stream-ordered; host values). */
smc_status smc_set_params(smc_ctx *ctx, double L, double eps);

/* Checkpoint and resume (not in the paper).  smc_save copies into HOST memory
 * buf (at least smc_state_bytes bytes) the state after the last completed
 * iteration: particles, gradients, log-densities and log-weights, the inverse
 * mass, each posterior's scalars (L, eps and their Adam and dual-averaging
 * moments, the moving average, the iteration counter k, the evidence
 * accumulator, the totals) and, with the flow preconditioner, the couplings,
 * their packed copies and Adam moments; it synchronises the stream and is
 * SMC_ESTATE between smc_step and chees_adapt.  smc_load restores such an
 * image into a context built from the same problem and parameters: the
 * randomness is counter-based (Philox keyed by seed and k), so the run goes
 * on bit-identically.  An image of another shape (B, J, row stride, n_max,
 * flow size, precision) is SMC_EINVAL; the caller owns keeping the problem
 * and the remaining parameters the same. */
size_t smc_state_bytes(const smc_ctx *ctx);
smc_status smc_save(smc_ctx *ctx, void *buf, size_t bytes);
smc_status smc_load(smc_ctx *ctx, const void *buf, size_t bytes);

void smc_destroy(smc_ctx *ctx);
const char *smc_last_error(const smc_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* CHEES_SMC_H */
