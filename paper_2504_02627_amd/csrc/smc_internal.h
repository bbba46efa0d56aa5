// Internal declarations shared by the kernels and the host orchestration of
// libchees_smc.so.  Not part of the public ABI (include/chees_smc.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smc {

// Particle tile of the fused leapfrog/likelihood kernels: 8 waves x SUB
// subtiles x 16 particles.  Particle counts are padded to a multiple of TJ per
// posterior.
constexpr int WAVES = 8;
constexpr int SUB = 1;
constexpr int TJ = WAVES * SUB * 16;
constexpr int WG = 64 * WAVES;
// waves per work group of the whole-trajectory kernel (16 particles each)
constexpr int TRAJ_WAVES = 4;
// blocks per posterior of the FP64 population reductions (ESS, ChEES sums)
constexpr int RED_G = 32;
// particle chunks of the flow's weighted covariance (partials summed in order)
constexpr int FCOV_CH = 8;
constexpr size_t TRAJ_LDS_MAX = 65536;  // LDS of one work group
constexpr int MAX_C2 = 13;          // d <= 16 * 13 = 208
constexpr int MAX_NMAX = 4096;      // cap on max_leapfrog
constexpr int LF_MAX_SPLIT = 64;    // data-row splits per tile and step
constexpr int QUANT_BITS = 40;      // fixed-point resolution of resampling weights
constexpr int NPRIMES = 1024;       // primes table for N-d Halton
constexpr int SOBOL_MAXDIM = 21201; // rows of Joe and Kuo's table
constexpr int SOBOL_MAXDEG = 18;    // its largest polynomial degree

// Philox stream ids (counter word 3)
constexpr uint32_t STREAM_INIT = 1, STREAM_MOMENTUM = 2, STREAM_MH = 3, STREAM_RESAMPLE = 4,
                   STREAM_FLOW = 5, STREAM_JITTER = 6, STREAM_SHUFFLE = 7;

// Flow preconditioner: affine couplings with a two-hidden-layer conditioner
// of width FH; FP particles per wave in the flow kernels.
constexpr int FH = 128;
constexpr int FMAXL = 8;
constexpr int FKSPLIT = 8;  // particle chunks of the flow parameter-gradient reduction

// One coupling layer: transformed coordinates [T0, T0 + dt), conditioning
// coordinates [C0, C0 + dc); offsets of its parameters in the flat vector
// (per layer W1 [FH][dc], b1 [FH], W2 [FH][FH], b2 [FH], W3 [2dt][FH], b3 [2dt]).
struct FlowLayerDesc {
  int T0, C0, dt, dc;
  int oW1, ob1, oW2, ob2, oW3, ob3;
  // packed A-operand copies (16 x 16 granules) of W1, W2, W3 and of their
  // transposes, offsets into the packed arrays
  int pW1, pW2, pW3, qW1, qW2, qW3;
};

struct FlowNet {
  int L;                  // coupling layers
  int d;                  // dimension
  int half;               // max(dt, dc) rounded up to a multiple of 4
  int tape_stride;        // floats per particle and layer of the move tape
  int train_stride;       // floats per particle and layer of the training record
  int nparams;            // length of the flat parameter vector
  int npacked;            // length of a packed weight array
  int ntrain;             // Adam steps per iteration
  float lr;               // Adam learning rate
  FlowLayerDesc ly[FMAXL];
};

// Constants of one posterior, resident in device memory.
struct Post {
  int N, d;        // data rows and features
  int C1, C2;      // GEMM1 K-chunks 4 C2; GEMM2 column tiles ceil(d/16)
  int NT;          // 16-row data tiles ceil(N/16)
  int NT2;         // 32-row data tiles ceil(N/32) (BF16 trajectories)
  int KC;          // BF16 GEMM1 K-chunks of 32 features, ceil(C2/2)
  int row0;        // first particle row of this posterior
  int ll_splits;   // N-splits of the log-likelihood pass
  int ll_base;     // first work item of this posterior in the log-likelihood plan
  long long xab;     // float offset into the packed X tiles
  long long xbf;     // uint4 offset into the packed BF16 tiles
  long long xb3;     // uint4 offset into the three-plane BF16 tiles of the energies
  long long uoff;    // offset of this posterior's block in caller (B*J) x d_b arrays
};

// Per-posterior scalar state, resident in device memory.
struct PState {
  double L, eps, Lbar;          // trajectory length, step size, moving average
  double am, av;                // Adam moments for log L
  double em, ev;                // Adam moments for log eps
  int at, et;                   // Adam step counts
  int k;                        // iteration counter (1-based after the first step)
  int adapted_k;                // last iteration adapted
  double log_c;                 // evidence accumulator
  double m, S, S2, ess;         // LSE terms and ESS of the current weights
  double ess_before;            // ESS that decided this step's resampling
  int flag_resample;            // resample at the start of the next step
  int resampled;                // resampling ran in this step
  int degenerate;               // every weight -inf/NaN
  int pad0;
  double L_used, eps_used;      // parameters used by this step
  double ghat, sum_alpha, chees, sum_alpha_all, sum_inv_alpha;
  double da_hbar, da_logbar, da_mu;  // dual averaging of log eps: H_bar, log eps_bar, mu
  long long grad_evals_step;
  long long tot_grad_evals, tot_resamples, tot_iters;
  double tot_ess;
};

struct Dev {                    // pointers carved from the workspace
  Post *posts;
  PState *ps;
  int B, J, Jcap, DS;           // posteriors, particles, padded particles, row stride
  int nmax, jitter, mh, resampling, precond;
  double prior_var, ess_frac;
  double adam_lr, adam_b1, adam_b2, adam_eps, avg_decay, target_accept;
  int adapt_eps, num_warmup;
  uint64_t seed;
  float *xab;                   // packed data tiles ([tile][lane][A | B | y])
  uint4 *xbf;                   // packed BF16 32-row tiles (BF16 trajectories)
  uint4 *xb3;                   // X~ = hi + mid + lo in bfloat16, 32-row tiles (BF16 energies)
  int bf16;                     // trajectory gradients on BF16 MFMA
  int *status;                  // [0]: a label other than 0 / 1 met by the BF16 packing
  float *theta, *grad;          // current state, B*Jcap x DS
  float *theta_t, *p_t, *grad_t;// trajectory buffers
  float *theta_n;               // theta' of the next leapfrog step, written by the split
                                // reduction (valid for the particles it finished);
                                // bfloat16, B*Jcap x DS, in the precision form
  double *logpi, *logpi_t, *logw;
  double *h, *l, *H0, *dH, *alpha, *ca, *cg;
  int *n, *perm, *active, *anc, *accepted;
  unsigned long long *cdf;
  double *red_part;             // [B][RED_G][4] per-block partial sums of the reductions
  int *red_cnt;                 // [B][2] blocks done (ESS, ChEES); zero between launches
  int *sort_cnt;                // [B][sort_chunks][256] bin counts of the sort's work groups
  int sort_chunks;              // ceil(Jcap / 1024)
  float *gpart;                 // split partial gradients, [wg][TJ][DS]
  int gpart_slots;              // number of [TJ][DS] slots
  float2 *llpart;               // log-likelihood partials [split][row]
  int ll_smax;
  int4 *ll_items;               // (posterior, tile, split, -) work items of the log-lik pass
  int ll_nitems;
  double *colpart;              // column partial sums [B][chunks][2][DS]
  int col_chunks;
  double *means;                // [B][2][DS]
  float *minv;                  // [B][DS] inverse mass diagonal
  int *primes;                  // NPRIMES
  double *sqrtp;                // NPRIMES: sqrt(P_k), correctly rounded (host)
  double golden;                // (sqrt 5 - 1) / 2 in binary64 (host)
  int jit_K;                    // K, columns of the jitter matrix
  uint32_t *sobol;              // [sobol_dims][32] direction numbers nu_b 2^32 (host)
  int sobol_dims;
  // synthetic targets (SMC_TARGET_GAUSSIAN / BANANA; 0 = logistic regression)
  int target;
  float *tmean, *tprec;         // Gaussian: mean [DS], precision [DS][DS] (zero padded)
  double tconst;                // constant of log pi (normalisation + log_const)
  double bs1, bb, bc;           // banana parameters
  double fsv;                   // funnel: standard deviation of v
  int lf_target;                // work groups per leapfrog launch and resident group per compute unit
  int lf_grid;                  // grid of a leapfrog launch
  int lf_nosplit;               // one split per tile: the leapfrog launch finishes each step
  int traj;                     // whole trajectories in one launch (k_traj), 0 = per step
  size_t traj_lds;              // its dynamic LDS: every packed data tile
  // leapfrog work plan, written once per iteration from the active counts:
  int4 *lf_post;                // [nmax][B] (first item, splits per tile, tiles with one more, tiles)
  int4 *lf_items;               // [group][nmax][lf_grid] (posterior, tile, split | S << 16, first item of tile)
  int *lf_count;                // [group][nmax] items of a launch
  int ngroups;                  // feature-tile groups (one leapfrog launch each per step)
  int split_cap;                // most data-row splits per tile in a step
  int group_c2[MAX_C2];         // C2 of group g
  int c2_group[MAX_C2 + 1];     // group of C2
  int lf_goff[MAX_C2];          // first partial-gradient slot of group g (groups own disjoint slots)
  // flow preconditioner (precond FLOW, one posterior)
  int flow;
  float *fz, *fz0, *fgz;        // latent position, pre-move latent, latent gradient [Jcap][DS]
  float *fld0, *fld1;           // log|det J_T| at z0 and at the current z [Jcap]
  float *fm;                    // base map theta = m + L u: m [DS]
  float *fL;                    // L, row-major d x d
  float *fAf, *fAb, *fAi;       // packed base products: L P^T, P L^T, P L^-1
  double *fcov, *fLd, *fLi;     // weighted covariance [FCOV_CH][d][d] (partials over
                                // particle chunks); the shrunk covariance (factorised
                                // in place for d > 128); L^-1 for d > 128 (FP64)
  float *fbase;                 // [0]: log|det L|
  float *fp;                    // FP32 parameters (flat)
  float *fpk, *fbk;             // packed weights (and transposes): FP32, bfloat16-rounded
  float *fbias;                 // BF16-rounded biases (flat offsets)
  float *fgrad, *fadm, *fadv;   // parameter gradient and Adam moments
  float *ftape;                 // per particle and layer activations
  int *fstate;                  // [1]: Adam steps taken by the fit; [2]: fitted moves
};

// Host copy of one posterior's packing sizes.
struct HostPost {
  int N, d, C1, C2, NT, NT2, KC;
  long long xab, xbf, xb3;
};

// Launchers (smc_kernels.hip).  All stream-ordered.
hipError_t launch_pack_one(const Dev &D, const void *X, const float *y, int x_dtype,
                           const HostPost &P, hipStream_t st);
hipError_t launch_pack_bf16(const Dev &D, const void *X, const float *y, int x_dtype,
                            const HostPost &P, hipStream_t st);
// BF16 leapfrog kernel: four waves of 32 particles per work group.
constexpr int B32_WAVES = 4;
constexpr int B32_WG = 64 * B32_WAVES;

// Resident leapfrog work groups per compute unit.  The FP32 kernel (8 waves)
// for up to 8 feature tiles is built for two (at most 128 VGPRs, LDS at most
// 80 KB), wider FP32 problems run one; the BF16 kernel (4 waves) runs two up
// to 10 feature tiles (at most 256 registers per lane, two LDS stages of at
// most 80 KB) and one beyond (its accumulators need more registers).
__host__ __device__ constexpr int lf_groups_per_cu(bool bf16, int c2) {
  return bf16 ? (c2 <= 10 ? 2 : 1) : (c2 <= 8 ? 2 : 1);
}

// uint4 per lane and 32-row tile in the BF16 packing: [A1: C2 | A2: 2 ceil(C2/2)],
// plus one zero slot when that is even
__host__ __device__ constexpr int bf16_lane_stride(int c2) { return (c2 + 2 * ((c2 + 1) / 2)) | 1; }
// 32-row data tiles per LDS stage of the BF16 kernel: two when the two stages
// of the resident work groups fit the compute unit's 160 KB of LDS (up to 9
// feature tiles at two groups per compute unit, 11-13 at one), one otherwise
// (10); a posterior's tiles are padded to whole stages (the pad rows are zero
// and add nothing).
__host__ __device__ constexpr int bf16_stage_tiles(int c2) {
  return 2 * 2 * 64 * bf16_lane_stride(c2) * 16 * lf_groups_per_cu(true, c2) <= 160 * 1024 ? 2 : 1;
}
// uint4 per lane and 32-row tile of the three-plane energy packing: the hi,
// mid and lo planes of GEMM1's A operand (C2 slots each), odd lane stride
__host__ __device__ constexpr int b3_lane_stride(int c2) { return (3 * c2) | 1; }
hipError_t fill_f32(float *p, long long n, float v, hipStream_t st);
hipError_t fill_i32(int *p, long long n, int v, hipStream_t st);
hipError_t fill_f64(double *p, long long n, double v, hipStream_t st);
hipError_t launch_init_theta(const Dev &D, const float *theta0, hipStream_t st);
hipError_t launch_init_weights(const Dev &D, hipStream_t st);
hipError_t launch_begin_step(const Dev &D, int conditional, const double *u, int count_iteration,
                             hipStream_t st);
hipError_t launch_mass(const Dev &D, int write_minv, hipStream_t st);
hipError_t launch_gather(const Dev &D, int *anc_out, hipStream_t st);
hipError_t launch_setup(const Dev &D, const float *momenta, int init_mode, hipStream_t st);
hipError_t launch_sort(const Dev &D, hipStream_t st);
// Work plan of every leapfrog launch of the iteration (after the sort, or the
// initial active counts).
hipError_t launch_lf_plan(const Dev &D, hipStream_t st);
// Synthetic targets (target_kernels.hip): one leapfrog step (or the gradient
// at theta_t), log pi(theta_t) into logpi_t, and the Gaussian's parameters.
hipError_t launch_target_step(const Dev &D, int step, int grad_only, hipStream_t st);
hipError_t launch_target_energy(const Dev &D, hipStream_t st);
hipError_t launch_target_pack(const Dev &D, const float *mean, const float *prec, int d,
                              hipStream_t st);
hipError_t launch_lf_partial(const Dev &D, int c2, int step, int zero_eps, hipStream_t st);
size_t traj_lds_bytes(int c2, int nt);
hipError_t launch_traj(const Dev &D, int c2, hipStream_t st);
// mode 0: full step; 1: zero step size (gradient at theta, state rewritten);
// 2: gradient only (theta given by the caller, p untouched)
// c2only > 0: only the posteriors of that feature-tile group
hipError_t launch_lf_reduce(const Dev &D, int step, int mode, hipStream_t st, int c2only = 0);
hipError_t launch_loglik(const Dev &D, int c2, int first, int count, hipStream_t st);
hipError_t launch_weights(const Dev &D, const double *mh_u, int init_mode, hipStream_t st);
hipError_t launch_chees(const Dev &D, hipStream_t st);
hipError_t launch_commit(const Dev &D, hipStream_t st);
hipError_t launch_ess(const Dev &D, int count, hipStream_t st);
hipError_t launch_adapt(const Dev &D, hipStream_t st);
hipError_t launch_set_params(const Dev &D, double L, double eps, hipStream_t st);
hipError_t launch_export_state(const Dev &D, float *theta, double *logw, double *logpi,
                               hipStream_t st);
// Flow preconditioner (flow_kernels.hip).
hipError_t launch_flow_init(const Dev &D, const FlowNet &F, hipStream_t st);
hipError_t launch_flow_base(const Dev &D, const FlowNet &F, hipStream_t st);
hipError_t launch_flow_train(const Dev &D, const FlowNet &F, int step, hipStream_t st);
hipError_t launch_flow_publish(const Dev &D, const FlowNet &F, hipStream_t st);
hipError_t launch_flow_set(const Dev &D, const FlowNet &F, hipStream_t st);
hipError_t launch_flow_gradsum(const Dev &D, const FlowNet &F, float *out, hipStream_t st);
hipError_t launch_flow_begin(const Dev &D, const FlowNet &F, hipStream_t st);
hipError_t launch_flow_drift(const Dev &D, const FlowNet &F, int step, hipStream_t st);
hipError_t launch_flow_kick(const Dev &D, const FlowNet &F, int step, hipStream_t st);
// the kick of step `step` and the drift of step `step + 1` in one launch
hipError_t launch_flow_kick_drift(const Dev &D, const FlowNet &F, int step, hipStream_t st);
hipError_t launch_resample_indices(const double *w, int J, const double *u, int scheme,
                                   int *anc, unsigned long long *cdf, double *wmax, int *err,
                                   hipStream_t st);
// Device address of the no-allocation resampling scratch on the current
// device (looked up once per device): CDF of RS_STATIC_MAX entries and the
// error flag.
constexpr int RS_STATIC_MAX = 1 << 20;
constexpr int RS_MAX_DEVICES = 64;
hipError_t static_resample_scratch(unsigned long long **cdf, int **err);

}  // namespace smc
