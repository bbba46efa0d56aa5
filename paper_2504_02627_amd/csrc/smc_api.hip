// Host side of libchees_smc.so: argument checks, workspace layout, and the
// order of kernel launches for each ABI call (include/chees_smc.h).
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "chees_smc.h"
#include "smc_internal.h"

using namespace smc;

constexpr int MAX_SIDE = 3;  // side streams: four lanes of group launches in all

struct smc_ctx {
  Dev D;
  hipStream_t st = nullptr;
  std::vector<HostPost> hp;
  std::vector<Post> posts;
  std::vector<PState> ps_host;
  std::vector<int> c2s;        // distinct GEMM2 tile counts among the posteriors
  std::vector<int3> ll_groups; // (C2, first item, count) of the log-likelihood pass
  std::vector<int4> ll_items;
  std::vector<int> primes;
  std::vector<double> sqrtp;   // sqrt of the primes (binary64, correctly rounded)
  std::vector<uint32_t> sobol; // direction numbers of the N-d Sobol schemes
  std::vector<float> minv;
  int stepped = 0;             // a step ran since the last adaptation
  int steps = 0;
  std::string err;
  // event timing of the hot kernels
  int timing = 0;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<std::pair<int, size_t>> ev_marks;  // (kind, index of the start event)
  // one SMC iteration (step + adaptation) captured as a graph for smc_run:
  // with n_max leapfrog launches, and (once the adaptation has frozen L and
  // eps) with as many launches as the longest trajectory can need
  FlowNet F{};
  hipStream_t cap_st = nullptr;
  hipGraph_t graph = nullptr, graph_b = nullptr;
  hipGraphExec_t gexec = nullptr, gexec_b = nullptr;
  int nl_b = 0;        // leapfrog launches of the bounded graph (0: none)
  int frozen = 0;      // L and eps are final and nl_b has been set
  // side streams on which the launches of several feature-tile groups run
  // side by side (created at smc_init when there is more than one group)
  hipStream_t side[MAX_SIDE] = {};
  hipEvent_t fork_ev = nullptr, join_ev[MAX_SIDE] = {};
  std::vector<int> group_lane;  // lane of each group: largest work first to the least loaded
  ~smc_ctx() {
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    if (gexec_b) (void)hipGraphExecDestroy(gexec_b);
    if (graph_b) (void)hipGraphDestroy(graph_b);
    if (cap_st) (void)hipStreamDestroy(cap_st);
    for (int i = 0; i < MAX_SIDE; ++i) {
      if (side[i]) (void)hipStreamDestroy(side[i]);
      if (join_ev[i]) (void)hipEventDestroy(join_ev[i]);
    }
    if (fork_ev) (void)hipEventDestroy(fork_ev);
  }
};

namespace {

struct Layout {
  int B = 0, J = 0, Jcap = 0, DS = 0, nmax = 0;
  int lf_target = 0, lf_grid = 0, ll_smax = 0, ll_nitems = 0, col_chunks = 0;
  int gpart_slots = 0, goff[MAX_C2] = {};
  int nosplit = 0;
  int traj = 0;
  int split_cap = LF_MAX_SPLIT;
  size_t traj_lds = 0;
  std::vector<HostPost> hp;
  std::vector<Post> posts;
  std::vector<int4> items;
  std::vector<int3> groups;  // (C2, first item, item count) of the log-likelihood pass
  size_t total = 0;
  // byte offsets
  size_t o_posts, o_ps, o_xab, o_xbf, o_xb3, o_theta, o_grad, o_theta_t, o_p_t, o_grad_t, o_theta_n;
  size_t o_logpi, o_logpi_t, o_logw, o_h, o_l, o_H0, o_dH, o_alpha, o_ca, o_cg;
  size_t o_n, o_perm, o_active, o_anc, o_acc, o_cdf, o_gpart, o_llpart;
  size_t o_redp = 0, o_redc = 0, o_sortc = 0, o_status = 0;
  size_t o_lf_post = 0, o_lf_items = 0, o_lf_count = 0;
  size_t o_tmean = 0, o_tprec = 0;
  size_t o_items, o_colpart, o_means, o_minv, o_primes, o_sqrtp = 0, o_sobol = 0;
  FlowNet F;
  size_t o_fz = 0, o_fz0 = 0, o_fgz = 0, o_fld0 = 0, o_fld1 = 0, o_fm = 0, o_fL = 0, o_fAf = 0,
         o_fAb = 0, o_fAi = 0, o_fcov = 0, o_fLd = 0, o_fLi = 0, o_fbase = 0;
  size_t o_fp = 0, o_fpk = 0, o_fbk = 0, o_fbias = 0, o_fgrad = 0, o_fadm = 0,
         o_fadv = 0, o_ftape = 0, o_fstate = 0;
};

// Layer table of the flow: even layers transform the first floor(d/2)
// coordinates given the rest, odd layers the rest given the first ones.
bool flow_net(int d, int layers, int width, FlowNet &F) {
  // layers = 0: the base map alone (theta = m + L u, a dense mass from the
  // weighted covariance)
  if (d < 2 || d > 16 * MAX_C2 || layers < 0 || layers > FMAXL || width != FH) return false;
  memset(&F, 0, sizeof(F));
  F.L = layers;
  F.d = d;
  const int da = d / 2;
  int o = 0, half = 0;
  for (int l = 0; l < layers; ++l) {
    FlowLayerDesc &Y = F.ly[l];
    if (l % 2 == 0) {
      Y.T0 = 0, Y.dt = da, Y.C0 = da, Y.dc = d - da;
    } else {
      Y.T0 = da, Y.dt = d - da, Y.C0 = 0, Y.dc = da;
    }
    Y.oW1 = o, o += FH * Y.dc;
    Y.ob1 = o, o += FH;
    Y.oW2 = o, o += FH * FH;
    Y.ob2 = o, o += FH;
    Y.oW3 = o, o += 2 * Y.dt * FH;
    Y.ob3 = o, o += 2 * Y.dt;
    half = std::max(half, std::max(Y.dt, Y.dc));
  }
  auto c16 = [](int v) { return (v + 15) / 16 * 16; };
  int q = 0;
  for (int l = 0; l < layers; ++l) {
    FlowLayerDesc &Y = F.ly[l];
    Y.pW1 = q, q += FH * c16(Y.dc);
    Y.pW2 = q, q += FH * FH;
    Y.pW3 = q, q += c16(2 * Y.dt) * FH;
    Y.qW1 = q, q += c16(Y.dc) * FH;
    Y.qW2 = q, q += FH * FH;
    Y.qW3 = q, q += FH * c16(2 * Y.dt);
  }
  F.npacked = q;
  F.half = (half + 3) / 4 * 4;  // tape rows and offsets stay multiples of 4 floats
  F.tape_stride = 2 * FH + 2 * F.half;
  F.train_stride = 5 * F.half + 4 * FH;
  F.nparams = o;
  return true;
}

size_t take(size_t &cur, size_t bytes) {
  const size_t o = (cur + 255) & ~(size_t)255;
  cur = o + bytes;
  return o;
}

// Direction numbers of the Sobol dimensions (Bratley and Fox; Joe and Kuo)
// from the table rows (polynomial mask, m_1..m_18): for the primitive
// polynomial x^s + a_1 x^(s-1) + .. + a_(s-1) x + 1 the direction integers
// after the s given ones follow
//   m_i = 2 a_1 m_(i-1) ^ .. ^ 2^(s-1) a_(s-1) m_(i-s+1) ^ 2^s m_(i-s) ^ m_(i-s),
// and V[b] = m_(b+1) 2^(31-b) is nu_(b+1) in 32-bit fixed point.  The mask 1
// (s = 0) gives m_i = 1.  Returns false for a malformed row (even mask, degree
// above 18, an m_i even or not below 2^i); V may be NULL (validation only).
bool sobol_directions(const uint32_t *tab, int dims, uint32_t *V) {
  for (int r = 0; r < dims; ++r) {
    const uint32_t *row = tab + (size_t)r * (1 + SOBOL_MAXDEG);
    const uint32_t poly = row[0];
    if (!(poly & 1u)) return false;
    const int s = 31 - __builtin_clz(poly);
    if (s > SOBOL_MAXDEG) return false;
    uint64_t m[32];
    for (int i = 0; i < 32; ++i) {
      if (s == 0) {
        m[i] = 1;
      } else if (i < s) {
        m[i] = row[1 + i];
        if (!(m[i] & 1u) || m[i] >= (2ull << i)) return false;
      } else {
        uint64_t v = m[i - s] ^ (m[i - s] << s);
        for (int t = 1; t < s; ++t)
          if ((poly >> (s - t)) & 1u) v ^= m[i - t] << t;
        m[i] = v;
      }
    }
    if (V)
      for (int b = 0; b < 32; ++b) V[(size_t)r * 32 + b] = (uint32_t)(m[b] << (31 - b));
  }
  return true;
}

const char *check(const smc_problem *pr, const smc_params *pa) {
  if (!pr || !pa) return "null problem or params";
  if (pr->num_posteriors < 1) return "num_posteriors must be >= 1";
  if (pr->target < SMC_TARGET_LOGISTIC || pr->target > SMC_TARGET_FUNNEL) return "target";
  if (!pr->dims) return "null problem arrays";
  if (pr->target == SMC_TARGET_LOGISTIC) {
    if (!pr->n_rows || !pr->X || !pr->y) return "null problem arrays";
    for (int b = 0; b < pr->num_posteriors; ++b) {
      if (pr->n_rows[b] < 1) return "n_rows must be >= 1";
      if (pr->dims[b] < 1 || pr->dims[b] > 16 * MAX_C2) return "dims must be in [1, 208]";
      if (!pr->X[b] || !pr->y[b]) return "null X or y";
    }
    if (pr->x_dtype != SMC_F32 && pr->x_dtype != SMC_BF16) return "x_dtype";
  } else {
    if (pr->num_posteriors != 1) return "a synthetic target takes one posterior";
    if (pr->dims[0] < 1 || pr->dims[0] > 16 * MAX_C2) return "dims must be in [1, 208]";
    if (pa && (pa->precond == SMC_PRECOND_FLOW || pa->precision != SMC_PRECISION_F32))
      return "synthetic targets run FP32 trajectories without the flow preconditioner";
    if (!std::isfinite(pr->log_const)) return "log_const must be finite";
    if (pr->target == SMC_TARGET_GAUSSIAN && (!pr->mean || !pr->precision))
      return "the Gaussian target needs mean and precision";
    if (pr->target == SMC_TARGET_BANANA &&
        (pr->dims[0] != 2 || !(pr->banana_s1 > 0.0) || !std::isfinite(pr->banana_b) ||
         !std::isfinite(pr->banana_c)))
      return "the banana target needs d = 2, s1 > 0 and finite b, c";
    if (pr->target == SMC_TARGET_FUNNEL &&
        (pr->dims[0] < 2 || !(pr->funnel_scale > 0.0) || !std::isfinite(pr->funnel_scale)))
      return "the funnel target needs d >= 2 and funnel_scale > 0";
  }
  if (!(pr->prior_var > 0.0)) return "prior_var must be > 0";
  if (pa->num_particles < 1 || pa->num_particles > 65536) return "num_particles in [1, 65536]";
  if (pa->max_leapfrog < 1 || pa->max_leapfrog > MAX_NMAX) return "max_leapfrog in [1, 4096]";
  if (pa->num_warmup < 1) return "num_warmup must be >= 1";
  if (pa->jitter < SMC_JITTER_HALTON1D || pa->jitter > SMC_JITTER_SOBOLND_INV) return "jitter";
  if (pa->jitter == SMC_JITTER_SOBOLND || pa->jitter == SMC_JITTER_SOBOLND_INV) {
    if (!pa->sobol_table || pa->sobol_dims < 1 || pa->sobol_dims > SOBOL_MAXDIM)
      return "the N-d Sobol schemes need sobol_table with sobol_dims in [1, 21201]";
    if (!sobol_directions(pa->sobol_table, pa->sobol_dims, nullptr))
      return "sobol_table: a row with a bad polynomial or direction integers";
    if (pa->jitter == SMC_JITTER_SOBOLND_INV &&
        (pa->num_iterations < 1 || pa->num_iterations > pa->sobol_dims))
      return "the inverse Sobol scheme needs num_iterations in [1, sobol_dims]";
  }
  if ((pa->jitter == SMC_JITTER_HALTONND_INV || pa->jitter == SMC_JITTER_PRIMES_INV) &&
      (pa->num_iterations < 1 || pa->num_iterations > NPRIMES))
    return "the inverse jitter schemes need num_iterations in [1, 1024]";
  if (pa->jitter == SMC_JITTER_GOLDEN && pa->num_iterations < 1)
    return "the golden-ratio jitter needs num_iterations >= 1";
  if (pa->resampling < 0 || pa->resampling > 1) return "resampling";
  if (pa->precision != SMC_PRECISION_F32 && pa->precision != SMC_PRECISION_BF16) return "precision";
  if (pa->precond < 0 || pa->precond > 2) return "precond";
  if (pa->precond == SMC_PRECOND_FLOW) {
    FlowNet F;
    if (pr->num_posteriors != 1) return "the flow preconditioner takes one posterior";
    if (!flow_net(pr->dims[0], pa->flow_layers, pa->flow_width, F))
      return "flow: d >= 2, flow_layers in [0, 8], flow_width 128";
    if (pa->flow_train_steps < 0 || pa->flow_train_steps > 100000) return "flow_train_steps";
    if (!(pa->flow_lr >= 0.0)) return "flow_lr >= 0";
  }
  if (!(pa->step_size > 0.0) || !(pa->traj_length > 0.0)) return "step_size, traj_length > 0";
  if (!(pa->ess_frac >= 0.0 && pa->ess_frac <= 1.0)) return "ess_frac in [0, 1]";
  if (!(pa->adam_lr >= 0.0) || !(pa->adam_b1 >= 0.0 && pa->adam_b1 < 1.0) ||
      !(pa->adam_b2 >= 0.0 && pa->adam_b2 < 1.0) || !(pa->adam_eps > 0.0))
    return "Adam hyperparameters";
  if (!(pa->avg_decay >= 0.0 && pa->avg_decay <= 1.0)) return "avg_decay in [0, 1]";
  if (pa->adapt_step_size < SMC_ADAPT_EPS_NONE || pa->adapt_step_size > SMC_ADAPT_EPS_DUAL_AVERAGING)
    return "adapt_step_size";
  if (pa->lf_items < 0 || pa->lf_items > 4096) return "lf_items in [0, 4096]";
  if (pa->lf_split_cap < 0 || pa->lf_split_cap > LF_MAX_SPLIT) return "lf_split_cap in [0, 64]";
  return nullptr;
}

void plan(const smc_problem *pr, const smc_params *pa, Layout &L) {
  const int B = pr->num_posteriors;
  L.B = B;
  L.J = pa->num_particles;
  L.Jcap = (L.J + TJ - 1) / TJ * TJ;
  L.nmax = pa->max_leapfrog;
  int maxc2 = 1;
  long long xoff = 0, uoff = 0, xboff = 0, x3off = 0;
  const bool bf16 = pa->precision == SMC_PRECISION_BF16;
  L.hp.resize(B);
  L.posts.resize(B);
  for (int b = 0; b < B; ++b) {
    HostPost &h = L.hp[b];
    h.N = pr->target == SMC_TARGET_LOGISTIC ? pr->n_rows[b] : 0;  // no data for a synthetic target
    h.d = pr->dims[b];
    h.C2 = (h.d + 15) / 16;
    h.C1 = 4 * h.C2;
    h.NT = (h.N + 15) / 16;
    {
      const int stt = bf16_stage_tiles(h.C2);
      h.NT2 = ((h.N + 31) / 32 + stt - 1) / stt * stt;
    }
    h.KC = (h.C2 + 1) / 2;
    h.xab = xoff;
    h.xbf = xboff;
    h.xb3 = x3off;
    xoff += (long long)h.NT * 64 * (8 * h.C2 + 4);
    if (bf16) {
      xboff += (long long)h.NT2 * 64 * bf16_lane_stride(h.C2);
      x3off += (long long)h.NT2 * 64 * b3_lane_stride(h.C2);
    }
    maxc2 = std::max(maxc2, h.C2);
    Post &p = L.posts[b];
    memset(&p, 0, sizeof(p));
    p.N = h.N;
    p.d = h.d;
    p.C1 = h.C1;
    p.C2 = h.C2;
    p.NT = h.NT;
    p.row0 = b * L.Jcap;
    p.xab = h.xab;
    p.xbf = h.xbf;
    p.xb3 = h.xb3;
    p.NT2 = h.NT2;
    p.KC = h.KC;
    p.uoff = uoff;
    uoff += (long long)L.J * h.d;
  }
  // row stride: the BF16 kernel reads theta' in chunks of 32 features
  L.DS = bf16 ? 32 * ((maxc2 + 1) / 2) : 16 * maxc2;
  // leapfrog launches: lf_target items per resident 8-wave work group of a
  // compute unit (256 CUs; two groups for the FP32 kernel up to d = 128)
  // (more items per launch for the batched form measured slower: each
  // feature-tile group already gets its own launch)
  L.lf_target = pa->lf_items > 0 ? pa->lf_items : 256;
  const int ntile = L.Jcap / TJ;
  // small data sets (at most 32 data tiles per posterior): one item per
  // particle tile holds the whole gradient and finishes the step, with no
  // reduction launch
  L.nosplit = 1;
  for (int b = 0; b < B; ++b) L.nosplit &= (bf16 ? L.hp[b].NT2 : L.hp[b].NT) <= 32;
  // whole trajectories in one launch when one posterior's packed data tiles
  // fit in a work group's LDS (unless CHEES_SMC_PER_STEP=1 asks for the
  // per-step launches)
  L.traj = 0;
  if (B == 1 && pr->target == SMC_TARGET_LOGISTIC && pa->precond != SMC_PRECOND_FLOW &&
      L.hp[0].C2 <= 2) {
    const int c2 = L.hp[0].C2;
    L.traj_lds = traj_lds_bytes(c2, L.hp[0].NT);
    const size_t fixed = (size_t)TRAJ_WAVES * 16 * (16 * c2 + 1) * sizeof(float);
    const char *env = getenv("CHEES_SMC_PER_STEP");
    L.traj = L.traj_lds + fixed <= TRAJ_LDS_MAX && !(env && env[0] == '1');
  }
  L.lf_grid = L.lf_target * lf_groups_per_cu(bf16, 1) + B * ntile;
  L.split_cap = pa->lf_split_cap > 0 ? pa->lf_split_cap : LF_MAX_SPLIT;
  // log-likelihood pass: every tile, static splits, one launch per
  // feature-tile group of about lf_target items per resident work group slot
  L.items.clear();
  L.ll_smax = 1;
  // items grouped by feature-tile count C2: one launch per group covers
  // exactly its own posteriors
  L.groups.clear();
  for (int b = 0; b < B; ++b) {
    bool seen = false;
    for (const auto &g : L.groups) seen |= (g.x == L.hp[b].C2);
    if (!seen) L.groups.push_back(make_int3(L.hp[b].C2, 0, 0));
  }
  for (auto &g : L.groups) {
    g.y = (int)L.items.size();
    long long U = 0;
    for (int b = 0; b < B; ++b)
      if (L.hp[b].C2 == g.x) U += (long long)ntile * L.hp[b].NT;
    // two resident log-likelihood work groups per compute unit while the
    // staging buffers fit twice in LDS (C2 <= 9), so twice the items
    const long long items = (long long)L.lf_target * (g.x <= 9 ? 2 : 1);
    const long long chunk = std::max(1LL, (U + items - 1) / items);
    for (int b = 0; b < B; ++b) {
      if (L.hp[b].C2 != g.x) continue;
      long long S = (L.hp[b].NT + chunk - 1) / chunk;
      S = std::max(1LL, std::min<long long>(S, L.hp[b].NT));
      L.posts[b].ll_splits = (int)S;
      L.posts[b].ll_base = (int)L.items.size();
      L.ll_smax = std::max(L.ll_smax, (int)S);
      for (int t = 0; t < ntile; ++t)
        for (int s = 0; s < S; ++s) L.items.push_back(make_int4(b, t, s, 0));
    }
    g.z = (int)L.items.size() - g.y;
  }
  L.ll_nitems = (int)L.items.size();
  L.col_chunks = std::max(1, std::min(64, (L.J + 127) / 128));

  const size_t rows = (size_t)B * L.Jcap, st = rows * L.DS * sizeof(float);
  size_t c = 0;
  L.o_posts = take(c, B * sizeof(Post));
  L.o_ps = take(c, B * sizeof(PState));
  L.o_xab = take(c, xoff * sizeof(float));
  L.o_xbf = take(c, xboff * 16);
  L.o_xb3 = take(c, x3off * 16);
  L.o_theta = take(c, st);
  L.o_grad = take(c, st);
  L.o_theta_t = take(c, st);
  L.o_theta_n = take(c, st);
  L.o_p_t = take(c, st);
  L.o_grad_t = take(c, st);
  L.o_logpi = take(c, rows * 8);
  L.o_logpi_t = take(c, rows * 8);
  L.o_logw = take(c, rows * 8);
  L.o_h = take(c, rows * 8);
  L.o_l = take(c, rows * 8);
  L.o_H0 = take(c, rows * 8);
  L.o_dH = take(c, rows * 8);
  L.o_alpha = take(c, rows * 8);
  L.o_ca = take(c, rows * 8);
  L.o_cg = take(c, rows * 8);
  L.o_n = take(c, rows * 4);
  L.o_perm = take(c, rows * 4);
  L.o_active = take(c, (size_t)B * (L.nmax + 1) * 4);
  L.o_lf_post = take(c, (size_t)L.nmax * B * sizeof(int4));
  L.o_lf_items = take(c, L.groups.size() * (size_t)L.nmax * L.lf_grid * sizeof(int4));
  L.o_lf_count = take(c, L.groups.size() * (size_t)L.nmax * sizeof(int));
  L.o_anc = take(c, rows * 4);
  L.o_acc = take(c, rows * 4);
  L.o_cdf = take(c, rows * 8);
  L.o_redp = take(c, (size_t)B * RED_G * 4 * sizeof(double));
  L.o_redc = take(c, (size_t)B * 2 * sizeof(int));
  L.o_status = take(c, 256);
  L.o_sortc = take(c, (size_t)B * ((L.Jcap + 1023) / 1024) * 256 * sizeof(int));
  // partial gradients: each feature-tile group owns the slots of its largest
  // launch, so one reduction per step serves every group
  L.gpart_slots = 0;
  for (size_t g = 0; g < L.groups.size(); ++g) {
    int Bg = 0;
    for (int b = 0; b < B; ++b) Bg += L.hp[b].C2 == L.groups[g].x;
    L.goff[g] = L.gpart_slots;
    L.gpart_slots += L.lf_target * lf_groups_per_cu(bf16, L.groups[g].x) + Bg * ntile;
  }
  L.o_gpart = take(c, (size_t)L.gpart_slots * TJ * L.DS * sizeof(float));

  L.o_llpart = take(c, (size_t)L.ll_smax * rows * sizeof(float2));
  L.o_items = take(c, (size_t)L.ll_nitems * sizeof(int4));
  L.o_colpart = take(c, (size_t)B * L.col_chunks * 2 * L.DS * 8);
  L.o_means = take(c, (size_t)B * 2 * L.DS * 8);
  L.o_minv = take(c, (size_t)B * L.DS * 4);
  L.o_tmean = take(c, (size_t)L.DS * 4);
  L.o_tprec = take(c, pr->target == SMC_TARGET_GAUSSIAN ? (size_t)L.DS * L.DS * 4 : 4);
  L.o_primes = take(c, NPRIMES * 4);
  L.o_sqrtp = take(c, NPRIMES * 8);
  const bool sobol = pa->jitter == SMC_JITTER_SOBOLND || pa->jitter == SMC_JITTER_SOBOLND_INV;
  L.o_sobol = take(c, sobol ? (size_t)pa->sobol_dims * 32 * 4 : 4);
  if (pa->precond == SMC_PRECOND_FLOW) {
    flow_net(pr->dims[0], pa->flow_layers, pa->flow_width, L.F);
    L.F.ntrain = L.F.L > 0 ? pa->flow_train_steps : 0;  // nothing to fit without couplings
    L.F.lr = (float)pa->flow_lr;
    const size_t np = (size_t)L.F.nparams;
    L.o_fz = take(c, st);
    L.o_fz0 = take(c, st);
    L.o_fgz = take(c, st);
    L.o_fld0 = take(c, rows * 4);
    L.o_fld1 = take(c, rows * 4);
    const size_t dd = (size_t)pr->dims[0] * pr->dims[0];
    const size_t d16 = (size_t)((pr->dims[0] + 15) / 16 * 16);
    L.o_fm = take(c, (size_t)L.DS * 4);
    L.o_fL = take(c, dd * 4);
    L.o_fAf = take(c, d16 * d16 * 4);
    L.o_fAb = take(c, d16 * d16 * 4);
    L.o_fAi = take(c, d16 * d16 * 4);
    L.o_fcov = take(c, (size_t)FCOV_CH * dd * 8);
    L.o_fLd = take(c, dd * 8);
    L.o_fLi = take(c, dd * 8);
    L.o_fbase = take(c, 256);
    L.o_fp = take(c, np * 4);
    L.o_fpk = take(c, (size_t)L.F.npacked * 4);
    L.o_fbk = take(c, (size_t)L.F.npacked * 4);
    L.o_fbias = take(c, np * 4);
    L.o_fgrad = take(c, (size_t)FKSPLIT * np * 4);
    L.o_fadm = take(c, np * 4);
    L.o_fadv = take(c, np * 4);
    L.o_ftape = take(c, rows * std::max(L.F.L, 1) * std::max(L.F.tape_stride, L.F.train_stride) * 4);
    L.o_fstate = take(c, 256);
  }
  L.total = (c + 255) & ~(size_t)255;
}

std::vector<int> first_primes(int n) {
  std::vector<int> p;
  for (int c = 2; (int)p.size() < n; ++c) {
    bool ok = true;
    for (int q : p) {
      if (q * q > c) break;
      if (c % q == 0) {
        ok = false;
        break;
      }
    }
    if (ok) p.push_back(c);
  }
  return p;
}

#define CK(call)                                                                     \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess) {                                                          \
      ctx->err = std::string(#call) + ": " + hipGetErrorString(e_);                   \
      return SMC_EDEVICE;                                                            \
    }                                                                                \
  } while (0)

smc_status fill_stats(smc_ctx *ctx, smc_stats *stats) {
  CK(hipMemcpyAsync(ctx->ps_host.data(), ctx->D.ps, ctx->D.B * sizeof(PState),
                    hipMemcpyDeviceToHost, ctx->st));
  CK(hipStreamSynchronize(ctx->st));
  const PState &S = ctx->ps_host[0];
  stats->ess = S.ess;
  stats->ess_before = S.ess_before;
  stats->mean_accept = S.sum_alpha_all / ctx->D.J;
  stats->chees = S.chees;
  stats->chees_grad = S.ghat;
  stats->L = S.L_used;
  stats->eps = S.eps_used;
  stats->log_z = S.log_c + S.m + log(S.S);
  stats->resampled = S.resampled;
  stats->iteration = S.k;
  stats->grad_evals = S.grad_evals_step;
  for (int b = 0; b < ctx->D.B; ++b)
    if (ctx->ps_host[b].degenerate) {
      ctx->err = "degenerate weights";
      return SMC_EDEGENERATE;
    }
  return SMC_OK;
}

}  // namespace

extern "C" {

size_t smc_workspace_bytes(const smc_problem *prob, const smc_params *par) {
  if (check(prob, par)) return 0;
  Layout L;
  plan(prob, par, L);
  return L.total;
}

smc_status smc_init(const smc_problem *prob, const smc_params *par, void *workspace,
                    size_t workspace_bytes, void *hip_stream, const float *theta0,
                    smc_ctx **out) {
  if (!out) return SMC_EINVAL;
  *out = nullptr;
  if (const char *why = check(prob, par)) {
    fprintf(stderr, "smc_init: %s\n", why);
    return SMC_EINVAL;
  }
  Layout L;
  plan(prob, par, L);
  if (!workspace || workspace_bytes < L.total) return SMC_ENOMEM;
  if (((uintptr_t)workspace & 255) != 0) return SMC_EINVAL;

  smc_ctx *ctx = new smc_ctx();
  ctx->st = (hipStream_t)hip_stream;
  char *w = (char *)workspace;
  Dev &D = ctx->D;
  memset(&D, 0, sizeof(D));
  D.B = L.B;
  D.J = L.J;
  D.Jcap = L.Jcap;
  D.DS = L.DS;
  D.nmax = L.nmax;
  D.jitter = par->jitter;
  D.jit_K = par->num_iterations;
  D.golden = (std::sqrt(5.0) - 1.0) / 2.0;
  D.mh = par->mh_accept ? 1 : 0;
  D.resampling = par->resampling;
  D.precond = par->precond;
  D.prior_var = prob->prior_var;
  D.ess_frac = par->ess_frac;
  D.adam_lr = par->adam_lr;
  D.adam_b1 = par->adam_b1;
  D.adam_b2 = par->adam_b2;
  D.adam_eps = par->adam_eps;
  D.avg_decay = par->avg_decay;
  D.target_accept = par->target_accept;
  D.adapt_eps = par->adapt_step_size;
  D.num_warmup = par->num_warmup;
  D.seed = par->seed;
  D.posts = (Post *)(w + L.o_posts);
  D.ps = (PState *)(w + L.o_ps);
  D.xab = (float *)(w + L.o_xab);
  D.xbf = (uint4 *)(w + L.o_xbf);
  D.xb3 = (uint4 *)(w + L.o_xb3);
  D.bf16 = par->precision == SMC_PRECISION_BF16 ? 1 : 0;
  D.status = (int *)(w + L.o_status);
  D.theta = (float *)(w + L.o_theta);
  D.grad = (float *)(w + L.o_grad);
  D.theta_t = (float *)(w + L.o_theta_t);
  D.theta_n = (float *)(w + L.o_theta_n);
  D.p_t = (float *)(w + L.o_p_t);
  D.grad_t = (float *)(w + L.o_grad_t);
  D.logpi = (double *)(w + L.o_logpi);
  D.logpi_t = (double *)(w + L.o_logpi_t);
  D.logw = (double *)(w + L.o_logw);
  D.h = (double *)(w + L.o_h);
  D.l = (double *)(w + L.o_l);
  D.H0 = (double *)(w + L.o_H0);
  D.dH = (double *)(w + L.o_dH);
  D.alpha = (double *)(w + L.o_alpha);
  D.ca = (double *)(w + L.o_ca);
  D.cg = (double *)(w + L.o_cg);
  D.n = (int *)(w + L.o_n);
  D.perm = (int *)(w + L.o_perm);
  D.active = (int *)(w + L.o_active);
  D.lf_post = (int4 *)(w + L.o_lf_post);
  D.lf_items = (int4 *)(w + L.o_lf_items);
  D.lf_count = (int *)(w + L.o_lf_count);
  D.ngroups = (int)L.groups.size();
  for (int c2 = 0; c2 <= MAX_C2; ++c2) D.c2_group[c2] = 0;
  for (int g = 0; g < D.ngroups; ++g) {
    D.group_c2[g] = L.groups[g].x;
    D.c2_group[L.groups[g].x] = g;
    D.lf_goff[g] = L.goff[g];
  }
  D.anc = (int *)(w + L.o_anc);
  D.accepted = (int *)(w + L.o_acc);
  D.cdf = (unsigned long long *)(w + L.o_cdf);
  D.red_part = (double *)(w + L.o_redp);
  D.red_cnt = (int *)(w + L.o_redc);
  D.sort_cnt = (int *)(w + L.o_sortc);
  D.sort_chunks = (L.Jcap + 1023) / 1024;
  D.gpart = (float *)(w + L.o_gpart);
  D.gpart_slots = L.gpart_slots;
  D.lf_nosplit = L.nosplit;
  D.traj = L.traj;
  D.traj_lds = L.traj_lds;
  D.llpart = (float2 *)(w + L.o_llpart);
  D.ll_smax = L.ll_smax;
  D.ll_items = (int4 *)(w + L.o_items);
  D.ll_nitems = L.ll_nitems;
  D.colpart = (double *)(w + L.o_colpart);
  D.col_chunks = L.col_chunks;
  D.means = (double *)(w + L.o_means);
  D.minv = (float *)(w + L.o_minv);
  D.tmean = (float *)(w + L.o_tmean);
  D.tprec = (float *)(w + L.o_tprec);
  D.target = prob->target;
  D.bs1 = prob->banana_s1;
  D.bb = prob->banana_b;
  D.bc = prob->banana_c;
  D.fsv = prob->funnel_scale;
  D.tconst = prob->log_const;
  D.primes = (int *)(w + L.o_primes);
  D.sqrtp = (double *)(w + L.o_sqrtp);
  D.sobol = (uint32_t *)(w + L.o_sobol);
  D.sobol_dims =
      (par->jitter == SMC_JITTER_SOBOLND || par->jitter == SMC_JITTER_SOBOLND_INV) ? par->sobol_dims
                                                                                    : 0;
  D.lf_target = L.lf_target;
  D.split_cap = L.split_cap;
  D.lf_grid = L.lf_grid;
  D.flow = par->precond == SMC_PRECOND_FLOW ? 1 : 0;
  if (D.flow) {
    D.fz = (float *)(w + L.o_fz);
    D.fz0 = (float *)(w + L.o_fz0);
    D.fgz = (float *)(w + L.o_fgz);
    D.fld0 = (float *)(w + L.o_fld0);
    D.fld1 = (float *)(w + L.o_fld1);
    D.fm = (float *)(w + L.o_fm);
    D.fL = (float *)(w + L.o_fL);
    D.fAf = (float *)(w + L.o_fAf);
    D.fAb = (float *)(w + L.o_fAb);
    D.fAi = (float *)(w + L.o_fAi);
    D.fcov = (double *)(w + L.o_fcov);
    D.fLd = (double *)(w + L.o_fLd);
    D.fLi = (double *)(w + L.o_fLi);
    D.fbase = (float *)(w + L.o_fbase);
    D.fp = (float *)(w + L.o_fp);
    D.fpk = (float *)(w + L.o_fpk);
    D.fbk = (float *)(w + L.o_fbk);
    D.fbias = (float *)(w + L.o_fbias);
    D.fgrad = (float *)(w + L.o_fgrad);
    D.fadm = (float *)(w + L.o_fadm);
    D.fadv = (float *)(w + L.o_fadv);
    D.ftape = (float *)(w + L.o_ftape);
    D.fstate = (int *)(w + L.o_fstate);
  }
  ctx->F = L.F;

  ctx->hp = L.hp;
  ctx->posts = L.posts;
  ctx->ll_items = L.items;
  ctx->ll_groups = L.groups;
  for (const int3 &g : L.groups) ctx->c2s.push_back(g.x);
  {
    // lanes of the groups: work ~ sum over the group's posteriors of data
    // tiles x feature tiles; largest first onto the least loaded lane
    const int ng = (int)ctx->c2s.size();
    std::vector<double> work(ng, 0.0), load(MAX_SIDE + 1, 0.0);
    for (const HostPost &h : L.hp)
      for (int g = 0; g < ng; ++g)
        if (ctx->c2s[g] == h.C2) work[g] += (double)h.NT * h.C2;
    std::vector<int> idx(ng);
    for (int g = 0; g < ng; ++g) idx[g] = g;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return work[a] > work[b]; });
    ctx->group_lane.assign(ng, 0);
    for (int g : idx) {
      const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      ctx->group_lane[g] = l;
      load[l] += work[g];
    }
  }
  ctx->primes = first_primes(NPRIMES);
  ctx->sqrtp.resize(NPRIMES);
  for (int i = 0; i < NPRIMES; ++i) ctx->sqrtp[i] = std::sqrt((double)ctx->primes[i]);
  ctx->minv.assign((size_t)L.B * L.DS, 1.0f);
  ctx->ps_host.resize(L.B);
  for (PState &s : ctx->ps_host) {
    memset(&s, 0, sizeof(s));
    s.L = par->traj_length;
    s.eps = par->step_size;
    s.da_mu = std::log(10.0 * par->step_size);
    s.adapted_k = 0;
  }

  smc_status rc = SMC_OK;
  auto fail = [&](smc_status r) {
    fprintf(stderr, "smc_init: %s\n", ctx->err.c_str());
    delete ctx;
    return r;
  };
#define CKI(call)                                                                    \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess) {                                                          \
      ctx->err = std::string(#call) + ": " + hipGetErrorString(e_);                   \
      return fail(SMC_EDEVICE);                                                      \
    }                                                                                \
  } while (0)
  CKI(fill_i32((int *)w, (long long)(L.total / 4), 0, ctx->st));
  if (ctx->c2s.size() > 1) {  // side streams for the group launches, default priority
    for (int i = 0; i < MAX_SIDE; ++i) {
      CKI(hipStreamCreateWithFlags(&ctx->side[i], hipStreamNonBlocking));
      CKI(hipEventCreateWithFlags(&ctx->join_ev[i], hipEventDisableTiming));
    }
    CKI(hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming));
  }
  CKI(hipMemcpyAsync(D.posts, ctx->posts.data(), L.B * sizeof(Post), hipMemcpyHostToDevice,
                     ctx->st));
  CKI(hipMemcpyAsync(D.ps, ctx->ps_host.data(), L.B * sizeof(PState), hipMemcpyHostToDevice,
                     ctx->st));
  CKI(hipMemcpyAsync(D.primes, ctx->primes.data(), NPRIMES * sizeof(int), hipMemcpyHostToDevice,
                     ctx->st));
  CKI(hipMemcpyAsync(D.sqrtp, ctx->sqrtp.data(), NPRIMES * sizeof(double), hipMemcpyHostToDevice,
                     ctx->st));
  if (D.sobol_dims > 0) {
    ctx->sobol.resize((size_t)D.sobol_dims * 32);
    sobol_directions(par->sobol_table, D.sobol_dims, ctx->sobol.data());
    CKI(hipMemcpyAsync(D.sobol, ctx->sobol.data(), ctx->sobol.size() * sizeof(uint32_t),
                       hipMemcpyHostToDevice, ctx->st));
  }
  CKI(hipMemcpyAsync(D.minv, ctx->minv.data(), ctx->minv.size() * sizeof(float),
                     hipMemcpyHostToDevice, ctx->st));
  CKI(hipMemcpyAsync(D.ll_items, ctx->ll_items.data(), ctx->ll_items.size() * sizeof(int4),
                     hipMemcpyHostToDevice, ctx->st));
  if (D.target == SMC_TARGET_GAUSSIAN) {
    // log N(theta; mu, P^{-1}) = 1/2 log det P - d/2 log 2 pi - 1/2 q: log det P
    // from a binary64 Cholesky factorisation of the FP32 precision
    const int d = L.hp[0].d;
    std::vector<float> P((size_t)d * d);
    CKI(hipMemcpyAsync(P.data(), prob->precision, P.size() * sizeof(float), hipMemcpyDeviceToHost,
                       ctx->st));
    CKI(hipStreamSynchronize(ctx->st));
    std::vector<double> Lc((size_t)d * d, 0.0);
    double logdet = 0.0;
    for (int i = 0; i < d; ++i)
      for (int j = 0; j <= i; ++j) {
        double v = P[(size_t)i * d + j];
        for (int k = 0; k < j; ++k) v -= Lc[(size_t)i * d + k] * Lc[(size_t)j * d + k];
        if (i == j) {
          if (!(v > 0.0)) {
            ctx->err = "the Gaussian precision is not positive definite";
            return fail(SMC_EINVAL);
          }
          Lc[(size_t)i * d + i] = std::sqrt(v);
          logdet += 2.0 * std::log(Lc[(size_t)i * d + i]);
        } else {
          Lc[(size_t)i * d + j] = v / Lc[(size_t)j * d + j];
        }
      }
    D.tconst = prob->log_const + 0.5 * logdet - 0.5 * d * std::log(2.0 * M_PI);
    CKI(launch_target_pack(D, prob->mean, prob->precision, d, ctx->st));
  }
  if (!D.target)
    for (int b = 0; b < L.B; ++b) {
      CKI(launch_pack_one(D, prob->X[b], prob->y[b], prob->x_dtype, L.hp[b], ctx->st));
      if (D.bf16) CKI(launch_pack_bf16(D, prob->X[b], prob->y[b], prob->x_dtype, L.hp[b], ctx->st));
    }
  CKI(launch_init_theta(D, theta0, ctx->st));
  if (D.target) {
    CKI(launch_target_step(D, 0, 1, ctx->st));
    CKI(launch_target_energy(D, ctx->st));
  } else {
    CKI(launch_lf_plan(D, ctx->st));
    for (int c2 : ctx->c2s) CKI(launch_lf_partial(D, c2, 0, 1, ctx->st));
    if (!D.lf_nosplit) CKI(launch_lf_reduce(D, 0, 1, ctx->st));
    for (const int3 &g : ctx->ll_groups) CKI(launch_loglik(D, g.x, g.y, g.z, ctx->st));
  }
  CKI(launch_init_weights(D, ctx->st));
  CKI(launch_ess(D, 0, ctx->st));
  if (D.flow) CKI(launch_flow_init(D, ctx->F, ctx->st));
  // the host copies above must stay alive until they have run
  int status = 0;
  CKI(hipMemcpyAsync(&status, D.status, sizeof(int), hipMemcpyDeviceToHost, ctx->st));
  CKI(hipStreamSynchronize(ctx->st));
  if (status) {
    ctx->err = "the BF16 precision form needs labels y in {0, 1}";
    return fail(SMC_EINVAL);
  }
  (void)rc;
  *out = ctx;
  return SMC_OK;
#undef CKI
}

namespace {
// Record an event pair around a launch when timing is on.
hipError_t timed_begin(smc_ctx *ctx, int kind, size_t &idx) {
  if (!ctx->timing) return hipSuccess;
  while (ctx->ev_pool.size() < ctx->ev_used + 2) {
    hipEvent_t e;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return r;
    ctx->ev_pool.push_back(e);
  }
  idx = ctx->ev_used;
  ctx->ev_used += 2;
  ctx->ev_marks.push_back({kind, idx});
  return hipEventRecord(ctx->ev_pool[idx], ctx->st);
}
hipError_t timed_end(smc_ctx *ctx, size_t idx) {
  if (!ctx->timing) return hipSuccess;
  return hipEventRecord(ctx->ev_pool[idx + 1], ctx->st);
}
// Launches fn(g, stream) for the feature-tile groups g = 0 .. n-1.  With one
// group, or with per-launch timing (events on the context's stream), in order
// on the context's stream; otherwise group g on lane g mod 4, lane 0 the
// context's stream and lanes 1..3 side streams forked from it and joined
// back into it afterwards (graph edges under capture).  The groups write
// disjoint memory, so the results do not depend on how they overlap.
extern "C++" template <typename Fn>
hipError_t for_groups(smc_ctx *ctx, int n, Fn fn) {
  if (n == 1 || ctx->timing || !ctx->fork_ev) {
    for (int g = 0; g < n; ++g) {
      const hipError_t e = fn(g, ctx->st);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  const int lanes = std::min(n, MAX_SIDE + 1);
  hipError_t e = hipEventRecord(ctx->fork_ev, ctx->st);
  for (int i = 1; i < lanes && e == hipSuccess; ++i)
    e = hipStreamWaitEvent(ctx->side[i - 1], ctx->fork_ev, 0);
  for (int g = 0; g < n && e == hipSuccess; ++g) {
    const int l = (int)ctx->group_lane.size() == n ? ctx->group_lane[g] % lanes : g % lanes;
    e = fn(g, l == 0 ? ctx->st : ctx->side[l - 1]);
  }
  for (int i = 1; i < lanes && e == hipSuccess; ++i) {
    e = hipEventRecord(ctx->join_ev[i - 1], ctx->side[i - 1]);
    if (e == hipSuccess) e = hipStreamWaitEvent(ctx->st, ctx->join_ev[i - 1], 0);
  }
  return e;
}
}  // namespace

namespace {
// Every launch of one smc_step (no host synchronisation, no memset, no copy).
// nl: leapfrog launches (n_max, or fewer when no trajectory can be longer).
smc_status enqueue_step(smc_ctx *ctx, const smc_inject *inject, int nl) {
  const Dev &D = ctx->D;
  size_t ei = 0;
  CK(launch_begin_step(D, 1, inject ? inject->resample_u : nullptr, 1, ctx->st));
  CK(launch_gather(D, nullptr, ctx->st));
  if (D.precond == SMC_PRECOND_DIAG) CK(launch_mass(D, 1, ctx->st));
  const FlowNet &F = ctx->F;
  if (D.flow) {
    // standardise the pre-move population, then fit the couplings to it
    CK(launch_mass(D, 0, ctx->st));
    CK(launch_flow_base(D, F, ctx->st));
    for (int i = 0; i < F.ntrain; ++i) {
      CK(timed_begin(ctx, 4, ei));
      CK(launch_flow_train(D, F, i, ctx->st));
      CK(timed_end(ctx, ei));
    }
  }
  CK(launch_setup(D, inject ? inject->momenta : nullptr, 0, ctx->st));
  if (D.flow) CK(launch_flow_begin(D, F, ctx->st));
  CK(launch_sort(D, ctx->st));
  if (D.target) {
    // synthetic target: one fused drift / gradient / kick launch per step
    for (int s = 0; s < nl; ++s) {
      CK(timed_begin(ctx, 0, ei));
      CK(launch_target_step(D, s, 0, ctx->st));
      CK(timed_end(ctx, ei));
    }
    CK(timed_begin(ctx, 1, ei));
    CK(launch_target_energy(D, ctx->st));
    CK(timed_end(ctx, ei));
  } else if (D.traj) {
    CK(timed_begin(ctx, 0, ei));
    CK(launch_traj(D, ctx->c2s[0], ctx->st));
    CK(timed_end(ctx, ei));
  } else {
    CK(launch_lf_plan(D, ctx->st));
  }
  const bool lanes = ctx->c2s.size() > 1 && !ctx->timing && ctx->fork_ev && !D.target &&
                     !D.traj && !D.flow;
  if (lanes) {
    // several feature-tile groups: each group's trajectories (step launches
    // and its own reductions) run on a stream lane of their own, joined once
    // after the last step
    CK(for_groups(ctx, (int)ctx->c2s.size(), [&](int g, hipStream_t stream) {
      hipError_t e = hipSuccess;
      for (int s = 0; s < nl && e == hipSuccess; ++s) {
        e = launch_lf_partial(D, ctx->c2s[g], s, 0, stream);
        if (e == hipSuccess && !D.lf_nosplit) e = launch_lf_reduce(D, s, 0, stream, ctx->c2s[g]);
      }
      return e;
    }));
  }
  for (int s = 0; s < (D.target || D.traj || lanes ? 0 : nl); ++s) {
    if (D.flow && s == 0) {  // one posterior, one group; later drifts join the kicks
      CK(timed_begin(ctx, 3, ei));
      CK(launch_flow_drift(D, F, s, ctx->st));
      CK(timed_end(ctx, ei));
    }
    CK(for_groups(ctx, (int)ctx->c2s.size(), [&](int g, hipStream_t stream) {
      hipError_t e = timed_begin(ctx, 0, ei);
      if (e == hipSuccess) e = launch_lf_partial(D, ctx->c2s[g], s, D.flow ? 2 : 0, stream);
      if (e == hipSuccess) e = timed_end(ctx, ei);
      return e;
    }));
    // one reduction for all groups (disjoint partial slots), unless every tile
    // is one item that finished its own step
    if (!D.lf_nosplit) {
      CK(timed_begin(ctx, 2, ei));
      CK(launch_lf_reduce(D, s, D.flow ? 2 : 0, ctx->st));
      CK(timed_end(ctx, ei));
    }
    if (D.flow) {
      CK(timed_begin(ctx, 3, ei));
      CK(s + 1 < nl ? launch_flow_kick_drift(D, F, s, ctx->st) : launch_flow_kick(D, F, s, ctx->st));
      CK(timed_end(ctx, ei));
    }
  }
  if (!D.target)
    CK(for_groups(ctx, (int)ctx->ll_groups.size(), [&](int i, hipStream_t stream) {
      const int3 &g = ctx->ll_groups[i];
      hipError_t e = timed_begin(ctx, 1, ei);
      if (e == hipSuccess) e = launch_loglik(D, g.x, g.y, g.z, stream);
      if (e == hipSuccess) e = timed_end(ctx, ei);
      return e;
    }));
  CK(launch_weights(D, inject ? inject->mh_uniforms : nullptr, 0, ctx->st));
  CK(launch_chees(D, ctx->st));
  CK(launch_commit(D, ctx->st));
  CK(launch_ess(D, 1, ctx->st));
  return SMC_OK;
}
}  // namespace

namespace {
// Capture one iteration (step with nl leapfrog launches, then the adaptation)
// on a private stream; kernel arguments are fixed for the life of the
// context, so the graph stays valid.
smc_status capture_iteration(smc_ctx *ctx, int nl, hipGraph_t *graph, hipGraphExec_t *gexec) {
  if (!ctx->cap_st) CK(hipStreamCreateWithFlags(&ctx->cap_st, hipStreamNonBlocking));
  const hipStream_t user = ctx->st;
  const int timing = ctx->timing;
  ctx->st = ctx->cap_st;
  ctx->timing = 0;
  hipError_t e = hipStreamBeginCapture(ctx->cap_st, hipStreamCaptureModeThreadLocal);
  smc_status r = SMC_EDEVICE;
  if (e == hipSuccess) {
    r = enqueue_step(ctx, nullptr, nl);
    if (r == SMC_OK && launch_adapt(ctx->D, ctx->cap_st) != hipSuccess) r = SMC_EDEVICE;
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(ctx->cap_st, &g);
    if (e == hipSuccess && r == SMC_OK) {
      e = hipGraphInstantiate(gexec, g, nullptr, nullptr, 0);
      if (e == hipSuccess) *graph = g;
    }
    if (e != hipSuccess || r != SMC_OK) {
      if (g) (void)hipGraphDestroy(g);
      *gexec = nullptr;
    }
  }
  ctx->st = user;
  ctx->timing = timing;
  if (e != hipSuccess) {
    ctx->err = std::string("graph capture of an iteration: ") + hipGetErrorString(e);
    return SMC_EDEVICE;
  }
  return r;
}

void drop_bounded(smc_ctx *ctx) {
  if (ctx->gexec_b) (void)hipGraphExecDestroy(ctx->gexec_b);
  if (ctx->graph_b) (void)hipGraphDestroy(ctx->graph_b);
  ctx->gexec_b = nullptr;
  ctx->graph_b = nullptr;
  ctx->nl_b = 0;
  ctx->frozen = 0;
}

// Once every posterior's adaptation has ended (its last adaptation ran at
// iteration k >= num_warmup), L and eps no longer change: each n_j =
// min(max(ceil(h_j L / eps), 1), n_max) with h_j <= h_max is at most
// min(max(ceil(h_max L / eps), 1), n_max) (binary64 rounding is monotone), and
// later leapfrog launches would find no active particle.  One synchronisation
// reads L and eps and sets nl_b (smc_run then captures a graph with that many
// launches; smc_step launches that many).
smc_status freeze_bound(smc_ctx *ctx) {
  const Dev &D = ctx->D;
  CK(hipMemcpyAsync(ctx->ps_host.data(), D.ps, D.B * sizeof(PState), hipMemcpyDeviceToHost,
                    ctx->st));
  CK(hipStreamSynchronize(ctx->st));
  const double hmax = D.jitter == 9 ? 1.0 + 0.1 : 1.0;  // scheme 9 adds 0.1 u to (y + 1) / J
  int nl = 1;
  for (int b = 0; b < D.B; ++b) {
    const PState &S = ctx->ps_host[b];
    if (S.adapted_k < D.num_warmup) return SMC_OK;  // still adapting: keep the full graph
    double nn = ceil(hmax * S.L / S.eps);
    nn = fmin(fmax(nn, 1.0), (double)D.nmax);
    nl = std::max(nl, (int)nn);
  }
  ctx->frozen = 1;
  ctx->nl_b = nl;
  return SMC_OK;
}

// Leapfrog launches of the next iteration: n_max until the adaptation has
// ended, then the bound (checked once, when the iteration count first
// reaches num_warmup with no step pending).
smc_status launch_count(smc_ctx *ctx, int *nl) {
  if (!ctx->frozen && !ctx->stepped && ctx->steps >= ctx->D.num_warmup) {
    const smc_status r = freeze_bound(ctx);
    if (r != SMC_OK) return r;
  }
  *nl = ctx->frozen ? ctx->nl_b : ctx->D.nmax;
  return SMC_OK;
}
}  // namespace

smc_status smc_step(smc_ctx *ctx, const smc_inject *inject, smc_stats *stats) {
  if (!ctx) return SMC_EINVAL;
  int nl = ctx->D.nmax;
  smc_status r = launch_count(ctx, &nl);
  if (r != SMC_OK) return r;
  r = enqueue_step(ctx, inject, nl);
  if (r != SMC_OK) return r;
  ctx->stepped = 1;
  ctx->steps += 1;
  if (stats) return fill_stats(ctx, stats);
  return SMC_OK;
}

smc_status smc_run(smc_ctx *ctx, int32_t iterations) {
  if (!ctx || iterations < 0) return SMC_EINVAL;
  if (ctx->stepped) {
    ctx->err = "smc_run after a smc_step that was not followed by chees_adapt";
    return SMC_ESTATE;
  }
  if (!ctx->gexec) {
    smc_status r = capture_iteration(ctx, ctx->D.nmax, &ctx->graph, &ctx->gexec);
    if (r != SMC_OK) return r;
  }
  int left = iterations;
  while (left > 0) {
    if (!ctx->frozen) {
      // iterations whose adaptation may still move L or eps (iteration k adapts
      // while k <= num_warmup; ctx->steps iterations have run)
      const int adapting = ctx->D.num_warmup - ctx->steps;
      if (adapting > 0) {
        const int n = std::min(left, adapting);
        for (int i = 0; i < n; ++i) CK(hipGraphLaunch(ctx->gexec, ctx->st));
        ctx->steps += n;
        left -= n;
        continue;
      }
    }
    int nl = ctx->D.nmax;
    smc_status r = launch_count(ctx, &nl);
    if (r != SMC_OK) return r;
    if (nl < ctx->D.nmax && !ctx->gexec_b) {
      r = capture_iteration(ctx, nl, &ctx->graph_b, &ctx->gexec_b);
      if (r != SMC_OK) return r;
    }
    // without a bound (adaptation not ended on the device: a restored or
    // re-parameterised state) the full graph runs
    hipGraphExec_t g = nl < ctx->D.nmax ? ctx->gexec_b : ctx->gexec;
    for (int i = 0; i < left; ++i) CK(hipGraphLaunch(g, ctx->st));
    ctx->steps += left;
    left = 0;
  }
  return SMC_OK;
}

smc_status chees_adapt(smc_ctx *ctx, smc_stats *stats) {
  if (!ctx) return SMC_EINVAL;
  if (!ctx->stepped) {
    ctx->err = "chees_adapt needs a step since the last adaptation";
    return SMC_ESTATE;
  }
  CK(launch_adapt(ctx->D, ctx->st));
  ctx->stepped = 0;
  if (stats) {
    smc_status r = fill_stats(ctx, stats);
    stats->L = ctx->ps_host[0].L;
    stats->eps = ctx->ps_host[0].eps;
    return r;
  }
  return SMC_OK;
}

smc_status resample(smc_ctx *ctx, const double *u, int32_t *ancestors_out) {
  if (!ctx) return SMC_EINVAL;
  const Dev &D = ctx->D;
  CK(launch_begin_step(D, 0, u, 0, ctx->st));
  CK(launch_gather(D, ancestors_out, ctx->st));
  CK(launch_setup(D, nullptr, 2, ctx->st));
  CK(launch_ess(D, 0, ctx->st));
  return SMC_OK;
}

size_t resample_workspace_bytes(int32_t J) {
  if (J < 1 || J > (1 << 24)) return 0;
  return ((size_t)J * 8 + 255) / 256 * 256 + 256;
}

smc_status resample_indices(const double *w, int32_t J, const double *u, int32_t scheme,
                            int32_t *ancestors, void *workspace, size_t workspace_bytes,
                            void *hip_stream) {
  if (!w || !u || !ancestors || !workspace || J < 1 || J > (1 << 24) ||
      (scheme != SMC_RESAMPLE_SYSTEMATIC && scheme != SMC_RESAMPLE_MULTINOMIAL))
    return SMC_EINVAL;
  if (workspace_bytes < resample_workspace_bytes(J)) return SMC_ENOMEM;
  hipStream_t st = (hipStream_t)hip_stream;
  unsigned long long *cdf = (unsigned long long *)workspace;
  int *err = (int *)((char *)workspace + ((size_t)J * 8 + 255) / 256 * 256);
  if (launch_resample_indices(w, J, u, scheme, ancestors, cdf, nullptr, err, st) != hipSuccess)
    return SMC_EDEVICE;
  int herr = 0;
  if (hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess)
    return SMC_EDEVICE;
  if (hipStreamSynchronize(st) != hipSuccess) return SMC_EDEVICE;
  return herr ? SMC_EDEGENERATE : SMC_OK;
}

int32_t resample_noalloc_max(void) { return RS_STATIC_MAX; }

smc_status resample_indices_noalloc(const double *w, int32_t J, const double *u, int32_t scheme,
                                    int32_t *ancestors, void *hip_stream) {
  if (!w || !u || !ancestors || J < 1 ||
      (scheme != SMC_RESAMPLE_SYSTEMATIC && scheme != SMC_RESAMPLE_MULTINOMIAL))
    return SMC_EINVAL;
  if (J > RS_STATIC_MAX) {
    fprintf(stderr, "resample_indices_noalloc: J = %d exceeds the static scratch (%d weights)\n",
            J, RS_STATIC_MAX);
    return SMC_EINVAL;
  }
  unsigned long long *cdf = nullptr;
  int *err = nullptr;
  if (static_resample_scratch(&cdf, &err) != hipSuccess) return SMC_EDEVICE;
  hipStream_t st = (hipStream_t)hip_stream;
  if (launch_resample_indices(w, J, u, scheme, ancestors, cdf, nullptr, err, st) != hipSuccess)
    return SMC_EDEVICE;
  int herr = 0;
  if (hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess)
    return SMC_EDEVICE;
  if (hipStreamSynchronize(st) != hipSuccess) return SMC_EDEVICE;
  return herr ? SMC_EDEGENERATE : SMC_OK;
}

smc_status log_evidence(smc_ctx *ctx, double *log_z_host, double *per_posterior_host) {
  if (!ctx) return SMC_EINVAL;
  CK(hipMemcpyAsync(ctx->ps_host.data(), ctx->D.ps, ctx->D.B * sizeof(PState),
                    hipMemcpyDeviceToHost, ctx->st));
  int fitted = 0;
  if (ctx->D.flow)
    CK(hipMemcpyAsync(&fitted, ctx->D.fstate + 2, sizeof(int), hipMemcpyDeviceToHost, ctx->st));
  CK(hipStreamSynchronize(ctx->st));
  smc_status r = SMC_OK;
  for (int b = 0; b < ctx->D.B; ++b) {
    const PState &S = ctx->ps_host[b];
    const double lz = S.S > 0.0 ? S.log_c + S.m + log(S.S) : -INFINITY;
    if (!(S.S > 0.0)) r = SMC_EDEGENERATE;
    if (b == 0 && log_z_host) *log_z_host = lz;
    if (per_posterior_host) per_posterior_host[b] = lz;
  }
  if (r == SMC_OK && fitted > 0) {
    ctx->err = "log_evidence: " + std::to_string(fitted) +
               " move(s) used flow couplings fitted to the population they moved; the estimate "
               "carries the bias of that adaptation";
    r = SMC_WADAPTIVE;
  }
  return r;
}

smc_status smc_get_state(smc_ctx *ctx, float *theta, double *logw, double *logpi) {
  if (!ctx) return SMC_EINVAL;
  CK(launch_export_state(ctx->D, theta, logw, logpi, ctx->st));
  return SMC_OK;
}

smc_status smc_get_trace(smc_ctx *ctx, smc_trace *t) {
  if (!ctx || !t) return SMC_EINVAL;
  t->h = ctx->D.h;
  t->l = ctx->D.l;
  t->n = ctx->D.n;
  t->dH = ctx->D.dH;
  t->alpha = ctx->D.alpha;
  t->ancestors = ctx->D.anc;
  t->p_final = ctx->D.p_t;
  t->theta_prop = ctx->D.theta_t;
  t->grad = ctx->D.grad_t;
  t->minv = ctx->D.minv;
  t->latent0 = ctx->D.flow ? ctx->D.fz0 : nullptr;
  t->latent = ctx->D.flow ? ctx->D.fz : nullptr;
  t->latent_grad = ctx->D.flow ? ctx->D.fgz : nullptr;
  t->logdet0 = ctx->D.flow ? ctx->D.fld0 : nullptr;
  t->logdet = ctx->D.flow ? ctx->D.fld1 : nullptr;
  t->dpad = ctx->D.DS;
  t->jcap = ctx->D.Jcap;
  t->order = ctx->D.perm;
  t->active = ctx->D.active;
  return SMC_OK;
}

smc_status smc_get_counters(smc_ctx *ctx, smc_counters *c) {
  if (!ctx || !c) return SMC_EINVAL;
  CK(hipMemcpyAsync(ctx->ps_host.data(), ctx->D.ps, ctx->D.B * sizeof(PState),
                    hipMemcpyDeviceToHost, ctx->st));
  CK(hipStreamSynchronize(ctx->st));
  memset(c, 0, sizeof(*c));
  c->iterations = ctx->ps_host[0].tot_iters;
  for (const PState &S : ctx->ps_host) {
    c->grad_evals += S.tot_grad_evals;
    c->ess_sum += S.tot_ess;
    c->resamples += S.tot_resamples;
  }
  return SMC_OK;
}

smc_status smc_set_timing(smc_ctx *ctx, int32_t enable) {
  if (!ctx) return SMC_EINVAL;
  ctx->timing = enable ? 1 : 0;
  return SMC_OK;
}

smc_status smc_get_timing(smc_ctx *ctx, smc_timing *out) {
  if (!ctx || !out) return SMC_EINVAL;
  memset(out, 0, sizeof(*out));
  CK(hipStreamSynchronize(ctx->st));
  for (const auto &m : ctx->ev_marks) {
    float ms = 0.f;
    CK(hipEventElapsedTime(&ms, ctx->ev_pool[m.second], ctx->ev_pool[m.second + 1]));
    if (m.first == 0) {
      out->leapfrog_ms += ms;
      out->leapfrog_launches += 1;
    } else if (m.first == 1) {
      out->loglik_ms += ms;
      out->loglik_launches += 1;
    } else if (m.first == 3) {
      out->flow_ms += ms;
      out->flow_launches += 1;
    } else if (m.first == 4) {
      out->train_ms += ms;
      out->train_launches += 1;
    } else {
      out->reduce_ms += ms;
      out->reduce_launches += 1;
    }
  }
  ctx->ev_marks.clear();
  ctx->ev_used = 0;
  return SMC_OK;
}

smc_status smc_set_params(smc_ctx *ctx, double L, double eps) {
  if (!ctx || !(L > 0.0) || !(eps > 0.0)) return SMC_EINVAL;
  drop_bounded(ctx);  // the launch bound depends on L and eps
  CK(launch_set_params(ctx->D, L, eps, ctx->st));
  return SMC_OK;
}

size_t smc_flow_param_count(int32_t d, int32_t layers, int32_t width) {
  FlowNet F;
  return flow_net(d, layers, width, F) ? (size_t)F.nparams : 0;
}

smc_status smc_get_flow(smc_ctx *ctx, float *params, float *m, float *L, float *grad) {
  if (!ctx) return SMC_EINVAL;
  if (!ctx->D.flow) {
    ctx->err = "no flow preconditioner in this context";
    return SMC_EINVAL;
  }
  const Dev &D = ctx->D;
  if (params)
    CK(hipMemcpyAsync(params, D.fp, (size_t)ctx->F.nparams * 4, hipMemcpyDeviceToDevice, ctx->st));
  if (m) CK(hipMemcpyAsync(m, D.fm, (size_t)ctx->F.d * 4, hipMemcpyDeviceToDevice, ctx->st));
  if (L)
    CK(hipMemcpyAsync(L, D.fL, (size_t)ctx->F.d * ctx->F.d * 4, hipMemcpyDeviceToDevice, ctx->st));
  if (grad) CK(launch_flow_gradsum(D, ctx->F, grad, ctx->st));
  return SMC_OK;
}

smc_status smc_set_flow(smc_ctx *ctx, const float *params) {
  if (!ctx || !params) return SMC_EINVAL;
  if (!ctx->D.flow) {
    ctx->err = "no flow preconditioner in this context";
    return SMC_EINVAL;
  }
  CK(hipMemcpyAsync(ctx->D.fp, params, (size_t)ctx->F.nparams * 4, hipMemcpyDeviceToDevice,
                    ctx->st));
  CK(launch_flow_set(ctx->D, ctx->F, ctx->st));
  return SMC_OK;
}

}  // extern "C"

namespace {
// Device arrays a checkpoint holds: what the next iteration reads (the
// trajectory buffers, plans and partials are rebuilt by every step).
std::vector<std::pair<void *, size_t>> state_pieces(const smc_ctx *ctx) {
  const Dev &D = ctx->D;
  const size_t rows = (size_t)D.B * D.Jcap;
  std::vector<std::pair<void *, size_t>> v = {{D.ps, (size_t)D.B * sizeof(PState)},
                                              {D.theta, rows * D.DS * sizeof(float)},
                                              {D.grad, rows * D.DS * sizeof(float)},
                                              {D.logpi, rows * sizeof(double)},
                                              {D.logw, rows * sizeof(double)},
                                              {D.minv, (size_t)D.B * D.DS * sizeof(float)}};
  if (D.flow) {
    const size_t np = (size_t)ctx->F.nparams * 4, npk = (size_t)ctx->F.npacked * 4;
    v.push_back({D.fp, np});
    v.push_back({D.fpk, npk});
    v.push_back({D.fbk, npk});
    v.push_back({D.fbias, np});
    v.push_back({D.fadm, np});
    v.push_back({D.fadv, np});
    v.push_back({D.fstate, 256});
  }
  return v;
}

struct StateHeader {
  char magic[8];
  int32_t B, J, Jcap, DS, nmax, flow, nparams, bf16;
  int64_t steps, bytes;
};

void state_header(const smc_ctx *ctx, StateHeader &h) {
  memset(&h, 0, sizeof(h));
  memcpy(h.magic, "CHEESMC1", 8);
  h.B = ctx->D.B;
  h.J = ctx->D.J;
  h.Jcap = ctx->D.Jcap;
  h.DS = ctx->D.DS;
  h.nmax = ctx->D.nmax;
  h.flow = ctx->D.flow;
  h.nparams = ctx->D.flow ? ctx->F.nparams : 0;
  h.bf16 = ctx->D.bf16;
  h.steps = ctx->steps;
  size_t bytes = sizeof(StateHeader);
  for (const auto &p : state_pieces(ctx)) bytes += p.second;
  h.bytes = (int64_t)bytes;
}
}  // namespace

extern "C" {

size_t smc_state_bytes(const smc_ctx *ctx) {
  if (!ctx) return 0;
  StateHeader h;
  state_header(ctx, h);
  return (size_t)h.bytes;
}

smc_status smc_save(smc_ctx *ctx, void *buf, size_t bytes) {
  if (!ctx || !buf) return SMC_EINVAL;
  if (ctx->stepped) {
    ctx->err = "smc_save between smc_step and chees_adapt";
    return SMC_ESTATE;
  }
  StateHeader h;
  state_header(ctx, h);
  if (bytes < (size_t)h.bytes) {
    ctx->err = "smc_save: buffer smaller than smc_state_bytes";
    return SMC_EINVAL;
  }
  char *out = (char *)buf;
  memcpy(out, &h, sizeof(h));
  size_t off = sizeof(h);
  for (const auto &p : state_pieces(ctx)) {
    CK(hipMemcpyAsync(out + off, p.first, p.second, hipMemcpyDeviceToHost, ctx->st));
    off += p.second;
  }
  CK(hipStreamSynchronize(ctx->st));
  return SMC_OK;
}

smc_status smc_load(smc_ctx *ctx, const void *buf, size_t bytes) {
  if (!ctx || !buf) return SMC_EINVAL;
  StateHeader mine, img;
  state_header(ctx, mine);
  if (bytes < sizeof(img)) {
    ctx->err = "smc_load: image too short";
    return SMC_EINVAL;
  }
  memcpy(&img, buf, sizeof(img));
  if (memcmp(img.magic, mine.magic, 8) != 0 || img.B != mine.B || img.J != mine.J ||
      img.Jcap != mine.Jcap || img.DS != mine.DS || img.nmax != mine.nmax ||
      img.flow != mine.flow || img.nparams != mine.nparams || img.bf16 != mine.bf16 ||
      img.bytes != mine.bytes || bytes < (size_t)img.bytes) {
    ctx->err = "smc_load: the image was saved from a context of another shape";
    return SMC_EINVAL;
  }
  const char *in = (const char *)buf;
  size_t off = sizeof(img);
  for (const auto &p : state_pieces(ctx)) {
    CK(hipMemcpyAsync(p.first, in + off, p.second, hipMemcpyHostToDevice, ctx->st));
    off += p.second;
  }
  CK(hipStreamSynchronize(ctx->st));
  ctx->steps = img.steps;
  ctx->stepped = 0;
  drop_bounded(ctx);  // the restored L and eps decide the launch bound afresh
  return SMC_OK;
}

void smc_destroy(smc_ctx *ctx) { delete ctx; }

const char *smc_last_error(const smc_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

}  // extern "C"
