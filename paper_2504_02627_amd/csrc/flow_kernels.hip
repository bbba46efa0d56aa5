// Flow preconditioner of the SMC/ChEES-HMC sampler (gfx950).
//
// The paper's exactness argument for the momentum L-kernel (Sec. III-A,
// eqs. proposal_momentum, l-kernel_momentum) needs only a volume-preserving
// bijection, so the leapfrog may run in the latent space of a bijection T
// that is fixed during an iteration, on the pushforward target
//   log pi_z(z) = log pi(T(z)) + log|det J_T(z)|.
// T: x = z; per coupling layer l: x_T <- x_T exp(s) + t with (s, t) from a
// tanh MLP (width FH) of the conditioning half x_C, s = tanh(.);
// theta_c = m_c + exp(a_c) x_q(c), q placing the even coordinates of theta
// first, then the odd ones.  m, a standardise the weighted pre-move population;
// the couplings are trained each iteration by a few Adam steps on the
// weighted maximum-likelihood objective of the population.
//
// Kernels work on FP = 4 particles per wave (one wave per block): every
// weight loaded from L2 feeds four particles; activations of the current
// layer sit in LDS, the per-layer activations the backward passes need in a
// per-particle tape in global memory.  Training uses the FP32 parameters,
// the moves the BF16-rounded weights with FP32 arithmetic.
#pragma clang fp contract(off)

#include <math.h>

#include "dev_common.h"
#include "smc_internal.h"

namespace smc {

namespace {

constexpr int MAXD = 16 * MAX_C2;  // largest padded dimension
constexpr int KSPLIT = FKSPLIT;

__device__ __forceinline__ float2 wpair(const uint16_t *w, int i) {
  const uint32_t u = *reinterpret_cast<const uint32_t *>(w + i);
  return make_float2(__uint_as_float(u << 16), __uint_as_float(u & 0xFFFF0000u));
}
__device__ __forceinline__ float2 wpair(const float *w, int i) {
  return *reinterpret_cast<const float2 *>(w + i);
}
__device__ __forceinline__ float wone(const uint16_t *w, int i) {
  return __uint_as_float((uint32_t)w[i] << 16);
}
__device__ __forceinline__ float wone(const float *w, int i) { return w[i]; }

__device__ __forceinline__ uint16_t bf16_bits(float f) {
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((u >> 16) | 0x40u);  // NaN stays NaN
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// out[p][u] = b[u] + sum_k Wt[k][u] in[p][k] for u < M, the lane holding the
// unit pairs (2q, 2q + 1), q = lane + 64 r.  Wt: transposed weights [K][M].
template <typename WT>
__device__ __forceinline__ void dense_fwd(const WT *Wt, const float *bias, int M, int K,
                                          const float *in, int ins, int lane, float acc[FP][2][2]) {
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int u = 2 * (lane + 64 * r);
#pragma unroll
    for (int p = 0; p < FP; ++p) {
      acc[p][r][0] = u < M ? bias[u] : 0.f;
      acc[p][r][1] = u + 1 < M ? bias[u + 1] : 0.f;
    }
  }
  const bool r1 = 2 * (lane + 64) < M;
  const bool r0 = 2 * lane < M;
#pragma unroll 4
  for (int k = 0; k < K; ++k) {
    float xv[FP];
#pragma unroll
    for (int p = 0; p < FP; ++p) xv[p] = in[p * ins + k];
    if (r0) {
      const float2 w = wpair(Wt, k * M + 2 * lane);
#pragma unroll
      for (int p = 0; p < FP; ++p) {
        acc[p][0][0] = fmaf(w.x, xv[p], acc[p][0][0]);
        acc[p][0][1] = fmaf(w.y, xv[p], acc[p][0][1]);
      }
    }
    if (r1) {
      const float2 w = wpair(Wt, k * M + 2 * (lane + 64));
#pragma unroll
      for (int p = 0; p < FP; ++p) {
        acc[p][1][0] = fmaf(w.x, xv[p], acc[p][1][0]);
        acc[p][1][1] = fmaf(w.y, xv[p], acc[p][1][1]);
      }
    }
  }
}

// Write a dense_fwd result to LDS rows out[p][u] (optionally tanh), and to the
// tape rows tp[p] + u when given.
__device__ __forceinline__ void store_units(float acc[FP][2][2], int M, bool act, float *out,
                                            int outs, float *const tp[FP], int lane) {
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int u = 2 * (lane + 64 * r) + e;
      if (u < M)
#pragma unroll
        for (int p = 0; p < FP; ++p) {
          const float v = act ? tanhf(acc[p][r][e]) : acc[p][r][e];
          out[p * outs + u] = v;
          if (tp[p]) tp[p][u] = v;
        }
    }
}

// out[p][k] = sum_u W[u][k] in[p][u] for k = lane + 64 r < K (K <= 128).
// W: row-major [M][K].
template <typename WT>
__device__ __forceinline__ void dense_bwd(const WT *W, int M, int K, const float *in, int ins,
                                          int lane, float out[FP][2]) {
#pragma unroll
  for (int p = 0; p < FP; ++p) out[p][0] = out[p][1] = 0.f;
  const bool r0 = lane < K, r1 = lane + 64 < K;
#pragma unroll 4
  for (int u = 0; u < M; ++u) {
    float g[FP];
#pragma unroll
    for (int p = 0; p < FP; ++p) g[p] = in[p * ins + u];
    if (r0) {
      const float w = wone(W, u * K + lane);
#pragma unroll
      for (int p = 0; p < FP; ++p) out[p][0] = fmaf(w, g[p], out[p][0]);
    }
    if (r1) {
      const float w = wone(W, u * K + lane + 64);
#pragma unroll
      for (int p = 0; p < FP; ++p) out[p][1] = fmaf(w, g[p], out[p][1]);
    }
  }
}

// Position of coordinate c of theta in the coupling state x: even
// coordinates first, then the odd ones, so that the halves of x split
// neighbouring coordinates.
__device__ __forceinline__ int xpos(int c, int d) { return (c & 1) ? (d + 1) / 2 + (c >> 1) : c >> 1; }

struct FlowLDS {
  float xs[FP][MAXD];  // coupling state x (or its cotangent)
  float h1[FP][FH];
  float h2[FP][FH];
  float ob[FP][MAXD];  // conditioner output (s~, t) or its cotangent
};

// Forward map of the four particles in xs (latent z on entry, the coupled x
// on exit), with the move tape [h1 | h2 | s | x_T before the update] per
// layer when tape rows are given; returns per-lane partial sums of s.
__device__ void forward_couplings(const FlowNet &F, const uint16_t *Wt, const float *bias,
                                  FlowLDS &S, float *const tape[FP], float ldl[FP], int lane) {
  for (int l = 0; l < F.L; ++l) {
    const FlowLayerDesc &Y = F.ly[l];
    float *t1[FP], *t2[FP], *ts[FP];
#pragma unroll
    for (int p = 0; p < FP; ++p) {
      float *b = tape[p] ? tape[p] + (long long)l * F.tape_stride : nullptr;
      t1[p] = b;
      t2[p] = b ? b + FH : nullptr;
      ts[p] = b ? b + 2 * FH : nullptr;
    }
    float acc[FP][2][2];
    dense_fwd(Wt + Y.oW1, bias + Y.ob1, FH, Y.dc, &S.xs[0][Y.C0], MAXD, lane, acc);
    store_units(acc, FH, true, &S.h1[0][0], FH, t1, lane);
    __syncthreads();
    dense_fwd(Wt + Y.oW2, bias + Y.ob2, FH, FH, &S.h1[0][0], FH, lane, acc);
    store_units(acc, FH, true, &S.h2[0][0], FH, t2, lane);
    __syncthreads();
    dense_fwd(Wt + Y.oW3, bias + Y.ob3, 2 * Y.dt, FH, &S.h2[0][0], FH, lane, acc);
    float *none[FP] = {nullptr, nullptr, nullptr, nullptr};
    store_units(acc, 2 * Y.dt, false, &S.ob[0][0], MAXD, none, lane);
    __syncthreads();
    for (int f = lane; f < Y.dt; f += 64)
#pragma unroll
      for (int p = 0; p < FP; ++p) {
        const float s = tanhf(S.ob[p][f]);
        const float t = S.ob[p][Y.dt + f];
        const float x = S.xs[p][Y.T0 + f];
        if (ts[p]) {
          ts[p][f] = s;
          ts[p][F.half + f] = x;
        }
        S.xs[p][Y.T0 + f] = fmaf(x, expf(s), t);
        ldl[p] += s;
      }
    __syncthreads();
  }
}

// Cotangent of z from the cotangent of x after the couplings (in xs), by
// reverse accumulation over the move tape; the log-determinant adds 1 to the
// cotangent of every s.
__device__ void vjp_couplings(const FlowNet &F, const uint16_t *W, FlowLDS &S,
                              const float *const tape[FP], int lane) {
  for (int l = F.L - 1; l >= 0; --l) {
    const FlowLayerDesc &Y = F.ly[l];
    const float *t1[FP], *t2[FP], *ts[FP];
#pragma unroll
    for (int p = 0; p < FP; ++p) {
      const float *b = tape[p] + (long long)l * F.tape_stride;
      t1[p] = b;
      t2[p] = b + FH;
      ts[p] = b + 2 * FH;
    }
    for (int f = lane; f < Y.dt; f += 64)
#pragma unroll
      for (int p = 0; p < FP; ++p) {
        const float s = ts[p][f], xT = ts[p][F.half + f];
        const float gy = S.xs[p][Y.T0 + f];
        const float es = expf(s);
        const float gs = fmaf(gy * xT, es, 1.f);
        S.ob[p][f] = gs * (1.f - s * s);
        S.ob[p][Y.dt + f] = gy;
        S.xs[p][Y.T0 + f] = gy * es;
      }
    __syncthreads();
    float o[FP][2];
    dense_bwd(W + Y.oW3, 2 * Y.dt, FH, &S.ob[0][0], MAXD, lane, o);
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int k = lane + 64 * r;
#pragma unroll
      for (int p = 0; p < FP; ++p) {
        const float h = t2[p][k];
        S.h2[p][k] = o[p][r] * (1.f - h * h);
      }
    }
    __syncthreads();
    dense_bwd(W + Y.oW2, FH, FH, &S.h2[0][0], FH, lane, o);
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int k = lane + 64 * r;
#pragma unroll
      for (int p = 0; p < FP; ++p) {
        const float h = t1[p][k];
        S.h1[p][k] = o[p][r] * (1.f - h * h);
      }
    }
    __syncthreads();
    dense_bwd(W + Y.oW1, FH, Y.dc, &S.h1[0][0], FH, lane, o);
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int k = lane + 64 * r;
      if (k < Y.dc)
#pragma unroll
        for (int p = 0; p < FP; ++p) S.xs[p][Y.C0 + k] += o[p][r];
    }
    __syncthreads();
  }
}

__device__ __forceinline__ float lane_sum_to_float(float v) { return (float)wave_sum((double)v); }

// ---------------------------------------------------------------------------
// Initial couplings: W1, W2 from the Philox stream FLOW (layer l: iterations
// 100 + 2l and 101 + 2l, row u as the particle index, column k in block k/4)
// scaled by 1/sqrt(fan-in); biases, W3, b3 and the Adam moments zero.
// ---------------------------------------------------------------------------
__global__ void k_flow_init(Dev D, FlowNet F) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < F.nparams; i += gridDim.x * blockDim.x) {
    float v = 0.f;
    for (int l = 0; l < F.L; ++l) {
      const FlowLayerDesc &Y = F.ly[l];
      int it = -1, K = 0, o = 0;
      if (i >= Y.oW1 && i < Y.ob1) {
        it = 100 + 2 * l;
        K = Y.dc;
        o = Y.oW1;
      } else if (i >= Y.oW2 && i < Y.ob2) {
        it = 101 + 2 * l;
        K = FH;
        o = Y.oW2;
      }
      if (it >= 0) {
        const int u = (i - o) / K, k = (i - o) % K;
        double z[4];
        box_muller4(philox_at(D.seed, (uint32_t)(k / 4), (uint32_t)u, (uint32_t)it, STREAM_FLOW), z);
        v = (float)(z[k % 4] / sqrt((double)K));
      }
    }
    D.fp[i] = v;
    D.fadm[i] = 0.f;
    D.fadv[i] = 0.f;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) D.fstate[0] = 0;
}

// ---------------------------------------------------------------------------
// Adam ascent on the couplings (update != 0), then the copies the kernels
// read: transposed FP32 weights (training forward), BF16 weights row-major and
// transposed, BF16-rounded biases (moves).  The gradient is the ordered sum of
// the KSPLIT particle-chunk partials.  Adam step t = (k - 1) ntrain + step + 1
// - offset, k the iteration counter of the device state.
// ---------------------------------------------------------------------------
__global__ void k_flow_adam(Dev D, FlowNet F, int step, int update, const float *part) {
  const int t = (D.ps[0].k - 1) * F.ntrain + step + 1 - D.fstate[0];
  const double c1 = 1.0 - pow(D.adam_b1, (double)t), c2 = 1.0 - pow(D.adam_b2, (double)t);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < F.nparams; i += gridDim.x * blockDim.x) {
    float pv = D.fp[i];
    if (update) {
      double g = 0.0;
      for (int s = 0; s < KSPLIT; ++s) g += (double)part[(long long)s * F.nparams + i];
      const double m = D.adam_b1 * (double)D.fadm[i] + (1.0 - D.adam_b1) * g;
      const double v = D.adam_b2 * (double)D.fadv[i] + (1.0 - D.adam_b2) * g * g;
      D.fadm[i] = (float)m;
      D.fadv[i] = (float)v;
      pv = (float)((double)pv + (double)F.lr * (m / c1) / (sqrt(v / c2) + D.adam_eps));
      D.fp[i] = pv;
    }
    const uint16_t hb = bf16_bits(pv);
    bool weight = false;
    for (int l = 0; l < F.L; ++l) {
      const FlowLayerDesc &Y = F.ly[l];
      int o = -1, rows = 0, cols = 0;
      if (i >= Y.oW1 && i < Y.ob1) {
        o = Y.oW1, rows = FH, cols = Y.dc;
      } else if (i >= Y.oW2 && i < Y.ob2) {
        o = Y.oW2, rows = FH, cols = FH;
      } else if (i >= Y.oW3 && i < Y.ob3) {
        o = Y.oW3, rows = 2 * Y.dt, cols = FH;
      }
      if (o >= 0) {
        const int u = (i - o) / cols, k = (i - o) % cols;
        const int ti = o + k * rows + u;
        D.fpt[ti] = pv;
        D.fwbt[ti] = hb;
        weight = true;
      }
    }
    D.fwb[i] = hb;
    D.fbias[i] = weight ? 0.f : __uint_as_float((uint32_t)hb << 16);
  }
}

// ---------------------------------------------------------------------------
// Standardisation m, a from the weighted column moments of the pre-move
// population (the two passes of k_mass_colsum): m = weighted mean,
// a = 1/2 log of the regularised weighted variance held in binary32.
// ---------------------------------------------------------------------------
__global__ void k_flow_base(Dev D, FlowNet F) {
  const double n = D.ps[0].ess_before;
  for (int c = threadIdx.x; c < D.DS; c += blockDim.x) {
    double s = 0.0;
    for (int ch = 0; ch < D.col_chunks; ++ch) s += D.colpart[(long long)ch * 2 * D.DS + c];
    const float v = (float)((n / (n + 5.0)) * s + 1e-3 * (5.0 / (n + 5.0)));
    D.fm[c] = c < F.d ? (float)D.means[c] : 0.f;
    D.fa[c] = c < F.d ? (float)(0.5 * log((double)v)) : 0.f;
  }
}

// ---------------------------------------------------------------------------
// One training pass over the population: the inverse map theta -> z with the
// FP32 parameters, recording per layer [x_C | h1 | h2 | s | x_T | d3 | d2 | d1]
// where d3, d2, d1 are the weighted cotangents of the conditioner output and
// pre-activations of the objective
//   sum_j W_j [log N(z_j; 0, I) + log|det J_{T^-1}(theta_j)|],
// W the normalised weights (uniform right after resampling).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_flow_train(Dev D, FlowNet F) {
  __shared__ FlowLDS S;
  const int lane = threadIdx.x;
  const int j0 = blockIdx.x * FP;
  const PState &PS = D.ps[0];
  const int rs = PS.resampled;
  const float *src = rs ? D.theta_t : D.theta;
  float wj[FP];
  float *rec[FP];
#pragma unroll
  for (int p = 0; p < FP; ++p) {
    const int j = j0 + p;
    const bool ok = j < D.J;
    double w = 0.0;
    if (ok) {
      const double lw = D.logw[j];
      w = rs ? 1.0 / D.J : ((lw == lw && lw > -INFINITY) ? exp(lw - PS.m) / PS.S : 0.0);
    }
    wj[p] = (float)w;
    rec[p] = ok ? D.ftape + (long long)j * F.L * F.train_stride : nullptr;
    for (int c = lane; c < MAXD; c += 64) {
      if (c < F.d)
        S.xs[p][xpos(c, F.d)] = ok ? (src[(long long)j * D.DS + c] - D.fm[c]) * expf(-D.fa[c]) : 0.f;
      else
        S.xs[p][c] = 0.f;
    }
  }
  __syncthreads();
  const float *Wt = D.fpt, *W = D.fp;
  const int h = F.half;
  // inverse couplings, last layer first
  for (int l = F.L - 1; l >= 0; --l) {
    const FlowLayerDesc &Y = F.ly[l];
    float *r[FP];
#pragma unroll
    for (int p = 0; p < FP; ++p) r[p] = rec[p] ? rec[p] + (long long)l * F.train_stride : nullptr;
    for (int c = lane; c < Y.dc; c += 64)
#pragma unroll
      for (int p = 0; p < FP; ++p)
        if (r[p]) r[p][c] = S.xs[p][Y.C0 + c];
    float acc[FP][2][2];
    float *t1[FP], *t2[FP];
#pragma unroll
    for (int p = 0; p < FP; ++p) {
      t1[p] = r[p] ? r[p] + h : nullptr;
      t2[p] = r[p] ? r[p] + h + FH : nullptr;
    }
    dense_fwd(Wt + Y.oW1, W + Y.ob1, FH, Y.dc, &S.xs[0][Y.C0], MAXD, lane, acc);
    store_units(acc, FH, true, &S.h1[0][0], FH, t1, lane);
    __syncthreads();
    dense_fwd(Wt + Y.oW2, W + Y.ob2, FH, FH, &S.h1[0][0], FH, lane, acc);
    store_units(acc, FH, true, &S.h2[0][0], FH, t2, lane);
    __syncthreads();
    dense_fwd(Wt + Y.oW3, W + Y.ob3, 2 * Y.dt, FH, &S.h2[0][0], FH, lane, acc);
    float *none[FP] = {nullptr, nullptr, nullptr, nullptr};
    store_units(acc, 2 * Y.dt, false, &S.ob[0][0], MAXD, none, lane);
    __syncthreads();
    for (int f = lane; f < Y.dt; f += 64)
#pragma unroll
      for (int p = 0; p < FP; ++p) {
        const float s = tanhf(S.ob[p][f]);
        const float t = S.ob[p][Y.dt + f];
        const float x = (S.xs[p][Y.T0 + f] - t) * expf(-s);
        S.xs[p][Y.T0 + f] = x;
        if (r[p]) {
          r[p][h + 2 * FH + f] = s;
          r[p][2 * h + 2 * FH + f] = x;
        }
      }
    __syncthreads();
  }
  // cotangent of z: -W_j z
  for (int c = lane; c < MAXD; c += 64)
#pragma unroll
    for (int p = 0; p < FP; ++p) S.xs[p][c] = -wj[p] * S.xs[p][c];
  __syncthreads();
  // reverse of the inverse order: layer 0 first
  for (int l = 0; l < F.L; ++l) {
    const FlowLayerDesc &Y = F.ly[l];
    float *r[FP];
#pragma unroll
    for (int p = 0; p < FP; ++p) r[p] = rec[p] ? rec[p] + (long long)l * F.train_stride : nullptr;
    for (int f = lane; f < Y.dt; f += 64)
#pragma unroll
      for (int p = 0; p < FP; ++p) {
        float s = 0.f, xT = 0.f;
        if (r[p]) {
          s = r[p][h + 2 * FH + f];
          xT = r[p][2 * h + 2 * FH + f];
        }
        const float gx = S.xs[p][Y.T0 + f];
        const float es = expf(-s);
        const float gs = -gx * xT - wj[p];
        const float d3s = gs * (1.f - s * s), d3t = -gx * es;
        S.ob[p][f] = d3s;
        S.ob[p][Y.dt + f] = d3t;
        S.xs[p][Y.T0 + f] = gx * es;
        if (r[p]) {
          r[p][3 * h + 2 * FH + f] = d3s;
          r[p][3 * h + 2 * FH + Y.dt + f] = d3t;
        }
      }
    __syncthreads();
    float o[FP][2];
    dense_bwd(W + Y.oW3, 2 * Y.dt, FH, &S.ob[0][0], MAXD, lane, o);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int k = lane + 64 * q;
#pragma unroll
      for (int p = 0; p < FP; ++p) {
        const float hh = r[p] ? r[p][h + FH + k] : 0.f;
        const float v = o[p][q] * (1.f - hh * hh);
        S.h2[p][k] = v;
        if (r[p]) r[p][5 * h + 2 * FH + k] = v;
      }
    }
    __syncthreads();
    dense_bwd(W + Y.oW2, FH, FH, &S.h2[0][0], FH, lane, o);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int k = lane + 64 * q;
#pragma unroll
      for (int p = 0; p < FP; ++p) {
        const float hh = r[p] ? r[p][h + k] : 0.f;
        const float v = o[p][q] * (1.f - hh * hh);
        S.h1[p][k] = v;
        if (r[p]) r[p][5 * h + 3 * FH + k] = v;
      }
    }
    __syncthreads();
    dense_bwd(W + Y.oW1, FH, Y.dc, &S.h1[0][0], FH, lane, o);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int k = lane + 64 * q;
      if (k < Y.dc)
#pragma unroll
        for (int p = 0; p < FP; ++p) S.xs[p][Y.C0 + k] += o[p][q];
    }
    __syncthreads();
  }
}

// Parameter gradient of one training pass: for every weight matrix
// dW[u][k] = sum_j delta_j[u] in_j[k] (W3: d3 x h2, W2: d2 x h1, W1: d1 x x_C)
// and every bias db[u] = sum_j delta_j[u], in 64 x 64 tiles (4 x 4 per
// thread), over KSPLIT particle chunks (blockIdx.y) in index order.
struct Gm {
  int rows, cols, off_delta, off_in, o, ob;
};
__device__ __forceinline__ Gm gm_of(const FlowNet &F, int l, int which) {
  const FlowLayerDesc &Y = F.ly[l];
  const int h = F.half;
  if (which == 0) return Gm{2 * Y.dt, FH, 3 * h + 2 * FH, h + FH, Y.oW3, Y.ob3};
  if (which == 1) return Gm{FH, FH, 5 * h + 2 * FH, h, Y.oW2, Y.ob2};
  return Gm{FH, Y.dc, 5 * h + 3 * FH, 0, Y.oW1, Y.ob1};
}

__global__ __launch_bounds__(256) void k_flow_wgrad(Dev D, FlowNet F, float *part) {
  __shared__ float4 As[32][16], Bs[32][16];
  // locate (layer, matrix, tile) or (layer, matrix, bias)
  int id = blockIdx.x, l = -1, which = 0, tile = 0, isbias = 0;
  for (int ll = 0; ll < F.L && l < 0; ++ll)
    for (int w = 0; w < 3 && l < 0; ++w) {
      const Gm g = gm_of(F, ll, w);
      const int nt = ((g.rows + 63) / 64) * ((g.cols + 63) / 64) + 1;
      if (id < nt) {
        l = ll;
        which = w;
        tile = id;
        isbias = id == nt - 1;
      } else {
        id -= nt;
      }
    }
  if (l < 0) return;
  const Gm g = gm_of(F, l, which);
  const int split = blockIdx.y;
  const int jc = (D.J + KSPLIT - 1) / KSPLIT;
  const int ja = split * jc, jb = min(D.J, ja + jc);
  float *out = part + (long long)split * F.nparams;
  const int t = threadIdx.x;
  const long long stride = (long long)F.L * F.train_stride;
  const float *base = D.ftape + (long long)l * F.train_stride;
  if (isbias) {
    for (int u = t; u < g.rows; u += blockDim.x) {
      float s = 0.f;
      for (int j = ja; j < jb; ++j) s += base[j * stride + g.off_delta + u];
      out[g.ob + u] = s;
    }
    return;
  }
  const int ntc = (g.cols + 63) / 64;
  const int u0 = (tile / ntc) * 64, k0 = (tile % ntc) * 64;
  const int ty = t >> 4, tx = t & 15;
  float acc[4][4] = {};
  for (int jj0 = ja; jj0 < jb; jj0 += 32) {
    // 32 particles x 64 delta rows / 64 input columns
    for (int idx = t; idx < 32 * 16; idx += 256) {
      const int jj = idx >> 4, c4 = idx & 15;
      const int j = jj0 + jj;
      float4 a = make_float4(0.f, 0.f, 0.f, 0.f), b = a;
      if (j < jb) {
        const float *r = base + j * stride;
        const int u = u0 + 4 * c4, k = k0 + 4 * c4;
        float av[4], bv[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          av[e] = (u + e < g.rows) ? r[g.off_delta + u + e] : 0.f;
          bv[e] = (k + e < g.cols) ? r[g.off_in + k + e] : 0.f;
        }
        a = make_float4(av[0], av[1], av[2], av[3]);
        b = make_float4(bv[0], bv[1], bv[2], bv[3]);
      }
      As[jj][c4] = a;
      Bs[jj][c4] = b;
    }
    __syncthreads();
#pragma unroll 4
    for (int jj = 0; jj < 32; ++jj) {
      const float4 a = As[jj][ty], b = Bs[jj][tx];
      const float av[4] = {a.x, a.y, a.z, a.w}, bv[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = fmaf(av[x], bv[y], acc[x][y]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int u = u0 + 4 * ty + x, k = k0 + 4 * tx + y;
      if (u < g.rows && k < g.cols) out[g.o + u * g.cols + k] = acc[x][y];
    }
}

// ---------------------------------------------------------------------------
// Start of the moves: z0 = T^-1(theta0) (BF16 weights), log|det J_T(z0)|,
// then the forward map from z0 with the move tape and the latent gradient
// grad_z log pi_z(z0) from the cached gradient of log pi at theta0; the
// initial energy gets -log|det J_T(z0)|.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_flow_begin(Dev D, FlowNet F) {
  __shared__ FlowLDS S;
  const int lane = threadIdx.x;
  const int j0 = blockIdx.x * FP;
  float *tape[FP];        // written by the forward pass (valid particles only)
  const float *rtape[FP]; // read by the backward pass
  float ldl[FP];
#pragma unroll
  for (int p = 0; p < FP; ++p) {
    const int j = j0 + p;
    const bool ok = j < D.J;
    tape[p] = ok ? D.ftape + (long long)j * F.L * F.tape_stride : nullptr;
    rtape[p] = D.ftape + (long long)(ok ? j : j0) * F.L * F.tape_stride;
    ldl[p] = 0.f;
    for (int c = lane; c < MAXD; c += 64) {
      if (c < F.d) {
        float x = 0.f;
        if (ok) {
          x = (D.theta_t[(long long)j * D.DS + c] - D.fm[c]) * expf(-D.fa[c]);
          ldl[p] -= D.fa[c];
        }
        S.xs[p][xpos(c, F.d)] = x;
      } else {
        S.xs[p][c] = 0.f;
      }
    }
  }
  __syncthreads();
  // inverse couplings (BF16 weights), last layer first
  for (int l = F.L - 1; l >= 0; --l) {
    const FlowLayerDesc &Y = F.ly[l];
    float acc[FP][2][2];
    float *none[FP] = {nullptr, nullptr, nullptr, nullptr};
    dense_fwd(D.fwbt + Y.oW1, D.fbias + Y.ob1, FH, Y.dc, &S.xs[0][Y.C0], MAXD, lane, acc);
    store_units(acc, FH, true, &S.h1[0][0], FH, none, lane);
    __syncthreads();
    dense_fwd(D.fwbt + Y.oW2, D.fbias + Y.ob2, FH, FH, &S.h1[0][0], FH, lane, acc);
    store_units(acc, FH, true, &S.h2[0][0], FH, none, lane);
    __syncthreads();
    dense_fwd(D.fwbt + Y.oW3, D.fbias + Y.ob3, 2 * Y.dt, FH, &S.h2[0][0], FH, lane, acc);
    store_units(acc, 2 * Y.dt, false, &S.ob[0][0], MAXD, none, lane);
    __syncthreads();
    for (int f = lane; f < Y.dt; f += 64)
#pragma unroll
      for (int p = 0; p < FP; ++p) {
        const float s = tanhf(S.ob[p][f]);
        S.xs[p][Y.T0 + f] = (S.xs[p][Y.T0 + f] - S.ob[p][Y.dt + f]) * expf(-s);
        ldl[p] -= s;
      }
    __syncthreads();
  }
#pragma unroll
  for (int p = 0; p < FP; ++p) {
    const int j = j0 + p;
    const float ld0 = -lane_sum_to_float(ldl[p]);   // log|det J_T(z0)|
    if (j < D.J) {
      for (int c = lane; c < D.DS; c += 64) {
        const float z = c < F.d ? S.xs[p][c] : 0.f;
        D.fz[(long long)j * D.DS + c] = z;
        D.fz0[(long long)j * D.DS + c] = z;
      }
      if (lane == 0) {
        D.fld0[j] = ld0;
        D.H0[j] -= (double)ld0;
      }
    }
    ldl[p] = 0.f;
  }
  __syncthreads();
  forward_couplings(F, D.fwbt, D.fbias, S, tape, ldl, lane);
  // cotangent of x: g_theta * exp(a), then back through the couplings
#pragma unroll
  for (int p = 0; p < FP; ++p) {
    const int j = j0 + p;
    for (int c = lane; c < MAXD; c += 64) {
      if (c < F.d)
        S.xs[p][xpos(c, F.d)] = j < D.J ? D.grad_t[(long long)j * D.DS + c] * expf(D.fa[c]) : 0.f;
      else
        S.xs[p][c] = 0.f;
    }
  }
  __syncthreads();
  vjp_couplings(F, D.fwb, S, rtape, lane);
#pragma unroll
  for (int p = 0; p < FP; ++p) {
    const int j = j0 + p;
    if (j < D.J)
      for (int c = lane; c < D.DS; c += 64)
        D.fgz[(long long)j * D.DS + c] = c < F.d ? S.xs[p][c] : 0.f;
  }
}

// Particles of a move launch: FP consecutive slots of the trajectory-length
// order (longest first), active while n > step.
__device__ __forceinline__ int move_rows(const Dev &D, int step, int rows[FP]) {
  int any = 0;
#pragma unroll
  for (int p = 0; p < FP; ++p) {
    const int slot = blockIdx.x * FP + p;
    int r = -1;
    if (slot < D.J) {
      const int j = D.perm[slot];
      if (j < D.J && D.n[j] > step) r = j;
    }
    rows[p] = r;
    any |= r >= 0;
  }
  return any;
}

// Leapfrog step `step`, first half: p += eps/2 g_z; z += eps p; theta = T(z)
// (BF16 weights) with the move tape and log|det J_T(z)|.  The likelihood
// gradient at theta follows (k_lf_partial / k_lf_reduce in gradient mode).
__global__ __launch_bounds__(64) void k_flow_drift(Dev D, FlowNet F, int step) {
  __shared__ FlowLDS S;
  int rows[FP];
  if (!move_rows(D, step, rows)) return;
  const int lane = threadIdx.x;
  const float eps = (float)D.ps[0].eps;
  const float he = 0.5f * eps;
  float *tape[FP];
  float ldl[FP];
#pragma unroll
  for (int p = 0; p < FP; ++p) {
    const int j = rows[p] >= 0 ? rows[p] : rows[0] >= 0 ? rows[0] : 0;
    tape[p] = rows[p] >= 0 ? D.ftape + (long long)j * F.L * F.tape_stride : nullptr;
    ldl[p] = 0.f;
    for (int c = lane; c < MAXD; c += 64) {
      float z = 0.f;
      if (rows[p] >= 0 && c < D.DS) {
        const long long e = (long long)rows[p] * D.DS + c;
        const float ph = fmaf(he, D.fgz[e], D.p_t[e]);
        z = fmaf(eps, ph, D.fz[e]);
        if (c >= F.d) z = 0.f;
        D.p_t[e] = c < F.d ? ph : 0.f;
        D.fz[e] = z;
      }
      S.xs[p][c] = z;
    }
  }
  __syncthreads();
  forward_couplings(F, D.fwbt, D.fbias, S, tape, ldl, lane);
#pragma unroll
  for (int p = 0; p < FP; ++p) {
    float sa = 0.f;
    for (int c = lane; c < F.d; c += 64) sa += D.fa[c];
    const float ld = lane_sum_to_float(ldl[p] + sa);
    if (rows[p] >= 0) {
      for (int c = lane; c < D.DS; c += 64)
        D.theta_t[(long long)rows[p] * D.DS + c] =
            c < F.d ? fmaf(expf(D.fa[c]), S.xs[p][xpos(c, F.d)], D.fm[c]) : 0.f;
      if (lane == 0) D.fld1[rows[p]] = ld;
    }
  }
}

// Leapfrog step `step`, second half: g_z = J_T^T grad log pi(theta) +
// grad log|det J_T| from the move tape; p += eps/2 g_z.
__global__ __launch_bounds__(64) void k_flow_kick(Dev D, FlowNet F, int step) {
  __shared__ FlowLDS S;
  int rows[FP];
  if (!move_rows(D, step, rows)) return;
  const int lane = threadIdx.x;
  const float he = 0.5f * (float)D.ps[0].eps;
  const float *tape[FP];
  int first = 0;
#pragma unroll
  for (int p = FP - 1; p >= 0; --p)
    if (rows[p] >= 0) first = rows[p];
#pragma unroll
  for (int p = 0; p < FP; ++p) {
    const int j = rows[p] >= 0 ? rows[p] : first;
    tape[p] = D.ftape + (long long)j * F.L * F.tape_stride;
    for (int c = lane; c < MAXD; c += 64) {
      if (c < F.d)
        S.xs[p][xpos(c, F.d)] =
            rows[p] >= 0 ? D.grad_t[(long long)rows[p] * D.DS + c] * expf(D.fa[c]) : 0.f;
      else
        S.xs[p][c] = 0.f;
    }
  }
  __syncthreads();
  vjp_couplings(F, D.fwb, S, tape, lane);
#pragma unroll
  for (int p = 0; p < FP; ++p)
    if (rows[p] >= 0)
      for (int c = lane; c < F.d; c += 64) {
        const long long e = (long long)rows[p] * D.DS + c;
        const float g = S.xs[p][c];
        D.fgz[e] = g;
        D.p_t[e] = fmaf(he, g, D.p_t[e]);
      }
}

// New parameters from the caller: restart the Adam moments, and count Adam
// steps from the next iteration on.
__global__ void k_flow_reset(Dev D, FlowNet F) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < F.nparams; i += gridDim.x * blockDim.x) {
    D.fadm[i] = 0.f;
    D.fadv[i] = 0.f;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) D.fstate[0] = D.ps[0].k * F.ntrain;
}

// The gradient the last Adam step used: the ordered sum of the chunk partials.
__global__ void k_flow_gradsum(FlowNet F, const float *part, float *out) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < F.nparams; i += gridDim.x * blockDim.x) {
    double g = 0.0;
    for (int s = 0; s < KSPLIT; ++s) g += (double)part[(long long)s * F.nparams + i];
    out[i] = (float)g;
  }
}

}  // namespace

hipError_t launch_flow_gradsum(const Dev &D, const FlowNet &F, float *out, hipStream_t st) {
  hipLaunchKernelGGL(k_flow_gradsum, dim3(256), dim3(256), 0, st, F, (const float *)D.fgrad, out);
  return hipGetLastError();
}

hipError_t launch_flow_set(const Dev &D, const FlowNet &F, hipStream_t st) {
  hipLaunchKernelGGL(k_flow_reset, dim3(256), dim3(256), 0, st, D, F);
  hipLaunchKernelGGL(k_flow_adam, dim3(256), dim3(256), 0, st, D, F, 0, 0, (const float *)nullptr);
  return hipGetLastError();
}

hipError_t launch_flow_init(const Dev &D, const FlowNet &F, hipStream_t st) {
  hipLaunchKernelGGL(k_flow_init, dim3(256), dim3(256), 0, st, D, F);
  hipLaunchKernelGGL(k_flow_adam, dim3(256), dim3(256), 0, st, D, F, 0, 0, (const float *)nullptr);
  return hipGetLastError();
}

hipError_t launch_flow_publish(const Dev &D, const FlowNet &F, hipStream_t st) {
  hipLaunchKernelGGL(k_flow_adam, dim3(256), dim3(256), 0, st, D, F, 0, 0, (const float *)nullptr);
  return hipGetLastError();
}

hipError_t launch_flow_base(const Dev &D, const FlowNet &F, hipStream_t st) {
  hipLaunchKernelGGL(k_flow_base, dim3(1), dim3(256), 0, st, D, F);
  return hipGetLastError();
}

hipError_t launch_flow_train(const Dev &D, const FlowNet &F, int step, hipStream_t st) {
  const int blocks = (D.J + FP - 1) / FP;
  hipLaunchKernelGGL(k_flow_train, dim3(blocks), dim3(64), 0, st, D, F);
  int nb = 0;
  for (int l = 0; l < F.L; ++l) {
    const FlowLayerDesc &Y = F.ly[l];
    const int rc[3][2] = {{2 * Y.dt, FH}, {FH, FH}, {FH, Y.dc}};
    for (int w = 0; w < 3; ++w) nb += ((rc[w][0] + 63) / 64) * ((rc[w][1] + 63) / 64) + 1;
  }
  hipLaunchKernelGGL(k_flow_wgrad, dim3(nb, KSPLIT), dim3(256), 0, st, D, F, D.fgrad);
  hipLaunchKernelGGL(k_flow_adam, dim3(256), dim3(256), 0, st, D, F, step, 1,
                     (const float *)D.fgrad);
  return hipGetLastError();
}

hipError_t launch_flow_begin(const Dev &D, const FlowNet &F, hipStream_t st) {
  hipLaunchKernelGGL(k_flow_begin, dim3((D.J + FP - 1) / FP), dim3(64), 0, st, D, F);
  return hipGetLastError();
}

hipError_t launch_flow_drift(const Dev &D, const FlowNet &F, int step, hipStream_t st) {
  hipLaunchKernelGGL(k_flow_drift, dim3((D.J + FP - 1) / FP), dim3(64), 0, st, D, F, step);
  return hipGetLastError();
}

hipError_t launch_flow_kick(const Dev &D, const FlowNet &F, int step, hipStream_t st) {
  hipLaunchKernelGGL(k_flow_kick, dim3((D.J + FP - 1) / FP), dim3(64), 0, st, D, F, step);
  return hipGetLastError();
}

}  // namespace smc
