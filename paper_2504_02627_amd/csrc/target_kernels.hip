// Synthetic targets on the device: those of Sec. IV -- the Gaussian (dense
// precision, the D = 5 and the ill-conditioned D = 100 examples) and the
// Rosenbrock (banana) density -- and Neal's funnel, which Sec. VI names as
// future work.  One posterior per context; rows are the particles of
// posterior 0 in the trajectory buffers.
//
// A leapfrog step (eqs. LF_p1/2, LF_theta, LF_p; gradient cached between
// steps) is one launch: drift, gradient at the new position and the second
// half kick, for the particles with n_j > s.  The Gaussian gradient
// g = -P (theta - mu) of a block of 16 particles is a 16 x d by d x d product
// on v_mfma_f32_16x16x4f32 (one wave per 16-feature output tile, P read from
// L2); the banana gradient is elementwise.  The log density at the end of a
// trajectory (and at theta_0) is evaluated in binary64 from the FP32 state.

#include <hip/hip_runtime.h>
#include <math.h>

#include "chees_smc.h"
#include "dev_common.h"
#include "smc_internal.h"

namespace smc {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int GT = 16;  // particles per Gaussian work group

// ---------------------------------------------------------------------------
// Gaussian step.  LDS: theta' and p + h g of the 16 particles, and
// theta' - mu (zero beyond d), row stride DS + 1 (bank spread).
// grad_only = 1: the gradient at the current theta (initial draw), written
// to grad_t only.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_gauss_step(Dev D, int s, int grad_only) {
  extern __shared__ float lds[];
  const int DS = D.DS, LS = DS + 1;
  float *th1 = lds, *phl = lds + GT * LS, *dl = lds + 2 * GT * LS;
  const int tile = blockIdx.x;
  if (tile * GT >= D.active[s]) return;  // sorted by n: no particle of the tile moves
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const float eps = grad_only ? 0.f : (float)D.ps[0].eps;
  const float he = 0.5f * eps;
  const int d = D.posts[0].d;
  for (int e = tid; e < GT * DS; e += blockDim.x) {
    const int i = e / DS, k = e - i * DS;
    const long long o = (long long)D.perm[tile * GT + i] * DS + k;
    const float t0 = D.theta_t[o], p0 = D.p_t[o], g0 = D.grad_t[o];
    const float ph = fmaf(he, g0, p0);
    const float t1 = fmaf(eps * D.minv[k], ph, t0);
    th1[i * LS + k] = t1;
    phl[i * LS + k] = ph;
    dl[i * LS + k] = k < d ? t1 - D.tmean[k] : 0.f;
  }
  __syncthreads();
  // output tile: particles 0..15 x features 16 wave .. 16 wave + 15
  const int f0 = 16 * wave;
  v4f acc = {0.f, 0.f, 0.f, 0.f};
  const float *Pc = D.tprec + f0 + (lane & 15);
  for (int k0 = 0; k0 < DS; k0 += 4) {
    const int k = k0 + (lane >> 4);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(dl[(lane & 15) * LS + k], Pc[(long long)k * DS], acc,
                                               0, 0, 0);
  }
  const int f = f0 + (lane & 15);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = 4 * (lane >> 4) + r;
    const int row = D.perm[tile * GT + i];
    if (D.n[row] <= s) continue;
    const long long o = (long long)row * DS + f;
    const float g1 = f < d ? -acc[r] : 0.f;
    D.grad_t[o] = g1;
    if (!grad_only) {
      D.theta_t[o] = th1[i * LS + f];
      D.p_t[o] = fmaf(he, g1, phl[i * LS + f]);
    }
  }
}

// ---------------------------------------------------------------------------
// Banana step: one thread per particle, d = 2.
//   grad_1 = -theta_1 / s1^2 + 2 b theta_1 r,  grad_2 = -r,
//   r = theta_2 - b (theta_1^2 - c).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_banana_step(Dev D, int s, int grad_only) {
  const int slot = blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= D.active[s]) return;
  const int row = D.perm[slot];
  const float eps = grad_only ? 0.f : (float)D.ps[0].eps;
  const float he = 0.5f * eps;
  const long long o = (long long)row * D.DS;
  float t[2], ph[2];
  for (int k = 0; k < 2; ++k) {
    ph[k] = fmaf(he, D.grad_t[o + k], D.p_t[o + k]);
    t[k] = fmaf(eps * D.minv[k], ph[k], D.theta_t[o + k]);
  }
  const float s1 = (float)D.bs1, bb = (float)D.bb, cc = (float)D.bc;
  const float r = t[1] - bb * (t[0] * t[0] - cc);
  const float g[2] = {-t[0] / (s1 * s1) + 2.f * bb * t[0] * r, -r};
  for (int k = 0; k < 2; ++k) {
    D.grad_t[o + k] = g[k];
    if (!grad_only) {
      D.theta_t[o + k] = t[k];
      D.p_t[o + k] = fmaf(he, g[k], ph[k]);
    }
  }
}

// ---------------------------------------------------------------------------
// Funnel step: one thread per particle, theta = (v, x_1..x_{d-1}).
//   grad_v = -v / sv^2 - (d - 1)/2 + e^{-v} |x|^2 / 2,  grad_x = -x e^{-v}.
// The drift is written first (theta', p + h g in the state rows), then the
// gradient at theta' and the kick read them back.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_funnel_step(Dev D, int s, int grad_only) {
  const int slot = blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= D.active[s]) return;
  const int row = D.perm[slot];
  const int d = D.posts[0].d;
  const float eps = grad_only ? 0.f : (float)D.ps[0].eps;
  const float he = 0.5f * eps;
  float *th = D.theta_t + (long long)row * D.DS, *p = D.p_t + (long long)row * D.DS,
        *g = D.grad_t + (long long)row * D.DS;
  float x2 = 0.f;
  for (int k = 0; k < d; ++k) {
    const float ph = fmaf(he, g[k], p[k]);
    const float t1 = fmaf(eps * D.minv[k], ph, th[k]);
    th[k] = t1;
    p[k] = ph;
    if (k > 0) x2 = fmaf(t1, t1, x2);
  }
  const float v = th[0], ev = __expf(-v), sv2 = (float)(D.fsv * D.fsv);
  for (int k = 0; k < d; ++k) {
    const float gk = k == 0 ? -v / sv2 - 0.5f * (float)(d - 1) + 0.5f * ev * x2 : -th[k] * ev;
    g[k] = gk;
    p[k] = fmaf(he, gk, p[k]);
  }
}

hipError_t launch_target_step(const Dev &D, int step, int grad_only, hipStream_t st) {
  if (D.target == SMC_TARGET_FUNNEL) {
    hipLaunchKernelGGL(k_funnel_step, dim3((D.Jcap + 255) / 256), dim3(256), 0, st, D, step,
                       grad_only);
  } else if (D.target == SMC_TARGET_GAUSSIAN) {
    const int threads = 64 * (D.DS / 16);
    const size_t lds = (size_t)3 * GT * (D.DS + 1) * sizeof(float);
    hipLaunchKernelGGL(k_gauss_step, dim3(D.Jcap / GT), dim3(threads), lds, st, D, step, grad_only);
  } else {
    hipLaunchKernelGGL(k_banana_step, dim3((D.Jcap + 255) / 256), dim3(256), 0, st, D, step,
                       grad_only);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// log pi(theta_t) in binary64 for every particle, written to logpi_t.  One
// wave per particle.
//   Gaussian: tconst - 1/2 (theta - mu)^T P (theta - mu), tconst = log_const
//             + 1/2 log det P - d/2 log 2 pi (host, Cholesky in binary64);
//   banana:   log N(theta_1; 0, s1^2) + log N(theta_2; b (theta_1^2 - c), 1)
//             + log_const;
//   funnel:   log N(v; 0, sv^2) + sum_i log N(x_i; 0, e^v) + log_const.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_target_energy(Dev D) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= D.J) return;
  const float *th = D.theta_t + (long long)j * D.DS;
  const int d = D.posts[0].d;
  if (D.target == SMC_TARGET_GAUSSIAN) {
    double q = 0.0;
    for (int k = lane; k < d; k += 64) {
      const double dk = (double)th[k] - (double)D.tmean[k];
      double row = 0.0;
      for (int l = 0; l < d; ++l)
        row += (double)D.tprec[(long long)k * D.DS + l] * ((double)th[l] - (double)D.tmean[l]);
      q += dk * row;
    }
    q = wave_sum(q);
    if (lane == 0) D.logpi_t[j] = D.tconst - 0.5 * q;
  } else if (D.target == SMC_TARGET_FUNNEL) {
    // log N(v; 0, sv^2) + sum_i log N(x_i; 0, e^v)
    const double v = th[0];
    double x2 = 0.0;
    for (int k = 1 + lane; k < d; k += 64) x2 += (double)th[k] * (double)th[k];
    x2 = wave_sum(x2);
    if (lane == 0) {
      const double z = v / D.fsv;
      D.logpi_t[j] = D.tconst - 0.5 * z * z - log(D.fsv) - 0.5 * exp(-v) * x2 -
                     0.5 * (d - 1) * v - 0.5 * d * 1.8378770664093454836;  // log 2 pi
    }
  } else if (lane == 0) {
    const double t1 = th[0], t2 = th[1];
    const double r = t2 - D.bb * (t1 * t1 - D.bc);
    const double z = t1 / D.bs1;
    D.logpi_t[j] = D.tconst - 0.5 * z * z - log(D.bs1) - 0.5 * r * r -
                   1.8378770664093454836;  // log 2 pi
  }
}

hipError_t launch_target_energy(const Dev &D, hipStream_t st) {
  hipLaunchKernelGGL(k_target_energy, dim3((D.J + 3) / 4), dim3(256), 0, st, D);
  return hipGetLastError();
}

// Copies the Gaussian's mean and precision into the workspace, zero padded to
// the row stride.
__global__ void k_target_pack(Dev D, const float *__restrict__ mean,
                              const float *__restrict__ prec, int d) {
  const long long tot = (long long)D.DS * D.DS;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(e / D.DS), c = (int)(e % D.DS);
    D.tprec[e] = (r < d && c < d) ? prec[(long long)r * d + c] : 0.f;
    if (r == 0) D.tmean[c] = c < d ? mean[c] : 0.f;
  }
}

hipError_t launch_target_pack(const Dev &D, const float *mean, const float *prec, int d,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_target_pack, dim3(256), dim3(256), 0, st, D, mean, prec, d);
  return hipGetLastError();
}

}  // namespace smc
