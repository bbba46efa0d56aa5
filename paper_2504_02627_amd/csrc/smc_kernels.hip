// Device kernels of libchees_smc.so for gfx950 (CDNA4, wave64).
//
// Method: SMC sampler with a ChEES-HMC proposal (arXiv 2504.02627).  Each
// kernel names the passage of the paper it computes.  Floating-point
// contraction is off in this file: every fused multiply-add is written as an
// explicit fmaf so that the two places that compute the same drift produce the
// same bits.
#pragma clang fp contract(off)

#include <math.h>

#include <mutex>

#include "smc_internal.h"
#include "dev_common.h"

namespace smc {

typedef float v4f __attribute__((ext_vector_type(4)));

// Block reduction helpers for 1024-thread single-posterior kernels.
template <typename T, typename Op>
__device__ T block_reduce(T v, T *sh, Op op) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = op(v, __shfl_xor(v, o, 64));
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  T r = sh[0];
  for (int i = 1; i < nw; ++i) r = op(r, sh[i]);
  __syncthreads();
  return r;
}

// Blocks of the reductions over a population: g of G blocks takes rows
// g T + i, g T + i + G T, ...  (T threads); the block that finishes last
// (a device-scope counter, reset by that block) combines the G partials in
// block order, so the result is the same on every run.
constexpr int RED_T = 256;

inline int red_grid(int J) {
  const int g = (J + 2 * RED_T - 1) / (2 * RED_T);
  return g < 1 ? 1 : (g > RED_G ? RED_G : g);
}

// Called by every thread of the block; true in the block that counted last,
// whose threads then see the partials every block wrote before counting.
__device__ __forceinline__ bool red_last(int *cnt, int G) {
  __shared__ int last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    last = atomicAdd(cnt, 1) == G - 1;
    if (last) {
      *cnt = 0;  // every block has counted: ready for the next launch
      __threadfence();
    }
  }
  __syncthreads();
  return last;
}

struct OpAdd {
  template <typename T>
  __device__ T operator()(T a, T b) const { return a + b; }
};
struct OpMax {
  __device__ double operator()(double a, double b) const { return a > b ? a : b; }
};

// ---------------------------------------------------------------------------
// Packing of X and y into the MFMA operand layouts (once, at init).  dp = 16 C2.
//
// A part (GEMM1, Z^T = X Theta^T with v_mfma_f32_16x16x4f32, M = data rows,
//   K = features): lane l of data tile t holds X[16t + l%16][(l/16) 4C2 + c]
//   in slot c < 4 C2 (the K index of MFMA c is (l/16) 4C2 + c).
// B part (GEMM2, G = R X, M = particles, N = 16 features, K = 4 data rows):
//   lane l holds X[16t + 4(l/16) + i][16 ct + l%16] in slot 4 ct + i.
// Y part: lane l holds y[16t + 4(l/16) + i], i = 0..3 (1/2 for padded rows,
//   which makes the padded residual y - sigmoid(0) exactly zero).
// Per tile and lane: [A: 4C2 | B: 4C2 | Y: 4] floats = 2 C2 + 1 float4, so a
// data tile is one contiguous block of 64 (2 C2 + 1) float4.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ float to_f32(T v);
template <>
__device__ __forceinline__ float to_f32<float>(float v) { return v; }
template <>
__device__ __forceinline__ float to_f32<uint16_t>(uint16_t v) {
  return __uint_as_float(((uint32_t)v) << 16);  // bfloat16 -> float is exact
}

template <typename T>
__global__ void k_pack(const T *__restrict__ X, const float *__restrict__ y, int N, int d, int C2,
                       int NT, float *__restrict__ xab) {
  const int K1 = 4 * C2;
  const int LF = 2 * K1 + 4;  // floats per lane and tile
  const long long tot = (long long)NT * 64 * LF;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < tot;
       idx += (long long)gridDim.x * blockDim.x) {
    const int slot = (int)(idx % LF);
    const long long r = idx / LF;
    const int lane = (int)(r % 64);
    const int t = (int)(r / 64);
    float v;
    if (slot < K1) {
      const int n = 16 * t + (lane & 15), k = (lane >> 4) * K1 + slot;
      v = (n < N && k < d) ? to_f32<T>(X[(long long)n * d + k]) : 0.f;
    } else if (slot < 2 * K1) {
      const int sb = slot - K1, ct = sb >> 2, i = sb & 3;
      const int n = 16 * t + 4 * (lane >> 4) + i, k = 16 * ct + (lane & 15);
      v = (n < N && k < d) ? to_f32<T>(X[(long long)n * d + k]) : 0.f;
    } else {
      const int n = 16 * t + 4 * (lane >> 4) + (slot - 2 * K1);
      v = n < N ? y[n] : 0.5f;
    }
    xab[idx] = v;
  }
}

hipError_t launch_pack_one(const Dev &D, const void *X, const float *y, int x_dtype,
                           const HostPost &P, hipStream_t st) {
  const long long tot = (long long)P.NT * 64 * (8 * P.C2 + 4);
  int grid = (int)((tot + 255) / 256);
  if (grid > 65535) grid = 65535;
  if (x_dtype == 0)
    hipLaunchKernelGGL(k_pack<float>, dim3(grid), dim3(256), 0, st, (const float *)X, y, P.N, P.d,
                       P.C2, P.NT, D.xab + P.xab);
  else
    hipLaunchKernelGGL(k_pack<uint16_t>, dim3(grid), dim3(256), 0, st, (const uint16_t *)X, y,
                       P.N, P.d, P.C2, P.NT, D.xab + P.xab);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Packing for BF16 trajectory gradients (v_mfma_f32_32x32x16_bf16, 32
// particles per wave).  Each row carries the sign of its label,
// x~_n = (2 y_n - 1) x_n: then y_n - sigmoid(x_n . theta) =
// (2 y_n - 1) sigmoid(-x~_n . theta), so the tile loop needs no labels and the
// residual of a well-classified row comes out with full relative precision
// (no 1 - sigmoid cancellation).  The sign flip is exact in bfloat16 and
// round-to-nearest-even is symmetric, so the rounded operands and products
// are those of X, theta' and R = y - sigmoid rounded to bfloat16.
// Per 32-row data tile T and lane l (h = l / 32), in 16-byte slots of eight
// bfloat16:
//   A of GEMM1 (Z^T = X~ Theta'^T), K-step c < C2:
//        x~[32T + l%32][16c + 8h + e];
//   A of GEMM2 (G^T = X~^T R^T), feature tile f < NF = ceil(C2/2), K-step q:
//        x~[32T + 16q + 8(e>>2) + 4h + (e&3)][phi(f, l%32)],
//        phi(f, i) = 32f + 16(i>>4) + 8((i>>2)&1) + 4((i>>3)&1) + (i&3).
//   The row order of GEMM2's K follows GEMM1's output layout (lane l, register
//   v holds row 8(v/4) + 4h + v%4), and phi makes GEMM2's output register v of
//   tile f hold feature 32f + 16(v>>3) + 8h + (v&7): the layout of theta' in
//   GEMM1's B operand (K-step c = 2f + (v>>3), element v&7).
//   Slots: [A1: C2 | A2: 2 NF ([f][q])] plus a zero slot when that is even
//   (odd lane stride: conflict-free 16-byte LDS reads).  Rows past N are zero.
// A label other than 0 or 1 sets *bad (the precision form needs binary y).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
template <typename T>
__device__ __forceinline__ uint16_t to_bf16(T v);
template <>
__device__ __forceinline__ uint16_t to_bf16<float>(float v) { return bf16_rne(v); }
template <>
__device__ __forceinline__ uint16_t to_bf16<uint16_t>(uint16_t v) { return v; }

__host__ __device__ constexpr int b32_phi(int f, int i) {
  return 32 * f + 16 * (i >> 4) + 8 * ((i >> 2) & 1) + 4 * ((i >> 3) & 1) + (i & 3);
}

template <typename T>
__global__ void k_pack_bf16(const T *__restrict__ X, const float *__restrict__ y, int N, int d,
                            int C2, int NF, int NT2, int LS, uint4 *__restrict__ xbf,
                            int *__restrict__ bad) {
  const long long tot = (long long)NT2 * 64 * LS;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < tot;
       idx += (long long)gridDim.x * blockDim.x) {
    const int slot = (int)(idx % LS);
    const long long r = idx / LS;
    const int lane = (int)(r % 64);
    const int tl = (int)(r / 64);
    const int h = lane >> 5, i = lane & 31;
    uint32_t w[4] = {0, 0, 0, 0};
    if (slot < C2 + 2 * NF) {
      uint16_t v[8];
      for (int e = 0; e < 8; ++e) {
        int n, k;
        if (slot < C2) {
          n = 32 * tl + i;
          k = 16 * slot + 8 * h + e;
        } else {
          const int f = (slot - C2) >> 1, q = (slot - C2) & 1;
          n = 32 * tl + 16 * q + 8 * (e >> 2) + 4 * h + (e & 3);
          k = b32_phi(f, i);
        }
        uint16_t u = 0;
        if (n < N && k < d) {
          const float yn = y[n];
          if (yn != 0.f && yn != 1.f) *bad = 1;
          u = to_bf16<T>(X[(long long)n * d + k]);
          if (yn == 0.f) u ^= 0x8000u;  // sign of the label (exact)
        }
        v[e] = u;
      }
      for (int q = 0; q < 4; ++q) w[q] = (uint32_t)v[2 * q] | ((uint32_t)v[2 * q + 1] << 16);
    }
    xbf[idx] = make_uint4(w[0], w[1], w[2], w[3]);
  }
}

// Three-plane packing for the precision form's energies: X~ (label sign
// folded, as above) written exactly as hi + mid + lo, each the bfloat16
// rounding (nearest even) of what the previous parts leave (the remainders
// are exact in FP32, and the last one has at most eight significant bits).
// Layout per 32-row tile and lane l: slots [hi: C2 | mid: C2 | lo: C2] (+ a
// zero slot, odd stride), slot c of a plane holding features 16c + 8h + e
// (h = l / 32, e = 0..7) of row 32 T + l % 32: GEMM1's A operand.
template <typename T>
__global__ void k_pack_b3(const T *__restrict__ X, const float *__restrict__ y, int N, int d, int C2,
                          int NT2, int LS, uint4 *__restrict__ xb3) {
  const long long tot = (long long)NT2 * 64 * LS;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < tot;
       idx += (long long)gridDim.x * blockDim.x) {
    const int slot = (int)(idx % LS);
    const long long r = idx / LS;
    const int lane = (int)(r % 64);
    const int tl = (int)(r / 64);
    const int h = lane >> 5, n = 32 * tl + (lane & 31);
    uint32_t w[4] = {0, 0, 0, 0};
    if (slot < 3 * C2) {
      const int plane = slot / C2, c = slot % C2;
      uint16_t v[8];
      for (int e = 0; e < 8; ++e) {
        const int k = 16 * c + 8 * h + e;
        uint16_t u = 0;
        if (n < N && k < d) {
          float x = to_f32<T>(X[(long long)n * d + k]);
          if (y[n] == 0.f) x = -x;                      // sign of the label (exact)
          const uint16_t hi = bf16_rne(x);
          const float r1 = x - __uint_as_float((uint32_t)hi << 16);
          const uint16_t mid = bf16_rne(r1);
          const float r2 = r1 - __uint_as_float((uint32_t)mid << 16);
          u = plane == 0 ? hi : (plane == 1 ? mid : bf16_rne(r2));
        }
        v[e] = u;
      }
      for (int q = 0; q < 4; ++q) w[q] = (uint32_t)v[2 * q] | ((uint32_t)v[2 * q + 1] << 16);
    }
    xb3[idx] = make_uint4(w[0], w[1], w[2], w[3]);
  }
}

hipError_t launch_pack_bf16(const Dev &D, const void *X, const float *y, int x_dtype,
                            const HostPost &P, hipStream_t st) {
  const int LS = bf16_lane_stride(P.C2);
  const long long tot = (long long)P.NT2 * 64 * LS;
  int grid = (int)((tot + 255) / 256);
  if (grid > 65535) grid = 65535;
  if (x_dtype == 0)
    hipLaunchKernelGGL(k_pack_bf16<float>, dim3(grid), dim3(256), 0, st, (const float *)X, y, P.N,
                       P.d, P.C2, P.KC, P.NT2, LS, D.xbf + P.xbf, D.status);
  else
    hipLaunchKernelGGL(k_pack_bf16<uint16_t>, dim3(grid), dim3(256), 0, st, (const uint16_t *)X, y,
                       P.N, P.d, P.C2, P.KC, P.NT2, LS, D.xbf + P.xbf, D.status);
  const int LS3 = b3_lane_stride(P.C2);
  const long long tot3 = (long long)P.NT2 * 64 * LS3;
  int grid3 = (int)((tot3 + 255) / 256);
  if (grid3 > 65535) grid3 = 65535;
  if (x_dtype == 0)
    hipLaunchKernelGGL(k_pack_b3<float>, dim3(grid3), dim3(256), 0, st, (const float *)X, y, P.N,
                       P.d, P.C2, P.NT2, LS3, D.xb3 + P.xb3);
  else
    hipLaunchKernelGGL(k_pack_b3<uint16_t>, dim3(grid3), dim3(256), 0, st, (const uint16_t *)X, y,
                       P.N, P.d, P.C2, P.NT2, LS3, D.xb3 + P.xb3);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fill helpers.
// ---------------------------------------------------------------------------
__global__ void k_fill_f32(float *p, long long n, float v) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_fill_i32(int *p, long long n, int v) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_fill_f64(double *p, long long n, double v) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t fill_f32(float *p, long long n, float v, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_f32, dim3(1024), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}
hipError_t fill_i32(int *p, long long n, int v, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_i32, dim3(256), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}
hipError_t fill_f64(double *p, long long n, double v, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_f64, dim3(256), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Initial draw theta_0 ~ q0 = N(0, prior_var I)  (eq. init_sample), or a copy of
// the caller's theta_0, into the trajectory buffer; momenta and gradients zero.
// One thread per (row, 4-column Philox block).
// ---------------------------------------------------------------------------
__global__ void k_init_theta(Dev D, const float *__restrict__ theta0) {
  const int nblk = D.DS / 4;
  const long long tot = (long long)D.B * D.Jcap * nblk;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < tot;
       idx += (long long)gridDim.x * blockDim.x) {
    const int blk = (int)(idx % nblk);
    const int row = (int)(idx / nblk);
    const int b = row / D.Jcap, j = row % D.Jcap;
    const Post P = D.posts[b];
    double v[4] = {0, 0, 0, 0};
    if (j < D.J) {
      if (theta0) {
        for (int q = 0; q < 4; ++q) {
          const int c = 4 * blk + q;
          if (c < P.d) v[q] = theta0[P.uoff + (long long)j * P.d + c];
        }
      } else if (4 * blk < P.d) {
        box_muller4(philox_at(D.seed, blk, (uint32_t)(b * D.J + j), 0, STREAM_INIT), v);
        const double s = sqrt(D.prior_var);
        for (int q = 0; q < 4; ++q) v[q] = (4 * blk + q < P.d) ? s * v[q] : 0.0;
      }
    }
    for (int q = 0; q < 4; ++q) {
      const long long o = (long long)row * D.DS + 4 * blk + q;
      D.theta_t[o] = (float)v[q];
      D.p_t[o] = 0.f;
      D.grad_t[o] = 0.f;
    }
    if (blk == 0) {
      D.n[row] = j < D.J ? 1 : 0;
      D.perm[row] = j;
    }
  }
  // one leapfrog "step" of size zero evaluates the gradient at theta_0
  const long long tb = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (tb < D.B) {
    int *a = D.active + tb * (D.nmax + 1);
    a[0] = D.J;
    for (int s = 1; s <= D.nmax; ++s) a[s] = 0;
  }
}

hipError_t launch_init_theta(const Dev &D, const float *theta0, hipStream_t st) {
  hipLaunchKernelGGL(k_init_theta, dim3(1024), dim3(256), 0, st, D, theta0);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fused leapfrog step with the batched logistic-regression gradient.
//
// Leapfrog (Sec. II-A, eqs. LF_p1/2, LF_theta, LF_p) with the gradient cached
// from the previous step:
//   p_half = p + eps/2 g;  theta' = theta + eps M^{-1} p_half;
//   g' = X^T (y - sigmoid(X theta')) - theta'/prior_var;  p' = p_half + eps/2 g'.
// Particles with n_j <= s are left alone (per-particle trajectory length).
//
// k_lf_partial: work item = (posterior, 128-particle tile, data-row split).
// Each of the 4 waves owns 2 x 16 particles.  Per 16-row data tile:
//   GEMM1  Z^T (16 rows x 16 particles) = X_A (16 x 4) Theta'^T (4 x 16),
//          4 C2 MFMAs (v_mfma_f32_16x16x4f32) accumulating over the features;
//   R = y - sigmoid(Z) elementwise on the accumulator registers;
//   GEMM2  G (16 particles x 16 features) += R (16 x 4) X_B (4 x 16): the
//          accumulator of GEMM1 is directly the A operand of GEMM2 (the data-row
//          index of GEMM2's K follows GEMM1's row layout), so Z never leaves
//          registers.
// Data tiles stream through LDS, double-buffered: the 256 threads load tile
// t+1 from global memory while the waves compute on tile t, and every wave
// reads its operands with 16-byte LDS reads (lane stride padded by 16 bytes to
// avoid bank conflicts).  The split writes its partial gradient.
// k_lf_reduce: sums the partials of each tile in split order (deterministic),
// adds the prior term and applies the second half kick.  The kernel boundary
// makes the partials visible; no cross-work-group synchronisation is needed.
// ---------------------------------------------------------------------------
struct Plan {
  int b, tile, split, S, wbase;
};

// Plan of the leapfrog launches at step s, written once per iteration by
// k_lf_plan from the active counts (one work group per step and feature-tile
// group).  About lf_target times the resident work groups per compute unit
// items (one wave of resident work groups on 256 compute units) are spread
// over the active tiles in proportion to their data tiles; within a posterior
// the tiles get split counts that differ by at most one, so items carry nearly
// equal work.  Items are enumerated posterior by posterior, tile by tile, split
// by split.  Per posterior the table lf_post holds (first item, splits per
// tile, tiles with one more split, active tiles); per launch lf_items holds
// each item's (posterior, tile, split | S << 16, first item of its tile).

// data units of a posterior in the leapfrog kernels: 16-row tiles (FP32) or
// LDS stages of 32-row tiles (BF16)
__device__ __forceinline__ int lf_units(const Dev &D, const Post &P) {
  return D.bf16 ? P.NT2 / bf16_stage_tiles(P.C2) : P.NT;
}

constexpr int PLAN_THREADS = 256;

__global__ __launch_bounds__(PLAN_THREADS) void k_lf_plan(Dev D) {
  __shared__ long long red[PLAN_THREADS];
  __shared__ int scan[PLAN_THREADS];
  const int s = blockIdx.x, g = blockIdx.y, c2 = D.group_c2[g], tid = threadIdx.x;
  const int *act = D.active + s;
  const int stride = D.nmax + 1;
  // U: data tiles times active particle tiles over the group's posteriors
  long long u = 0;
  for (int b = tid; b < D.B; b += PLAN_THREADS) {
    const Post &P = D.posts[b];
    if (P.C2 == c2) u += (long long)((act[b * stride] + TJ - 1) / TJ) * lf_units(D, P);
  }
  red[tid] = u;
  __syncthreads();
  for (int h = PLAN_THREADS / 2; h > 0; h >>= 1) {
    if (tid < h) red[tid] += red[tid + h];
    __syncthreads();
  }
  const long long U = red[0];
  const long long share = (long long)D.lf_target * lf_groups_per_cu(D.bf16, c2);
  // per posterior: item count, splits per tile; exclusive prefix of the counts
  int run = 0;
  for (int b0 = 0; b0 < D.B; b0 += PLAN_THREADS) {
    const int b = b0 + tid;
    int T = 0, items = 0, base = 0, extra = 0;
    bool mine = false;
    if (b < D.B) {
      const Post &P = D.posts[b];
      mine = P.C2 == c2;
      if (mine) T = (act[b * stride] + TJ - 1) / TJ;
      if (T > 0 && U > 0) {
        const int NU = lf_units(D, P);
        long long G = (share * T * NU) / U;  // this posterior's share of the items
        if (G < T || D.lf_nosplit) G = T;
        const long long cap = (long long)T * (NU < D.split_cap ? NU : D.split_cap);
        if (G > cap) G = cap;
        base = (int)(G / T);
        extra = (int)(G % T);
        items = (int)G;
      } else {
        T = 0;
      }
    }
    __syncthreads();  // scan[] of the previous chunk has been read
    scan[tid] = items;
    __syncthreads();
    for (int h = 1; h < PLAN_THREADS; h <<= 1) {
      const int v = tid >= h ? scan[tid - h] : 0;
      __syncthreads();
      scan[tid] += v;
      __syncthreads();
    }
    if (mine) D.lf_post[(long long)s * D.B + b] = make_int4(run + scan[tid] - items, base, extra, T);
    run += scan[PLAN_THREADS - 1];
  }
  if (tid == 0) D.lf_count[g * D.nmax + s] = run < D.lf_grid ? run : D.lf_grid;
  __syncthreads();  // lf_post of this block is visible to the whole block
  int4 *it = D.lf_items + ((long long)g * D.nmax + s) * D.lf_grid;
  for (int b = 0; b < D.B; ++b) {
    if (D.posts[b].C2 != c2) continue;
    const int4 q = D.lf_post[(long long)s * D.B + b];
    if (q.w == 0) continue;
    const int items = q.w * q.y + q.z, big = q.z * (q.y + 1);
    for (int w = tid; w < items; w += PLAN_THREADS) {
      int tile, split, S;
      if (w < big) {
        tile = w / (q.y + 1);
        split = w % (q.y + 1);
        S = q.y + 1;
      } else {
        tile = q.z + (w - big) / q.y;
        split = (w - big) % q.y;
        S = q.y;
      }
      const int wid = q.x + w;
      if (wid < D.lf_grid)
        it[wid] = make_int4(b, tile, split | (S << 16), q.x + tile * q.y + (tile < q.z ? tile : q.z));
    }
  }
}

hipError_t launch_lf_plan(const Dev &D, hipStream_t st) {
  hipLaunchKernelGGL(k_lf_plan, dim3(D.nmax, D.ngroups), dim3(PLAN_THREADS), 0, st, D);
  return hipGetLastError();
}

// Item of this work group in a leapfrog launch (false: nothing to do).
__device__ __forceinline__ bool lf_item(const Dev &D, int c2, int s, int wid, Plan &pl) {
  const int g = D.c2_group[c2];
  const long long slot = (long long)g * D.nmax + s;
  const int cnt = D.lf_count[slot];
  const int4 e = D.lf_items[slot * D.lf_grid + wid];
  if (wid >= cnt) return false;
  pl.b = e.x;
  pl.tile = e.y;
  pl.split = e.z & 0xffff;
  pl.S = e.z >> 16;
  pl.wbase = e.w;
  return true;
}

// softplus(z) = max(z, 0) + ln 2 log2(1 + 2^(-|z| log2 e)) with the hardware
// exp2/log2; the absolute error per term is a few 1e-8.
__device__ __forceinline__ float softplusf_hw(float z) {
  const float e = __builtin_amdgcn_exp2f(-fabsf(z) * 1.4426950408889634f);
  return fmaxf(z, 0.f) + 0.6931471805599453f * __builtin_amdgcn_logf(1.0f + e);
}

__device__ __forceinline__ float sigmoidf_fast(float z) {
  // 1 / (1 + 2^(-z log2 e)) with the hardware exp2 and reciprocal
  const float e = __builtin_amdgcn_exp2f(-z * 1.4426950408889634f);
  return __builtin_amdgcn_rcpf(1.0f + e);
}

// LDS staging of packed data tiles, two 16-row tiles per stage, double
// buffered, with gfx950's direct global-to-LDS loads (global_load_lds_dwordx4:
// each lane's 16 bytes land at the wave-uniform LDS base + 16 * lane), so the
// prefetch of the next stage holds no registers.  A tile is copied verbatim:
// 64 lanes x (2 C2 + 1) float4 (A | B | y); the odd lane stride keeps the
// per-lane 16-byte operand reads free of bank conflicts.  Load m of a stage
// moves float4 [64 m, 64 m + 64) of it, which lie in tile m / (2 C2 + 1).
template <int C2>
struct Tiles {
  static constexpr int LSTR = 2 * C2 + 1;     // float4 per lane and tile
  static constexpr int TILE = 64 * LSTR;      // float4 per tile
  static constexpr int STAGE = 2 * TILE;      // two tiles
  static constexpr int NINST = STAGE / 64;    // wave-wide loads per stage
};

typedef __attribute__((address_space(3))) void lds_void;

template <int C2>
__device__ __forceinline__ void stage_issue(float4 *xs, const float4 *__restrict__ xab, int t,
                                            int t1, int wave, int lane) {
  using TL = Tiles<C2>;
  const float4 *src = xab + (long long)t * TL::TILE + lane;
#pragma unroll
  for (int k = 0; k < (TL::NINST + WAVES - 1) / WAVES; ++k) {
    const int m = wave + k * WAVES;
    // wave-uniform: skip loads past the split's last tile
    if (m < TL::NINST && t + m / TL::LSTR < t1)
      __builtin_amdgcn_global_load_lds((const void *)(src + 64 * m), (lds_void *)(xs + 64 * m), 16,
                                       0, 0);
  }
}

// End of a leapfrog step for one (particle row, feature) with the full
// likelihood gradient G: the arithmetic of the split reduction.
__device__ __forceinline__ void lf_finish(const Dev &D, long long row, int k, float G, float eps,
                                          float he, const float *minv, int mode) {
  const long long e = row * D.DS + k;
  const float inv_pv = (float)(1.0 / D.prior_var);
  const float t0 = D.theta_t[e];
  if (mode == 2) {  // gradient only: theta' was written by the caller
    D.grad_t[e] = G - t0 * inv_pv;
    return;
  }
  const float ph = fmaf(he, D.grad_t[e], D.p_t[e]);
  const float th1 = fmaf(eps * minv[k], ph, t0);
  const float gn = G - th1 * inv_pv;
  D.theta_t[e] = th1;
  D.p_t[e] = fmaf(he, gn, ph);
  D.grad_t[e] = gn;
}

// One work item of the FP32 fused step (posterior, particle tile, data-row
// split): each wave's 16 particles' partial likelihood gradient over the
// split's rows, in the output layout of GEMM2 (gacc[ct][rr]: particle slot
// 16 wave + 4 (lane / 16) + rr, feature 16 ct + lane % 16).  given: theta'
// of this step was formed by the previous reduction (theta_n).
template <int C2>
__device__ __forceinline__ void lf_unit_f32(const Dev &D, const Plan &pl, int s, int zero_eps,
                                            bool given, float4 (&xs)[2][Tiles<C2>::STAGE],
                                            v4f (&gacc)[SUB][C2]) {
  constexpr int K1 = 4 * C2;
  using TL = Tiles<C2>;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, kq = lane >> 4;
  const Post P = D.posts[pl.b];
  const float eps = zero_eps ? 0.f : (float)D.ps[pl.b].eps;
  const float he = 0.5f * eps;
  const float *minv = D.minv + (long long)pl.b * D.DS;
  const int *perm = D.perm + P.row0;

  // the first stage of data tiles is in flight while theta' is formed
  const int t0 = (int)((long long)pl.split * P.NT / pl.S);
  const int t1 = (int)((long long)(pl.split + 1) * P.NT / pl.S);
  const float4 *xab = reinterpret_cast<const float4 *>(D.xab + P.xab);
  stage_issue<C2>(xs[0], xab, t0, t1, wave, lane);

  // theta' of this wave's particles in the B-operand layout of GEMM1: after
  // the first step of the split path the previous reduction has written it
  // (the same arithmetic), so one array is read instead of three
  float th[SUB][K1];
#pragma unroll
  for (int sb = 0; sb < SUB; ++sb) {
    const int slot = pl.tile * TJ + (wave * SUB + sb) * 16 + (lane & 15);
    const long long base = (long long)(P.row0 + perm[slot]) * D.DS + kq * K1;
    if (given) {
#pragma unroll
      for (int c = 0; c < K1; ++c) th[sb][c] = D.theta_n[base + c];
    } else {
#pragma unroll
      for (int c = 0; c < K1; ++c) {
        const float t0 = D.theta_t[base + c], p0 = D.p_t[base + c], g0 = D.grad_t[base + c];
        const float ph = fmaf(he, g0, p0);
        // eps = 0 (gradient at the given theta): t0 + 0 * ph = t0 for finite
        // ph; written without a select, which costs this kernel its schedule
        th[sb][c] = fmaf(eps * minv[kq * K1 + c], ph, t0);
      }
    }
  }

#pragma unroll
  for (int sb = 0; sb < SUB; ++sb)
#pragma unroll
    for (int ct = 0; ct < C2; ++ct) gacc[sb][ct] = v4f{0.f, 0.f, 0.f, 0.f};

  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  int cur = 0;
  for (int t = t0; t < t1; t += 2) {
    const bool more = t + 2 < t1;
    if (more) stage_issue<C2>(xs[cur ^ 1], xab, t + 2, t1, wave, lane);
    const int ntt = (t + 1 < t1) ? 2 : 1;
    for (int tt = 0; tt < ntt; ++tt) {
      const float4 *xl = xs[cur] + tt * TL::TILE + lane * TL::LSTR;
      const float4 y4 = xl[2 * C2];
      const float ya[4] = {y4.x, y4.y, y4.z, y4.w};
#pragma unroll
      for (int sb = 0; sb < SUB; ++sb) {
        v4f z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < C2; ++q) {
          const float4 a = xl[q];
          z = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, th[sb][4 * q + 0], z, 0, 0, 0);
          z = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, th[sb][4 * q + 1], z, 0, 0, 0);
          z = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, th[sb][4 * q + 2], z, 0, 0, 0);
          z = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, th[sb][4 * q + 3], z, 0, 0, 0);
        }
        float r[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) r[i] = ya[i] - sigmoidf_fast(z[i]);
#pragma unroll
        for (int ct = 0; ct < C2; ++ct) {
          const float4 bb = xl[C2 + ct];
          gacc[sb][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(r[0], bb.x, gacc[sb][ct], 0, 0, 0);
          gacc[sb][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(r[1], bb.y, gacc[sb][ct], 0, 0, 0);
          gacc[sb][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(r[2], bb.z, gacc[sb][ct], 0, 0, 0);
          gacc[sb][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(r[3], bb.w, gacc[sb][ct], 0, 0, 0);
        }
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    cur ^= 1;
  }
}

// Partial gradient of an FP32 work item into a [TJ][DS] slot.
template <int C2>
__device__ __forceinline__ void lf_store_f32(const Dev &D, float *gp, const v4f (&gacc)[SUB][C2]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, kq = lane >> 4;
#pragma unroll
  for (int sb = 0; sb < SUB; ++sb)
#pragma unroll
    for (int ct = 0; ct < C2; ++ct)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int slot = (wave * SUB + sb) * 16 + 4 * kq + rr;
        gp[(long long)slot * D.DS + 16 * ct + (lane & 15)] = gacc[sb][ct][rr];
      }
}

// FIN: the plan has one split per tile (small data sets), so the item holds
// its particles' whole likelihood gradient and finishes the step itself
// (prior, second half kick, or the gradient only for zero_eps = 2), exactly as
// the split reduction does; no reduction launch follows.
template <int C2, bool FIN>
__global__ __launch_bounds__(WG, 2 * lf_groups_per_cu(false, C2)) void k_lf_partial(Dev D, int s, int zero_eps) {
  using TL = Tiles<C2>;
  __shared__ float4 xs[2][TL::STAGE];
  __shared__ Plan spl;
  if (threadIdx.x == 0) {
    Plan pl;
    if (!lf_item(D, C2, s, blockIdx.x, pl)) pl.b = -1;
    spl = pl;
  }
  __syncthreads();
  const Plan pl = spl;
  if (pl.b < 0) return;
  v4f gacc[SUB][C2];
  lf_unit_f32<C2>(D, pl, s, zero_eps, !FIN && s > 0 && !zero_eps, xs, gacc);

  if constexpr (FIN) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, kq = lane >> 4;
    const Post P = D.posts[pl.b];
    const float eps = zero_eps ? 0.f : (float)D.ps[pl.b].eps;
    const float he = 0.5f * eps;
    const float *minv = D.minv + (long long)pl.b * D.DS;
    const int *perm = D.perm + P.row0;
#pragma unroll
    for (int sb = 0; sb < SUB; ++sb)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int slot = (wave * SUB + sb) * 16 + 4 * kq + rr;
        const long long row = P.row0 + perm[pl.tile * TJ + slot];
        if (D.n[row] <= s) continue;
#pragma unroll
        for (int ct = 0; ct < C2; ++ct)
          lf_finish(D, row, 16 * ct + (lane & 15), gacc[sb][ct][rr], eps, he, minv, zero_eps);
      }
    return;
  }
  // partial gradient of this split: gpart[group's first slot + work item][slot][k]
  lf_store_f32<C2>(D, D.gpart + (long long)(D.lf_goff[D.c2_group[C2]] + blockIdx.x) * TJ * D.DS, gacc);
}

// ---------------------------------------------------------------------------
// Whole trajectories in one launch, for one posterior whose packed data tiles
// fit in LDS (small N d).  Each wave owns 16 sorted particle slots and runs
// their leapfrog steps s < n_j back to back with theta, p and the gradient in
// registers, in the output layout of GEMM2 (particle 4 (lane / 16) + r,
// feature 16 ct + lane % 16).  Per step: drift; theta' moved into the
// B-operand layout of GEMM1 through a per-wave LDS tile; GEMM1 -> sigmoid ->
// GEMM2 over every data tile; prior; second half kick; a particle past its
// n_j keeps its state.  The arithmetic is that of the one-split step kernel
// (k_lf_partial with FIN) except GEMM1's K order: the features are
// interleaved over the lane groups so that the MFMAs on the padding of d to
// 16 C2 are skipped (d = 5: 2 of 4), which changes the order of Z's sum only.
// BF: the precision form's operands, theta', X and R rounded to bfloat16
// (nearest even), on the FP32 MFMA: the products are exact and accumulate in
// FP32, as on the BF16 MFMA.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float bf16_val(float x) { return (float)(__bf16)x; }

// GEMM1 of one data tile in the whole-trajectory kernel, K interleaved over
// the lane groups (MFMA m takes features 4m .. 4m + 3, lane group kq feature
// 4m + kq), issuing only the RL MFMAs of the last group that reach a real
// feature (ceil(d/4) - 4 (C2 - 1)); the rest would multiply zero padding.
template <int C2, int RL>
__device__ __forceinline__ v4f traj_gemm1(const float4 *xl, const float *tB) {
  v4f z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int q = 0; q < C2 - 1; ++q) {
    const float4 a = xl[q];
    z = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, tB[4 * q + 0], z, 0, 0, 0);
    z = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, tB[4 * q + 1], z, 0, 0, 0);
    z = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, tB[4 * q + 2], z, 0, 0, 0);
    z = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, tB[4 * q + 3], z, 0, 0, 0);
  }
  const float4 a = xl[C2 - 1];
  const float *tq = tB + 4 * (C2 - 1);
  z = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, tq[0], z, 0, 0, 0);
  if constexpr (RL > 1) z = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, tq[1], z, 0, 0, 0);
  if constexpr (RL > 2) z = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, tq[2], z, 0, 0, 0);
  if constexpr (RL > 3) z = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, tq[3], z, 0, 0, 0);
  return z;
}

// The leapfrog steps of one wave's 16 particles (k_traj below), with RL
// GEMM1 MFMAs in the last operand group.
template <int C2, bool BF, int RL>
__device__ __forceinline__ void traj_steps(const Dev &D, const Post &P, const float4 *xall,
                                           float *T) {
  using TL = Tiles<C2>;
  constexpr int K1 = 4 * C2, FS = 16 * C2 + 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, kq = lane >> 4, col = lane & 15;
  const float eps = (float)D.ps[0].eps, he = 0.5f * eps;
  const float inv_pv = (float)(1.0 / D.prior_var);
  const int *perm = D.perm + P.row0;
  const int base = blockIdx.x * (16 * TRAJ_WAVES) + wave * 16;
  long long row[4];
  int nn[4];
  float th[C2][4], pp[C2][4], gg[C2][4], em[C2];
#pragma unroll
  for (int ct = 0; ct < C2; ++ct) em[ct] = eps * D.minv[16 * ct + col];
#pragma unroll
  for (int rr = 0; rr < 4; ++rr) {
    row[rr] = P.row0 + perm[base + 4 * kq + rr];
    nn[rr] = D.n[row[rr]];
#pragma unroll
    for (int ct = 0; ct < C2; ++ct) {
      const long long e = row[rr] * D.DS + 16 * ct + col;
      th[ct][rr] = D.theta_t[e];
      pp[ct][rr] = D.p_t[e];
      gg[ct][rr] = D.grad_t[e];
    }
  }
  // steps of this wave: the largest n_j of its 16 particles
  int nw = D.n[P.row0 + perm[base + col]];
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) nw = max(nw, __shfl_xor(nw, o));
  nw = __builtin_amdgcn_readfirstlane(nw);
  __syncthreads();  // the data tiles are in LDS

  for (int s = 0; s < nw; ++s) {
    float ph[C2][4], t1[C2][4];
#pragma unroll
    for (int ct = 0; ct < C2; ++ct)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        ph[ct][rr] = fmaf(he, gg[ct][rr], pp[ct][rr]);
        t1[ct][rr] = fmaf(em[ct], ph[ct][rr], th[ct][rr]);
        T[(4 * kq + rr) * FS + 16 * ct + col] = t1[ct][rr];
      }
    __builtin_amdgcn_wave_barrier();
    float tB[K1];  // tB[c] is feature 4c + kq
#pragma unroll
    for (int c = 0; c < K1; ++c) {
      tB[c] = T[col * FS + 4 * c + kq];
      if constexpr (BF) tB[c] = bf16_val(tB[c]);
    }
    v4f gacc[C2];
#pragma unroll
    for (int ct = 0; ct < C2; ++ct) gacc[ct] = v4f{0.f, 0.f, 0.f, 0.f};
    for (int t = 0; t < P.NT; ++t) {
      const float4 *xl = xall + t * TL::TILE + lane * TL::LSTR;
      const float4 y4 = xl[2 * C2];
      const float ya[4] = {y4.x, y4.y, y4.z, y4.w};
      const v4f z = traj_gemm1<C2, RL>(xl, tB);
      float r[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        r[i] = ya[i] - sigmoidf_fast(z[i]);
        if constexpr (BF) r[i] = bf16_val(r[i]);
      }
#pragma unroll
      for (int ct = 0; ct < C2; ++ct) {
        const float4 bb = xl[C2 + ct];
        gacc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(r[0], bb.x, gacc[ct], 0, 0, 0);
        gacc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(r[1], bb.y, gacc[ct], 0, 0, 0);
        gacc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(r[2], bb.z, gacc[ct], 0, 0, 0);
        gacc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(r[3], bb.w, gacc[ct], 0, 0, 0);
      }
    }
#pragma unroll
    for (int ct = 0; ct < C2; ++ct)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const float gn = gacc[ct][rr] - t1[ct][rr] * inv_pv;
        const bool on = s < nn[rr];
        th[ct][rr] = on ? t1[ct][rr] : th[ct][rr];
        pp[ct][rr] = on ? fmaf(he, gn, ph[ct][rr]) : pp[ct][rr];
        gg[ct][rr] = on ? gn : gg[ct][rr];
      }
    __builtin_amdgcn_wave_barrier();
  }
#pragma unroll
  for (int rr = 0; rr < 4; ++rr) {
    if (nn[rr] <= 0) continue;
#pragma unroll
    for (int ct = 0; ct < C2; ++ct) {
      const long long e = row[rr] * D.DS + 16 * ct + col;
      D.theta_t[e] = th[ct][rr];
      D.p_t[e] = pp[ct][rr];
      D.grad_t[e] = gg[ct][rr];
    }
  }
}

template <int C2, bool BF>
__global__ __launch_bounds__(64 * TRAJ_WAVES) void k_traj(Dev D) {
  using TL = Tiles<C2>;
  constexpr int K1 = 4 * C2, LF = 4 * TL::LSTR, FS = 16 * C2 + 1;
  extern __shared__ float4 xall[];                // every data tile of the posterior
  __shared__ float tb[TRAJ_WAVES][16 * FS];        // per-wave theta' transpose
  const Post P = D.posts[0];
  const int tid = threadIdx.x;
  // the packed tiles into LDS; the GEMM1 operands re-ordered on the way to
  // the interleaved K order (slot c of lane (n, kq) <- feature 4c + kq, which
  // the packing holds in lane (n, f / K1), slot f mod K1)
  const float *xf = D.xab + P.xab;
  const int nx = P.NT * TL::TILE;
  for (int e = tid; e < nx; e += 64 * TRAJ_WAVES) {
    const int t = e / TL::TILE, r = e - t * TL::TILE;
    const int ln = r / TL::LSTR, q = r - ln * TL::LSTR;
    float v[4];
    if (q < C2) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int f = 4 * (4 * q + i) + (ln >> 4);
        v[i] = xf[((long long)t * 64 + (ln & 15) + 16 * (f / K1)) * LF + f % K1];
      }
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) v[i] = xf[((long long)t * 64 + ln) * LF + 4 * q + i];
    }
    if constexpr (BF) {
#pragma unroll
      for (int i = 0; i < 4; ++i) v[i] = bf16_val(v[i]);  // labels, 1/2 padding exact
    }
    xall[e] = make_float4(v[0], v[1], v[2], v[3]);
  }
  float *T = tb[threadIdx.x >> 6];
  switch ((P.d + 3) / 4 - 4 * (C2 - 1)) {
    case 1: traj_steps<C2, BF, 1>(D, P, xall, T); break;
    case 2: traj_steps<C2, BF, 2>(D, P, xall, T); break;
    case 3: traj_steps<C2, BF, 3>(D, P, xall, T); break;
    default: traj_steps<C2, BF, 4>(D, P, xall, T);
  }
}

size_t traj_lds_bytes(int c2, int nt) { return (size_t)nt * 64 * (2 * c2 + 1) * 16; }

hipError_t launch_traj(const Dev &D, int c2, hipStream_t st) {
  const dim3 grid(D.Jcap / (16 * TRAJ_WAVES)), block(64 * TRAJ_WAVES);
  const size_t lds = D.traj_lds;
  if (c2 == 1 && D.bf16)
    hipLaunchKernelGGL((k_traj<1, true>), grid, block, lds, st, D);
  else if (c2 == 1)
    hipLaunchKernelGGL((k_traj<1, false>), grid, block, lds, st, D);
  else if (c2 == 2 && D.bf16)
    hipLaunchKernelGGL((k_traj<2, true>), grid, block, lds, st, D);
  else if (c2 == 2)
    hipLaunchKernelGGL((k_traj<2, false>), grid, block, lds, st, D);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fused leapfrog step with BF16 trajectory gradients (precision form):
// theta', X and R in bfloat16 on v_mfma_f32_32x32x16_bf16 with FP32
// accumulation.  Work item as in k_lf_partial (posterior, 128-particle tile,
// data-row split); a work group is four waves of 32 particles.  Per 32-row
// data tile and wave:
//   GEMM1  Z~^T (32 rows x 32 particles) = X~ Theta'^T, C2 MFMAs (K = 16
//          features each);
//   R = sigmoid(-Z~) on the lane's 16 accumulator values (with the label
//          signs folded into X~, this is (2y - 1)(y - sigmoid(Z))), rounded
//          to bfloat16 as GEMM2's B operand (two K-steps of 16 rows);
//   GEMM2  G^T (32 features x 32 particles) += X~^T R^T, 2 NF MFMAs.
// theta' stays in registers as GEMM1's B operand; G's registers line up with
// it, so the step's end needs no shuffle.  Data tiles are staged through two
// named LDS buffers by direct global-to-LDS loads (global_load_lds_dwordx4);
// because the buffers are distinct objects, the compiler need not wait for
// the next stage's loads before reading the current buffer, and the
// prefetch holds no registers.  Two tiles per stage wherever both stages of
// the resident work groups fit the LDS (every width but 10 feature tiles),
// one otherwise.
// The drift, the partials and the reduction are those of the FP32 kernel.
// Exactness of the weights does not depend on the gradient's precision: the
// leapfrog map with any position-only force field is volume preserving and
// reversible, and the energies are recomputed from the FP32 data.
// ---------------------------------------------------------------------------
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

__device__ __forceinline__ v8bf as_v8bf(uint4 u) { return __builtin_bit_cast(v8bf, u); }

template <int C2>
struct B32 {
  static constexpr int NF = (C2 + 1) / 2;          // 32-feature tiles of GEMM2
  static constexpr int LS = bf16_lane_stride(C2);  // uint4 per lane and 32-row tile
  static constexpr int TILE = 64 * LS;             // uint4 per tile
  static constexpr int STT = bf16_stage_tiles(C2);  // tiles per stage
  static constexpr int STAGE = STT * TILE;
  static constexpr int NINST = STAGE / 64;         // wave-wide 16-byte loads per stage
};

// Direct loads of the stage starting at data tile t into `buf` (every tile of
// a stage exists: the tile count is padded to whole stages).
template <int C2>
__device__ __forceinline__ void b32_issue(uint4 *__restrict__ buf, const uint4 *__restrict__ xbf,
                                          int t, int wave, int lane) {
  using TL = B32<C2>;
  const uint4 *src = xbf + (long long)t * TL::TILE + lane;
#pragma unroll
  for (int k = 0; k < (TL::NINST + B32_WAVES - 1) / B32_WAVES; ++k) {
    const int m = wave + k * B32_WAVES;
    if (m < TL::NINST)
      __builtin_amdgcn_global_load_lds((const void *)(src + 64 * m), (lds_void *)(buf + 64 * m), 16,
                                       0, 0);
  }
}

// R = sigmoid(-z~) = 1 / (1 + 2^(z~ log2 e)), hardware exp2 and reciprocal,
// rounded to bfloat16 (nearest even) as GEMM2's B operand: half H holds the
// lane's values 8 H .. 8 H + 7 (GEMM2's K-step H).
template <int H>
__device__ __forceinline__ void b32_residual_half(const v16f &z, v8bf &r) {
#pragma unroll
  for (int v = 0; v < 8; ++v)
    r[v] = (__bf16)__builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(z[8 * H + v] * 1.4426950408889634f));
}
// Both halves together (the single-tile stage).
__device__ __forceinline__ void b32_residual(const v16f &z, v8bf &r0, v8bf &r1) {
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    r0[v] = (__bf16)__builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(z[v] * 1.4426950408889634f));
    r1[v] = (__bf16)__builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(z[8 + v] * 1.4426950408889634f));
  }
}

// The STT tiles of one stage in buffer xs (lane's slots at xs + lane * LS).
template <int C2>
__device__ __forceinline__ void b32_stage(const uint4 *__restrict__ xs, const v8bf (&thb)[C2],
                                          v16f (&g)[B32<C2>::NF]) {
  using TL = B32<C2>;
  constexpr int NF = TL::NF;
  if constexpr (TL::STT == 2) {
    // both tiles' GEMM1 first: the first tile's residuals overlap the second's MFMAs
    const uint4 *x0 = xs, *x1 = xs + TL::TILE;
    v16f z0 = {}, z1 = {};
#pragma unroll
    for (int c = 0; c < C2; ++c) z0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_v8bf(x0[c]), thb[c], z0, 0, 0, 0);
#pragma unroll
    for (int c = 0; c < C2; ++c) z1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_v8bf(x1[c]), thb[c], z1, 0, 0, 0);
    // each g[f] takes tile a's K-steps 0 and 1, then tile b's, as in the
    // one-tile stage; the first K-steps of all f go before the second ones,
    // so that each residual half is due only when its K-step starts
    v8bf ra0, ra1, rb0, rb1;
    b32_residual_half<0>(z0, ra0);
    b32_residual_half<1>(z0, ra1);
#pragma unroll
    for (int f = 0; f < NF; ++f)
      g[f] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_v8bf(x0[C2 + 2 * f]), ra0, g[f], 0, 0, 0);
#pragma unroll
    for (int f = 0; f < NF; ++f)
      g[f] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_v8bf(x0[C2 + 2 * f + 1]), ra1, g[f], 0, 0, 0);
    b32_residual_half<0>(z1, rb0);
    b32_residual_half<1>(z1, rb1);
#pragma unroll
    for (int f = 0; f < NF; ++f)
      g[f] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_v8bf(x1[C2 + 2 * f]), rb0, g[f], 0, 0, 0);
#pragma unroll
    for (int f = 0; f < NF; ++f)
      g[f] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_v8bf(x1[C2 + 2 * f + 1]), rb1, g[f], 0, 0, 0);
    // issue order (scheduling groups: 0x008 MFMA, 0x002 VALU, 0x400
    // transcendental, 0x100 LDS read): tile a's GEMM1 (reading tile b's GEMM1
    // operands), tile b's GEMM1 beside the first half of tile a's residuals,
    // then the GEMM2 K-steps of a (0, 1) and b (0) each beside the next
    // residual half (a: second; b: first, second), then b's K-step 1; a wave's
    // VALU work runs while its own MFMAs execute, and each phase reads the
    // next phase's LDS operands
    constexpr int HV = 20, HT = 16;  // VALU and transcendental ops per residual half
    constexpr int V1 = (HV + C2 - 1) / C2, T1 = (HT + C2 - 1) / C2;
    constexpr int V2 = (HV + NF - 1) / NF, T2 = (HT + NF - 1) / NF;
    constexpr int D1 = (2 * NF + C2 - 1) / C2, D2 = 2;
    __builtin_amdgcn_sched_group_barrier(0x100, C2, 0);
#pragma unroll
    for (int c = 0; c < C2; ++c) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    }
#pragma unroll
    for (int c = 0; c < C2; ++c) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x100, D1, 0);
      __builtin_amdgcn_sched_group_barrier(0x002, V1, 0);
      __builtin_amdgcn_sched_group_barrier(0x400, T1, 0);
    }
#pragma unroll
    for (int f = 0; f < 3 * NF; ++f) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x100, D2, 0);
      __builtin_amdgcn_sched_group_barrier(0x002, V2, 0);
      __builtin_amdgcn_sched_group_barrier(0x400, T2, 0);
    }
    __builtin_amdgcn_sched_group_barrier(0x008, NF, 0);
  } else {
    v16f z = {};
#pragma unroll
    for (int c = 0; c < C2; ++c) z = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_v8bf(xs[c]), thb[c], z, 0, 0, 0);
    v8bf r0, r1;
    b32_residual(z, r0, r1);
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      g[f] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_v8bf(xs[C2 + 2 * f]), r0, g[f], 0, 0, 0);
      g[f] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_v8bf(xs[C2 + 2 * f + 1]), r1, g[f], 0, 0, 0);
    }
  }
}

// One work item of the BF16 fused step: the partial gradient of this wave's
// 32 particles over the split's rows; register v of g[f] holds feature
// 32f + 16(v>>3) + 8h + (v&7) of particle slot 32 wave + lane % 32.
template <int C2>
__device__ __forceinline__ void lf_unit_b32(const Dev &D, const Plan &pl, int s, int zero_eps,
                                            bool given, uint4 *__restrict__ bufA,
                                            uint4 *__restrict__ bufB, v16f (&g)[B32<C2>::NF]) {
  using TL = B32<C2>;
  constexpr int NF = TL::NF;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, h = lane >> 5;
  const Post P = D.posts[pl.b];
  const float eps = zero_eps ? 0.f : (float)D.ps[pl.b].eps;
  const float he = 0.5f * eps;
  const float *minv = D.minv + (long long)pl.b * D.DS;
  const int *perm = D.perm + P.row0;

  // the split's stages [s0, s1) of STT tiles each (the tile count is padded to
  // whole stages)
  const int ns = P.NT2 / TL::STT;
  const int s0 = (int)((long long)pl.split * ns / pl.S);
  const int s1 = (int)((long long)(pl.split + 1) * ns / pl.S);
  const uint4 *xbf = D.xbf + P.xbf;
  // an odd stage count runs its first stage from bufB before the loop, so
  // that the loop body always holds two stages (no exit in its middle)
  const bool odd = (s1 - s0) & 1;
  if (odd)
    b32_issue<C2>(bufB, xbf, s0 * TL::STT, wave, lane);
  else if (s0 < s1)
    b32_issue<C2>(bufA, xbf, s0 * TL::STT, wave, lane);

  // theta' (bfloat16, B operand of GEMM1): K-step c holds features 16c + 8h + e
  // of particle slot 32 wave + lane % 32; on the split path the set-up (first
  // step) or the previous reduction (later steps) has formed it with the
  // arithmetic of the other branch, which the one-split and gradient-only
  // launches use
  const int slot = wave * 32 + (lane & 31);
  const long long rowp = P.row0 + perm[pl.tile * TJ + slot];
  // the branch sits outside the K-step loops, so that all of a path's loads
  // are issued before the first conversion waits for them
  v8bf thb[C2];
  if (given) {
    // bfloat16 theta' from the reduction, 8 features (16 bytes) per K-step
    const uint4 *trow =
        reinterpret_cast<const uint4 *>(reinterpret_cast<const uint16_t *>(D.theta_n) + rowp * D.DS + 8 * h);
#pragma unroll
    for (int c = 0; c < C2; ++c) thb[c] = as_v8bf(trow[2 * c]);
  } else {
#pragma unroll
    for (int c = 0; c < C2; ++c) {
      const long long base = rowp * D.DS + 16 * c + 8 * h;
      const int kb = 16 * c + 8 * h;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float t0v = D.theta_t[base + e], p0 = D.p_t[base + e], g0 = D.grad_t[base + e];
        const float ph = fmaf(he, g0, p0);
        // eps = 0 (gradient at the given theta): t0 + 0 * ph = t0 for finite ph
        thb[c][e] = (__bf16)fmaf(eps * minv[kb + e], ph, t0v);
      }
    }
  }

#pragma unroll
  for (int f = 0; f < NF; ++f) g[f] = v16f{};

  __syncthreads();  // the first stage has landed (the compiler waits for the loads here)
  if (odd) {
    if (s0 + 1 < s1) b32_issue<C2>(bufA, xbf, (s0 + 1) * TL::STT, wave, lane);
    b32_stage<C2>(bufB + lane * TL::LS, thb, g);
    __syncthreads();
  }
  for (int st = s0 + (odd ? 1 : 0); st < s1; st += 2) {
    // stage st in bufA (stage st + 1 exists: the remaining count is even);
    // stage st + 1 goes to bufB meanwhile
    b32_issue<C2>(bufB, xbf, (st + 1) * TL::STT, wave, lane);
    b32_stage<C2>(bufA + lane * TL::LS, thb, g);
    __syncthreads();
    if (st + 2 < s1) b32_issue<C2>(bufA, xbf, (st + 2) * TL::STT, wave, lane);
    b32_stage<C2>(bufB + lane * TL::LS, thb, g);
    __syncthreads();
  }
}

// Partial gradient of a BF16 work item into a [TJ][DS] slot.
template <int C2>
__device__ __forceinline__ void lf_store_b32(const Dev &D, float *gp0, const v16f (&g)[B32<C2>::NF]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, h = lane >> 5;
  float *gp = gp0 + (long long)(wave * 32 + (lane & 31)) * D.DS;
#pragma unroll
  for (int f = 0; f < B32<C2>::NF; ++f)
#pragma unroll
    for (int hv = 0; hv < 2; ++hv) {
      float4 *o = reinterpret_cast<float4 *>(gp + 32 * f + 16 * hv + 8 * h);
      o[0] = make_float4(g[f][8 * hv + 0], g[f][8 * hv + 1], g[f][8 * hv + 2], g[f][8 * hv + 3]);
      o[1] = make_float4(g[f][8 * hv + 4], g[f][8 * hv + 5], g[f][8 * hv + 6], g[f][8 * hv + 7]);
    }
}

// Resident groups per compute unit = waves per SIMD (four waves per group);
// the one-split variant finishes the step in registers: one group per
// compute unit beyond 7 feature tiles.
template <int C2, bool FIN>
constexpr int b32_groups() { return FIN ? (C2 <= 7 ? 2 : 1) : lf_groups_per_cu(true, C2); }

template <int C2, bool FIN>
__global__ __launch_bounds__(B32_WG, (b32_groups<C2, FIN>())) void k_lf_partial_bf16(Dev D, int s, int zero_eps) {
  using TL = B32<C2>;
  constexpr int NF = TL::NF;
  __shared__ uint4 bufA[TL::STAGE];
  __shared__ uint4 bufB[TL::STAGE];
  __shared__ Plan spl;
  if (threadIdx.x == 0) {
    Plan pl;
    if (!lf_item(D, C2, s, blockIdx.x, pl)) pl.b = -1;
    spl = pl;
  }
  __syncthreads();
  const Plan pl = spl;
  if (pl.b < 0) return;
  v16f g[NF];
  // theta' in bfloat16 from the set-up (first step) or the split reduction
  lf_unit_b32<C2>(D, pl, s, zero_eps, !FIN && !zero_eps, bufA, bufB, g);

  // register v of tile f: feature 32f + 16(v>>3) + 8h + (v&7)
  if constexpr (FIN) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, h = lane >> 5;
    const Post P = D.posts[pl.b];
    const long long rowp = P.row0 + D.perm[P.row0 + pl.tile * TJ + wave * 32 + (lane & 31)];
    if (D.n[rowp] <= s) return;
    const float eps = zero_eps ? 0.f : (float)D.ps[pl.b].eps;
    const float he = 0.5f * eps;
    const float *minv = D.minv + (long long)pl.b * D.DS;
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int v = 0; v < 16; ++v)
        lf_finish(D, rowp, 32 * f + 16 * (v >> 3) + 8 * h + (v & 7), g[f][v], eps, he, minv,
                  zero_eps);
    return;
  }
  lf_store_b32<C2>(D, D.gpart + (long long)(D.lf_goff[D.c2_group[C2]] + blockIdx.x) * TJ * D.DS, g);
}

// grid: (B * tiles per posterior, slices of RED_SLOTS float4 of a tile's
// 128 x d gradient block).  A work group is RED_GROUPS groups of RED_SLOTS
// threads: group q sums splits [q S / RED_GROUPS, (q + 1) S / RED_GROUPS) of
// its float4 slot in split order (eight loads in flight per round), and the
// first group adds the group sums in group order, so every sum has a fixed
// order and the loads of many splits are in flight at once whatever S is.
// Every thread reads the tile's plan itself (uniform loads).
constexpr int RED_THREADS = 256;
constexpr int RED_ROUND = 8;
constexpr int RED_GROUPS = 4;
constexpr int RED_SLOTS = RED_THREADS / RED_GROUPS;

__global__ __launch_bounds__(RED_THREADS) void k_lf_reduce(Dev D, int s, int zero_eps, int c2only) {
  __shared__ float4 part[RED_GROUPS - 1][RED_SLOTS];
  const int tj = TJ, ntile = D.Jcap / tj;
  const int b = blockIdx.x / ntile, tile = blockIdx.x % ntile;
  const Post P = D.posts[b];
  if (c2only && P.C2 != c2only) return;  // another group's posterior (uniform)
  const int4 q = D.lf_post[(long long)s * D.B + b];
  if (tile >= q.w) return;                // inactive tile (uniform)
  const int dq = 4 * P.C2;  // float4 per particle row
  const int sl = threadIdx.x % RED_SLOTS, grp = threadIdx.x / RED_SLOTS;
  const int idx = blockIdx.y * RED_SLOTS + sl;
  const bool live = idx < tj * dq;
  const int S = q.y + (tile < q.z ? 1 : 0);
  const int wbase = D.lf_goff[D.c2_group[P.C2]] + q.x + tile * q.y + (tile < q.z ? tile : q.z);
  const int slot = live ? idx / dq : 0, k4 = live ? idx - slot * dq : 0;
  const float4 *g0p = reinterpret_cast<const float4 *>(D.gpart + (long long)wbase * tj * D.DS);
  const long long sstride = (long long)tj * D.DS / 4;  // float4 between splits
  const long long o4 = (long long)slot * D.DS / 4 + k4;
  // the first group issues the row index and the state loads before its sums
  const bool fin = grp == 0 && live;
  long long row = 0, e = 0;
  float4 t0, p0, g0, mv;
  int nrow = 0;
  if (fin) {
    row = P.row0 + D.perm[P.row0 + tile * tj + slot];
    e = (row * D.DS) / 4 + k4;
    t0 = reinterpret_cast<const float4 *>(D.theta_t)[e];
    p0 = reinterpret_cast<const float4 *>(D.p_t)[e];
    g0 = reinterpret_cast<const float4 *>(D.grad_t)[e];
    mv = reinterpret_cast<const float4 *>(D.minv + (long long)b * D.DS)[k4];
    nrow = D.n[row];
  }
  // this group's splits, in order: ((p_a + p_a+1) + ...) + p_b-1
  const int sa = grp * S / RED_GROUPS, sb = (grp + 1) * S / RED_GROUPS;
  float4 G = make_float4(0.f, 0.f, 0.f, 0.f);
  if (live && sa < sb) {
    G = g0p[sa * sstride + o4];
    for (int sp0 = sa + 1; sp0 < sb; sp0 += RED_ROUND) {
      float4 v[RED_ROUND];
#pragma unroll
      for (int u = 0; u < RED_ROUND; ++u)
        if (sp0 + u < sb) v[u] = g0p[(sp0 + u) * sstride + o4];
#pragma unroll
      for (int u = 0; u < RED_ROUND; ++u)
        if (sp0 + u < sb) {
          G.x += v[u].x;
          G.y += v[u].y;
          G.z += v[u].z;
          G.w += v[u].w;
        }
    }
  }
  if (grp > 0) part[grp - 1][sl] = G;
  __syncthreads();
  if (!fin) return;
  // group sums in group order (a group with no split adds nothing)
#pragma unroll
  for (int r = 1; r < RED_GROUPS; ++r)
    if (r * S / RED_GROUPS < (r + 1) * S / RED_GROUPS) {
      const float4 v = part[r - 1][sl];
      G.x += v.x;
      G.y += v.y;
      G.z += v.z;
      G.w += v.w;
    }
  if (nrow <= s) return;
  const float eps = zero_eps ? 0.f : (float)D.ps[b].eps;
  const float he = 0.5f * eps;
  const float inv_pv = (float)(1.0 / D.prior_var);
  float4 th1, pn, gn;
#define LF_LANE(c)                                       \
  {                                                      \
    const float ph = fmaf(he, g0.c, p0.c);               \
    th1.c = fmaf(eps * mv.c, ph, t0.c);                  \
    gn.c = G.c - th1.c * inv_pv;                         \
    pn.c = fmaf(he, gn.c, ph);                           \
  }
  if (zero_eps == 2) {
    // gradient only: theta' was written by the caller
    gn = make_float4(G.x - t0.x * inv_pv, G.y - t0.y * inv_pv, G.z - t0.z * inv_pv,
                     G.w - t0.w * inv_pv);
    reinterpret_cast<float4 *>(D.grad_t)[e] = gn;
    return;
  }
  LF_LANE(x) LF_LANE(y) LF_LANE(z) LF_LANE(w)
#undef LF_LANE
  reinterpret_cast<float4 *>(D.theta_t)[e] = th1;
  reinterpret_cast<float4 *>(D.p_t)[e] = pn;
  reinterpret_cast<float4 *>(D.grad_t)[e] = gn;
  if (!zero_eps) {
    // theta' of the next step from the state just written, exactly as the
    // leapfrog prologue would form it
    float4 tn;
#define LF_NEXT(c) tn.c = fmaf(eps * mv.c, fmaf(he, gn.c, pn.c), th1.c);
    LF_NEXT(x) LF_NEXT(y) LF_NEXT(z) LF_NEXT(w)
#undef LF_NEXT
    if (D.bf16) {
      // the precision form's leapfrog reads theta' as its bfloat16 operand:
      // rounded here (nearest even, the conversion the kernel would apply),
      // half the bytes for every split item that reads it
      typedef __bf16 v4bf __attribute__((ext_vector_type(4)));
      const v4bf tb = {(__bf16)tn.x, (__bf16)tn.y, (__bf16)tn.z, (__bf16)tn.w};
      reinterpret_cast<uint2 *>(D.theta_n)[e] = __builtin_bit_cast(uint2, tb);
    } else {
      reinterpret_cast<float4 *>(D.theta_n)[e] = tn;
    }
  }
}

template <int C2>
static hipError_t launch_lf_c2(const Dev &D, int step, int zero_eps, hipStream_t st) {
  if (D.bf16 && D.lf_nosplit)
    hipLaunchKernelGGL((k_lf_partial_bf16<C2, true>), dim3(D.lf_grid), dim3(B32_WG), 0, st, D, step,
                       zero_eps);
  else if (D.bf16)
    hipLaunchKernelGGL((k_lf_partial_bf16<C2, false>), dim3(D.lf_grid), dim3(B32_WG), 0, st, D, step,
                       zero_eps);
  else if (D.lf_nosplit)
    hipLaunchKernelGGL((k_lf_partial<C2, true>), dim3(D.lf_grid), dim3(WG), 0, st, D, step,
                       zero_eps);
  else
    hipLaunchKernelGGL((k_lf_partial<C2, false>), dim3(D.lf_grid), dim3(WG), 0, st, D, step,
                       zero_eps);
  return hipGetLastError();
}

hipError_t launch_lf_reduce(const Dev &D, int step, int zero_eps, hipStream_t st, int c2only) {
  // TJ * 4 C2 float4 per tile, for the widest group (or the one group)
  int c2max = c2only;
  for (int g = 0; g < D.ngroups && !c2only; ++g)
    c2max = D.group_c2[g] > c2max ? D.group_c2[g] : c2max;
  const int slices = (TJ * 4 * c2max + RED_SLOTS - 1) / RED_SLOTS;
  hipLaunchKernelGGL(k_lf_reduce, dim3(D.B * (D.Jcap / TJ), slices), dim3(RED_THREADS), 0, st, D,
                     step, zero_eps, c2only);
  return hipGetLastError();
}


hipError_t launch_lf_partial(const Dev &D, int c2, int step, int zero_eps, hipStream_t st) {
  switch (c2) {
    case 1: return launch_lf_c2<1>(D, step, zero_eps, st);
    case 2: return launch_lf_c2<2>(D, step, zero_eps, st);
    case 3: return launch_lf_c2<3>(D, step, zero_eps, st);
    case 4: return launch_lf_c2<4>(D, step, zero_eps, st);
    case 5: return launch_lf_c2<5>(D, step, zero_eps, st);
    case 6: return launch_lf_c2<6>(D, step, zero_eps, st);
    case 7: return launch_lf_c2<7>(D, step, zero_eps, st);
    case 8: return launch_lf_c2<8>(D, step, zero_eps, st);
    case 9: return launch_lf_c2<9>(D, step, zero_eps, st);
    case 10: return launch_lf_c2<10>(D, step, zero_eps, st);
    case 11: return launch_lf_c2<11>(D, step, zero_eps, st);
    case 12: return launch_lf_c2<12>(D, step, zero_eps, st);
    case 13: return launch_lf_c2<13>(D, step, zero_eps, st);
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Log-likelihood at the trajectory end points, recomputed for the energies:
//   sum_n [ y_n z_n - log(1 + e^{z_n}) ],  z = X theta'   (Sec. IV model)
// GEMM1 as above (A part of the packed tiles only), softplus from the hardware
// exp2 and log2 (softplusf_hw: absolute error a few 1e-8 per term) and a
// Neumaier-compensated FP32 sum per lane; the four lanes of a particle are
// merged with error-free TwoSum, the splits in order by the weights kernel.
// ---------------------------------------------------------------------------
struct Neu {
  float s, c;
};
__device__ __forceinline__ void neu_add(Neu &a, float x) {
  const float t = a.s + x;
  const float e = (fabsf(a.s) >= fabsf(x)) ? ((a.s - t) + x) : ((x - t) + a.s);
  a.c += e;
  a.s = t;
}
__device__ __forceinline__ Neu neu_merge(Neu a, Neu b) {
  Neu r;
  const float t = a.s + b.s;
  const float bp = t - a.s;
  const float e = (a.s - (t - bp)) + (b.s - bp);  // TwoSum error
  r.s = t;
  r.c = (a.c + b.c) + e;
  return r;
}

template <int C2>
__global__ __launch_bounds__(WG) void k_loglik(Dev D, int first) {
  constexpr int K1 = 4 * C2;
  using TL = Tiles<C2>;
  __shared__ float4 xs[2][TL::STAGE];
  const int4 it = D.ll_items[first + blockIdx.x];
  const int b = it.x, tile = it.y, split = it.z;
  const Post P = D.posts[b];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, kq = lane >> 4;
  const int S = P.ll_splits;
  const int t0 = (int)((long long)split * P.NT / S);
  const int t1 = (int)((long long)(split + 1) * P.NT / S);
  const float4 *xab = reinterpret_cast<const float4 *>(D.xab + P.xab);
  stage_issue<C2>(xs[0], xab, t0, t1, wave, lane);  // in flight with the theta loads
  float th[SUB][K1];
#pragma unroll
  for (int sb = 0; sb < SUB; ++sb) {
    const long long base =
        (long long)(P.row0 + tile * TJ + (wave * SUB + sb) * 16 + (lane & 15)) * D.DS + kq * K1;
#pragma unroll
    for (int c = 0; c < K1; ++c) th[sb][c] = D.theta_t[base + c];
  }
  Neu acc[SUB];
#pragma unroll
  for (int sb = 0; sb < SUB; ++sb) acc[sb] = Neu{0.f, 0.f};
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  int cur = 0;
  for (int t = t0; t < t1; t += 2) {
    const bool more = t + 2 < t1;
    if (more) stage_issue<C2>(xs[cur ^ 1], xab, t + 2, t1, wave, lane);
    const int ntt = (t + 1 < t1) ? 2 : 1;
    for (int tt = 0; tt < ntt; ++tt) {
      const float4 *xl = xs[cur] + tt * TL::TILE + lane * TL::LSTR;
      const float4 y4 = xl[2 * C2];
      const float ya[4] = {y4.x, y4.y, y4.z, y4.w};
#pragma unroll
      for (int sb = 0; sb < SUB; ++sb) {
        v4f z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < C2; ++q) {
          const float4 a = xl[q];
          z = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, th[sb][4 * q + 0], z, 0, 0, 0);
          z = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, th[sb][4 * q + 1], z, 0, 0, 0);
          z = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, th[sb][4 * q + 2], z, 0, 0, 0);
          z = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, th[sb][4 * q + 3], z, 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          // y z - softplus(z) = -softplus(-z) for y = 1, -softplus(z) for y = 0
          const float zz = ya[i] > 0.5f ? -z[i] : z[i];
          const float sp = softplusf_hw(zz);
          const int n = 16 * (t + tt) + 4 * kq + i;
          neu_add(acc[sb], n < P.N ? -sp : 0.f);
        }
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    cur ^= 1;
  }
  // merge the four lanes (kq = 0..3) that hold the same particle
#pragma unroll
  for (int sb = 0; sb < SUB; ++sb) {
    Neu a = acc[sb];
    for (int o = 16; o <= 32; o <<= 1) {
      Neu bq;
      bq.s = __shfl_xor(a.s, o, 64);
      bq.c = __shfl_xor(a.c, o, 64);
      // merge in a fixed (lower lane first) order so both lanes agree
      a = (lane & o) ? neu_merge(bq, a) : neu_merge(a, bq);
    }
    if (kq == 0) {
      const long long row = P.row0 + tile * TJ + (wave * SUB + sb) * 16 + lane;
      D.llpart[(long long)split * D.B * D.Jcap + row] = make_float2(a.s, a.c);
    }
  }
}

// The same terms for the precision form, GEMM1 on v_mfma_f32_32x32x16_bf16:
// X~ in its three exact bfloat16 planes (k_pack_b3) and theta' split the same
// way in registers; of the nine plane products per K-step the six of order
// 2^-16 of the full product or larger are taken (hi hi, hi mid, mid hi,
// hi lo, mid mid, lo hi; mid lo, lo mid and lo lo are of order 2^-24 or
// smaller, below the FP32 rounding of the sum), accumulated in FP32.  With the label sign folded into X~, every
// row contributes -softplus(-z~).  Each wave takes 32 particles (a work
// group the TJ particles of its tile); one 32-row tile per LDS stage, double
// buffered by direct global-to-LDS loads.  Lane l, register v of the
// accumulator holds row 8 (v/4) + 4 (l/32) + v%4 of particle l % 32; the two
// lanes of a particle merge their Neumaier sums with TwoSum at the end.
template <int C2>
__global__ __launch_bounds__(B32_WG) void k_loglik_b3(Dev D, int first) {
  constexpr int LS = b3_lane_stride(C2);
  constexpr int TILE = 64 * LS;   // uint4 per 32-row tile
  __shared__ uint4 xs[2][TILE];
  const int4 it = D.ll_items[first + blockIdx.x];
  const int b = it.x, tile = it.y, split = it.z;
  const Post P = D.posts[b];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, h = lane >> 5;
  const int S = P.ll_splits;
  const int t0 = (int)((long long)split * P.NT2 / S);
  const int t1 = (int)((long long)(split + 1) * P.NT2 / S);
  const uint4 *xb = D.xb3 + P.xb3;
  auto issue = [&](uint4 *buf, int t) {
    const uint4 *src = xb + (long long)t * TILE + lane;
#pragma unroll
    for (int k = 0; k < (LS + B32_WAVES - 1) / B32_WAVES; ++k) {
      const int m = wave + k * B32_WAVES;
      if (m < LS)
        __builtin_amdgcn_global_load_lds((const void *)(src + 64 * m), (lds_void *)(buf + 64 * m), 16,
                                         0, 0);
    }
  };
  if (t0 < t1) issue(xs[0], t0);
  // theta' in three planes, B-operand layout: K-step c holds features
  // 16c + 8h + e of particle slot 32 wave + l % 32
  const long long base = (long long)(P.row0 + tile * TJ + wave * 32 + (lane & 31)) * D.DS;
  v8bf th[3][C2];
#pragma unroll
  for (int c = 0; c < C2; ++c) {
    const float4 a = *reinterpret_cast<const float4 *>(D.theta_t + base + 16 * c + 8 * h);
    const float4 q = *reinterpret_cast<const float4 *>(D.theta_t + base + 16 * c + 8 * h + 4);
    const float v[8] = {a.x, a.y, a.z, a.w, q.x, q.y, q.z, q.w};
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const uint16_t hi = bf16_rne(v[e]);
      const float r1 = v[e] - __uint_as_float((uint32_t)hi << 16);
      const uint16_t mid = bf16_rne(r1);
      const float r2 = r1 - __uint_as_float((uint32_t)mid << 16);
      th[0][c][e] = __builtin_bit_cast(__bf16, hi);
      th[1][c][e] = __builtin_bit_cast(__bf16, mid);
      th[2][c][e] = __builtin_bit_cast(__bf16, bf16_rne(r2));
    }
  }
  Neu acc = Neu{0.f, 0.f};
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  // Z~ of one staged tile: the six plane products per K-step
  auto gemm = [&](const uint4 *xl) {
    v16f z = {};
#pragma unroll
    for (int c = 0; c < C2; ++c) {
      const v8bf ah = as_v8bf(xl[c]), am = as_v8bf(xl[C2 + c]), al = as_v8bf(xl[2 * C2 + c]);
      z = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, th[0][c], z, 0, 0, 0);
      z = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, th[1][c], z, 0, 0, 0);
      z = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, th[0][c], z, 0, 0, 0);
      z = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, th[2][c], z, 0, 0, 0);
      z = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, th[1][c], z, 0, 0, 0);
      z = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, th[0][c], z, 0, 0, 0);
    }
    return z;
  };
  // the rows of tile t into the compensated sum, in row order; a pad row
  // (z~ = 0, a finite term) adds a zero, written as a product so that the
  // term is computed without a branch
  auto rows = [&](const v16f &z, int t) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int n = 32 * t + 8 * (v >> 2) + 4 * h + (v & 3);
      neu_add(acc, -softplusf_hw(-z[v]) * (n < P.N ? 1.f : 0.f));
    }
  };
  // software pipeline: tile t's products beside tile t - 1's softplus terms
  // (independent work, so a wave's VALU runs while its MFMAs execute); the
  // terms enter the sum in the same order as tile by tile
  if (t0 < t1) {
    int cur = 0;
    if (t0 + 1 < t1) issue(xs[1], t0 + 1);
    v16f zp = gemm(xs[0] + lane * LS);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    cur = 1;
    for (int t = t0 + 1; t < t1; ++t) {
      if (t + 1 < t1) issue(xs[cur ^ 1], t + 1);
      const v16f z = gemm(xs[cur] + lane * LS);
      rows(zp, t - 1);
      zp = z;
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      cur ^= 1;
    }
    rows(zp, t1 - 1);
  }
  // the two lanes of a particle (h = 0, 1), in a fixed order
  Neu o;
  o.s = __shfl_xor(acc.s, 32, 64);
  o.c = __shfl_xor(acc.c, 32, 64);
  const Neu m = h ? neu_merge(o, acc) : neu_merge(acc, o);
  if (h == 0) {
    const long long row = P.row0 + tile * TJ + wave * 32 + lane;
    D.llpart[(long long)split * D.B * D.Jcap + row] = make_float2(m.s, m.c);
  }
}

template <int C2>
static hipError_t launch_ll_b3(const Dev &D, int first, int count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_loglik_b3<C2>, dim3(count), dim3(B32_WG), 0, st, D, first);
  return hipGetLastError();
}

template <int C2>
static hipError_t launch_ll_c2(const Dev &D, int first, int count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_loglik<C2>, dim3(count), dim3(WG), 0, st, D, first);
  return hipGetLastError();
}

// items [first, first + count) all belong to posteriors with this C2
hipError_t launch_loglik(const Dev &D, int c2, int first, int count, hipStream_t st) {
  if (D.bf16) {  // the precision form: three-plane BF16 products
    switch (c2) {
      case 1: return launch_ll_b3<1>(D, first, count, st);
      case 2: return launch_ll_b3<2>(D, first, count, st);
      case 3: return launch_ll_b3<3>(D, first, count, st);
      case 4: return launch_ll_b3<4>(D, first, count, st);
      case 5: return launch_ll_b3<5>(D, first, count, st);
      case 6: return launch_ll_b3<6>(D, first, count, st);
      case 7: return launch_ll_b3<7>(D, first, count, st);
      case 8: return launch_ll_b3<8>(D, first, count, st);
      case 9: return launch_ll_b3<9>(D, first, count, st);
      case 10: return launch_ll_b3<10>(D, first, count, st);
      case 11: return launch_ll_b3<11>(D, first, count, st);
      case 12: return launch_ll_b3<12>(D, first, count, st);
      case 13: return launch_ll_b3<13>(D, first, count, st);
    }
    return hipErrorInvalidValue;
  }
  switch (c2) {
    case 1: return launch_ll_c2<1>(D, first, count, st);
    case 2: return launch_ll_c2<2>(D, first, count, st);
    case 3: return launch_ll_c2<3>(D, first, count, st);
    case 4: return launch_ll_c2<4>(D, first, count, st);
    case 5: return launch_ll_c2<5>(D, first, count, st);
    case 6: return launch_ll_c2<6>(D, first, count, st);
    case 7: return launch_ll_c2<7>(D, first, count, st);
    case 8: return launch_ll_c2<8>(D, first, count, st);
    case 9: return launch_ll_c2<9>(D, first, count, st);
    case 10: return launch_ll_c2<10>(D, first, count, st);
    case 11: return launch_ll_c2<11>(D, first, count, st);
    case 12: return launch_ll_c2<12>(D, first, count, st);
    case 13: return launch_ll_c2<13>(D, first, count, st);
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Per-row helpers: LPR lanes of a wave per particle row (a power of two up
// to 64; sums over a row's lanes by a butterfly inside its lane group).
// ---------------------------------------------------------------------------
template <int LPR>
__device__ __forceinline__ double seg_sum(double v) {
#pragma unroll
  for (int o = LPR / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Lanes per row for a row stride of DS floats: about four columns a lane.
__host__ __device__ constexpr int row_lanes(int DS) {
  return DS <= 16 ? 4 : DS <= 32 ? 8 : DS <= 64 ? 16 : DS <= 128 ? 32 : 64;
}

// Launch of a row kernel templated on LPR: 256 threads, 256 / LPR rows each.
#define LAUNCH_ROWS(KERNEL, DS, ROWS, STREAM, ...)                                          \
  do {                                                                                      \
    const long long rows_ = (ROWS);                                                         \
    switch (row_lanes(DS)) {                                                                \
      case 4:                                                                               \
        hipLaunchKernelGGL(KERNEL<4>, dim3((unsigned)((rows_ + 63) / 64)), dim3(256), 0,     \
                           STREAM, __VA_ARGS__);                                            \
        break;                                                                              \
      case 8:                                                                               \
        hipLaunchKernelGGL(KERNEL<8>, dim3((unsigned)((rows_ + 31) / 32)), dim3(256), 0,     \
                           STREAM, __VA_ARGS__);                                            \
        break;                                                                              \
      case 16:                                                                              \
        hipLaunchKernelGGL(KERNEL<16>, dim3((unsigned)((rows_ + 15) / 16)), dim3(256), 0,    \
                           STREAM, __VA_ARGS__);                                            \
        break;                                                                              \
      case 32:                                                                              \
        hipLaunchKernelGGL(KERNEL<32>, dim3((unsigned)((rows_ + 7) / 8)), dim3(256), 0,      \
                           STREAM, __VA_ARGS__);                                            \
        break;                                                                              \
      default:                                                                              \
        hipLaunchKernelGGL(KERNEL<64>, dim3((unsigned)((rows_ + 3) / 4)), dim3(256), 0,      \
                           STREAM, __VA_ARGS__);                                            \
    }                                                                                       \
  } while (0)
__device__ __forceinline__ double row_loglik(const Dev &D, const Post &P, long long row) {
  double ll = 0.0;
  for (int sp = 0; sp < P.ll_splits; ++sp) {
    const float2 v = D.llpart[(long long)sp * D.B * D.Jcap + row];
    ll += (double)v.x + (double)v.y;
  }
  return ll;
}

// log q0(theta) = -|theta|^2 / (2 prior_var) - d/2 log(2 pi prior_var), FP64.
template <int LPR>
__device__ __forceinline__ double row_log_prior(const Dev &D, const Post &P, const float *th,
                                                int lane) {
  double sq = 0.0;
  for (int c = lane; c < P.d; c += LPR) sq += (double)th[c] * (double)th[c];
  sq = seg_sum<LPR>(sq);
  return -0.5 * sq / D.prior_var - 0.5 * P.d * log(2.0 * 3.141592653589793 * D.prior_var);
}

// 1/2 p^T M^{-1} p, FP64 (kinetic energy, Sec. II-A).
template <int LPR>
__device__ __forceinline__ double row_kinetic(const Dev &D, const Post &P, const float *p,
                                              const float *mv, int lane) {
  double k = 0.0;
  for (int c = lane; c < P.d; c += LPR) k += (double)mv[c] * (double)p[c] * (double)p[c];
  return 0.5 * seg_sum<LPR>(k);
}

// ---------------------------------------------------------------------------
// Initial weights (eq. init_weights): log w = log pi - log q0 - log J, which is
// the log-likelihood minus log J; log pi and the gradient become the state.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_init_weights(Dev D) {
  const int lane = threadIdx.x & 63;
  const long long row = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= (long long)D.B * D.Jcap) return;
  const int b = (int)(row / D.Jcap), j = (int)(row % D.Jcap);
  const Post P = D.posts[b];
  const float *th = D.theta_t + row * D.DS;
  for (int c = lane; c < D.DS; c += 64) {
    D.theta[row * D.DS + c] = th[c];
    D.grad[row * D.DS + c] = D.grad_t[row * D.DS + c];
  }
  if (j >= D.J) {
    if (lane == 0) {
      D.logw[row] = -INFINITY;
      D.logpi[row] = 0.0;
    }
    return;
  }
  if (D.target) {
    // log w = log pi - log q0 - log J, q0 = N(0, prior_var I) the initial draw
    const double logq0 = row_log_prior<64>(D, P, th, lane);
    if (lane == 0) {
      const double lp = D.logpi_t[row];
      D.logpi[row] = lp;
      D.logw[row] = lp - logq0 - log((double)D.J);
    }
    return;
  }
  const double ll = row_loglik(D, P, row);
  const double lp = row_log_prior<64>(D, P, th, lane);
  if (lane == 0) {
    D.logpi[row] = ll + lp;
    D.logw[row] = ll - log((double)D.J);
  }
}

hipError_t launch_init_weights(const Dev &D, hipStream_t st) {
  const long long rows = (long long)D.B * D.Jcap;
  hipLaunchKernelGGL(k_init_weights, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, st, D);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Start of an SMC iteration (Alg. smc_BNN): count k, and when J_eff < ess_frac J
// (or unconditionally for an explicit resample) resample with probability
// w~ (Sec. III).  One 1024-thread work group per posterior.
//
// Integer fixed-point scheme: Q_j = floor(exp(log w_j - m) 2^40), exact uint64
// inclusive scan C, T = C_J.  Systematic: a_i = min{j : C_j (J 2^32) >
// (i 2^32 + U) T} with U = floor(u 2^32), compared exactly in 128 bits.
// Multinomial: a_i = min{j : C_j 2^32 > U_i T}.  The evidence accumulator
// takes LSE(log w) = m + log S before the weights are reset to 1/J.
// ---------------------------------------------------------------------------
__device__ int upper_search(const unsigned long long *C, int J, unsigned __int128 lhs_num,
                            unsigned long long scale) {
  // smallest j with C[j] * scale > lhs_num
  int lo = 0, hi = J - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if ((unsigned __int128)C[mid] * scale > lhs_num)
      hi = mid;
    else
      lo = mid + 1;
  }
  return lo;
}

// The same search in two levels: idx[b] = C[min(J, (b + 1) s) - 1], the last
// entry of each block of s entries (in LDS), is searched first, then the one
// block of C whose last entry passes (C is non-decreasing, so the answer lies
// in the first such block).  Requires C[J - 1] * scale > lhs_num.
__device__ int upper_search2(const unsigned long long *C, const unsigned long long *idx, int J,
                             int s, int nb, unsigned __int128 lhs_num, unsigned long long scale) {
  int lo = 0, hi = nb - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if ((unsigned __int128)idx[mid] * scale > lhs_num)
      hi = mid;
    else
      lo = mid + 1;
  }
  int jl = lo * s, jh = min(J, (lo + 1) * s) - 1;
  while (jl < jh) {
    const int mid = (jl + jh) >> 1;
    if ((unsigned __int128)C[mid] * scale > lhs_num)
      jh = mid;
    else
      jl = mid + 1;
  }
  return jl;
}

__device__ void quantise_scan(const double *lw, double m, int J, unsigned long long *cdf,
                              unsigned long long *sh) {
  // each thread takes a contiguous chunk; chunk sums are scanned in LDS
  const int nt = blockDim.x, t = threadIdx.x;
  const int chunk = (J + nt - 1) / nt;
  const int j0 = min(J, t * chunk), j1 = min(J, j0 + chunk);
  unsigned long long local = 0;
  for (int j = j0; j < j1; ++j) {
    const double v = lw[j];
    unsigned long long q = 0;
    if (v == v && v > -INFINITY) q = (unsigned long long)floor(exp(v - m) * 1099511627776.0);
    local += q;
    cdf[j] = local;
  }
  sh[t] = local;
  __syncthreads();
  // inclusive Hillis-Steele scan over the chunk sums
  for (int o = 1; o < nt; o <<= 1) {
    const unsigned long long v = t >= o ? sh[t - o] : 0ull;
    __syncthreads();
    sh[t] += v;
    __syncthreads();
  }
  const unsigned long long off = t > 0 ? sh[t - 1] : 0ull;
  for (int j = j0; j < j1; ++j) cdf[j] += off;
  __syncthreads();
}

__device__ __forceinline__ unsigned long long u_to_u32(double u) {
  double v = floor(u * 4294967296.0);
  if (v < 0.0) v = 0.0;
  if (v > 4294967295.0) v = 4294967295.0;
  return (unsigned long long)v;
}

__global__ __launch_bounds__(1024) void k_begin_step(Dev D, int conditional, const double *u,
                                                     int count_iteration) {
  __shared__ unsigned long long sh[1024];
  const int b = blockIdx.x, t = threadIdx.x;
  PState &S = D.ps[b];
  const Post P = D.posts[b];
  const int J = D.J;
  const int k = S.k + (count_iteration ? 1 : 0);
  const int doit = conditional ? S.flag_resample : 1;
  const int ok = S.S > 0.0;
  __syncthreads();
  if (t == 0) {
    if (count_iteration) {
      S.k = k;
      S.grad_evals_step = 0;
      S.ess_before = S.ess;
    }
    S.resampled = (doit && ok) ? 1 : 0;
  }
  if (!(doit && ok)) return;
  unsigned long long *cdf = D.cdf + P.row0;
  quantise_scan(D.logw + P.row0, S.m, J, cdf, sh);
  const unsigned long long T = cdf[J - 1];
  // search index in LDS (the scan buffer, free again): the last entry of
  // every block of bs entries, at most 1024 blocks
  const int bs = (J + 1023) / 1024, nb = (J + bs - 1) / bs;
  for (int q = t; q < nb; q += blockDim.x) sh[q] = cdf[min(J, (q + 1) * bs) - 1];
  __syncthreads();
  const int chunk = (J + blockDim.x - 1) / blockDim.x;
  const int i0 = min(J, t * chunk), i1 = min(J, i0 + chunk);
  // every target below is < C[J - 1] * scale, so each search has an answer
  if (D.resampling == 0) {
    const double u0 = u ? u[b] : u01(philox_at(D.seed, 0, (uint32_t)b, (uint32_t)k, STREAM_RESAMPLE).x);
    const unsigned long long U = u_to_u32(u0);
    const unsigned long long scale = (unsigned long long)J << 32;
    for (int i = i0; i < i1; ++i) {
      const unsigned __int128 lhs = (unsigned __int128)(((unsigned long long)i << 32) + U) * T;
      D.anc[P.row0 + i] = upper_search2(cdf, sh, J, bs, nb, lhs, scale);
    }
  } else {
    for (int i = i0; i < i1; ++i) {
      const double ui = u ? u[(long long)b * J + i]
                          : u01(philox_at(D.seed, 0, (uint32_t)(b * J + i), (uint32_t)k, STREAM_RESAMPLE).x);
      const unsigned __int128 lhs = (unsigned __int128)u_to_u32(ui) * T;
      D.anc[P.row0 + i] = upper_search2(cdf, sh, J, bs, nb, lhs, 4294967296ull);
    }
  }
  if (t == 0) {
    S.log_c += S.m + log(S.S);
    S.tot_resamples += 1;
  }
}

hipError_t launch_begin_step(const Dev &D, int conditional, const double *u, int count_iteration,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_begin_step, dim3(D.B), dim3(1024), 0, st, D, conditional, u,
                     count_iteration);
  return hipGetLastError();
}

// Gather the chosen ancestors into the trajectory buffers and reset the weights
// to 1/J (Alg. smc_BNN).  One wave per row.
__global__ __launch_bounds__(256) void k_gather(Dev D, int *anc_out) {
  const int lane = threadIdx.x & 63;
  const long long row = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= (long long)D.B * D.Jcap) return;
  const int b = (int)(row / D.Jcap), j = (int)(row % D.Jcap);
  if (j >= D.J || !D.ps[b].resampled) return;
  const long long src = (long long)b * D.Jcap + D.anc[row];
  for (int c = lane; c < D.DS; c += 64) {
    D.theta_t[row * D.DS + c] = D.theta[src * D.DS + c];
    D.grad_t[row * D.DS + c] = D.grad[src * D.DS + c];
  }
  if (lane == 0) {
    D.logpi_t[row] = D.logpi[src];
    D.logw[row] = -log((double)D.J);
    if (anc_out) anc_out[(long long)b * D.J + j] = D.anc[row];
  }
}

hipError_t launch_gather(const Dev &D, int *anc_out, hipStream_t st) {
  const long long rows = (long long)D.B * D.Jcap;
  hipLaunchKernelGGL(k_gather, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, st, D, anc_out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Trajectory set-up (Alg. smc_ChEES): momenta p = xi M^{1/2}, jitter h_jk,
// l_j = h_j L, n_j = min(max(ceil(l_j / eps), 1), n_max) in binary64, initial
// energy H0 = -log pi + 1/2 p^T M^{-1} p, and the step-count histogram.
// Also moves a freshly resampled population back into the state buffers, or
// copies the state into the trajectory buffers.  One wave per row.
// init_mode = 2: copy the trajectory buffers back only (explicit resample).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double radical_inverse(unsigned long long i, unsigned long long base) {
  unsigned long long r = 0, bm = 1;
  while (i > 0) {
    const unsigned long long dig = i % base;
    i /= base;
    r = r * base + dig;
    bm *= base;
  }
  return (double)r / (double)bm;
}

__device__ __forceinline__ double radical_inverse2(unsigned long long i) {
  const int m = 64 - __clzll((long long)i);
  const unsigned long long r = __builtin_bitreverse64(i) >> (64 - m);
  return (double)r / (double)(1ull << m);
}

// Shuffle of the equidistant jitter schemes: a 4-round Feistel network on
// 2 half bits (Luby and Rackoff), round r's function word 0 of the Philox
// block (R, 4 b + r, k, STREAM_SHUFFLE) masked to half bits.  It permutes
// [0, 2^(2 half)); cycle walking (Black and Rogaway) restricts it to [0, J):
// the walk from x < J ends because x's cycle returns to x.
__device__ uint32_t feistel(const Dev &D, uint32_t x, int half, uint32_t b, uint32_t k) {
  const uint32_t mask = (1u << half) - 1u;
  uint32_t lo = x & mask, hi = x >> half;
  for (uint32_t r = 0; r < 4; ++r) {
    const uint32_t f = philox_at(D.seed, lo, 4 * b + r, k, STREAM_SHUFFLE).x & mask;
    const uint32_t t = hi ^ f;
    hi = lo;
    lo = t;
  }
  return (hi << half) | lo;
}

__device__ uint32_t shuffle_index(const Dev &D, uint32_t x, uint32_t b, uint32_t k) {
  int half = 1;
  while ((1ull << (2 * half)) < (unsigned long long)D.J) ++half;
  uint32_t y = feistel(D, x, half, b, k);
  while (y >= (uint32_t)D.J) y = feistel(D, y, half, b, k);
  return y;
}

// Jitter h_jk of Sec. III-B-1 for particle j (0-based) of posterior b at
// iteration k (1-based); the schemes and readings are listed with the
// SMC_JITTER_* constants of the C interface.
__device__ double jitter_h(const Dev &D, int b, int j, int k) {
  const unsigned long long jj = (unsigned long long)j + 1;  // 1-based particle
  const int K = D.jit_K;
  const int krev = K > 0 ? K - (k - 1) % K : k;               // reversed column
  const uint32_t particle = (uint32_t)(b * D.J + j);
  switch (D.jitter) {
    case 1: return 1.0;
    case 2: return radical_inverse(jj, (unsigned long long)D.primes[min(k, NPRIMES) - 1]);
    case 3: return u01(philox_at(D.seed, 0, particle, (uint32_t)k, STREAM_JITTER).x);
    case 4: return radical_inverse(jj, (unsigned long long)D.primes[krev - 1]);
    case 5:
    case 6: {
      const double x = (double)jj * D.sqrtp[(D.jitter == 5 ? min(k, NPRIMES) : krev) - 1];
      return x - floor(x);
    }
    case 7: {
      const double x = (double)((unsigned long long)j * K + k) * D.golden;
      return x - floor(x);
    }
    case 8:
    case 9: {
      const uint32_t y = shuffle_index(D, (uint32_t)j, (uint32_t)b, (uint32_t)k);
      double h = (double)(y + 1) / (double)D.J;
      if (D.jitter == 9) h += 0.1 * u01(philox_at(D.seed, 0, particle, (uint32_t)k, STREAM_JITTER).x);
      return h;
    }
    case 10: {
      // first Sobol dimension, nu_b = 2^-b: the bit reversal of the Gray code
      const unsigned long long i = (unsigned long long)(k - 1) * D.J + jj;
      return (double)__builtin_bitreverse64(i ^ (i >> 1)) * 0x1p-64;
    }
    case 11:
    case 12: {
      const int dim = D.jitter == 11 ? min(k, D.sobol_dims) : krev;
      const uint32_t *V = D.sobol + (size_t)(dim - 1) * 32;
      uint32_t g = (uint32_t)(jj ^ (jj >> 1)), x = 0;
      for (int b = 0; g; ++b, g >>= 1)
        if (g & 1u) x ^= V[b];
      return (double)x * 0x1p-32;
    }
    default: return radical_inverse2((unsigned long long)(k - 1) * D.J + jj);
  }
}

template <int LPR>
__global__ __launch_bounds__(256) void k_setup(Dev D, const float *__restrict__ momenta,
                                               int init_mode) {
  const int lane = threadIdx.x % LPR;  // lane within the row's group
  const long long row = (long long)blockIdx.x * (256 / LPR) + threadIdx.x / LPR;
  if (row >= (long long)D.B * D.Jcap) return;
  const int b = (int)(row / D.Jcap), j = (int)(row % D.Jcap);
  PState &S = D.ps[b];
  const Post P = D.posts[b];
  const long long o = row * D.DS;
  if (j >= D.J) {
    if (lane == 0 && init_mode != 2) {
      D.n[row] = 0;
      D.h[row] = 0.0;
      D.l[row] = 0.0;
    }
    return;
  }
  const int resampled = S.resampled;
  if (resampled) {
    for (int c = lane; c < D.DS; c += LPR) {
      D.theta[o + c] = D.theta_t[o + c];
      D.grad[o + c] = D.grad_t[o + c];
    }
    if (lane == 0) D.logpi[row] = D.logpi_t[row];
  } else if (init_mode != 2) {
    for (int c = lane; c < D.DS; c += LPR) {
      D.theta_t[o + c] = D.theta[o + c];
      D.grad_t[o + c] = D.grad[o + c];
    }
  }
  if (init_mode == 2) return;
  const int k = S.k;
  const float *mv = D.minv + (long long)b * D.DS;
  // momenta: lane q covers columns 4q .. 4q+3 (one Philox block); the kinetic
  // energy is accumulated from the values written
  double kin = 0.0;
  // precision form: theta' of the first leapfrog step in bfloat16, as the
  // split reduction forms it for the later steps (the same FP32 arithmetic
  // as the leapfrog prologue); read from the array not written here
  const bool first_theta = D.bf16 && !D.flow && !D.traj && !D.target;
  const float eps1 = (float)S.eps, he1 = 0.5f * eps1;
  const float *t_src = resampled ? D.theta_t : D.theta;
  const float *g_src = resampled ? D.grad_t : D.grad;
  for (int q = lane; q * 4 < D.DS; q += LPR) {
    double xi[4] = {0, 0, 0, 0};
    if (4 * q < P.d) {
      if (momenta) {
        for (int r = 0; r < 4; ++r)
          if (4 * q + r < P.d) xi[r] = momenta[P.uoff + (long long)j * P.d + 4 * q + r];
      } else {
        box_muller4(philox_at(D.seed, q, (uint32_t)(b * D.J + j), (uint32_t)k, STREAM_MOMENTUM), xi);
      }
    }
    for (int r = 0; r < 4; ++r) {
      const int c = 4 * q + r;
      float pv = 0.f;
      if (c < P.d) {
        const float x = (float)xi[r];
        pv = D.precond ? x / sqrtf(mv[c]) : x;
        kin += (double)mv[c] * (double)pv * (double)pv;
      }
      D.p_t[o + c] = pv;
      if (first_theta) {
        const float tn = fmaf(eps1 * mv[c], fmaf(he1, g_src[o + c], pv), t_src[o + c]);
        reinterpret_cast<__bf16 *>(D.theta_n)[o + c] = (__bf16)tn;
      }
    }
  }
  const double K0 = 0.5 * seg_sum<LPR>(kin);
  if (lane == 0) {
    const double h = jitter_h(D, b, j, k);
    const double L = S.L, eps = S.eps;
    const double l = h * L;
    double nn = ceil(l / eps);
    nn = fmin(fmax(nn, 1.0), (double)D.nmax);
    const int n = (int)nn;
    D.h[row] = h;
    D.l[row] = l;
    D.n[row] = n;
    D.H0[row] = -D.logpi[row] + K0;
    if (j == 0) {
      S.L_used = L;
      S.eps_used = eps;
    }
  }
}

hipError_t launch_setup(const Dev &D, const float *momenta, int init_mode, hipStream_t st) {
  LAUNCH_ROWS(k_setup, D.DS, (long long)D.B * D.Jcap, st, D, momenta, init_mode);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Counting sort of the particles by n_j, longest first, so that a leapfrog
// tile holds particles of similar trajectory length; active[s] = #{j: n_j > s}
// and the step's gradient count sum_j n_j.  One work group per posterior; the
// histogram is built with LDS atomics (its counts do not depend on their
// order).  Placement is stable: within a bin particles keep their index
// order, so the tiles, and with them each particle's split count and
// gradient summation order, are the same on every run.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_sort(Dev D) {
  extern __shared__ int lds[];  // hist[nmax + 1], cur[nmax + 1]
  int *hist = lds, *cur = lds + (D.nmax + 1);
  const int b = blockIdx.x;
  const int row0 = b * D.Jcap;
  for (int i = threadIdx.x; i <= D.nmax; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  for (int j = threadIdx.x; j < D.Jcap; j += blockDim.x) atomicAdd(&hist[D.n[row0 + j]], 1);
  __syncthreads();
  if (threadIdx.x == 0) {
    int pos = 0;
    long long evals = 0;
    for (int n = D.nmax; n >= 0; --n) {
      cur[n] = pos;
      pos += hist[n];
      evals += (long long)n * hist[n];
    }
    int *act = D.active + b * (D.nmax + 1);
    for (int s = 0; s <= D.nmax; ++s) act[s] = (s < D.nmax) ? cur[s] : 0;
    D.ps[b].grad_evals_step = evals;
  }
  __syncthreads();
  // chunks of blockDim.x particles in index order; inside a wave, a particle's
  // rank among the lanes below it with the same n; across the waves of a
  // chunk, the bin cursors advance wave by wave
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
  for (int c0 = 0; c0 < D.Jcap; c0 += blockDim.x) {
    const int j = c0 + threadIdx.x;
    const int n = j < D.Jcap ? D.n[row0 + j] : -1;
    unsigned long long left = __ballot(1), peers = 0;
    while (left) {
      const int v = __shfl(n, __ffsll((long long)left) - 1);
      const unsigned long long m = __ballot(n == v);
      if (n == v) peers = m;
      left &= ~m;
    }
    const int rank = __popcll(peers & below);
    int base = 0;
    for (int w = 0; w < nw; ++w) {
      if (wave == w && rank == 0 && n >= 0) {
        base = cur[n];
        cur[n] = base + __popcll(peers);
      }
      __syncthreads();
    }
    base = __shfl(base, __ffsll((long long)peers) - 1);
    if (n >= 0) D.perm[row0 + base + rank] = j;
  }
}

// The same stable counting sort over many work groups, for n_max < 256.
// Work group c of a posterior owns the particles [1024 c, 1024 c + 1024),
// its wave w the quarter [256 w, 256 w + 256) of those.  k_sort_count writes
// each group's bin counts; k_sort_place, a later launch (so every count is
// visible to it), gives each wave a cursor per bin: the bin's start (bins
// longest first) + the counts of the groups before it + those of the waves
// before it in its group; the wave then places its quarter in index order.
// Inside a wave, keys are ranked by nine per-bit ballots.  The placement
// equals that of k_sort.
constexpr int SORT_BINS = 256;    // the multi-group sort takes n_max < 256
constexpr int SORT_CHUNK = 1024;  // particles per work group: 4 waves x 256

// Lanes of the wave holding the same 9-bit key as this lane: the
// intersection over the key's bits of the ballot of that bit (or of its
// complement), nine ballots whatever the number of distinct keys.
__device__ __forceinline__ unsigned long long peers9(int v) {
  unsigned long long peers = ~0ull;
#pragma unroll
  for (int bit = 0; bit < 9; ++bit) {
    const bool on = (v >> bit) & 1;
    const unsigned long long m = __ballot(on);
    peers &= on ? m : ~m;
  }
  return peers;
}

// Keys of this wave's quarter of the group's particles [j0, j1): four
// 64-particle chunks, 511 where there is no particle.
__device__ __forceinline__ void sort_keys(const Dev &D, int row0, int j0, int j1, int (&nv)[4]) {
  const int lane = threadIdx.x & 63, q0 = j0 + 256 * (threadIdx.x >> 6);
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int j = q0 + 64 * u + lane;
    nv[u] = j < j1 ? D.n[row0 + j] : 511;
  }
}

// Per-wave bin counts of the group's quarters into hw (zeroed here).  The
// lowest lane of each key adds its peer count: the keys' leaders are
// distinct lanes and hw[wave] is the wave's own row.
__device__ __forceinline__ void sort_wave_counts(const int (&nv)[4], int (*hw)[SORT_BINS]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
  for (int i = threadIdx.x; i < 4 * SORT_BINS; i += blockDim.x) (&hw[0][0])[i] = 0;
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const unsigned long long peers = peers9(nv[u]);
    if (nv[u] != 511 && !(peers & below)) hw[wave][nv[u]] += __popcll(peers);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
}

__global__ __launch_bounds__(256) void k_sort_count(Dev D) {
  __shared__ int hw[4][SORT_BINS];
  const int b = blockIdx.y, c = blockIdx.x, nb = D.nmax + 1;
  const int j0 = c * SORT_CHUNK, j1 = min(D.Jcap, j0 + SORT_CHUNK);
  int nv[4];
  sort_keys(D, b * D.Jcap, j0, j1, nv);
  sort_wave_counts(nv, hw);
  int *out = D.sort_cnt + ((long long)b * D.sort_chunks + c) * SORT_BINS;
  for (int n = threadIdx.x; n < nb; n += blockDim.x) out[n] = hw[0][n] + hw[1][n] + hw[2][n] + hw[3][n];
}

__global__ __launch_bounds__(256) void k_sort_place(Dev D) {
  __shared__ int hw[4][SORT_BINS];  // counts, then cursors
  __shared__ int ts[SORT_BINS];
  __shared__ double shr[4];
  const int b = blockIdx.y, c = blockIdx.x, nb = D.nmax + 1, row0 = b * D.Jcap;
  const int j0 = c * SORT_CHUNK, j1 = min(D.Jcap, j0 + SORT_CHUNK);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  int nv[4];
  sort_keys(D, row0, j0, j1, nv);
  sort_wave_counts(nv, hw);
  // index t holds bin n = n_max - t (longest first): its total over the
  // groups, and the counts of the groups before this one
  int tot = 0, bef = 0;
  if (t < nb) {
    const int *cn = D.sort_cnt + (long long)b * D.sort_chunks * SORT_BINS + (D.nmax - t);
    for (int cc = 0; cc < D.sort_chunks; ++cc) {
      const int v = cn[(long long)cc * SORT_BINS];
      tot += v;
      bef += cc < c ? v : 0;
    }
    ts[t] = tot;
  }
  __syncthreads();
  for (int off = 1; off < nb; off <<= 1) {  // inclusive scan of the totals
    const int v = (t < nb && t >= off) ? ts[t - off] : 0;
    __syncthreads();
    if (t < nb) ts[t] += v;
    __syncthreads();
  }
  int *act = D.active + b * nb;
  if (t < nb) {
    const int n = D.nmax - t;
    const int start = ts[t] - tot;  // particles with n_j > n
    if (c == 0 && n < D.nmax) act[n] = start;
    int pos = start + bef;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int k = hw[w][n];
      hw[w][n] = pos;
      pos += k;
    }
  }
  if (c == 0) {  // uniform in the work group
    if (t == 0) act[D.nmax] = 0;
    const double ev = block_reduce(t < nb ? (double)(D.nmax - t) * tot : 0.0, shr, OpAdd());
    if (t == 0) D.ps[b].grad_evals_step = (long long)ev;  // exact: below 2^53
  }
  __syncthreads();
  const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
  const int q0 = j0 + 256 * wave;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int n = nv[u];
    const unsigned long long peers = peers9(n);
    const int rank = __popcll(peers & below);
    const int base = n != 511 ? hw[wave][n] : 0;
    __builtin_amdgcn_wave_barrier();
    if (n != 511 && rank == 0) hw[wave][n] = base + __popcll(peers);
    __builtin_amdgcn_wave_barrier();
    if (n != 511) D.perm[row0 + base + rank] = q0 + 64 * u + lane;
  }
}

hipError_t launch_sort(const Dev &D, hipStream_t st) {
  if (D.nmax < SORT_BINS) {
    const dim3 grid(D.sort_chunks, D.B);
    hipLaunchKernelGGL(k_sort_count, grid, dim3(256), 0, st, D);
    hipLaunchKernelGGL(k_sort_place, grid, dim3(256), 0, st, D);
  } else {
    hipLaunchKernelGGL(k_sort, dim3(D.B), dim3(1024), 2 * (D.nmax + 1) * sizeof(int), st, D);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Energies and weights after the trajectories.
//   Delta H = H(theta', p') - H(theta, p), non-finite -> +inf   (Sec. II-A)
//   alpha = min(1, exp(-Delta H))                 (eq. HMC_accept_reject)
//   SMC-ChEES (no accept/reject, Sec. III-A): log w += -Delta H, the
//     momentum change-of-variables L-kernel (eqs. proposal_momentum,
//     l-kernel_momentum, l_weights) whose Jacobians cancel;
//   MH mode: accept iff u < alpha (eq. mh_ratio_rn), weight unchanged.
// One wave per row.
// ---------------------------------------------------------------------------
template <int LPR>
__global__ __launch_bounds__(256) void k_weights(Dev D, const double *__restrict__ mh_u) {
  const int lane = threadIdx.x % LPR;  // lane within the row's group
  const long long row = (long long)blockIdx.x * (256 / LPR) + threadIdx.x / LPR;
  if (row >= (long long)D.B * D.Jcap) return;
  const int b = (int)(row / D.Jcap), j = (int)(row % D.Jcap);
  if (j >= D.J) return;
  const Post P = D.posts[b];
  const PState &S = D.ps[b];
  const float *th = D.theta_t + row * D.DS;
  const float *mv = D.minv + (long long)b * D.DS;
  // synthetic targets: log pi(theta') was evaluated by the target's energy pass
  const double ll = D.target ? 0.0 : row_loglik(D, P, row);
  const double lp = D.target ? D.logpi_t[row] : row_log_prior<LPR>(D, P, th, lane);
  const double K1 = row_kinetic<LPR>(D, P, D.p_t + row * D.DS, mv, lane);
  if (lane != 0) return;
  const double logpi1 = ll + lp;
  double dh = (-logpi1 + K1) - D.H0[row];
  if (D.flow) dh = (-logpi1 - (double)D.fld1[row] + K1) - D.H0[row];
  if (!(dh == dh) || dh == INFINITY || dh == -INFINITY) dh = INFINITY;
  const double alpha = fmin(1.0, exp(-dh));
  D.logpi_t[row] = logpi1;
  D.dH[row] = dh;
  D.alpha[row] = alpha;
  if (D.mh) {
    const double u = mh_u ? mh_u[(long long)b * D.J + j]
                          : u01(philox_at(D.seed, 0, (uint32_t)(b * D.J + j), (uint32_t)S.k, STREAM_MH).x);
    D.accepted[row] = u < alpha ? 1 : 0;
  } else {
    D.accepted[row] = 1;
    const double w = D.logw[row];
    D.logw[row] = (dh == INFINITY) ? -INFINITY : w - dh;
  }
}

hipError_t launch_weights(const Dev &D, const double *mh_u, int init_mode, hipStream_t st) {
  (void)init_mode;
  LAUNCH_ROWS(k_weights, D.DS, (long long)D.B * D.Jcap, st, D, mh_u);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// ChEES statistics (Sec. II-C, Alg. smc_ChEES), FP64 accumulation:
//   theta_hat' = mean theta', theta_hat = mean theta (unweighted),
//   a_j = |theta'_j - theta_hat'|^2 - |theta_j - theta_hat|^2,
//   g_j = l_j a_j (theta'_j - theta_hat')^T M^{-1} p'_j,
//   g_hat = sum alpha_j g_j / sum alpha_j,  ChEES = 1/4 mean a_j^2.
// Under the flow preconditioner the positions are the latent z (the
// trajectories run there).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_colsum(Dev D) {
  // grid (col_chunks, B); 4 row lanes x 64 columns per column group
  __shared__ double sh[2][4][64];
  const int b = blockIdx.y, ch = blockIdx.x;
  const int rl = threadIdx.x >> 6, cl = threadIdx.x & 63;
  const int rows_per = (D.J + D.col_chunks - 1) / D.col_chunks;
  const int r0 = ch * rows_per, r1 = min(D.J, r0 + rows_per);
  for (int cg = 0; cg * 64 < D.DS; ++cg) {
    const int c = cg * 64 + cl;
    double s0 = 0.0, s1 = 0.0;
    if (c < D.DS)
#pragma unroll 8
      for (int r = r0 + rl; r < r1; r += 4) {  // unrolled: the loads overlap, the sum order stays
        const long long o = ((long long)b * D.Jcap + r) * D.DS + c;
        s0 += (double)(D.flow ? D.fz0 : D.theta)[o];
        s1 += (double)(D.flow ? D.fz : D.theta_t)[o];
      }
    sh[0][rl][cl] = s0;
    sh[1][rl][cl] = s1;
    __syncthreads();
    if (rl == 0 && c < D.DS) {
      double *out = D.colpart + (((long long)b * D.col_chunks + ch) * 2) * D.DS;
      out[c] = ((sh[0][0][cl] + sh[0][1][cl]) + sh[0][2][cl]) + sh[0][3][cl];
      out[D.DS + c] = ((sh[1][0][cl] + sh[1][1][cl]) + sh[1][2][cl]) + sh[1][3][cl];
    }
    __syncthreads();
  }
}

__global__ void k_colmean(Dev D) {
  const int b = blockIdx.x;
  for (int c = threadIdx.x; c < 2 * D.DS; c += blockDim.x) {
    const int which = c / D.DS, col = c % D.DS;
    double s = 0.0;
#pragma unroll 8
    for (int ch = 0; ch < D.col_chunks; ++ch)
      s += D.colpart[(((long long)b * D.col_chunks + ch) * 2 + which) * D.DS + col];
    D.means[((long long)b * 2 + which) * D.DS + col] = s / D.J;
  }
}

template <int LPR>
__global__ __launch_bounds__(256) void k_chees_row(Dev D) {
  const int lane = threadIdx.x % LPR;  // lane within the row's group
  const long long row = (long long)blockIdx.x * (256 / LPR) + threadIdx.x / LPR;
  if (row >= (long long)D.B * D.Jcap) return;
  const int b = (int)(row / D.Jcap), j = (int)(row % D.Jcap);
  if (j >= D.J) return;
  const Post P = D.posts[b];
  const double *mo = D.means + (long long)b * 2 * D.DS;  // theta_hat
  const double *mn = mo + D.DS;                           // theta_hat'
  const float *mv = D.minv + (long long)b * D.DS;
  const long long o = row * D.DS;
  double an = 0.0, ao = 0.0, dt = 0.0;
  for (int c = lane; c < P.d; c += LPR) {
    const double cn = (double)(D.flow ? D.fz : D.theta_t)[o + c] - mn[c];
    const double co = (double)(D.flow ? D.fz0 : D.theta)[o + c] - mo[c];
    an += cn * cn;
    ao += co * co;
    dt += cn * (double)mv[c] * (double)D.p_t[o + c];
  }
  an = seg_sum<LPR>(an);
  ao = seg_sum<LPR>(ao);
  dt = seg_sum<LPR>(dt);
  if (lane == 0) {
    const double a = an - ao;
    D.ca[row] = a;
    D.cg[row] = D.l[row] * a * dt;
  }
}

__global__ __launch_bounds__(RED_T) void k_chees_reduce(Dev D) {
  __shared__ double sh[RED_T / 64];
  const int b = blockIdx.y, g = blockIdx.x, G = gridDim.x;
  const long long r0 = (long long)b * D.Jcap;
  double sag = 0, sa = 0, sa2 = 0, sinv = 0;
#pragma unroll 4
  for (int j = g * RED_T + threadIdx.x; j < D.J; j += G * RED_T) {
    const double al = D.alpha[r0 + j], a = D.ca[r0 + j];
    sag += al * D.cg[r0 + j];
    sa += al;
    sa2 += a * a;
    sinv += 1.0 / fmax(al, 1e-20);
  }
  sag = block_reduce(sag, sh, OpAdd());
  sa = block_reduce(sa, sh, OpAdd());
  sa2 = block_reduce(sa2, sh, OpAdd());
  sinv = block_reduce(sinv, sh, OpAdd());
  double *part = D.red_part + (long long)b * RED_G * 4;
  if (threadIdx.x == 0) {
    part[4 * g] = sag;
    part[4 * g + 1] = sa;
    part[4 * g + 2] = sa2;
    part[4 * g + 3] = sinv;
  }
  if (!red_last(D.red_cnt + 2 * b + 1, G)) return;
  const bool own = threadIdx.x < G;  // thread g takes partial g (fixed order)
  sag = block_reduce(own ? part[4 * threadIdx.x] : 0.0, sh, OpAdd());
  sa = block_reduce(own ? part[4 * threadIdx.x + 1] : 0.0, sh, OpAdd());
  sa2 = block_reduce(own ? part[4 * threadIdx.x + 2] : 0.0, sh, OpAdd());
  sinv = block_reduce(own ? part[4 * threadIdx.x + 3] : 0.0, sh, OpAdd());
  if (threadIdx.x != 0) return;
  PState &S = D.ps[b];
  S.sum_alpha = sa;
  S.ghat = sa > 0.0 ? sag / sa : 0.0;
  S.chees = 0.25 * sa2 / D.J;
  S.sum_alpha_all = sa;
  S.sum_inv_alpha = sinv;
}

hipError_t launch_chees(const Dev &D, hipStream_t st) {
  const long long rows = (long long)D.B * D.Jcap;
  hipLaunchKernelGGL(k_colsum, dim3(D.col_chunks, D.B), dim3(256), 0, st, D);
  hipLaunchKernelGGL(k_colmean, dim3(D.B), dim3(256), 0, st, D);
  LAUNCH_ROWS(k_chees_row, D.DS, rows, st, D);
  hipLaunchKernelGGL(k_chees_reduce, dim3(red_grid(D.J), D.B), dim3(RED_T), 0, st, D);
  return hipGetLastError();
}

// Diagonal inverse mass matrix from the pre-move population (preconditioner
// DIAG, the diagonal-mass fallback; the paper uses M = I):
//   M^{-1}_c = n/(n+5) Var_W[theta_c] + 1e-3 * 5/(n+5),
// W the normalised weights (uniform right after resampling), n their
// effective sample size before any resampling; two FP64 passes (mean, then
// squared deviations) over the same column chunks as the ChEES means.  The
// mean lands in the first half of `means`, which the ChEES statistics
// overwrite later in the step.
constexpr int MASS_ROWS = 1024;  // row weights held in LDS per round

__global__ __launch_bounds__(256) void k_mass_colsum(Dev D, int pass) {
  __shared__ double sh[4][64];
  __shared__ double wr[MASS_ROWS];   // normalised weights of this round's rows
  const int b = blockIdx.y, ch = blockIdx.x;
  const int rl = threadIdx.x >> 6, cl = threadIdx.x & 63;
  const PState &S = D.ps[b];
  const int rs = S.resampled;
  const float *src = rs ? D.theta_t : D.theta;
  const double m = S.m, inv = 1.0 / S.S, uni = 1.0 / D.J;
  const double *mean = D.means + (long long)b * 2 * D.DS;
  const int rows_per = (D.J + D.col_chunks - 1) / D.col_chunks;
  const int r0 = ch * rows_per, r1 = min(D.J, r0 + rows_per);
  constexpr int MAXCG = (32 * ((MAX_C2 + 1) / 2) + 63) / 64;  // widest state row
  double acc[MAXCG];
#pragma unroll
  for (int g = 0; g < MAXCG; ++g) acc[g] = 0.0;
  // each row's weight once per block (one exponential per row, not per
  // column), then every thread's rows in the same order as before
  for (int rb = r0; rb < r1; rb += MASS_ROWS) {
    const int re = min(r1, rb + MASS_ROWS);
    __syncthreads();
    for (int r = rb + (int)threadIdx.x; r < re; r += 256) {
      const double lw = D.logw[(long long)b * D.Jcap + r];
      wr[r - rb] = rs ? uni : ((lw == lw && lw > -INFINITY) ? exp(lw - m) * inv : 0.0);
    }
    __syncthreads();
#pragma unroll
    for (int g = 0; g < MAXCG; ++g) {
      const int c = g * 64 + cl;
      if (c < D.DS)
        for (int r = rb + rl; r < re; r += 4) {
          const long long row = (long long)b * D.Jcap + r;
          const double w = wr[r - rb];
          const double x = (double)src[row * D.DS + c];
          acc[g] += pass == 0 ? w * x : w * ((x - mean[c]) * (x - mean[c]));
        }
    }
  }
#pragma unroll
  for (int g = 0; g < MAXCG; ++g) {
    const int c = g * 64 + cl;
    sh[rl][cl] = acc[g];
    __syncthreads();
    if (rl == 0 && c < D.DS)
      D.colpart[((long long)b * D.col_chunks + ch) * 2 * D.DS + c] =
          ((sh[0][cl] + sh[1][cl]) + sh[2][cl]) + sh[3][cl];
    __syncthreads();
  }
}

__global__ void k_mass_finish(Dev D, int pass) {
  const int b = blockIdx.x;
  const Post P = D.posts[b];
  const double n = D.ps[b].ess_before;
  for (int c = threadIdx.x; c < D.DS; c += blockDim.x) {
    double s = 0.0;
    for (int ch = 0; ch < D.col_chunks; ++ch)
      s += D.colpart[((long long)b * D.col_chunks + ch) * 2 * D.DS + c];
    if (pass == 0)
      D.means[(long long)b * 2 * D.DS + c] = s;
    else
      D.minv[(long long)b * D.DS + c] =
          c < P.d ? (float)((n / (n + 5.0)) * s + 1e-3 * (5.0 / (n + 5.0))) : 1.0f;
  }
}

// write_minv = 0: the weighted mean only (the flow preconditioner's base map
// takes it from there).
hipError_t launch_mass(const Dev &D, int write_minv, hipStream_t st) {
  for (int pass = 0; pass < (write_minv ? 2 : 1); ++pass) {
    hipLaunchKernelGGL(k_mass_colsum, dim3(D.col_chunks, D.B), dim3(256), 0, st, D, pass);
    hipLaunchKernelGGL(k_mass_finish, dim3(D.B), dim3(256), 0, st, D, pass);
  }
  return hipGetLastError();
}

// Accepted proposals become the state (all of them in SMC-ChEES mode).
__global__ void k_commit(Dev D) {
  const long long tot = (long long)D.B * D.Jcap * D.DS;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (long long)gridDim.x * blockDim.x) {
    const long long row = e / D.DS;
    const int j = (int)(row % D.Jcap);
    if (j >= D.J || !D.accepted[row]) continue;
    D.theta[e] = D.theta_t[e];
    D.grad[e] = D.grad_t[e];
    if (e % D.DS == 0) D.logpi[row] = D.logpi_t[row];
  }
}

hipError_t launch_commit(const Dev &D, hipStream_t st) {
  hipLaunchKernelGGL(k_commit, dim3(2048), dim3(256), 0, st, D);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Normalisation terms and ESS (eqs. normalise_smc2, ess_smc), FP64:
//   m = max log w, S = sum e^{log w - m}, S2 = sum e^{2(log w - m)},
//   J_eff = S^2 / S2; resample next iff J_eff < ess_frac J.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(RED_T) void k_ess(Dev D, int count) {
  __shared__ double sh[RED_T / 64];
  const int b = blockIdx.y, g = blockIdx.x, G = gridDim.x;
  const double *lw = D.logw + (long long)b * D.Jcap;
  const int j0 = g * RED_T + threadIdx.x, js = G * RED_T;
  double m = -INFINITY;
#pragma unroll 4
  for (int j = j0; j < D.J; j += js) {
    const double v = lw[j];
    if (v == v && v > m) m = v;
  }
  m = block_reduce(m, sh, OpMax());
  double s = 0.0, s2 = 0.0;
  if (m > -INFINITY)
#pragma unroll 4
    for (int j = j0; j < D.J; j += js) {
      const double v = lw[j];
      if (v == v && v > -INFINITY) {
        const double e = exp(v - m);
        s += e;
        s2 += e * e;
      }
    }
  s = block_reduce(s, sh, OpAdd());
  s2 = block_reduce(s2, sh, OpAdd());
  double *part = D.red_part + (long long)b * RED_G * 4;
  if (threadIdx.x == 0) {
    part[4 * g] = m;
    part[4 * g + 1] = s;
    part[4 * g + 2] = s2;
  }
  if (!red_last(D.red_cnt + 2 * b, G)) return;
  // m = max m_g, S = sum S_g e^{m_g - m}, S2 = sum S2_g e^{2 (m_g - m)}:
  // thread g takes partial g (fixed reduction order)
  const double mg = threadIdx.x < G ? part[4 * threadIdx.x] : -INFINITY;
  const double M = block_reduce(mg, sh, OpMax());
  double sg = 0.0, s2g = 0.0;
  if (M > -INFINITY && mg > -INFINITY) {
    const double f = exp(mg - M);
    sg = part[4 * threadIdx.x + 1] * f;
    s2g = part[4 * threadIdx.x + 2] * f * f;
  }
  const double S = block_reduce(sg, sh, OpAdd());
  const double S2 = block_reduce(s2g, sh, OpAdd());
  if (threadIdx.x != 0) return;
  PState &St = D.ps[b];
  St.m = M;
  St.S = S;
  St.S2 = S2;
  St.ess = S > 0.0 ? S * S / S2 : 0.0;
  St.degenerate = !(S > 0.0);
  St.flag_resample = St.ess < D.ess_frac * D.J;
  if (count) {
    St.tot_iters += 1;
    St.tot_ess += St.ess;
    St.tot_grad_evals += St.grad_evals_step;
  }
}

hipError_t launch_ess(const Dev &D, int count, hipStream_t st) {
  hipLaunchKernelGGL(k_ess, dim3(red_grid(D.J), D.B), dim3(RED_T), 0, st, D, count);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Warm-up adaptation after step k (Alg. smc_ChEES): Adam ascent on log L with
// g_hat (Kingma and Ba), L_bar moving average, freeze at k = M_warmup.
// Optional Adam on log eps toward a harmonic-mean acceptance target.
// ---------------------------------------------------------------------------
__device__ double adam_ascend(double x, double g, double &m, double &v, int &t, double lr,
                              double b1, double b2, double ae) {
  t += 1;
  m = b1 * m + (1.0 - b1) * g;
  v = b2 * v + (1.0 - b2) * g * g;
  const double mhat = m / (1.0 - pow(b1, (double)t));
  const double vhat = v / (1.0 - pow(b2, (double)t));
  return x + lr * mhat / (sqrt(vhat) + ae);
}

__global__ void k_adapt(Dev D) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= D.B) return;
  PState &S = D.ps[b];
  const int k = S.k;
  if (k < D.num_warmup) {
    if (S.sum_alpha > 0.0)
      S.L = exp(adam_ascend(log(S.L), S.ghat, S.am, S.av, S.at, D.adam_lr, D.adam_b1, D.adam_b2,
                            D.adam_eps));
    S.Lbar = D.avg_decay * S.Lbar + (1.0 - D.avg_decay) * S.L;
    if (D.adapt_eps == 1) {
      const double hm = (double)D.J / S.sum_inv_alpha;
      S.eps = exp(adam_ascend(log(S.eps), hm - D.target_accept, S.em, S.ev, S.et, D.adam_lr,
                              D.adam_b1, D.adam_b2, D.adam_eps));
    } else if (D.adapt_eps == 2) {
      // dual averaging (Hoffman and Gelman 2014, with gamma 0.05, t0 10,
      // kappa 0.75) at adaptation iteration m = k on the mean acceptance
      const double m = (double)k, w = 1.0 / (m + 10.0);
      const double abar = S.sum_alpha_all / (double)D.J;
      S.da_hbar = (1.0 - w) * S.da_hbar + w * (D.target_accept - abar);
      const double le = S.da_mu - sqrt(m) / 0.05 * S.da_hbar;
      const double mk = pow(m, -0.75);
      S.da_logbar = mk * le + (1.0 - mk) * S.da_logbar;
      S.eps = exp(le);
    }
  } else if (k == D.num_warmup) {
    S.L = S.Lbar;
    if (D.adapt_eps == 2) S.eps = exp(S.da_logbar);
  }
  S.adapted_k = k;
}

hipError_t launch_adapt(const Dev &D, hipStream_t st) {
  hipLaunchKernelGGL(k_adapt, dim3((D.B + 63) / 64), dim3(64), 0, st, D);
  return hipGetLastError();
}

__global__ void k_set_params(Dev D, double L, double eps) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= D.B) return;
  D.ps[b].L = L;
  D.ps[b].eps = eps;
}

hipError_t launch_set_params(const Dev &D, double L, double eps, hipStream_t st) {
  hipLaunchKernelGGL(k_set_params, dim3((D.B + 63) / 64), dim3(64), 0, st, D, L, eps);
  return hipGetLastError();
}

// State export to caller layouts: theta (B*J) x d_b FP32, logw, logpi (B*J).
__global__ void k_export(Dev D, float *theta, double *logw, double *logpi) {
  const long long tot = (long long)D.B * D.J * D.DS;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (long long)gridDim.x * blockDim.x) {
    const int c = (int)(e % D.DS);
    const long long bj = e / D.DS;
    const int b = (int)(bj / D.J), j = (int)(bj % D.J);
    const Post &P = D.posts[b];
    const long long row = (long long)b * D.Jcap + j;
    if (theta && c < P.d) theta[P.uoff + (long long)j * P.d + c] = D.theta[row * D.DS + c];
    if (c == 0) {
      if (logw) logw[bj] = D.logw[row];
      if (logpi) logpi[bj] = D.logpi[row];
    }
  }
}

hipError_t launch_export_state(const Dev &D, float *theta, double *logw, double *logpi,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_export, dim3(1024), dim3(256), 0, st, D, theta, logw, logpi);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Stateless resampling of nonnegative weights (same integer scheme as above,
// with e_j = w_j / max w).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_resample_indices(const double *w, int J, const double *u,
                                                           int scheme, int *anc,
                                                           unsigned long long *cdf, int *err) {
  __shared__ unsigned long long sh[1024];
  __shared__ double shd[16];
  const int t = threadIdx.x;
  const int chunk = (J + blockDim.x - 1) / blockDim.x;
  const int j0 = min(J, t * chunk), j1 = min(J, j0 + chunk);
  double mx = 0.0;
  for (int j = j0; j < j1; ++j) mx = fmax(mx, w[j]);
  mx = block_reduce(mx, shd, OpMax());
  if (!(mx > 0.0)) {
    if (t == 0) *err = 1;
    return;
  }
  unsigned long long local = 0;
  for (int j = j0; j < j1; ++j) {
    const double v = w[j] / mx;
    const unsigned long long q = (v > 0.0) ? (unsigned long long)floor(v * 1099511627776.0) : 0ull;
    local += q;
    cdf[j] = local;
  }
  sh[t] = local;
  __syncthreads();
  for (int o = 1; o < (int)blockDim.x; o <<= 1) {
    const unsigned long long v = t >= o ? sh[t - o] : 0ull;
    __syncthreads();
    sh[t] += v;
    __syncthreads();
  }
  const unsigned long long off = t > 0 ? sh[t - 1] : 0ull;
  for (int j = j0; j < j1; ++j) cdf[j] += off;
  __syncthreads();
  const unsigned long long T = cdf[J - 1];
  if (t == 0) *err = 0;
  if (scheme == 0) {
    const unsigned long long U = u_to_u32(u[0]);
    const unsigned long long scale = (unsigned long long)J << 32;
    for (int i = j0; i < j1; ++i) {
      const unsigned __int128 lhs = (unsigned __int128)(((unsigned long long)i << 32) + U) * T;
      anc[i] = upper_search(cdf, J, lhs, scale);
    }
  } else {
    for (int i = j0; i < j1; ++i) {
      const unsigned __int128 lhs = (unsigned __int128)u_to_u32(u[i]) * T;
      anc[i] = upper_search(cdf, J, lhs, 4294967296ull);
    }
  }
}

hipError_t launch_resample_indices(const double *w, int J, const double *u, int scheme, int *anc,
                                   unsigned long long *cdf, double *wmax, int *err,
                                   hipStream_t st) {
  (void)wmax;
  hipLaunchKernelGGL(k_resample_indices, dim3(1), dim3(1024), 0, st, w, J, u, scheme, anc, cdf,
                     err);
  return hipGetLastError();
}

// Scratch of the no-allocation resampling entry point: the integer CDF of at
// most RS_STATIC_MAX weights, then 256 bytes for the error flag.  One copy per
// device, held until the process ends.  Host code never passes the array's
// name to a kernel (in host code it is a stand-in, not a device address): the
// device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned long long scratch[RS_STATIC_MAX + 32];

hipError_t static_resample_scratch(unsigned long long **cdf, int **err) {
  static std::mutex mu;
  static void *addr[RS_MAX_DEVICES] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= RS_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[dev] = p;
  }
  *cdf = static_cast<unsigned long long *>(addr[dev]);
  *err = reinterpret_cast<int *>(*cdf + RS_STATIC_MAX);
  return hipSuccess;
}

}  // namespace smc
