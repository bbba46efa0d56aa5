// Flow preconditioner of the SMC/ChEES-HMC sampler (gfx950).
//
// The paper's exactness argument for the momentum L-kernel (Sec. III-A,
// eqs. proposal_momentum, l-kernel_momentum) needs only a volume-preserving
// bijection, so the leapfrog may run in the latent space of a bijection T
// that is fixed during an iteration, on the pushforward target
//   log pi_z(z) = log pi(T(z)) + log|det J_T(z)|.
// T: x = z; per coupling layer l: x_T <- x_T exp(s) + t with (s, t) from a
// tanh MLP (width FH) of the conditioning half x_C, s = tanh(.);
// theta = m + L u with u_c = x_q(c), q placing the even coordinates of theta
// first, then the odd ones.  m and the Cholesky factor L standardise the
// weighted pre-move population; the couplings are trained each iteration by a
// few Adam steps on the weighted maximum-likelihood objective of the
// population.
//
// A block of eight waves carries 16 particles.  Every dense layer of the
// conditioners runs on v_mfma_f32_16x16x4f32 with a 16-unit tile of the
// weight matrix as A (the waves take the tiles in turn) and the 16 particles'
// activations, held in LDS, as B; the weights are pre-packed in the A-operand
// order so that each lane reads four K-steps with one 16-byte load.  The
// per-layer activations the backward passes need sit in a per-particle tape
// in global memory.  Training uses the FP32 parameters on
// v_mfma_f32_16x16x4f32.  The moves use the weights rounded to bfloat16 on
// v_mfma_f32_16x16x32_bf16: the weights are exact bfloat16 operands, and each
// FP32 activation enters as the sum of three bfloat16 parts (hi, mid, lo;
// split once per layer into LDS planes), so every product is exact and the
// sums accumulate in FP32 -- the FP32 arithmetic of the weights' values, at
// three bfloat16 products per 32 inputs instead of eight FP32 ones per 4.
// The moves need that precision: the latent start z0 = T^-1(theta_0) and the
// end point theta' = T(z') must come from the same map to FP32 rounding, or
// the weights would not be those of the latent target.
#pragma clang fp contract(off)

#include <math.h>

#include "dev_common.h"
#include "smc_internal.h"

namespace smc {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int MAXD = 16 * MAX_C2;  // largest dimension
constexpr int PB = 16;             // particles per block
constexpr int NT = 512;            // threads per block: one wave per 16-row output tile of a
                                   // 128-wide layer (J = 4096 gives one block per compute unit)
constexpr int LPP = NT / PB;       // lanes per particle in the element-wise parts
constexpr int XP = MAXD + 17;      // LDS pitch of state rows: a padded K chunk stays in the row
constexpr int HP = FH + 1;         // LDS pitch of hidden rows
constexpr int BKP = 232;           // bfloat16 plane pitch: >= 32 ceil(MAXD / 32), 8 x odd for
                                   // conflict-free 16-byte reads
constexpr int KSPLIT = FKSPLIT;

// Position of coordinate c of theta in the coupling state x: even
// coordinates first, then the odd ones, so that the halves of x split
// neighbouring coordinates.
__device__ __forceinline__ int xpos(int c, int d) { return (c & 1) ? (d + 1) / 2 + (c >> 1) : c >> 1; }

__device__ __forceinline__ uint16_t bf16_bits(float f) {
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((u >> 16) | 0x40u);  // NaN stays NaN
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// Element A[u][k] of an M x K matrix in the packed A-operand order:
// [u/16][k/16][lane][j] with lane = u%16 + 16 (k%4), j = (k%16)/4, so that
// lane l's float4 at (tile, chunk) holds A[16 tile + l%16][16 chunk + 4 j + l/16].
__device__ __forceinline__ int pk_index(int u, int k, int K16) {
  const int kk = k & 15;
  const int lane = (u & 15) + 16 * (kk & 3);
  return (((u >> 4) * (K16 >> 4) + (k >> 4)) * 64 + lane) * 4 + (kk >> 2);
}

static_assert(NT % PB == 0 && LPP % 2 == 0, "row-parallel loops: LPP threads per particle");
static_assert(BKP >= 32 * ((MAXD + 31) / 32) && BKP % 8 == 0 && (BKP / 8) % 2 == 1, "plane pitch");

struct BlockLDS {
  uint16_t bs[3][PB][BKP];  // an input of a move layer split into three bfloat16 planes
  float xs[PB][XP];   // coupling state x (or its cotangent)
  float h1[PB][HP];
  float h2[PB][HP];
  float ob[PB][XP];   // conditioner output (s~, t) or its cotangent
  float *tw[PB];      // tape rows written (nullptr for absent particles)
  const float *tr[PB];// tape rows read (a present particle's for absent ones)
  int rows[PB];
  float wj[PB];
};

enum { ST_PLAIN = 0, ST_TANH = 1, ST_DTANH = 2, ST_ADD = 3 };

// Epilogue of one 16-row output tile t (accumulator acc, tape quad axq, the
// lane's four biases bq).
__device__ __forceinline__ void mdense_out(int t, const v4f &acc, const float4 &axq,
                                           const float *bq, int M, const float *bias, float *out,
                                           int outs, int mode, float *tp, const float *ax, int pn,
                                           int kq) {
  const int u0 = 16 * t + 4 * kq;
  const bool quad = u0 + 3 < M;
  const float axv[4] = {axq.x, axq.y, axq.z, axq.w};
  float vq[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int u = u0 + i;
    vq[i] = 0.f;
    if (u >= M) continue;
    float v = acc[i];
    if (bias) v += bq[i];
    if (mode == ST_TANH) {
      v = tanhf(v);
    } else if (mode == ST_DTANH) {
      const float h = quad ? axv[i] : ax[u];
      v *= 1.f - h * h;
    }
    if (mode == ST_ADD)
      out[pn * outs + u] += v;
    else
      out[pn * outs + u] = v;
    vq[i] = v;
  }
  if (tp) {
    if (quad) {
      *reinterpret_cast<float4 *>(tp + u0) = make_float4(vq[0], vq[1], vq[2], vq[3]);
    } else {
      for (int i = 0; i < 4; ++i)
        if (u0 + i < M) tp[u0 + i] = vq[i];
    }
  }
}

// NTL (1 or 2) output tiles t, t + NT / 64 of one wave in one pass: the
// tiles' MFMA chains interleave and share the B operand read from LDS; each
// tile's MFMAs run in the same order as alone.  A chunks are loaded four at a
// time so that a group's loads are in flight together, and the biases and
// the tape values of ST_DTANH before the MFMAs (at typical populations each
// SIMD holds one wave, so latency, not the MFMAs, sets the pace).  The lane's outputs u0 .. u0 + 3
// are consecutive in a tape row; tape rows and offsets are multiples of 4
// floats, so whole quads move as single 16-byte accesses.
template <int NTL>
__device__ __forceinline__ void mdense_tiles(const float *Ap, int t, int M, int C16,
                                             const float *bias, const float *ip0, float *out,
                                             int outs, int mode, float *tp, const float *ax,
                                             int pn, int kq, int lane) {
  int tt[NTL];
  float4 axq[NTL];
  float bq[NTL][4];
  v4f acc[NTL];
  const float4 *ap[NTL];
#pragma unroll
  for (int g = 0; g < NTL; ++g) {
    tt[g] = t + g * (NT / 64);
    const int u0 = 16 * tt[g] + 4 * kq;
    axq[g] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (ax && u0 + 3 < M) axq[g] = *reinterpret_cast<const float4 *>(ax + u0);
#pragma unroll
    for (int i = 0; i < 4; ++i) bq[g][i] = (bias && u0 + i < M) ? bias[u0 + i] : 0.f;
    acc[g] = v4f{0.f, 0.f, 0.f, 0.f};
    ap[g] = reinterpret_cast<const float4 *>(Ap) + (long long)tt[g] * C16 * 64 + lane;
  }
  int c = 0;
  for (; c + 4 <= C16; c += 4) {
    float4 a[NTL][4];
#pragma unroll
    for (int g = 0; g < NTL; ++g)
#pragma unroll
      for (int u = 0; u < 4; ++u) a[g][u] = ap[g][(c + u) * 64];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const float *ip = ip0 + 16 * (c + u);
      const float b0 = ip[0], b1 = ip[4], b2 = ip[8], b3 = ip[12];
#pragma unroll
      for (int g = 0; g < NTL; ++g) {
        acc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[g][u].x, b0, acc[g], 0, 0, 0);
        acc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[g][u].y, b1, acc[g], 0, 0, 0);
        acc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[g][u].z, b2, acc[g], 0, 0, 0);
        acc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[g][u].w, b3, acc[g], 0, 0, 0);
      }
    }
  }
  for (; c < C16; ++c) {
    const float *ip = ip0 + 16 * c;
    const float b0 = ip[0], b1 = ip[4], b2 = ip[8], b3 = ip[12];
#pragma unroll
    for (int g = 0; g < NTL; ++g) {
      const float4 a = ap[g][c * 64];
      acc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b0, acc[g], 0, 0, 0);
      acc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b1, acc[g], 0, 0, 0);
      acc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b2, acc[g], 0, 0, 0);
      acc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, b3, acc[g], 0, 0, 0);
    }
  }
#pragma unroll
  for (int g = 0; g < NTL; ++g)
    mdense_out(tt[g], acc[g], axq[g], bq[g], M, bias, out, outs, mode, tp, ax, pn, kq);
}

// One dense layer for the block's 16 particles:
//   v[p][u] = sum_k A[u][k] in[p][k] (+ bias[u]),  u < M, k < K,
// then out[p][u] = v (ST_PLAIN), tanh(v) (ST_TANH), v (1 - aux[u]^2)
// (ST_DTANH, aux the particle's tape of tanh outputs) or out += v (ST_ADD);
// the stored value also goes to tape + toff when the particle has a tape.
// Lane (pn = lane % 16, kq = lane / 16) gives B[kq][pn] = in[pn][4 c + kq].
__device__ void mdense(const float *Ap, int M, int K, const float *bias, const float *in, int ins,
                       float *out, int outs, int mode, const BlockLDS &S, int toff, int aoff,
                       int wave, int lane) {
  const int T = (M + 15) >> 4, C16 = (K + 15) >> 4;
  const int pn = lane & 15, kq = lane >> 4;
  const float *ip0 = in + pn * ins + kq;
  float *tp = (toff >= 0 && S.tw[pn]) ? S.tw[pn] + toff : nullptr;
  const float *ax = mode == ST_DTANH ? S.tr[pn] + aoff : nullptr;
  constexpr int NW = NT / 64;
  // two tiles per pass in the backward layers; the forward layers (tanh
  // epilogue) measured faster one tile at a time
  const bool pair = mode == ST_DTANH || mode == ST_ADD;
  for (int t = wave; t < T; t += (pair ? 2 : 1) * NW) {
    if (pair && t + NW < T)
      mdense_tiles<2>(Ap, t, M, C16, bias, ip0, out, outs, mode, tp, ax, pn, kq, lane);
    else
      mdense_tiles<1>(Ap, t, M, C16, bias, ip0, out, outs, mode, tp, ax, pn, kq, lane);
  }
}

// Element A[u][k] of an M x K bfloat16-exact matrix in the packed A-operand
// order of v_mfma_f32_16x16x32_bf16: [u/16][k/32][lane][e] with lane =
// u%16 + 16 ((k%32)/8), e = k%8, so that lane l's 16 bytes at (tile, chunk)
// hold A[16 tile + l%16][32 chunk + 8 (l/16) + e], e = 0..7.
__device__ __forceinline__ int pk16_index(int u, int k, int C32) {
  return (((u >> 4) * C32 + (k >> 5)) * 64 + (u & 15) + 16 * ((k & 31) >> 3)) * 8 + (k & 7);
}

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// v = hi + mid + lo in bfloat16 (round to nearest even each), exact to a
// unit in the last place of FP32; two values at a time (element 0 in the low
// halves), by the hardware's pair conversion, which rounds as bf16_bits does.
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
typedef float v2f __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t bf16_pair(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((v2f){a, b}, v2bf));
}

__device__ __forceinline__ void split3_pair(float v0, float v1, uint32_t &h, uint32_t &m,
                                            uint32_t &l) {
  h = bf16_pair(v0, v1);
  const float r0 = v0 - __uint_as_float(h << 16), r1 = v1 - __uint_as_float(h & 0xFFFF0000u);
  m = bf16_pair(r0, r1);
  const float q0 = r0 - __uint_as_float(m << 16), q1 = r1 - __uint_as_float(m & 0xFFFF0000u);
  l = bf16_pair(q0, q1);
}

// NTL output tiles of one wave from the bfloat16 weights (Ab: the layer's
// packed array) and the three planes of the input (lane (pn, kq) reads eight
// consecutive inputs of particle pn per plane and chunk).
template <int NTL>
__device__ __forceinline__ void mdense_tiles_bf(const uint4 *Ab, int t, int M, int C32,
                                                const float *bias, const BlockLDS &S, float *out,
                                                int outs, int mode, float *tp, const float *ax,
                                                int pn, int kq, int lane) {
  int tt[NTL];
  float4 axq[NTL];
  float bq[NTL][4];
  v4f acc[NTL];
  const uint4 *ap[NTL];
#pragma unroll
  for (int g = 0; g < NTL; ++g) {
    tt[g] = t + g * (NT / 64);
    const int u0 = 16 * tt[g] + 4 * kq;
    axq[g] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (ax && u0 + 3 < M) axq[g] = *reinterpret_cast<const float4 *>(ax + u0);
#pragma unroll
    for (int i = 0; i < 4; ++i) bq[g][i] = (bias && u0 + i < M) ? bias[u0 + i] : 0.f;
    acc[g] = v4f{0.f, 0.f, 0.f, 0.f};
    ap[g] = Ab + (long long)tt[g] * C32 * 64 + lane;
  }
  for (int c = 0; c < C32; ++c) {
    uint4 a[NTL];
#pragma unroll
    for (int g = 0; g < NTL; ++g) a[g] = ap[g][c * 64];
    const int ko = 32 * c + 8 * kq;
    const v8bf b0 = *reinterpret_cast<const v8bf *>(&S.bs[0][pn][ko]);
    const v8bf b1 = *reinterpret_cast<const v8bf *>(&S.bs[1][pn][ko]);
    const v8bf b2 = *reinterpret_cast<const v8bf *>(&S.bs[2][pn][ko]);
#pragma unroll
    for (int g = 0; g < NTL; ++g) {
      const v8bf av = __builtin_bit_cast(v8bf, a[g]);
      acc[g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b2, acc[g], 0, 0, 0);
      acc[g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b1, acc[g], 0, 0, 0);
      acc[g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b0, acc[g], 0, 0, 0);
    }
  }
#pragma unroll
  for (int g = 0; g < NTL; ++g)
    mdense_out(tt[g], acc[g], axq[g], bq[g], M, bias, out, outs, mode, tp, ax, pn, kq);
}

constexpr int MAXC32 = (MAXD + 31) / 32;  // 32-input chunks of the widest layer input

// One move layer (bfloat16-exact weights, packed by pk16_index) for the
// block's 16 particles, with the semantics of mdense.  The input rows are
// first split into the three planes (every thread, one barrier); the caller
// synchronises before (input complete) and after (planes free) as for mdense.
// When every wave has at most one output tile (layers up to 128 wide), the
// wave's weights, biases and tape values do not depend on the input and are
// loaded before the split, so their latency passes with the split's barrier.
__device__ void mdense_bf(const uint16_t *Ab16, int M, int K, const float *bias, const float *in,
                          int ins, float *out, int outs, int mode, BlockLDS &S, int toff, int aoff,
                          int wave, int lane) {
  const int T = (M + 15) >> 4, C32 = (K + 31) >> 5, KP = 32 * C32;
  const int tid = wave * 64 + lane;
  const int pn = lane & 15, kq = lane >> 4;
  float *tp = (toff >= 0 && S.tw[pn]) ? S.tw[pn] + toff : nullptr;
  const float *ax = mode == ST_DTANH ? S.tr[pn] + aoff : nullptr;
  const uint4 *Ab = reinterpret_cast<const uint4 *>(Ab16);
  constexpr int NW = NT / 64;
  const bool one = T <= NW;
  uint4 apre[MAXC32];
  float4 axq = make_float4(0.f, 0.f, 0.f, 0.f);
  float bq[4] = {0.f, 0.f, 0.f, 0.f};
  if (one && wave < T) {
    const int u0 = 16 * wave + 4 * kq;
    if (ax && u0 + 3 < M) axq = *reinterpret_cast<const float4 *>(ax + u0);
#pragma unroll
    for (int i = 0; i < 4; ++i) bq[i] = (bias && u0 + i < M) ? bias[u0 + i] : 0.f;
    const uint4 *ap = Ab + (long long)wave * C32 * 64 + lane;
#pragma unroll
    for (int c = 0; c < MAXC32; ++c)
      if (c < C32) apre[c] = ap[c * 64];
  }
  {
    // LPP threads per particle row, two neighbouring inputs each: one 32-bit
    // store per plane, no division by the run-time row length
    const int q = tid / LPP;
    const float *row = in + q * ins;
    for (int k = 2 * (tid % LPP); k < KP; k += 2 * LPP) {
      uint32_t h, m, l;
      split3_pair(k < K ? row[k] : 0.f, k + 1 < K ? row[k + 1] : 0.f, h, m, l);
      *reinterpret_cast<uint32_t *>(&S.bs[0][q][k]) = h;
      *reinterpret_cast<uint32_t *>(&S.bs[1][q][k]) = m;
      *reinterpret_cast<uint32_t *>(&S.bs[2][q][k]) = l;
    }
  }
  __syncthreads();
  if (one) {
    if (wave >= T) return;
    v4f acc = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < MAXC32; ++c) {
      if (c >= C32) break;
      const int ko = 32 * c + 8 * kq;
      const v8bf av = __builtin_bit_cast(v8bf, apre[c]);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
          av, *reinterpret_cast<const v8bf *>(&S.bs[2][pn][ko]), acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
          av, *reinterpret_cast<const v8bf *>(&S.bs[1][pn][ko]), acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
          av, *reinterpret_cast<const v8bf *>(&S.bs[0][pn][ko]), acc, 0, 0, 0);
    }
    mdense_out(wave, acc, axq, bq, M, bias, out, outs, mode, tp, ax, pn, kq);
    return;
  }
  const bool pair = mode == ST_DTANH || mode == ST_ADD;
  for (int t = wave; t < T; t += (pair ? 2 : 1) * NW) {
    if (pair && t + NW < T)
      mdense_tiles_bf<2>(Ab, t, M, C32, bias, S, out, outs, mode, tp, ax, pn, kq, lane);
    else
      mdense_tiles_bf<1>(Ab, t, M, C32, bias, S, out, outs, mode, tp, ax, pn, kq, lane);
  }
}

// Forward map of the block's particles (xs: latent z on entry, coupled x on
// exit), with the move tape [h1 | h2 | s | x_T before the update] per layer;
// returns the thread's partial sum of s (particle tid / 16).
__device__ float forward_couplings(const FlowNet &F, const uint16_t *Ap, const float *bias,
                                   BlockLDS &S, int wave, int lane, int tid) {
  const int p = tid / LPP, r = tid % LPP;
  float ldp = 0.f;
  for (int l = 0; l < F.L; ++l) {
    const FlowLayerDesc &Y = F.ly[l];
    const int lo = l * F.tape_stride;
    mdense_bf(Ap + 2 * Y.pW1, FH, Y.dc, bias + Y.ob1, &S.xs[0][Y.C0], XP, &S.h1[0][0], HP, ST_TANH,
              S, lo, 0, wave, lane);
    __syncthreads();
    mdense_bf(Ap + 2 * Y.pW2, FH, FH, bias + Y.ob2, &S.h1[0][0], HP, &S.h2[0][0], HP, ST_TANH, S,
              lo + FH, 0, wave, lane);
    __syncthreads();
    mdense_bf(Ap + 2 * Y.pW3, 2 * Y.dt, FH, bias + Y.ob3, &S.h2[0][0], HP, &S.ob[0][0], XP,
              ST_PLAIN, S, -1, 0, wave, lane);
    __syncthreads();
    float *tp = S.tw[p] ? S.tw[p] + lo + 2 * FH : nullptr;
    for (int f = r; f < Y.dt; f += LPP) {
      const float s = tanhf(S.ob[p][f]);
      const float t = S.ob[p][Y.dt + f];
      const float x = S.xs[p][Y.T0 + f];
      if (tp) {
        tp[f] = s;
        tp[F.half + f] = x;
      }
      S.xs[p][Y.T0 + f] = fmaf(x, expf(s), t);
      ldp += s;
    }
    __syncthreads();
  }
  return ldp;
}

// Cotangent of z from the cotangent of x after the couplings (in xs), by
// reverse accumulation over the move tape; the log-determinant adds 1 to the
// cotangent of every s.  Bp: the transposed weights, packed.
__device__ void vjp_couplings(const FlowNet &F, const uint16_t *Bp, BlockLDS &S, int wave, int lane,
                              int tid) {
  const int p = tid / LPP, r = tid % LPP;
  for (int l = F.L - 1; l >= 0; --l) {
    const FlowLayerDesc &Y = F.ly[l];
    const int lo = l * F.tape_stride;
    const float *ts = S.tr[p] + lo + 2 * FH;
    for (int f = r; f < Y.dt; f += LPP) {
      const float s = ts[f], xT = ts[F.half + f];
      const float gy = S.xs[p][Y.T0 + f];
      const float es = expf(s);
      S.ob[p][f] = fmaf(gy * xT, es, 1.f) * (1.f - s * s);
      S.ob[p][Y.dt + f] = gy;
      S.xs[p][Y.T0 + f] = gy * es;
    }
    __syncthreads();
    mdense_bf(Bp + 2 * Y.qW3, FH, 2 * Y.dt, nullptr, &S.ob[0][0], XP, &S.h2[0][0], HP, ST_DTANH, S,
              -1, lo + FH, wave, lane);
    __syncthreads();
    mdense_bf(Bp + 2 * Y.qW2, FH, FH, nullptr, &S.h2[0][0], HP, &S.h1[0][0], HP, ST_DTANH, S, -1, lo,
              wave, lane);
    __syncthreads();
    mdense_bf(Bp + 2 * Y.qW1, Y.dc, FH, nullptr, &S.h1[0][0], HP, &S.xs[0][Y.C0], XP, ST_ADD, S, -1,
              0, wave, lane);
    __syncthreads();
  }
}

// Sum of the LPP partials of a particle (lanes LPP p .. LPP p + LPP - 1 of a
// wave), fixed order.
__device__ __forceinline__ float sum_lpp(float v) {
#pragma unroll
  for (int o = LPP / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, LPP);
  return v;
}

// Zero the pad columns of the LDS state rows.
__device__ __forceinline__ void clear_rows(BlockLDS &S, int tid) {
  for (int i = tid; i < PB * XP; i += NT) {
    (&S.xs[0][0])[i] = 0.f;
    (&S.ob[0][0])[i] = 0.f;
  }
}

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
  if (blockIdx.x == 0 && threadIdx.x == 0) D.fstate[1] = 0;
}

// ---------------------------------------------------------------------------
// Adam ascent on the couplings (update != 0), then the copies the kernels
// read: packed A-operand copies of every weight matrix and of its transpose,
// FP32 (training) and bfloat16-rounded (moves), and the bfloat16-rounded
// biases.  The gradient is the ordered sum of the KSPLIT particle-chunk
// partials.  Reading: the fit runs only on iterations that did not resample
// (a resampled population holds duplicates, which a maximum-likelihood fit
// would collapse onto); Adam's step count counts the steps taken.
// ---------------------------------------------------------------------------
__global__ void k_flow_adam(Dev D, FlowNet F, int step, int update, const float *part) {
  if (update && D.ps[0].resampled) return;  // no fit on a resampled iteration
  // Adam steps taken before this iteration's fit, plus this one (step: its
  // index in the fit; the count advances once, after the fit's last step)
  const int t = D.fstate[1] + step + 1;
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
    const float hb = __uint_as_float((uint32_t)bf16_bits(pv) << 16);
    bool weight = false;
    for (int l = 0; l < F.L; ++l) {
      const FlowLayerDesc &Y = F.ly[l];
      int o = -1, rows = 0, cols = 0, pf = 0, pb = 0;
      if (i >= Y.oW1 && i < Y.ob1) {
        o = Y.oW1, rows = FH, cols = Y.dc, pf = Y.pW1, pb = Y.qW1;
      } else if (i >= Y.oW2 && i < Y.ob2) {
        o = Y.oW2, rows = FH, cols = FH, pf = Y.pW2, pb = Y.qW2;
      } else if (i >= Y.oW3 && i < Y.ob3) {
        o = Y.oW3, rows = 2 * Y.dt, cols = FH, pf = Y.pW3, pb = Y.qW3;
      }
      if (o >= 0) {
        const int u = (i - o) / cols, k = (i - o) % cols;
        D.fpk[pf + pk_index(u, k, (cols + 15) / 16 * 16)] = pv;
        D.fpk[pb + pk_index(k, u, (rows + 15) / 16 * 16)] = pv;
        // the moves' bfloat16 copies, in the region of the FP32 layout (at most
        // half of it: K padded to 32 in bfloat16 against 16 in FP32)
        uint16_t *wb = reinterpret_cast<uint16_t *>(D.fbk);
        const uint16_t hbits = bf16_bits(pv);
        wb[2 * pf + pk16_index(u, k, (cols + 31) / 32)] = hbits;
        wb[2 * pb + pk16_index(k, u, (rows + 31) / 32)] = hbits;
        weight = true;
      }
    }
    D.fbias[i] = weight ? 0.f : hb;
  }
}

// ---------------------------------------------------------------------------
// Base map theta = m + L u of the flow from the weighted pre-move population:
// m its weighted mean (the first column pass of k_mass_colsum), L the Cholesky
// factor of its weighted covariance shrunk toward 1e-3 I,
//   n/(n+5) C + 1e-3 5/(n+5) I,  n the effective sample size,
// all in FP64; then FP32 copies of m and L, the packed A-operand matrices of
// the three base products (x -> L u, its transpose for the latent gradient,
// theta - m -> x via L^-1, with u_c = x_q(c)) and log|det L|.
// ---------------------------------------------------------------------------
constexpr int FCOV_G = 4;  // particle groups of 256 threads per covariance block

__global__ __launch_bounds__(256 * FCOV_G) void k_flow_cov(Dev D, FlowNet F) {
  // one 16 x 16 tile of the lower triangle of C and one of FCOV_CH particle
  // chunks per block (its partial sum goes to its own slice); each of the
  // FCOV_G thread groups takes every FCOV_G-th slab of 64 particles of the
  // chunk, and the group sums are added in group order
  __shared__ double Xa[FCOV_G][64][17], Xb[FCOV_G][64][17];
  __shared__ double Wc[FCOV_G][64];
  __shared__ double red[FCOV_G - 1][256];
  const int d = F.d;
  const int bt = blockIdx.x;
  int ta = (int)((sqrt(8.0 * bt + 1.0) - 1.0) * 0.5);
  while (ta * (ta + 1) / 2 > bt) --ta;
  while ((ta + 1) * (ta + 2) / 2 <= bt) ++ta;
  const int tb = bt - ta * (ta + 1) / 2, ch = blockIdx.y;
  const int g = threadIdx.x >> 8, t = threadIdx.x & 255;
  const int ty = t >> 4, tx = t & 15;
  const int c = 16 * ta + ty, k = 16 * tb + tx;
  const PState &PS = D.ps[0];
  const int rs = PS.resampled;
  const float *src = rs ? D.theta_t : D.theta;
  const double *mean = D.means;
  const int per = ((D.J + FCOV_CH - 1) / FCOV_CH + 63) / 64 * 64;
  const int jb = ch * per, je = min(D.J, jb + per);
  const int nit = (max(je - jb, 0) + 64 * FCOV_G - 1) / (64 * FCOV_G);
  double acc = 0.0;
  for (int it = 0; it < nit; ++it) {
    const int j0 = jb + 64 * (g + FCOV_G * it);
    for (int i = t; i < 64 * 16; i += 256) {
      const int jj = i >> 4, cc = i & 15, j = j0 + jj;
      const int ca = 16 * ta + cc, cb = 16 * tb + cc;
      Xa[g][jj][cc] = (j < je && ca < d) ? (double)src[(long long)j * D.DS + ca] - mean[ca] : 0.0;
      Xb[g][jj][cc] = (j < je && cb < d) ? (double)src[(long long)j * D.DS + cb] - mean[cb] : 0.0;
    }
    if (t < 64) {
      const int j = j0 + t;
      double w = 0.0;
      if (j < je) {
        const double lw = D.logw[j];
        w = rs ? 1.0 / D.J : ((lw == lw && lw > -INFINITY) ? exp(lw - PS.m) / PS.S : 0.0);
      }
      Wc[g][t] = w;
    }
    __syncthreads();
    for (int jj = 0; jj < 64; ++jj) acc += Wc[g][jj] * (Xa[g][jj][ty] * Xb[g][jj][tx]);
    __syncthreads();
  }
  if (g > 0) red[g - 1][t] = acc;
  __syncthreads();
  if (g == 0 && c < d && k < d) {
    for (int q = 0; q < FCOV_G - 1; ++q) acc += red[q][t];
    double *out = D.fcov + (long long)ch * d * d;
    out[(long long)c * d + k] = acc;
    out[(long long)k * d + c] = acc;
  }
}

// C = sum of the chunk partials in chunk order, shrunk: n/(n+5) C + 1e-3 5/(n+5) I,
// into fLd (d x d, FP64), the factorisations' input.
__global__ __launch_bounds__(256) void k_flow_covsum(Dev D, FlowNet F) {
  const int d = F.d, i = blockIdx.x * 256 + threadIdx.x;
  if (i >= d * d) return;
  const double n = D.ps[0].ess_before;
  const double sc = n / (n + 5.0), sh = 1e-3 * (5.0 / (n + 5.0));
  double v = 0.0;
  for (int ch = 0; ch < FCOV_CH; ++ch) v += D.fcov[(long long)ch * d * d + i];
  D.fLd[i] = sc * v + ((i / d == i % d) ? sh : 0.0);
}

__global__ __launch_bounds__(256) void k_flow_chol(Dev D, FlowNet F) {
  const int d = F.d, tid = threadIdx.x;
  double *A = D.fLd, *X = D.fLi;  // A: the shrunk covariance, factorised in place
  // right-looking Cholesky, lower triangle in place
  for (int k = 0; k < d; ++k) {
    if (tid == 0) A[(long long)k * d + k] = sqrt(A[(long long)k * d + k]);
    __syncthreads();
    const double lkk = A[(long long)k * d + k];
    for (int i = k + 1 + tid; i < d; i += 256) A[(long long)i * d + k] /= lkk;
    __syncthreads();
    const int m = d - k - 1;
    for (int e = tid; e < m * m; e += 256) {
      const int i = k + 1 + e / m, j = k + 1 + e % m;
      if (j <= i) A[(long long)i * d + j] -= A[(long long)i * d + k] * A[(long long)j * d + k];
    }
    __syncthreads();
  }
  // L^-1 column by column (forward substitution)
  for (int j = tid; j < d; j += 256)
    for (int i = 0; i < d; ++i) {
      double v = 0.0;
      if (i >= j) {
        v = (i == j) ? 1.0 : 0.0;
        for (int q = j; q < i; ++q) v -= A[(long long)i * d + q] * X[(long long)q * d + j];
        v /= A[(long long)i * d + i];
      }
      X[(long long)i * d + j] = v;
    }
  __syncthreads();
  const int K16 = (d + 15) / 16 * 16;
  for (int e = tid; e < d * d; e += 256) {
    const int c = e / d, k = e % d;
    const float l = k <= c ? (float)A[e] : 0.f;
    const float li = (float)X[e];
    D.fL[e] = l;
    D.fAf[pk_index(c, xpos(k, d), K16)] = l;          // theta - m = L u, u_k = x_q(k)
    D.fAb[pk_index(xpos(k, d), c, K16)] = l;          // cotangent of x: L^T g
    D.fAi[pk_index(xpos(c, d), k, K16)] = li;         // x_q(c) = (L^-1 (theta - m))_c
  }
  for (int c = tid; c < D.DS; c += 256) D.fm[c] = c < d ? (float)D.means[c] : 0.f;
  if (tid == 0) {
    double s = 0.0;
    for (int c = 0; c < d; ++c) s += log(A[(long long)c * d + c]);
    D.fbase[0] = (float)s;
  }
}

// The same for d <= FCHOL_LDS in one work group of FCHOL_W waves, as one pass
// of symmetric Gaussian elimination on [C_s | I], C_s = S^-1 C S^-1 the
// covariance scaled to unit diagonal (S = diag(sqrt(C_cc))).  Pivot k turns
// every row i > k into row_i - (s_ik / s_kk) row_k; afterwards the left block
// holds the pivots delta_k and the right block E = L_u^-1, the inverse of the
// unit lower factor of C_s = L_u diag(delta) L_u^T.  Hence
//   L = S L_u diag(delta)^1/2,  L^-1 = diag(delta)^-1/2 E S^-1.
// Layout: wave w keeps rows w, w + FCHOL_W, ... in registers, lane l holding
// columns l and l + 64, the full row (upper part included: by symmetry row k
// of the Schur complement is also its column k).  Row k as it stands when it
// becomes the pivot, v_k = (E_k0 .. E_k,k-1, s_kk, s_k,k+1 ..), is published
// to LDS row k by its owner, with 1/s_kk; one barrier per pivot.  Every
// position then takes the same update a_ij -= s_ik (v_k[j] / s_kk), with
// v_k[k] read as 1: the position (i, k) so becomes s_ik - s_ik / s_kk, i.e.
// E_ik plus s_ik, an offset no later update changes (updates are linear in
// the row), which the owner subtracts when it publishes row i (the s_ik are
// v_k[i], in LDS).  The unit diagonal keeps that offset no larger than the
// E entries it is added to (s_kk <= 1).  At the end LDS row k holds v_k:
// E_kj for j < k, delta_k, and s_jk for j > k (column k of L_u diag(delta)).
// Rows at or above the pivot keep taking the update; nothing reads them again.
// The blocked right-looking form (a panel of 16 pivots factored in one wave,
// then the trailing update, and L^-1 by block rows) took 0.21 ms at d = 100,
// the pivot-by-pivot form with two barriers per pivot 0.20 ms.
constexpr int FCHOL_LDS = 128;
constexpr int FCHOL_W = 16;                   // waves of the work group
constexpr int FCHOL_NT = 64 * FCHOL_W;
constexpr int FCHOL_RW = FCHOL_LDS / FCHOL_W; // rows per wave
constexpr int FCHOL_P = FCHOL_LDS + 1;        // largest LDS row pitch (odd: conflict-free columns)

// 1/x for x > 0 normal: the hardware estimate and two Newton-Raphson steps
// r <- r + r (1 - x r), each squaring the relative error.
__device__ __forceinline__ double rcp_newton(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  return fma(fma(-x, r, 1.0), r, r);
}

__global__ __launch_bounds__(FCHOL_NT) void k_flow_chol_lds(Dev D, FlowNet F) {
  __shared__ double M[FCHOL_LDS * FCHOL_P];   // row k: v_k
  __shared__ double rc[FCHOL_LDS];            // 1 / s_kk
  __shared__ double sd[FCHOL_LDS], isd[FCHOL_LDS], sq[FCHOL_LDS], rs[FCHOL_LDS];
  const int d = F.d, tid = threadIdx.x, P = d | 1, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const double *C = D.fLd;                    // the shrunk covariance
  for (int c = tid; c < d; c += FCHOL_NT) {
    const double x = C[c * d + c];
    sd[c] = sqrt(x);
    isd[c] = 1.0 / sd[c];
  }
  __syncthreads();
  const int j0 = min(lane, d - 1), j1 = min(lane + 64, d - 1);
  double a0[FCHOL_RW], a1[FCHOL_RW];
  {
    const double is0 = isd[j0], is1 = isd[j1];
#pragma unroll
    for (int r = 0; r < FCHOL_RW; ++r) {
      const int i = w + FCHOL_W * r;
      double x0 = 0.0, x1 = 0.0;
      if (i < d) {
        const double isi = isd[i];
        if (lane < d) x0 = C[i * d + lane] * isi * is0;
        if (lane + 64 < d) x1 = C[i * d + lane + 64] * isi * is1;
        if (i == 0) {                           // v_0: row 0 of C_s
          if (lane < d) M[lane] = x0;
          if (lane + 64 < d) M[lane + 64] = x1;
          if (lane == 0) rc[0] = rcp_newton(x0);
        }
      }
      a0[r] = x0;
      a1[r] = x1;
    }
  }
  for (int k = 0; k + 1 < d; ++k) {
    __syncthreads();
    const double rk = rc[k];
    const double *vk = M + k * P;
    double *vn = M + (k + 1) * P;
    const double w0 = lane == k ? rk : rk * vk[j0];
    const double w1 = lane + 64 == k ? rk : rk * vk[j1];
    double vi[FCHOL_RW];
#pragma unroll
    for (int r = 0; r < FCHOL_RW; ++r) vi[r] = vk[min(w + FCHOL_W * r, d - 1)];  // s_ik
#pragma unroll
    for (int r = 0; r < FCHOL_RW; ++r) {
      a0[r] = fma(-vi[r], w0, a0[r]);
      a1[r] = fma(-vi[r], w1, a1[r]);
    }
    const int nx = k + 1;
    if (nx % FCHOL_W == w) {                    // this wave owns the next pivot row
      const int rn = nx / FCHOL_W;
      double p0 = a0[0], p1 = a1[0];
#pragma unroll
      for (int r = 1; r < FCHOL_RW; ++r)
        if (r == rn) { p0 = a0[r]; p1 = a1[r]; }
      // E positions j < nx carry + s_{nx,j} = v_j[nx]
      if (lane < d) vn[lane] = lane < nx ? p0 - M[lane * P + nx] : p0;
      if (lane + 64 < d) vn[lane + 64] = lane + 64 < nx ? p1 - M[(lane + 64) * P + nx] : p1;
      if (lane == (nx & 63)) rc[nx] = rcp_newton(nx < 64 ? p0 : p1);
    }
  }
  __syncthreads();
  for (int c = tid; c < d; c += FCHOL_NT) {
    sq[c] = sqrt(M[c * P + c]);                 // delta_c^1/2
    rs[c] = 1.0 / sq[c];
    rc[c] = log(sq[c] * sd[c]);                 // log L_cc (rc is free again)
  }
  __syncthreads();
  const int K16 = (d + 15) / 16 * 16;
  // row c of L and of L^-1: wave w takes rows w, w + FCHOL_W, ..., lanes the columns
  for (int c = w; c < d; c += FCHOL_W)
    for (int k = lane; k < d; k += 64) {
      const double l = k < c ? M[k * P + c] * rs[k] * sd[c] : (k == c ? sq[c] * sd[c] : 0.0);
      const double li = k < c ? M[c * P + k] * rs[c] * isd[k] : (k == c ? rs[c] * isd[c] : 0.0);
      D.fL[c * d + k] = (float)l;
      D.fAf[pk_index(c, xpos(k, d), K16)] = (float)l;        // theta - m = L u, u_k = x_q(k)
      D.fAb[pk_index(xpos(k, d), c, K16)] = (float)l;        // cotangent of x: L^T g
      D.fAi[pk_index(xpos(c, d), k, K16)] = (float)li;       // x_q(c) = (L^-1 (theta - m))_c
    }
  for (int c = tid; c < D.DS; c += FCHOL_NT) D.fm[c] = c < d ? (float)D.means[c] : 0.f;
  if (tid == 0) {
    double s = 0.0;
    for (int c = 0; c < d; ++c) s += rc[c];
    D.fbase[0] = (float)s;
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
__global__ __launch_bounds__(NT) void k_flow_train(Dev D, FlowNet F) {
  if (D.ps[0].resampled) return;
  __shared__ BlockLDS S;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int p = tid / LPP, r = tid % LPP;
  const int j0 = blockIdx.x * PB;
  const PState &PS = D.ps[0];
  const int rs = PS.resampled;
  const float *src = rs ? D.theta_t : D.theta;
  if (tid < PB) {
    const int j = j0 + tid;
    const bool ok = j < D.J;
    double w = 0.0;
    if (ok) {
      const double lw = D.logw[j];
      w = rs ? 1.0 / D.J : ((lw == lw && lw > -INFINITY) ? exp(lw - PS.m) / PS.S : 0.0);
    }
    S.wj[tid] = (float)w;
    S.rows[tid] = ok ? j : -1;
    float *rec = D.ftape + (long long)(ok ? j : j0) * F.L * F.train_stride;
    S.tw[tid] = ok ? rec : nullptr;
    S.tr[tid] = rec;
  }
  clear_rows(S, tid);
  __syncthreads();
  for (int q = tid / LPP, c = tid % LPP; c < F.d; c += LPP) {
    const int j = S.rows[q];
    S.ob[q][c] = j >= 0 ? src[(long long)j * D.DS + c] - D.fm[c] : 0.f;
  }
  __syncthreads();
  mdense(D.fAi, F.d, F.d, nullptr, &S.ob[0][0], XP, &S.xs[0][0], XP, ST_PLAIN, S, -1, 0, wave, lane);
  __syncthreads();
  const float *W = D.fp;
  const int h = F.half, TS = F.train_stride;
  // inverse couplings, last layer first
  for (int l = F.L - 1; l >= 0; --l) {
    const FlowLayerDesc &Y = F.ly[l];
    const int lo = l * TS;
    if (S.tw[p])
      for (int c = r; c < Y.dc; c += LPP) S.tw[p][lo + c] = S.xs[p][Y.C0 + c];
    mdense(D.fpk + Y.pW1, FH, Y.dc, W + Y.ob1, &S.xs[0][Y.C0], XP, &S.h1[0][0], HP, ST_TANH, S,
           lo + h, 0, wave, lane);
    __syncthreads();
    mdense(D.fpk + Y.pW2, FH, FH, W + Y.ob2, &S.h1[0][0], HP, &S.h2[0][0], HP, ST_TANH, S,
           lo + h + FH, 0, wave, lane);
    __syncthreads();
    mdense(D.fpk + Y.pW3, 2 * Y.dt, FH, W + Y.ob3, &S.h2[0][0], HP, &S.ob[0][0], XP, ST_PLAIN, S,
           -1, 0, wave, lane);
    __syncthreads();
    for (int f = r; f < Y.dt; f += LPP) {
      const float s = tanhf(S.ob[p][f]);
      const float t = S.ob[p][Y.dt + f];
      const float x = (S.xs[p][Y.T0 + f] - t) * expf(-s);
      S.xs[p][Y.T0 + f] = x;
      if (S.tw[p]) {
        S.tw[p][lo + h + 2 * FH + f] = s;
        S.tw[p][lo + 2 * h + 2 * FH + f] = x;
      }
    }
    __syncthreads();
  }
  // cotangent of z: -W_j z
  for (int c = r; c < MAXD; c += LPP) S.xs[p][c] = -S.wj[p] * S.xs[p][c];
  __syncthreads();
  // reverse of the inverse order: layer 0 first
  for (int l = 0; l < F.L; ++l) {
    const FlowLayerDesc &Y = F.ly[l];
    const int lo = l * TS;
    const float *rr = S.tr[p] + lo;
    for (int f = r; f < Y.dt; f += LPP) {
      const float s = rr[h + 2 * FH + f], xT = rr[2 * h + 2 * FH + f];
      const float gx = S.xs[p][Y.T0 + f];
      const float es = expf(-s);
      const float gs = -gx * xT - S.wj[p];
      const float d3s = gs * (1.f - s * s), d3t = -gx * es;
      S.ob[p][f] = d3s;
      S.ob[p][Y.dt + f] = d3t;
      S.xs[p][Y.T0 + f] = gx * es;
      if (S.tw[p]) {
        S.tw[p][lo + 3 * h + 2 * FH + f] = d3s;
        S.tw[p][lo + 3 * h + 2 * FH + Y.dt + f] = d3t;
      }
    }
    __syncthreads();
    mdense(D.fpk + Y.qW3, FH, 2 * Y.dt, nullptr, &S.ob[0][0], XP, &S.h2[0][0], HP, ST_DTANH, S,
           lo + 5 * h + 2 * FH, lo + h + FH, wave, lane);
    __syncthreads();
    mdense(D.fpk + Y.qW2, FH, FH, nullptr, &S.h2[0][0], HP, &S.h1[0][0], HP, ST_DTANH, S,
           lo + 5 * h + 3 * FH, lo + h, wave, lane);
    __syncthreads();
    mdense(D.fpk + Y.qW1, Y.dc, FH, nullptr, &S.h1[0][0], HP, &S.xs[0][Y.C0], XP, ST_ADD, S, -1, 0,
           wave, lane);
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
  if (D.ps[0].resampled) return;
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
      const float *q = base + g.off_delta + u;
      float s = 0.f;
      int j = ja;
      for (; j + 8 <= jb; j += 8) {  // eight loads in flight, summed in index order
        float v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = q[(j + e) * stride];
#pragma unroll
        for (int e = 0; e < 8; ++e) s += v[e];
      }
      for (; j < jb; ++j) s += q[j * stride];
      out[g.ob + u] = s;
    }
    return;
  }
  const int ntc = (g.cols + 63) / 64;
  const int u0 = (tile / ntc) * 64, k0 = (tile % ntc) * 64;
  const int ty = t >> 4, tx = t & 15;
  // one round: 32 particles x 64 delta rows / 64 input columns, two float4
  // pairs per thread (tape rows and offsets are multiples of 4 floats); the
  // next round's loads are issued before this round's FMAs
  auto fetch = [&](int j0, float4 *a, float4 *b) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int idx = t + 256 * q, jj = idx >> 4, c4 = idx & 15;
      const int j = j0 + jj;
      a[q] = make_float4(0.f, 0.f, 0.f, 0.f);
      b[q] = a[q];
      if (j < jb) {
        const float *r = base + j * stride;
        const int u = u0 + 4 * c4, k = k0 + 4 * c4;
        if (u + 3 < g.rows) {
          a[q] = *reinterpret_cast<const float4 *>(r + g.off_delta + u);
        } else {
          float av[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) av[e] = (u + e < g.rows) ? r[g.off_delta + u + e] : 0.f;
          a[q] = make_float4(av[0], av[1], av[2], av[3]);
        }
        if (k + 3 < g.cols) {
          b[q] = *reinterpret_cast<const float4 *>(r + g.off_in + k);
        } else {
          float bv[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) bv[e] = (k + e < g.cols) ? r[g.off_in + k + e] : 0.f;
          b[q] = make_float4(bv[0], bv[1], bv[2], bv[3]);
        }
      }
    }
  };
  float acc[4][4] = {};
  float4 pa[2], pb[2];
  fetch(ja, pa, pb);
  for (int jj0 = ja; jj0 < jb; jj0 += 32) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int idx = t + 256 * q;
      As[idx >> 4][idx & 15] = pa[q];
      Bs[idx >> 4][idx & 15] = pb[q];
    }
    __syncthreads();
    if (jj0 + 32 < jb) fetch(jj0 + 32, pa, pb);
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
// Start of the moves: z0 = T^-1(theta0) (BF16 weights) and log|det J_T(z0)|;
// the initial energy gets -log|det J_T(z0)|.  The latent gradient at z0
// follows from the forward pass with its tape and the backward pass on the
// cached gradient of log pi at theta0 (k_flow_drift / k_flow_kick, init).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(NT) void k_flow_inverse(Dev D, FlowNet F) {
  __shared__ BlockLDS S;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int p = tid / LPP, r = tid % LPP;
  const int j0 = blockIdx.x * PB;
  if (tid < PB) {
    const int j = j0 + tid;
    S.rows[tid] = j < D.J ? j : -1;
    S.tw[tid] = nullptr;
    S.tr[tid] = nullptr;
  }
  clear_rows(S, tid);
  __syncthreads();
  for (int q = tid / LPP, c = tid % LPP; c < F.d; c += LPP) {
    const int j = S.rows[q];
    S.ob[q][c] = j >= 0 ? D.theta_t[(long long)j * D.DS + c] - D.fm[c] : 0.f;
  }
  __syncthreads();
  mdense(D.fAi, F.d, F.d, nullptr, &S.ob[0][0], XP, &S.xs[0][0], XP, ST_PLAIN, S, -1, 0, wave, lane);
  __syncthreads();
  float ldp = r == 0 ? -D.fbase[0] : 0.f;
  for (int l = F.L - 1; l >= 0; --l) {
    const FlowLayerDesc &Y = F.ly[l];
    const uint16_t *Wb = reinterpret_cast<const uint16_t *>(D.fbk);
    mdense_bf(Wb + 2 * Y.pW1, FH, Y.dc, D.fbias + Y.ob1, &S.xs[0][Y.C0], XP, &S.h1[0][0], HP,
              ST_TANH, S, -1, 0, wave, lane);
    __syncthreads();
    mdense_bf(Wb + 2 * Y.pW2, FH, FH, D.fbias + Y.ob2, &S.h1[0][0], HP, &S.h2[0][0], HP, ST_TANH,
              S, -1, 0, wave, lane);
    __syncthreads();
    mdense_bf(Wb + 2 * Y.pW3, 2 * Y.dt, FH, D.fbias + Y.ob3, &S.h2[0][0], HP, &S.ob[0][0], XP,
              ST_PLAIN, S, -1, 0, wave, lane);
    __syncthreads();
    for (int f = r; f < Y.dt; f += LPP) {
      const float s = tanhf(S.ob[p][f]);
      S.xs[p][Y.T0 + f] = (S.xs[p][Y.T0 + f] - S.ob[p][Y.dt + f]) * expf(-s);
      ldp -= s;
    }
    __syncthreads();
  }
  const float ld0 = -sum_lpp(ldp);   // log|det J_T(z0)|
  const int j = S.rows[p];
  if (j >= 0) {
    for (int c = r; c < D.DS; c += LPP) {
      const float z = c < F.d ? S.xs[p][c] : 0.f;
      D.fz[(long long)j * D.DS + c] = z;
      D.fz0[(long long)j * D.DS + c] = z;
    }
    if (r == 0) {
      D.fld0[j] = ld0;
      D.H0[j] -= (double)ld0;
    }
  }
}

// Particles of a move launch: 16 consecutive slots of the trajectory-length
// order (longest first), active while n > step; init: every particle, in
// index order.  Returns whether any is active (the same in every thread).
__device__ __forceinline__ bool move_rows(const Dev &D, const FlowNet &F, BlockLDS &S, int step,
                                          int init, int tid) {
  int act = 0;
  if (tid < PB) {
    const int slot = blockIdx.x * PB + tid;
    int r = -1;
    if (slot < D.J) {
      const int j = init ? slot : D.perm[slot];
      if (j < D.J && (init || D.n[j] > step)) r = j;
    }
    S.rows[tid] = r;
    act = r >= 0;
  }
  const bool any = __syncthreads_or(act);
  if (!any) return false;
  if (tid < PB) {
    int first = 0;
    for (int q = PB - 1; q >= 0; --q)
      if (S.rows[q] >= 0) first = S.rows[q];
    const int r = S.rows[tid];
    S.tw[tid] = r >= 0 ? D.ftape + (long long)r * F.L * F.tape_stride : nullptr;
    S.tr[tid] = D.ftape + (long long)(r >= 0 ? r : first) * F.L * F.tape_stride;
  }
  clear_rows(S, tid);
  __syncthreads();
  return true;
}

// Leapfrog step `step`, first half: p += eps/2 g_z; z += eps p; theta = T(z)
// (BF16 weights) with the move tape and log|det J_T(z)|.  The likelihood
// gradient at theta follows (k_lf_partial / k_lf_reduce in gradient mode).
// init: only the forward pass from z0, for the tape of the latent gradient.
__device__ __forceinline__ void drift_body(const Dev &D, const FlowNet &F, BlockLDS &S, int init,
                                           int tid) {
  const int lane = tid & 63, wave = tid >> 6;
  const int p = tid / LPP, r = tid % LPP;
  const float eps = (float)D.ps[0].eps;
  const float he = 0.5f * eps;
  for (int q = tid / LPP, c = tid % LPP; c < F.d; c += LPP) {
    const int j = S.rows[q];
    if (j < 0) continue;
    const long long e = (long long)j * D.DS + c;
    float z;
    if (init) {
      z = D.fz[e];
    } else {
      const float ph = fmaf(he, D.fgz[e], D.p_t[e]);
      z = fmaf(eps, ph, D.fz[e]);
      D.p_t[e] = ph;
      D.fz[e] = z;
    }
    S.xs[q][c] = z;
  }
  __syncthreads();
  float ldp = forward_couplings(F, reinterpret_cast<const uint16_t *>(D.fbk), D.fbias, S, wave,
                               lane, tid);
  if (init) return;
  mdense(D.fAf, F.d, F.d, nullptr, &S.xs[0][0], XP, &S.ob[0][0], XP, ST_PLAIN, S, -1, 0, wave, lane);
  if (r == 0) ldp += D.fbase[0];
  const float ld = sum_lpp(ldp);
  __syncthreads();
  const int j = S.rows[p];
  if (j >= 0) {
    for (int c = r; c < D.DS; c += LPP)
      D.theta_t[(long long)j * D.DS + c] = c < F.d ? D.fm[c] + S.ob[p][c] : 0.f;
    if (r == 0) D.fld1[j] = ld;
  }
}

__global__ __launch_bounds__(NT) void k_flow_drift(Dev D, FlowNet F, int step, int init) {
  __shared__ BlockLDS S;
  if (!move_rows(D, F, S, step, init, threadIdx.x)) return;
  drift_body(D, F, S, init, threadIdx.x);
}

// Leapfrog step `step`, second half: g_z = J_T^T grad log pi(theta) +
// grad log|det J_T| from the move tape; p += eps/2 g_z.  init: the latent
// gradient at z0 from the cached gradient at theta0, no kick.
__device__ __forceinline__ void kick_body(const Dev &D, const FlowNet &F, BlockLDS &S, int init,
                                          int tid) {
  const int lane = tid & 63, wave = tid >> 6;
  const float he = 0.5f * (float)D.ps[0].eps;
  for (int q = tid / LPP, c = tid % LPP; c < F.d; c += LPP) {
    const int j = S.rows[q];
    S.ob[q][c] = j >= 0 ? D.grad_t[(long long)j * D.DS + c] : 0.f;
  }
  __syncthreads();
  mdense(D.fAb, F.d, F.d, nullptr, &S.ob[0][0], XP, &S.xs[0][0], XP, ST_PLAIN, S, -1, 0, wave, lane);
  __syncthreads();
  for (int i = tid; i < PB * XP; i += NT) (&S.ob[0][0])[i] = 0.f;
  __syncthreads();
  vjp_couplings(F, reinterpret_cast<const uint16_t *>(D.fbk), S, wave, lane, tid);
  for (int q = tid / LPP, c = tid % LPP; c < F.d; c += LPP) {
    const int j = S.rows[q];
    if (j < 0) continue;
    const long long e = (long long)j * D.DS + c;
    const float g = S.xs[q][c];
    D.fgz[e] = g;
    if (!init) D.p_t[e] = fmaf(he, g, D.p_t[e]);
  }
}

__global__ __launch_bounds__(NT) void k_flow_kick(Dev D, FlowNet F, int step, int init) {
  __shared__ BlockLDS S;
  if (!move_rows(D, F, S, step, init, threadIdx.x)) return;
  kick_body(D, F, S, init, threadIdx.x);
}

// The kick of step `step` and the drift of step `step + 1` in one launch (one
// kernel boundary fewer per step).  Both work on the block's own particles
// only: a particle moving at step + 1 moves at step too, and its p and g_z
// pass from the kick to the drift through global memory within the block.
__global__ __launch_bounds__(NT) void k_flow_kick_drift(Dev D, FlowNet F, int step) {
  __shared__ BlockLDS S;
  const int tid = threadIdx.x;
  if (!move_rows(D, F, S, step, 0, tid)) return;
  kick_body(D, F, S, 0, tid);
  __syncthreads();  // the kick's LDS reads and global writes before the drift's set-up
  if (!move_rows(D, F, S, step + 1, 0, tid)) return;
  drift_body(D, F, S, 0, tid);
}

// New parameters from the caller: restart the Adam moments, and count Adam
// steps from the next iteration on.
__global__ void k_flow_reset(Dev D, FlowNet F) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < F.nparams; i += gridDim.x * blockDim.x) {
    D.fadm[i] = 0.f;
    D.fadv[i] = 0.f;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) D.fstate[1] = 0;
}

// Count the Adam steps of an iteration's fit (after its last k_flow_adam), and
// the iterations whose move used couplings fitted to the population it moved
// (never reset: the evidence estimate carries every such iteration).
__global__ void k_flow_tick(Dev D, int steps) {
  if (!D.ps[0].resampled) {
    D.fstate[1] += steps;
    D.fstate[2] += 1;
  }
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
  const int nt = (F.d + 15) / 16;
  hipLaunchKernelGGL(k_flow_cov, dim3(nt * (nt + 1) / 2, FCOV_CH), dim3(256 * FCOV_G), 0, st, D, F);
  hipLaunchKernelGGL(k_flow_covsum, dim3((F.d * F.d + 255) / 256), dim3(256), 0, st, D, F);
  if (F.d <= FCHOL_LDS)
    hipLaunchKernelGGL(k_flow_chol_lds, dim3(1), dim3(FCHOL_NT), 0, st, D, F);
  else
    hipLaunchKernelGGL(k_flow_chol, dim3(1), dim3(256), 0, st, D, F);
  return hipGetLastError();
}

hipError_t launch_flow_train(const Dev &D, const FlowNet &F, int step, hipStream_t st) {
  hipLaunchKernelGGL(k_flow_train, dim3((D.J + PB - 1) / PB), dim3(NT), 0, st, D, F);
  int nb = 0;
  for (int l = 0; l < F.L; ++l) {
    const FlowLayerDesc &Y = F.ly[l];
    const int rc[3][2] = {{2 * Y.dt, FH}, {FH, FH}, {FH, Y.dc}};
    for (int w = 0; w < 3; ++w) nb += ((rc[w][0] + 63) / 64) * ((rc[w][1] + 63) / 64) + 1;
  }
  hipLaunchKernelGGL(k_flow_wgrad, dim3(nb, KSPLIT), dim3(256), 0, st, D, F, D.fgrad);
  hipLaunchKernelGGL(k_flow_adam, dim3(256), dim3(256), 0, st, D, F, step, 1,
                     (const float *)D.fgrad);
  if (step == F.ntrain - 1) hipLaunchKernelGGL(k_flow_tick, dim3(1), dim3(1), 0, st, D, F.ntrain);
  return hipGetLastError();
}

hipError_t launch_flow_begin(const Dev &D, const FlowNet &F, hipStream_t st) {
  const dim3 grid((D.J + PB - 1) / PB);
  hipLaunchKernelGGL(k_flow_inverse, grid, dim3(NT), 0, st, D, F);
  hipLaunchKernelGGL(k_flow_drift, grid, dim3(NT), 0, st, D, F, 0, 1);
  hipLaunchKernelGGL(k_flow_kick, grid, dim3(NT), 0, st, D, F, 0, 1);
  return hipGetLastError();
}

hipError_t launch_flow_drift(const Dev &D, const FlowNet &F, int step, hipStream_t st) {
  hipLaunchKernelGGL(k_flow_drift, dim3((D.J + PB - 1) / PB), dim3(NT), 0, st, D, F, step, 0);
  return hipGetLastError();
}

hipError_t launch_flow_kick(const Dev &D, const FlowNet &F, int step, hipStream_t st) {
  hipLaunchKernelGGL(k_flow_kick, dim3((D.J + PB - 1) / PB), dim3(NT), 0, st, D, F, step, 0);
  return hipGetLastError();
}

hipError_t launch_flow_kick_drift(const Dev &D, const FlowNet &F, int step, hipStream_t st) {
  hipLaunchKernelGGL(k_flow_kick_drift, dim3((D.J + PB - 1) / PB), dim3(NT), 0, st, D, F, step);
  return hipGetLastError();
}

}  // namespace smc
