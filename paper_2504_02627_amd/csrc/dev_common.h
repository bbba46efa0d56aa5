// Device helpers shared by the kernel sources of libchees_smc.so: Philox
// counter-based normals and fixed-order wave reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace smc {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC 2011) and Box--Muller normals.
// Counter = (block, particle, iteration, stream), key = (seed lo, seed hi).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(0xD2511F53u, c.x), lo0 = 0xD2511F53u * c.x;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z), lo1 = 0xCD9E8D57u * c.z;
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

__device__ __forceinline__ double u01(uint32_t x) { return ((double)x + 0.5) / 4294967296.0; }

__device__ __forceinline__ uint4 philox_at(uint64_t seed, uint32_t block, uint32_t particle,
                                           uint32_t iteration, uint32_t stream) {
  return philox10(make_uint4(block, particle, iteration, stream), (uint32_t)seed,
                  (uint32_t)(seed >> 32));
}

// Four standard normals from one Philox block: pairs (w0, w1), (w2, w3).
__device__ __forceinline__ void box_muller4(uint4 w, double out[4]) {
  const double two_pi = 2.0 * 3.141592653589793;
  double r = sqrt(-2.0 * log(u01(w.x)));
  double t = two_pi * u01(w.y);
  out[0] = r * cos(t);
  out[1] = r * sin(t);
  r = sqrt(-2.0 * log(u01(w.z)));
  t = two_pi * u01(w.w);
  out[2] = r * cos(t);
  out[3] = r * sin(t);
}

// ---------------------------------------------------------------------------
// Wave64 reductions in a fixed order (butterfly), deterministic.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

}  // namespace smc
