// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and Box-Muller, device side.
#pragma once
#include <hip/hip_runtime.h>

namespace sq {

struct P4 { unsigned x, y, z, w; };

// Ten rounds of Philox4x32: two 32x32->64 products per round, key advanced by the
// Weyl constants between rounds.
__device__ __forceinline__ P4 philox10(P4 c, unsigned k0, unsigned k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    const unsigned a = c.x, b = c.z;
    const unsigned hi0 = __umulhi(0xD2511F53u, a), lo0 = 0xD2511F53u * a;
    const unsigned hi1 = __umulhi(0xCD9E8D57u, b), lo1 = 0xCD9E8D57u * b;
    c = P4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
  }
  return c;
}

// 23 random bits plus one half, scaled into (0, 1): exact in FP32.
__device__ __forceinline__ float uniform23(unsigned w) {
  return ((float)(w >> 9) + 0.5f) * 1.1920928955078125e-7f;  // 2^-23
}

__device__ __forceinline__ float box_muller(unsigned w0, unsigned w1) {
  const float u1 = uniform23(w0), u2 = uniform23(w1);
  return sqrtf(-2.0f * logf(u1)) * cosf(6.283185307179586f * u2);
}

}  // namespace sq
