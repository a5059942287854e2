// bfloat16 helpers: round-to-nearest-even from FP32, kept as raw 16-bit patterns.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sq {

__device__ __forceinline__ uint16_t bf16_bits(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_round(float f) {
  return __uint_as_float(((unsigned)bf16_bits(f)) << 16);
}

}  // namespace sq
