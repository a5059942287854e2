// bfloat16 helpers: round-to-nearest-even from FP32 on the gfx950 conversion
// instruction (v_cvt_pk_bf16_f32), kept as raw 16-bit patterns.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sq {

__device__ __forceinline__ uint16_t bf16_bits(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

__device__ __forceinline__ float bf16_round(float f) { return (float)(__bf16)f; }

}  // namespace sq
