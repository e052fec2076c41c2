// bfloat16 helpers and matrix-core operand types shared by the bf16 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>

namespace hx {

typedef short bf16x4 __attribute__((ext_vector_type(4)));  // 4 bf16 operands of a 16x16x16 MFMA
typedef float f32x4 __attribute__((ext_vector_type(4)));   // its 4 FP32 accumulators
typedef short bf16x8 __attribute__((ext_vector_type(8)));  // 8 bf16 operands (bit patterns) of a 16x16x32 MFMA
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));  // the same bits as that builtin's operand type

// round to nearest even
__host__ __device__ inline uint16_t f32_to_bf16_bits(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_bits_to_f32(uint16_t h) { return __builtin_bit_cast(float, (uint32_t)h << 16); }

__device__ __forceinline__ float to_float(float v) { return v; }
__device__ __forceinline__ float to_float(uint16_t v) { return bf16_bits_to_f32(v); }
__device__ __forceinline__ void store_as(float *p, float v) { *p = v; }
__device__ __forceinline__ void store_as(uint16_t *p, float v) { *p = f32_to_bf16_bits(v); }

}  // namespace hx
