// Shared pieces of the MLP kernels: parameter offsets, bfloat16 rounding,
// matrix-core wrappers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

typedef __bf16 nb_bf16x8 __attribute__((ext_vector_type(8)));
typedef float nb_floatx4 __attribute__((ext_vector_type(4)));

// Offsets into theta for an in_dim -> W^NH -> 1 network (linear-layer layout):
// layer l's weight matrix starts at nb_w_off(l), its bias at nb_b_off(l).
__host__ __device__ inline int64_t nb_w_off(int l, int in_dim, int W) {
  return l == 0 ? 0 : (int64_t)W * in_dim + W + (int64_t)(l - 1) * ((int64_t)W * W + W);
}
__host__ __device__ inline int64_t nb_b_off(int l, int in_dim, int W, int NH) {
  return nb_w_off(l, in_dim, W) + (int64_t)(l == 0 ? in_dim : W) * (l == NH ? 1 : W);
}

// bfloat16 round-to-nearest-even of a float32, from its bit pattern.
__host__ __device__ inline uint16_t nb_bf16_bits(float v) {
  uint32_t u;
  __builtin_memcpy(&u, &v, 4);
  u = u + 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__host__ __device__ inline float nb_bf16_value(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float v;
  __builtin_memcpy(&v, &u, 4);
  return v;
}

__device__ __forceinline__ nb_floatx4 nb_mfma_bf16(nb_bf16x8 a, nb_bf16x8 b, nb_floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Number of compute units of the current device (cached per device).
int nb_cu_count();
