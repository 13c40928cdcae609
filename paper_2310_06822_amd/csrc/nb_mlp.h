// Shared pieces of the MLP kernels: parameter offsets, bfloat16 rounding,
// matrix-core wrappers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

typedef __bf16 nb_bf16x8 __attribute__((ext_vector_type(8)));
typedef float nb_floatx4 __attribute__((ext_vector_type(4)));

typedef __bf16 nb_bf16x2 __attribute__((ext_vector_type(2)));
typedef float nb_float2 __attribute__((ext_vector_type(2)));
typedef short nb_short2 __attribute__((ext_vector_type(2)));
typedef unsigned nb_uint4 __attribute__((ext_vector_type(4)));

// max(z, 0) in one instruction for every finite z (+inf becomes FLT_MAX).
__device__ __forceinline__ float nb_relu(float z) { return __builtin_amdgcn_fmed3f(z, 0.0f, 3.40282347e38f); }

// max(v_j, 0) rounded to bfloat16 for 8 values: each pair is rounded to
// nearest even by one packed conversion, then a packed signed 16-bit max with
// 0 clears the negative ones (a bfloat16 with its sign bit set is a negative
// 16-bit integer).  The same bits as rounding max(v_j, 0), NaN aside, in 8
// instructions.
__device__ __forceinline__ nb_bf16x8 nb_relu_bf16x8(const float (&v)[8]) {
  nb_uint4 u;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const nb_float2 f = {v[2 * p], v[2 * p + 1]};
    const nb_bf16x2 b = __builtin_convertvector(f, nb_bf16x2);
    const nb_short2 m = __builtin_elementwise_max(__builtin_bit_cast(nb_short2, b), (nb_short2)0);
    u[p] = __builtin_bit_cast(unsigned, m);
  }
  return __builtin_bit_cast(nb_bf16x8, u);
}

// Offsets into theta for an in_dim -> W^NH -> 1 network (linear-layer layout):
// layer l's weight matrix starts at nb_w_off(l), its bias at nb_b_off(l).
__host__ __device__ inline int64_t nb_w_off(int l, int in_dim, int W) {
  return l == 0 ? 0 : (int64_t)W * in_dim + W + (int64_t)(l - 1) * ((int64_t)W * W + W);
}
__host__ __device__ inline int64_t nb_b_off(int l, int in_dim, int W, int NH) {
  return nb_w_off(l, in_dim, W) + (int64_t)(l == 0 ? in_dim : W) * (l == NH ? 1 : W);
}

// Writes the value of float32 weight p to every packed-fragment slot that
// holds it, in the layout the float32 forward and training kernels read
// (KIN = ceil(in_dim / 4) input steps, RB = W / 16 row blocks; lane
// 16 g + c of a fragment):
//   first layer W0[row][k]: fragment (row / 16) KIN + k / 4, g = k % 4,
//     c = row % 16;
//   hidden W_l[row][col]: forward fragment (mo, mi, r) = (row / 16, col / 16,
//     col % 4) with g = (col % 16) / 4, c = row % 16, and the transposed copy
//     (mo, mi, r) = (col / 16, row / 16, row % 4) with g = (row % 16) / 4,
//     c = col % 16.
// Biases and output weights are read from theta and have no slot.
__device__ inline void nb_f32_pack_put(int64_t p, float v, float* __restrict__ pack, int in_dim, int W, int NH) {
  const int RB = W / 16, KIN = (in_dim + 3) / 4, F1 = RB * KIN, FH = RB * RB * 4, NFWD = F1 + (NH - 1) * FH;
  if (p < (int64_t)W * in_dim) {
    const int row = (int)(p / in_dim), k = (int)(p % in_dim);
    pack[(int64_t)((row >> 4) * KIN + (k >> 2)) * 64 + (k & 3) * 16 + (row & 15)] = v;
    return;
  }
  for (int l = 1; l < NH; ++l) {
    const int64_t off = nb_w_off(l, in_dim, W);
    if (p >= off && p < off + (int64_t)W * W) {
      const int e = (int)(p - off), row = e / W, col = e % W;
      pack[(int64_t)(F1 + (l - 1) * FH + ((row >> 4) * RB + (col >> 4)) * 4 + (col & 3)) * 64 +
           ((col & 15) >> 2) * 16 + (row & 15)] = v;
      pack[(int64_t)(NFWD + (l - 1) * FH + ((col >> 4) * RB + (row >> 4)) * 4 + (row & 3)) * 64 +
           ((row & 15) >> 2) * 16 + (col & 15)] = v;
      return;
    }
  }
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

// Element e (bfloat16 bits) of a bound's forward fragment pack, from its
// float32 parameters th: e = (f*64 + lane)*8 + j with c = lane % 16,
// g = lane / 16:
//   f < RB            first layer, block mo = f, "bf16x3" split:
//                       g = 0, 1: W0_hi[16mo + c][j];  g = 2: W0_lo[16mo + c][j];
//                       g = 3: 0;  (0 for j >= in_dim)
//   otherwise         hidden layer l (1-based), fragment (mo, ks),
//                       f = RB + (l-1)*FH + mo*KS + ks:
//                       W_l[16mo + c][32ks + 16(j/4) + 4g + (j%4)]
__host__ __device__ inline uint16_t nb_bf16_pack_elem(const float* th, int in_dim, int W, int NH, int64_t e) {
  (void)NH;
  const int j = (int)(e & 7), lane = (int)((e >> 3) & 63);
  const int f = (int)(e >> 9);
  const int c = lane & 15, g = lane >> 4;
  const int RB = W / 16, KS = W / 32, FH = RB * KS;
  if (f < RB) {
    if (j >= in_dim || g == 3) return 0;
    const float w = th[(int64_t)(16 * f + c) * in_dim + j];
    const uint16_t hi = nb_bf16_bits(w);
    return g < 2 ? hi : nb_bf16_bits(w - nb_bf16_value(hi));
  }
  const int t = f - RB;
  const int l = 1 + t / FH, rem = t % FH, mo = rem / KS, ks = rem % KS;
  const float* Wl = th + nb_w_off(l, in_dim, W);
  return nb_bf16_bits(Wl[(int64_t)(16 * mo + c) * W + 32 * ks + 16 * (j / 4) + 4 * g + (j % 4)]);
}

// Element e of the transposed (backward) pack of the hidden layers:
// packT[((l-1)*FH + mo*KS + ks)*64 + lane][j] = W_l[32ks + 8g + j][16mo + c]
// (the A operand of W_l^T D with the reduction over W_l's outputs in order).
__host__ __device__ inline uint16_t nb_bf16_pack_t_elem(const float* th, int in_dim, int W, int NH, int64_t e) {
  (void)NH;
  const int j = (int)(e & 7), lane = (int)((e >> 3) & 63), f = (int)(e >> 9);
  const int c = lane & 15, g = lane >> 4;
  const int RB = W / 16, KS = W / 32, FH = RB * KS;
  const int l = 1 + f / FH, rem = f % FH, mo = rem / KS, ks = rem % KS;
  const float* Wl = th + nb_w_off(l, in_dim, W);
  return nb_bf16_bits(Wl[(int64_t)(32 * ks + 8 * g + j) * W + 16 * mo + c]);
}

// Number of 16-byte fragment slices of the forward / transposed packs.
__host__ __device__ inline int64_t nb_bf16_fwd_slices(int W, int NH) {
  return (int64_t)(W / 16 + (NH - 1) * (W / 16) * (W / 32)) * 64;
}
__host__ __device__ inline int64_t nb_bf16_t_slices(int W, int NH) {
  return (int64_t)(NH - 1) * (W / 16) * (W / 32) * 64;
}

// Number of compute units of the current device (cached per device).
int nb_cu_count();
