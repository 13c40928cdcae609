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

// Reduce-scatter over the 16 lanes of a row: lane c ends with the row sums
// of the values i = c + 16 k (k < V / 16), each in a fixed order.  Step t
// pairs lane c with c ^ (1 << bt) for bt = 3, 0, 1, 2 and keeps the half of
// its remaining values whose bit bt of i matches the lane's, adding the
// partner's copy of that half.  The position of value i among the remaining
// ones is i with the bits split so far taken out (nb_rs_compress).
__host__ __device__ constexpr int nb_rs_compress(int i, int mask) {
  int r = 0, o = 0;
  for (int b = 0; b < 8; ++b)
    if (!((mask >> b) & 1)) r |= ((i >> b) & 1) << o++;
  return r;
}
__host__ __device__ constexpr int nb_rs_expand(int j, int mask) {   // j with zero bits put in at the mask's positions
  int r = 0, o = 0;
  for (int b = 0; b < 8; ++b) {
    if ((mask >> b) & 1) continue;
    r |= ((j >> o++) & 1) << b;
  }
  return r;
}

template <int V>
__device__ __forceinline__ void nb_row_reduce_scatter(const float (&x)[V], int c, float (&out)[V / 16]) {
  static_assert(V % 16 == 0 && V <= 64, "values per lane: a multiple of 16");
  float a[V];
#pragma unroll
  for (int i = 0; i < V; ++i) a[i] = x[i];
  constexpr int order[4] = {3, 0, 1, 2};
  int mask = 0;   // bits split so far
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    const int bt = order[st];
    const bool hi = (c >> bt) & 1;
    const int nmask = mask | (1 << bt);
    float nx[V / 2];
#pragma unroll
    for (int j = 0; j < (V >> (st + 1)); ++j) {
      const int i0 = nb_rs_expand(j, nmask), i1 = i0 | (1 << bt);
      const float v0 = a[nb_rs_compress(i0, mask)], v1 = a[nb_rs_compress(i1, mask)];
      const float keep = hi ? v1 : v0, send = hi ? v0 : v1;
      float got;
      if (bt == 3)
        got = __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, send), 0x128, 0xF, 0xF, false));
      else if (bt == 0)
        got = __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, send), 0xB1, 0xF, 0xF, false));
      else if (bt == 1)
        got = __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, send), 0x4E, 0xF, 0xF, false));
      else   // lane c ^ 4 (swizzle, bit mode: and 0x1f, xor 4)
        got = __builtin_bit_cast(float, __builtin_amdgcn_ds_swizzle(__builtin_bit_cast(int, send), 0x101F));
      nx[j] = keep + got;
    }
#pragma unroll
    for (int j = 0; j < (V >> (st + 1)); ++j) a[j] = nx[j];
    mask = nmask;
  }
#pragma unroll
  for (int k = 0; k < V / 16; ++k) out[k] = a[k];
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

// First layer at float32 accuracy on the bfloat16 matrix cores.  A float32
// value v is cut exactly into three bfloat16 pieces by truncation:
// v1 = v with its low 16 bits cleared, v2 = (v - v1) likewise, and
// v3 = v - v1 - v2 (at most 8 significant bits: a bfloat16 itself).  W x is
// the sum of the six piece products whose size can exceed about 2^-16 |w||x|,
//   product p:   0        1        2        3        4        5
//   (w, x):      (w1,x1)  (w1,x2)  (w2,x1)  (w1,x3)  (w3,x1)  (w2,x2)
// (the three left out sum to less than 2^-20 |w||x|), laid out along K of
// v_mfma_f32_16x16x32_bf16, lane group g holding k = 8g .. 8g + 7:
//   in_dim <= 4: one step; group g holds product 2g for features 0..3
//                (k = 8g .. 8g+3) and product 2g + 1 for features 0..3
//                (k = 8g+4 .. 8g+7); group 3 is zero;
//   in_dim 5..8: two steps; in step s group g holds product 4s + g for
//                features 0..7 (step 1, groups 2 and 3 zero).
__host__ __device__ inline float nb_trunc_bf16(float v) {
  uint32_t u;
  __builtin_memcpy(&u, &v, 4);
  u &= 0xFFFF0000u;
  float r;
  __builtin_memcpy(&r, &u, 4);
  return r;
}
// Piece k (1, 2 or 3) of v.
__host__ __device__ inline float nb_piece(float v, int k) {
  const float v1 = nb_trunc_bf16(v);
  if (k == 1) return v1;
  const float r = v - v1;
  const float v2 = nb_trunc_bf16(r);
  return k == 2 ? v2 : r - v2;
}
// Weight and input piece of product p.
__host__ __device__ inline int nb_first_wpiece(int p) { return p == 2 || p == 5 ? 2 : (p == 4 ? 3 : 1); }
__host__ __device__ inline int nb_first_xpiece(int p) { return p == 1 || p == 5 ? 2 : (p == 3 ? 3 : 1); }
// Bits of a float32 that is a bfloat16 (its low 16 bits are zero).
__host__ __device__ inline uint16_t nb_hi16(float v) {
  uint32_t u;
  __builtin_memcpy(&u, &v, 4);
  return (uint16_t)(u >> 16);
}

// Element e (bfloat16 bits) of a bound's forward fragment pack, from its
// float32 parameters th: e = (f*64 + lane)*8 + j with c = lane % 16,
// g = lane / 16.  With NFWD = RB + (NH-1)*FH:
//   f < RB            first layer, step 0, row block mo = f (layout above);
//   RB <= f < NFWD    hidden layer l (1-based), fragment (mo, ks),
//                       f = RB + (l-1)*FH + mo*KS + ks:
//                       W_l[16mo + c][32ks + 16(j/4) + 4g + (j%4)];
//   NFWD <= f         first layer, step 1, row block mo = f - NFWD (zero
//                     when in_dim <= 4).
__host__ __device__ inline uint16_t nb_bf16_pack_elem(const float* th, int in_dim, int W, int NH, int64_t e) {
  const int j = (int)(e & 7), lane = (int)((e >> 3) & 63);
  const int f = (int)(e >> 9);
  const int c = lane & 15, g = lane >> 4;
  const int RB = W / 16, KS = W / 32, FH = RB * KS, NFWD = RB + (NH - 1) * FH;
  if (f < RB || f >= NFWD) {
    const int step = f < RB ? 0 : 1, mo = f < RB ? f : f - NFWD;
    const int p = in_dim <= 4 ? (step ? 6 : 2 * g + j / 4) : 4 * step + g;
    const int k = in_dim <= 4 ? j % 4 : j;
    if (p >= 6 || k >= in_dim) return 0;
    return nb_hi16(nb_piece(th[(int64_t)(16 * mo + c) * in_dim + k], nb_first_wpiece(p)));
  }
  const int t = f - RB;
  const int l = 1 + t / FH, rem = t % FH, mo = rem / KS, ks = rem % KS;
  const float* Wl = th + nb_w_off(l, in_dim, W);
  return nb_bf16_bits(Wl[(int64_t)(16 * mo + c) * W + 32 * ks + 16 * (j / 4) + 4 * g + (j % 4)]);
}

// Two float32 values that are bfloat16 numbers, packed (a in the low half).
__device__ __forceinline__ unsigned nb_pack_hi16(float a, float b) {
  return (__float_as_uint(a) >> 16) | (__float_as_uint(b) & 0xFFFF0000u);
}

// B operands of the first layer's one (wide = false: in_dim <= 4) or two
// (wide: in_dim 5..8) K = 32 steps, from the raw inputs of the lane's query
// column: the lane's group picks the input piece of its product (layout in
// nb_mlp.h).  Pieces by truncation: x1 = x with its low 16 bits cleared,
// x2 = (x - x1) likewise, x3 = x - x1 - x2; all three sums are exact.
template <int NB>
__device__ __forceinline__ void nb_first_operands(const float (&xr)[NB][8], int grp, bool wide, nb_bf16x8 (&x0)[NB],
                                               nb_bf16x8 (&x1)[NB]) {
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    float p1[8], p2[8], p3[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      p1[j] = __uint_as_float(__float_as_uint(xr[nb][j]) & 0xFFFF0000u);
      const float r = xr[nb][j] - p1[j];
      p2[j] = __uint_as_float(__float_as_uint(r) & 0xFFFF0000u);
      p3[j] = r - p2[j];
    }
    nb_uint4 u0, u1;
    if (!wide) {
      // features 0..3: group g holds products 2g and 2g + 1
      //   g = 0: (x1 | x2)   g = 1: (x1 | x3)   g = 2: (x1 | x2)   g = 3: 0
      float lo[4], hi[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        lo[j] = grp == 3 ? 0.0f : p1[j];
        hi[j] = grp == 3 ? 0.0f : (grp == 1 ? p3[j] : p2[j]);
      }
      u0 = nb_uint4{nb_pack_hi16(lo[0], lo[1]), nb_pack_hi16(lo[2], lo[3]), nb_pack_hi16(hi[0], hi[1]),
                    nb_pack_hi16(hi[2], hi[3])};
      u1 = nb_uint4{0u, 0u, 0u, 0u};
    } else {
      // step 0: group g holds product g (x1, x2, x1, x3); step 1: product
      // 4 + g (x1, x2, 0, 0)
      float a[8], b[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        a[j] = grp == 1 ? p2[j] : (grp == 3 ? p3[j] : p1[j]);
        b[j] = grp == 0 ? p1[j] : (grp == 1 ? p2[j] : 0.0f);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        u0[i] = nb_pack_hi16(a[2 * i], a[2 * i + 1]);
        u1[i] = nb_pack_hi16(b[2 * i], b[2 * i + 1]);
      }
    }
    x0[nb] = __builtin_bit_cast(nb_bf16x8, u0);
    x1[nb] = __builtin_bit_cast(nb_bf16x8, u1);
  }
}

// Neuron at position p of a K = 32 operand in "operand order": within each
// 32-neuron block, position 8g + j holds neuron 4g + j for j < 4 and
// 16 + 4g + (j - 4) for j >= 4 -- the order in which a lane of group g holds
// the values of row blocks 2ks and 2ks + 1 after a layer's products.
__host__ __device__ inline int nb_op_neuron(int p) {
  return (p & ~31) + 16 * ((p >> 2) & 1) + 4 * ((p >> 3) & 3) + (p & 3);
}

// Element e of the transposed (backward) pack of the hidden layers:
// packT[((l-1)*FH + mo*KS + ks)*64 + lane][j] = W_l[k(32ks + 8g + j)][16mo + c]
// (the A operand of W_l^T D, the reduction running over W_l's outputs), with
// k(p) = p when D is read in neuron order (the layer-wise kernels) and
// k(p) = nb_op_neuron(p) when D comes straight from a layer's accumulators
// (the fused training kernel).
__host__ __device__ inline uint16_t nb_bf16_pack_t_elem(const float* th, int in_dim, int W, int NH, int64_t e,
                                                        bool op) {
  (void)NH;
  const int j = (int)(e & 7), lane = (int)((e >> 3) & 63), f = (int)(e >> 9);
  const int c = lane & 15, g = lane >> 4;
  const int RB = W / 16, KS = W / 32, FH = RB * KS;
  const int l = 1 + f / FH, rem = f % FH, mo = rem / KS, ks = rem % KS;
  const float* Wl = th + nb_w_off(l, in_dim, W);
  const int p = 32 * ks + 8 * g + j;
  return nb_bf16_bits(Wl[(int64_t)(op ? nb_op_neuron(p) : p) * W + 16 * mo + c]);
}

// Shapes the fused bfloat16 training step covers (their transposed packs are
// in operand order).
__host__ __device__ inline bool nb_bf16_fused_shape(int in_dim, int n_hidden, int width) {
  return in_dim >= 1 && in_dim <= 8 && n_hidden >= 2 && n_hidden <= 4 && (width == 32 || width == 64 || width == 128);
}

// Number of 16-byte fragment slices of the forward pack (both first-layer
// steps and the hidden layers) / of the transposed pack.
__host__ __device__ inline int64_t nb_bf16_fwd_slices(int W, int NH) {
  return (int64_t)(2 * (W / 16) + (NH - 1) * (W / 16) * (W / 32)) * 64;
}
__host__ __device__ inline int64_t nb_bf16_t_slices(int W, int NH) {
  return (int64_t)(NH - 1) * (W / 16) * (W / 32) * 64;
}

// Number of compute units of the current device (cached per device).
int nb_cu_count();
