// Training of a bfloat16 bound (Alg. 1 steps 4-5, gradient of Eq. 1),
// layer by layer on the matrix cores (v_mfma_f32_16x16x32_bf16, float32
// accumulation), with the same rounding points as the bfloat16 forward: a
// float32-accurate first layer (three bfloat16 pieces per value, nb_mlp.h),
// bfloat16 hidden layers, a float32 output layer.
//
// One kernel per layer keeps a single layer's weights in LDS (at most
// 128 KiB for width 256); activations A_l (post-ReLU, bfloat16) and
// back-propagated gradients D_l (bfloat16) live in HBM as row-major
// [queries][width] arrays.
//
//   first   x -> A_0
//   hidden  A_{l-1} -> A_l                         (l = 1 .. H-2)
//   head    A_{H-2} -> layer H-1 -> z (float32 output layer), Eq. 1 loss,
//           dz = dL/dz, D_{H-1} = dz w_out [a > 0], dw_out, db_out
//   data    D_{l-1} = (W_l^T D_l) [A_{l-1} > 0]     (transposed weight fragments)
//   weight  dW_l = sum_q D_l[q] A_{l-1}[q]^T, db_l = sum_q D_l[q]
//           (both operands transposed through LDS; K = queries)
//   first'  dW_0 = sum_q D_0[q] x[q]^T, db_0 = sum_q D_0[q]   (float32 inputs)
//
// The batch is cut into fixed chunks, one per workgroup; every kernel that
// produces gradient terms writes one partial per chunk, summed afterwards in
// a fixed order, so a step is bit-reproducible.
#include <algorithm>

#include "nb_bf16_train.h"
#include "nb_internal.h"

namespace {

// ---------------------------------------------------------- transposed pack
//
// packT[((l-1)*FH + mo*KS + ks)*64 + lane][j] = W_l[k(32ks + 8g + j)][16mo + c]:
// the A operand of (W_l^T D), the reduction over W_l's output neurons in
// natural order for the layer-wise kernels, in operand order for the fused
// step (nb_bf16_pack_t_elem).
__global__ void k_pack_bf16_t(const float* __restrict__ theta, int in_dim, int W, int NH, uint16_t* __restrict__ pack,
                              int64_t total, bool op) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  pack[idx] = nb_bf16_pack_t_elem(theta, in_dim, W, NH, idx, op);
}

// ------------------------------------------------------------ first layer

template <int W>
__global__ __launch_bounds__(256) void k_tr_first(const float* __restrict__ q, int64_t n, int in_dim, int64_t Bp,
                                                  const bf16x8* __restrict__ pack, const float* __restrict__ theta,
                                                  int NH, uint16_t* __restrict__ A0, TrObjs T) {
  constexpr int RB = W / 16;
  const TrObj ob = tr_obj(T);
  q += ob.o * T.q_stride * in_dim;
  pack += T.pkoff ? T.pkoff[ob.o] : 0;
  theta += ob.poff;
  A0 += ob.member * T.ms_a;
  const bool wide = in_dim > 4;
  // the first layer's two steps: fragments 0 .. RB-1 and, after the hidden
  // layers', the second step's RB fragments
  __shared__ bf16x8 sw[2 * RB * 64];
  __shared__ float sb[W];
  const bf16x8* ext = pack + (int64_t)(RB + (NH - 1) * RB * (W / 32)) * 64;
  for (int i = threadIdx.x; i < RB * 64; i += blockDim.x) {
    sw[i] = pack[i];
    if (wide) sw[RB * 64 + i] = ext[i];
  }
  for (int i = threadIdx.x; i < W; i += blockDim.x) sb[i] = theta[(int64_t)W * in_dim + i];
  __syncthreads();
  const int lane = threadIdx.x & 63, c = lane & 15, grp = lane >> 4;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t blk = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); blk < Bp / 16; blk += waves) {
    const int64_t qi = blk * 16 + c;
    const bool valid = qi < n;
    float xr[1][8];
#pragma unroll
    for (int j = 0; j < 8; ++j) xr[0][j] = (valid && j < in_dim) ? q[qi * in_dim + j] : 0.0f;
    bf16x8 xb[1], xb1[1];
    nb_first_operands<1>(xr, grp, wide, xb, xb1);
    uint16_t* out = A0 + qi * W;
#pragma unroll
    for (int ks = 0; ks < RB / 2; ++ks) {
      floatx4 acc[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int mo = 2 * ks + h;
        const float* b = sb + 16 * mo + 4 * grp;
        acc[h] = nb_mfma_bf16(sw[mo * 64 + lane], xb[0], floatx4{b[0], b[1], b[2], b[3]});
        if (wide) acc[h] = nb_mfma_bf16(sw[(RB + mo) * 64 + lane], xb1[0], acc[h]);
      }
      *reinterpret_cast<uint4*>(out + 32 * ks + 8 * grp) = relu_pair(acc[0], acc[1]);
    }
  }
}

// ------------------------------------------------- hidden layers and head

template <int W>
struct TrHidden {
  static constexpr int RB = W / 16, KS = W / 32, FH = RB * KS;
  static constexpr size_t lds_bytes() { return (size_t)FH * 64 * 16 + (size_t)(2 * W + 1) * 4; }
};

// Threads per workgroup of the hidden-layer and data-gradient kernels.  A
// width-256 layer's fragments fill 128 KB of LDS, one workgroup per CU of 8
// waves (two per SIMD: one wave's loads overlap the other's products).  The
// head runs one workgroup per chunk of the batch (one partial each) with 8
// waves up to width 128; at width 256 its per-lane accumulators (the layer's
// 64 outputs and 64 output-weight gradients per lane, plus the next block's
// operands in flight) need more than the 256 registers of two waves per
// SIMD, so it runs one wave per SIMD with up to 512.
template <int W, bool HEAD>
constexpr int tr_threads() { return HEAD ? (W >= 256 ? 256 : 512) : (W >= 256 ? 512 : 256); }
// Blocks of 16 queries a wave multiplies per weight fragment it reads from
// LDS in the layer kernels (k_tr_layer, k_tr_data): every fragment read
// feeds this many matrix-core instructions, so that the LDS bandwidth (128
// bytes per clock per CU) stays below what four busy SIMDs draw.  A divisor
// of 4 (the padded batch is a multiple of 64 queries).
template <int W>
constexpr int kTrNB() { return W >= 256 ? 4 : 2; }
// Row blocks unrolled per step of the output-neuron loop: all of them up to
// width 64; two from width 128 on, where full unrolling hoists more fragment
// loads than the registers of several waves per SIMD hold.
template <int W>
constexpr int kMoUnroll() { return W >= 128 ? 2 : W / 16; }

// A_l = relu(W_l A_{l-1} + b_l) over the padded batch: each wave takes NB
// blocks of 16 queries at a time, so one LDS fragment read feeds NB products.
template <int W>
__global__ __launch_bounds__((tr_threads<W, false>())) void k_tr_layer(const uint16_t* __restrict__ Ain, int64_t Bp,
                                                                      int l, int in_dim, int NH,
                                                                      const bf16x8* __restrict__ pack,
                                                                      const float* __restrict__ theta,
                                                                      uint16_t* __restrict__ Aout, TrObjs TO) {
  using T = TrHidden<W>;
  constexpr int RB = T::RB, KS = T::KS, NB = kTrNB<W>();
  const TrObj ob = tr_obj(TO);
  pack += TO.pkoff ? TO.pkoff[ob.o] : 0;
  theta += ob.poff;
  Ain += ob.member * TO.ms_a;
  Aout += ob.member * TO.ms_a;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  bf16x8* sw = reinterpret_cast<bf16x8*>(smem_raw);
  float* sb = reinterpret_cast<float*>(smem_raw + (size_t)T::FH * 64 * 16);
  const bf16x8* src = pack + (RB + (l - 1) * T::FH) * 64;
  for (int i = threadIdx.x; i < T::FH * 64; i += blockDim.x) sw[i] = src[i];
  for (int i = threadIdx.x; i < W; i += blockDim.x) sb[i] = theta[nb_b_off(l, in_dim, W, NH) + i];
  __syncthreads();
  const int lane = threadIdx.x & 63, c = lane & 15, grp = lane >> 4;
  const int64_t groups = Bp / (16 * NB);   // Bp is a multiple of 64 and NB divides 4
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t gi = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); gi < groups; gi += waves) {
    bf16x8 bop[NB][KS];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const uint16_t* row = Ain + ((gi * NB + nb) * 16 + c) * W;
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) bop[nb][ks] = load_fwd_operand(row, ks, grp);
    }
    // row blocks in pairs: a pair's activations are one 16-byte store per query
#pragma unroll(kMoUnroll<W>() / 2)
    for (int kp = 0; kp < RB / 2; ++kp) {
      floatx4 acc[2][NB];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int mo = 2 * kp + h;
        const floatx4 bi = *reinterpret_cast<const floatx4*>(sb + 16 * mo + 4 * grp);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[h][nb] = bi;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          const bf16x8 f = sw[(mo * KS + ks) * 64 + lane];
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) acc[h][nb] = nb_mfma_bf16(f, bop[nb][ks], acc[h][nb]);
        }
      }
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        *reinterpret_cast<uint4*>(Aout + ((gi * NB + nb) * 16 + c) * W + 32 * kp + 8 * grp) =
            relu_pair(acc[0][nb], acc[1][nb]);
    }
  }
}

// The last hidden layer and the head: layer NH-1, the output logit, Eq. 1
// and its gradient, D_{NH-1}; one workgroup per chunk of the batch writes
// the chunk's output-layer partials.
template <int W>
__global__ __launch_bounds__((tr_threads<W, true>())) void k_tr_head(const uint16_t* __restrict__ Ain, int64_t n,
                                                                    int64_t CH, int l, int in_dim, int NH,
                                                                    const bf16x8* __restrict__ pack,
                                                                    const float* __restrict__ theta,
                                                                    uint16_t* __restrict__ Dout,
                                                                    const uint8_t* __restrict__ y, float alpha,
                                                                    float beta, float inv_n, float tau,
                                                                    float* __restrict__ partial,
                                                                    float* __restrict__ aux, TrObjs TO) {
  using T = TrHidden<W>;
  constexpr int RB = T::RB, KS = T::KS;
  const TrObj ob = tr_obj(TO);
  const int64_t P = ob.P;
  pack += TO.pkoff ? TO.pkoff[ob.o] : 0;
  theta += ob.poff;
  Ain += ob.member * TO.ms_a;
  Dout += ob.member * TO.ms_d;
  if (TO.alpha) alpha = TO.alpha[ob.o];
  y += ob.o * TO.q_stride;
  partial += (int64_t)gridDim.x * ob.poff;
  aux += (int64_t)ob.o * gridDim.x * 8;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  bf16x8* sw = reinterpret_cast<bf16x8*>(smem_raw);
  float* sb = reinterpret_cast<float*>(smem_raw + (size_t)T::FH * 64 * 16);   // [W] bias, [W] w_out, b_out
  const bf16x8* src = pack + (RB + (l - 1) * T::FH) * 64;
  for (int i = threadIdx.x; i < T::FH * 64; i += blockDim.x) sw[i] = src[i];
  for (int i = threadIdx.x; i < W; i += blockDim.x) sb[i] = theta[nb_b_off(l, in_dim, W, NH) + i];
  for (int i = threadIdx.x; i < W + 1; i += blockDim.x) sb[W + i] = theta[nb_w_off(NH, in_dim, W) + i];
  __syncthreads();

  const int lane = threadIdx.x & 63, c = lane & 15, grp = lane >> 4, wave = threadIdx.x >> 6;
  const int64_t base = (int64_t)blockIdx.x * CH;
  const int64_t nblk = CH / 16;
  float gwo[RB * 4];
#pragma unroll
  for (int i = 0; i < RB * 4; ++i) gwo[i] = 0.0f;
  float gbo = 0.0f, lsum = 0.0f;
  unsigned cnt[4] = {0u, 0u, 0u, 0u};

  // the next block's operands load while this block computes
  bf16x8 nxt[KS];
  if (wave < nblk) {
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) nxt[ks] = load_fwd_operand(Ain + (base + wave * 16 + c) * W, ks, grp);
  }
  for (int64_t blk = wave; blk < nblk; blk += (blockDim.x >> 6)) {
    const int64_t qi = base + blk * 16 + c;
    bf16x8 bop[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) bop[ks] = nxt[ks];
    if (blk + (blockDim.x >> 6) < nblk) {
      const uint16_t* row = Ain + (qi + 16 * (int64_t)(blockDim.x >> 6)) * W;
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) nxt[ks] = load_fwd_operand(row, ks, grp);
    }
    {
      // every row block stays in registers (unrolled in full); a scheduling
      // barrier after each row block keeps its fragment loads from being
      // hoisted above the earlier blocks' products (which would need a
      // register per loaded fragment)
      floatx4 acc[RB];
#pragma unroll
      for (int mo = 0; mo < RB; ++mo) {
        const float* b = sb + 16 * mo + 4 * grp;
        acc[mo] = floatx4{b[0], b[1], b[2], b[3]};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) acc[mo] = nb_mfma_bf16(sw[(mo * KS + ks) * 64 + lane], bop[ks], acc[mo]);
        __builtin_amdgcn_sched_barrier(0);
      }
      const float* wo = sb + W;
      float p = 0.0f;
#pragma unroll
      for (int mo = 0; mo < RB; ++mo)
#pragma unroll
        for (int r = 0; r < 4; ++r) p = fmaf(wo[16 * mo + 4 * grp + r], fmaxf(acc[mo][r], 0.0f), p);
      p += __shfl_xor(p, 16);
      p += __shfl_xor(p, 32);
      const float z = p + wo[W];
      const bool valid = qi < n;
      const bool yv = valid && y[qi] != 0;
      const float e = expf(-fabsf(z));
      const float inv1pe = 1.0f / (1.0f + e);
      const float sig = z >= 0.0f ? inv1pe : e * inv1pe;
      const float sigm = z >= 0.0f ? e * inv1pe : inv1pe;
      const float dz = valid ? inv_n * (yv ? -alpha * sigm : beta * sig) : 0.0f;
      const bool own = grp == 0 && valid;
      if (own) {
        const float sp = log1pf(e);
        lsum += yv ? alpha * (fmaxf(-z, 0.0f) + sp) : beta * (fmaxf(z, 0.0f) + sp);
        gbo += dz;
      }
      const bool pos = !(z < tau);
      cnt[0] += __popcll(__ballot(own && pos && yv));
      cnt[1] += __popcll(__ballot(own && pos && !yv));
      cnt[2] += __popcll(__ballot(own && !pos && !yv));
      cnt[3] += __popcll(__ballot(own && !pos && yv));
      uint16_t* out = Dout + qi * W;   // D_{H-1}
#pragma unroll
      for (int mo = 0; mo < RB; ++mo) {
        float d[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float a = fmaxf(acc[mo][r], 0.0f);
          gwo[mo * 4 + r] = fmaf(dz, a, gwo[mo * 4 + r]);
          d[r] = acc[mo][r] > 0.0f ? dz * wo[16 * mo + 4 * grp + r] : 0.0f;
        }
        *reinterpret_cast<uint2*>(out + 16 * mo + 4 * grp) = pack4(d[0], d[1], d[2], d[3]);
      }
    }
  }
  {
    // fixed-order workgroup reduction of the output-layer terms
    __syncthreads();
    float* red = reinterpret_cast<float*>(smem_raw);   // reuse the weight area: [W + 1] + [4][8]
    float* saux = red + W + 8;
#pragma unroll
    for (int i = 0; i < RB * 4; ++i)
#pragma unroll
      for (int m = 1; m < 16; m <<= 1) gwo[i] += __shfl_xor(gwo[i], m);
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
      gbo += __shfl_xor(gbo, m);
      lsum += __shfl_xor(lsum, m);
    }
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      if (wave == w) {
        if (c == 0) {
#pragma unroll
          for (int mo = 0; mo < RB; ++mo)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int i = 16 * mo + 4 * grp + r;
              red[i] = w == 0 ? gwo[mo * 4 + r] : red[i] + gwo[mo * 4 + r];
            }
        }
        if (lane == 0) {
          red[W] = w == 0 ? gbo : red[W] + gbo;
          saux[w * 8] = lsum;
          for (int i = 0; i < 4; ++i) saux[w * 8 + 1 + i] = __uint_as_float(cnt[i]);
        }
      }
      __syncthreads();
    }
    float* out = partial + (int64_t)blockIdx.x * P;
    for (int i = threadIdx.x; i < W + 1; i += blockDim.x) out[nb_w_off(NH, in_dim, W) + i] = red[i];
    if (threadIdx.x == 0) {
      float ls = 0.0f;
      unsigned cs[4] = {0u, 0u, 0u, 0u};
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
        ls += saux[w * 8];
        for (int i = 0; i < 4; ++i) cs[i] += __float_as_uint(saux[w * 8 + 1 + i]);
      }
      aux[blockIdx.x * 8] = ls;
      for (int i = 0; i < 4; ++i) aux[blockIdx.x * 8 + 1 + i] = __uint_as_float(cs[i]);
    }
  }
}

// ------------------------------------------------------- data gradient

// D_{l-1} = (W_l^T D_l) * [A_{l-1} > 0], NB blocks of 16 queries per wave
// at a time (one LDS fragment read feeds NB products).
template <int W>
__global__ __launch_bounds__((tr_threads<W, false>())) void k_tr_data(const uint16_t* __restrict__ Dl, const uint16_t* __restrict__ Aprev,
                                                 int64_t Bp, int l, const bf16x8* __restrict__ packT,
                                                 uint16_t* __restrict__ Dprev, TrObjs TO) {
  using T = TrHidden<W>;
  const TrObj ob = tr_obj(TO);
  packT += TO.ptoff ? TO.ptoff[ob.o] : 0;
  Dl += ob.member * TO.ms_d;
  Dprev += ob.member * TO.ms_d;
  Aprev += ob.member * TO.ms_a;
  constexpr int RB = T::RB, KS = T::KS, NB = kTrNB<W>();
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  bf16x8* sw = reinterpret_cast<bf16x8*>(smem_raw);
  const bf16x8* src = packT + (l - 1) * T::FH * 64;
  for (int i = threadIdx.x; i < T::FH * 64; i += blockDim.x) sw[i] = src[i];
  __syncthreads();
  const int lane = threadIdx.x & 63, c = lane & 15, grp = lane >> 4;
  const int64_t groups = Bp / (16 * NB);
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t gi = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); gi < groups; gi += waves) {
    bf16x8 bop[NB][KS];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int64_t qi = (gi * NB + nb) * 16 + c;
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) bop[nb][ks] = *reinterpret_cast<const bf16x8*>(Dl + qi * W + 32 * ks + 8 * grp);
    }
    // row blocks in pairs: a pair's ReLU mask is one 16-byte load of A_{l-1}
    // (operand order), loaded ahead of the pair's products
#pragma unroll(kMoUnroll<W>() / 2)
    for (int kp = 0; kp < RB / 2; ++kp) {
      uint4 am[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        am[nb] = *reinterpret_cast<const uint4*>(Aprev + ((gi * NB + nb) * 16 + c) * W + 32 * kp + 8 * grp);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int mo = 2 * kp + h;
        floatx4 acc[NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          const bf16x8 f = sw[(mo * KS + ks) * 64 + lane];
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) acc[nb] = nb_mfma_bf16(f, bop[nb][ks], acc[nb]);
        }
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          float a[4];
          unpack4(h ? uint2{am[nb].z, am[nb].w} : uint2{am[nb].x, am[nb].y}, a);
          *reinterpret_cast<uint2*>(Dprev + ((gi * NB + nb) * 16 + c) * W + 16 * mo + 4 * grp) =
              pack4(a[0] > 0.0f ? acc[nb][0] : 0.0f, a[1] > 0.0f ? acc[nb][1] : 0.0f,
                    a[2] > 0.0f ? acc[nb][2] : 0.0f, a[3] > 0.0f ? acc[nb][3] : 0.0f);
        }
      }
    }
  }
}

// ----------------------------------------------------- weight gradient

constexpr int kTS = 40;   // LDS row stride of a [width][32 queries] bfloat16 tile (+ 8 pad)

// Staging: thread t owns the neuron pair (2p, 2p + 1), p = t % (W/2), and
// QPT consecutive queries of the 32-query slab, group j = t / (W/2); per
// query it loads 4 bytes (a wave reads whole 256-byte rows, coalesced) and
// writes QPT consecutive bf16 per neuron into the [neuron][query] tiles.
template <int W, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_tr_weight(const uint16_t* __restrict__ Dl,
                                                          const uint16_t* __restrict__ Aprev, int64_t CH, int l,
                                                          int in_dim, int NH, float* __restrict__ partial, TrObjs TO) {
  constexpr int RB = W / 16, TILES = RB * RB, TPW = TILES / WAVES;
  const TrObj ob = tr_obj(TO);
  const int64_t P = ob.P;
  Dl += ob.member * TO.ms_d;
  Aprev += ob.member * TO.ms_a;
  partial += (int64_t)gridDim.x * ob.poff;
  static_assert(TILES % WAVES == 0, "tiles must split evenly over the waves");
  constexpr int THREADS = WAVES * 64;
  constexpr int PAIRS = W / 2;
  constexpr int GROUPS = THREADS / PAIRS;      // query groups per slab
  constexpr int QPT = 32 / GROUPS;             // queries per thread per slab
  static_assert(THREADS % PAIRS == 0 && 32 % GROUPS == 0 && QPT % 2 == 0, "staging shape");
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  uint16_t (*sD)[W * kTS] = reinterpret_cast<uint16_t (*)[W * kTS]>(smem_raw);
  uint16_t (*sA)[W * kTS] = reinterpret_cast<uint16_t (*)[W * kTS]>(smem_raw + 2 * W * kTS * 2);
  float (*sdb)[W] = reinterpret_cast<float (*)[W]>(smem_raw + 4 * W * kTS * 2);
  const int lane = threadIdx.x & 63, c = lane & 15, grp = lane >> 4, wave = threadIdx.x >> 6;
  const int pr = threadIdx.x % PAIRS, gq = threadIdx.x / PAIRS;
  const int64_t base = (int64_t)blockIdx.x * CH;
  floatx4 acc[TPW];
#pragma unroll
  for (int i = 0; i < TPW; ++i) acc[i] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
  float db0 = 0.0f, db1 = 0.0f;
  uint32_t pd[QPT], pa[QPT];
  auto fetch = [&](int64_t k0) {
#pragma unroll
    for (int i = 0; i < QPT; ++i) {
      const int64_t qi = base + k0 + gq * QPT + i;
      pd[i] = *reinterpret_cast<const uint32_t*>(Dl + qi * W + 2 * pr);
      pa[i] = *reinterpret_cast<const uint32_t*>(Aprev + qi * W + 2 * pr);
    }
  };
  auto stash = [&](int bufi) {
    uint16_t d0[QPT], d1[QPT], a0[QPT], a1[QPT];
#pragma unroll
    for (int i = 0; i < QPT; ++i) {
      d0[i] = (uint16_t)(pd[i] & 0xFFFF);
      d1[i] = (uint16_t)(pd[i] >> 16);
      a0[i] = (uint16_t)(pa[i] & 0xFFFF);
      a1[i] = (uint16_t)(pa[i] >> 16);
      db0 += (float)bf16_of(d0[i]);
      db1 += (float)bf16_of(d1[i]);
    }
    uint16_t* rd0 = sD[bufi] + (2 * pr) * kTS + gq * QPT;
    uint16_t* ra0 = sA[bufi] + act_neuron(2 * pr) * kTS + gq * QPT;   // positions 2pr, 2pr+1: two consecutive neurons
#pragma unroll
    for (int i = 0; i < QPT; i += 2) {
      *reinterpret_cast<uint32_t*>(rd0 + i) = (uint32_t)d0[i] | ((uint32_t)d0[i + 1] << 16);
      *reinterpret_cast<uint32_t*>(rd0 + kTS + i) = (uint32_t)d1[i] | ((uint32_t)d1[i + 1] << 16);
      *reinterpret_cast<uint32_t*>(ra0 + i) = (uint32_t)a0[i] | ((uint32_t)a0[i + 1] << 16);
      *reinterpret_cast<uint32_t*>(ra0 + kTS + i) = (uint32_t)a1[i] | ((uint32_t)a1[i + 1] << 16);
    }
  };
  fetch(0);
  stash(0);
  __syncthreads();
  int buf = 0;
  for (int64_t k0 = 0; k0 < CH; k0 += 32) {
    const bool more = k0 + 32 < CH;
    if (more) fetch(k0 + 32);              // next slab in flight during this step's products
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int T = wave * TPW + t, no = T / RB, ko = T % RB;
      const bf16x8 a = *reinterpret_cast<const bf16x8*>(sD[buf] + (16 * no + c) * kTS + 8 * grp);
      const bf16x8 b = *reinterpret_cast<const bf16x8*>(sA[buf] + (16 * ko + c) * kTS + 8 * grp);
      acc[t] = nb_mfma_bf16(a, b, acc[t]);
    }
    if (more) stash(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  sdb[gq][2 * pr] = db0;
  sdb[gq][2 * pr + 1] = db1;
  float* out = partial + (int64_t)blockIdx.x * P;
  const int64_t wo = nb_w_off(l, in_dim, W);
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int T = wave * TPW + t, no = T / RB, ko = T % RB;
#pragma unroll
    for (int r = 0; r < 4; ++r) out[wo + (int64_t)(16 * no + 4 * grp + r) * W + 16 * ko + c] = acc[t][r];
  }
  __syncthreads();
  if (threadIdx.x < W) {
    float db = sdb[0][threadIdx.x];
    for (int j = 1; j < GROUPS; ++j) db += sdb[j][threadIdx.x];
    out[nb_b_off(l, in_dim, W, NH) + threadIdx.x] = db;
  }
}

// dW_0 = sum_q D_0[q] x[q]^T, db_0 = sum_q D_0[q].  1024 threads: thread t
// takes neuron t % W and every S-th query of each 256-query slab (S = 1024 / W,
// subset t / W); the slab's inputs sit in LDS; the S subset sums are added in
// subset order at the end.
constexpr int kFG = 512;

// dW_0 = sum_i delta_0 x^T and db_0 = sum_i delta_0 over a chunk of the batch,
// one partial per workgroup.  A lane takes 8 neurons of a sample (one 16-byte
// load of delta_0); the lanes of a wave holding the same neurons are summed by
// a fixed butterfly, then the waves in order through LDS (deterministic).
template <int W>
__global__ __launch_bounds__(kFG) void k_tr_first_grad(const uint16_t* __restrict__ D0, const float* __restrict__ q,
                                                       int64_t n, int64_t CH, int in_dim, int NH,
                                                       float* __restrict__ partial, TrObjs TO) {
  constexpr int G = W / 8;        // lanes per sample
  constexpr int S = kFG / G;      // samples per workgroup pass
  static_assert(64 % G == 0, "a wave holds whole samples");
  const TrObj ob = tr_obj(TO);
  const int64_t P = ob.P;
  D0 += ob.member * TO.ms_d;
  q += ob.o * TO.q_stride * in_dim;
  partial += (int64_t)gridDim.x * ob.poff;
  __shared__ float red[G * 72];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane % G, sub = threadIdx.x / G;
  const int64_t base = (int64_t)blockIdx.x * CH;
  const int64_t end = base + CH < n ? base + CH : n;
  float acc[8][9];   // neuron 8 g + e: dW_0 row (8 inputs), then db_0
#pragma unroll
  for (int e = 0; e < 8; ++e)
#pragma unroll
    for (int k = 0; k < 9; ++k) acc[e][k] = 0.0f;
  // U samples' loads in flight per lane before their products (the lanes of
  // a sample read the same input row: one transaction); a sample past the
  // chunk loads row `base` and adds zeros, so there are no branches and each
  // lane's sums keep the order i = base + sub, + S, ...
  constexpr int U = 8;
  for (int64_t i0 = base + sub; i0 < end; i0 += U * S) {
    uint4 v[U];
    float xs[U][8];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + (int64_t)u * S;
      const int64_t ic = i < end ? i : base;
      v[u] = *reinterpret_cast<const uint4*>(D0 + ic * W + 8 * g);
#pragma unroll
      for (int k = 0; k < 8; ++k) xs[u][k] = k < in_dim ? q[ic * in_dim + k] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool valid = i0 + (int64_t)u * S < end;
      float d[8];
      unpack4(uint2{v[u].x, v[u].y}, d);
      unpack4(uint2{v[u].z, v[u].w}, d + 4);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float de = valid ? d[e] : 0.0f;
        acc[e][8] += de;
#pragma unroll
        for (int k = 0; k < 8; ++k)
          if (k < in_dim) acc[e][k] = fmaf(de, xs[u][k], acc[e][k]);
      }
    }
  }
#pragma unroll
  for (int off = G; off < 64; off <<= 1)
#pragma unroll
    for (int e = 0; e < 8; ++e)
#pragma unroll
      for (int k = 0; k < 9; ++k) acc[e][k] += __shfl_xor(acc[e][k], off);
  for (int w = 0; w < kFG / 64; ++w) {
    if (wave == w && lane < G)
#pragma unroll
      for (int e = 0; e < 8; ++e)
#pragma unroll
        for (int k = 0; k < 9; ++k) red[g * 72 + e * 9 + k] = (w == 0 ? 0.0f : red[g * 72 + e * 9 + k]) + acc[e][k];
    __syncthreads();
  }
  float* out = partial + (int64_t)blockIdx.x * P;
  for (int t = threadIdx.x; t < W * 9; t += kFG) {
    const int nn = t / 9, k = t % 9;
    const float tot = red[(nn / 8) * 72 + (nn % 8) * 9 + k];
    if (k < in_dim) out[(int64_t)nn * in_dim + k] = tot;
    else if (k == 8) out[nb_b_off(0, in_dim, W, NH) + nn] = tot;
  }
}

// One training pass over `members` same-width bounds (gridDim.y).
struct TrainJob {
  int in_dim = 0, NH = 0, members = 1;
  int64_t n = 0;                    // valid queries per bound
  BF16TrainPlan plan;
  const float* q = nullptr;
  const uint8_t* y = nullptr;
  const float* theta = nullptr;
  const bf16x8* pack = nullptr;
  const bf16x8* packT = nullptr;
  uint16_t* act = nullptr;          // member 0: activation slots, slot(l) at act + slot(l) * Bp * W
  int every = 0;                    // checkpoint interval of the activation recomputation (0: keep all)
  bool stream_fwd = false;          // width 256: the forward half in one streamed launch, and every
                                    // backward layer's data and weight gradient in one launch
  uint16_t* grad = nullptr;         // member 0: D ping-pong at grad + k * Bp * W
  float* partial = nullptr;
  float* aux = nullptr;
  float alpha = 1, beta = 1, inv_n = 1, tau = 0;
  TrObjs T{};
};

// Activation slots of the layer-wise training pass.  every = 0 keeps every
// hidden activation A_0 .. A_{NH-2}.  every = k >= 2 keeps the checkpoints
// A_0, A_k, A_2k, ... and one segment of k - 1 scratch slots: the forward
// writes each segment's other activations into the scratch slots, and the
// backward recomputes a segment's activations from its checkpoint (the same
// kernel, so the same bits) when it moves down into that segment.
struct ActSlots {
  int every = 0, n_act = 0, n_ckpt = 0;
  int slot(int l) const {
    if (every < 2) return l;
    return l % every == 0 ? l / every : n_ckpt + (l % every) - 1;
  }
  int count() const { return every < 2 ? n_act : n_ckpt + std::min(every - 1, n_act - 1); }
  int segment(int l) const { return every < 2 ? 0 : l / every; }
};

ActSlots act_slots(int NH, int every) {
  ActSlots a;
  a.every = every;
  a.n_act = NH - 1;
  a.n_ckpt = every < 2 ? 0 : (NH - 2) / every + 1;
  return a;
}

template <int W>
nb_status train_w(const TrainJob& J, hipStream_t s) {
  using T = TrHidden<W>;
  const int NH = J.NH, in_dim = J.in_dim;
  const int64_t CH = J.plan.chunk;
  const dim3 grid((unsigned)J.plan.n_wg, (unsigned)J.members);
  const size_t lds = T::lds_bytes();
  const int64_t stride = J.plan.padded * W;
  const ActSlots S = act_slots(NH, J.every);
  auto A = [&](int l) { return J.act + (int64_t)S.slot(l) * stride; };
  uint16_t* D[2] = {J.grad, J.grad + stride};
  // workgroups of the layer kernels: as many as fit the CUs at once (the
  // width-256 ones hold 128 KB of LDS each: one per CU), each striding over
  // the batch, so every workgroup loads the layer's weights once
  const int64_t fit = W >= 256 ? 1 : 4;
  const unsigned wx = (unsigned)std::max<int64_t>(
      1, std::min<int64_t>(J.plan.padded / 64, std::max<int64_t>(1, fit * (int64_t)nb_cu_count() / J.members)));
  const dim3 wide(wx, (unsigned)J.members);

  NB_TRY(allow_lds(k_tr_layer<W>, lds));
  NB_TRY(allow_lds(k_tr_head<W>, lds));
  NB_TRY(allow_lds(k_tr_data<W>, (size_t)T::FH * 64 * 16));
  auto hidden = [&](int l) -> nb_status {   // A_l = relu(W_l A_{l-1} + b_l)
    k_tr_layer<W><<<wide, tr_threads<W, false>(), lds, s>>>(A(l - 1), J.plan.padded, l, in_dim, NH, J.pack, J.theta,
                                                          A(l), J.T);
    NB_LAUNCHED();
    return NB_OK;
  };
  int cur = 0;
  if (W == 256 && J.stream_fwd && J.members == 1 && bf16_stream_forward_supported(in_dim, NH, W)) {
    // one streamed launch: the activations the backward reads first (every
    // one, or the checkpoints and the last segment), D_{NH-1}, output layer
    StreamJob F;
    F.in_dim = in_dim;
    F.NH = NH;
    F.n = J.n;
    F.P = J.T.P;
    F.plan = J.plan;
    F.q = J.q;
    F.y = J.y;
    F.theta = J.theta;
    F.pack = J.pack;
    F.act = J.act;
    F.act_stride = stride;
    for (int l = 0; l < 8; ++l) {
      const bool keep = l <= NH - 2 && (S.every < 2 || l % S.every == 0 || S.segment(l) == S.segment(NH - 2));
      F.slots.s[l] = keep ? S.slot(l) : -1;
    }
    F.Dout = D[cur];
    F.partial = J.partial;
    F.aux = J.aux;
    F.alpha = J.alpha;
    F.beta = J.beta;
    F.inv_n = J.inv_n;
    F.tau = J.tau;
    NB_TRY(bf16_stream_forward(F, s));
  } else {
    k_tr_first<W><<<wide, 256, 0, s>>>(J.q, J.n, in_dim, J.plan.padded, J.pack, J.theta, NH, A(0), J.T);
    NB_LAUNCHED();
    for (int l = 1; l < NH - 1; ++l) NB_TRY(hidden(l));
    // head: layer NH-1, output layer, loss, D_{NH-1}
    k_tr_head<W><<<grid, tr_threads<W, true>(), lds, s>>>(A(NH - 2), J.n, CH, NH - 1, in_dim, NH, J.pack, J.theta,
                                                         D[cur], J.y, J.alpha, J.beta, J.inv_n, J.tau, J.partial,
                                                         J.aux, J.T);
    NB_LAUNCHED();
  }
  constexpr int WW = W >= 256 ? 8 : 4;
  const size_t wlds = (size_t)4 * W * kTS * 2 + (size_t)(WW * 64 / (W / 2)) * W * 4;
  NB_TRY(allow_lds(k_tr_weight<W, WW>, wlds));
  int valid_seg = S.segment(NH - 2);   // the segment whose activations the scratch slots hold
  for (int l = NH - 1; l >= 1; --l) {
    if (S.segment(l - 1) != valid_seg) {
      valid_seg = S.segment(l - 1);
      const int c = valid_seg * S.every, c1 = std::min(c + S.every - 1, NH - 2);
      if (W == 256 && J.stream_fwd && J.members == 1 && c1 > c) {
        // the segment's layers in one streamed launch from the checkpoint
        RecomputeJob R;
        R.in_dim = in_dim;
        R.NH = NH;
        R.l0 = c + 1;
        R.l1 = c1;
        R.plan = J.plan;
        R.ain = A(c);
        R.pack = J.pack;
        R.theta = J.theta;
        R.act = J.act;
        R.act_stride = stride;
        for (int r = 0; r < 8; ++r) R.slots.s[r] = r >= R.l0 && r <= R.l1 ? S.slot(r) : -1;
        NB_TRY(bf16_recompute256(R, s));
      } else {
        for (int r = c + 1; r <= c1; ++r) NB_TRY(hidden(r));
      }
    }
    if (W == 256 && J.stream_fwd && J.members == 1) {
      // data and weight gradient in one launch: D_l, A_{l-1} read once
      Back256Job B;
      B.in_dim = in_dim;
      B.NH = NH;
      B.l = l;
      B.P = J.T.P;
      B.plan = J.plan;
      B.Dl = D[cur];
      B.Aprev = A(l - 1);
      B.packT = J.packT;
      B.Dprev = D[cur ^ 1];
      B.partial = J.partial;
      NB_TRY(bf16_back256(B, s));
    } else {
      k_tr_weight<W, WW><<<grid, WW * 64, wlds, s>>>(D[cur], A(l - 1), CH, l, in_dim, NH, J.partial, J.T);
      NB_LAUNCHED();
      k_tr_data<W><<<wide, tr_threads<W, false>(), (size_t)T::FH * 64 * 16, s>>>(D[cur], A(l - 1), J.plan.padded,
                                                                               l, J.packT, D[cur ^ 1], J.T);
      NB_LAUNCHED();
    }
    cur ^= 1;
  }
  k_tr_first_grad<W><<<grid, kFG, 0, s>>>(D[cur], J.q, J.n, CH, in_dim, NH, J.partial, J.T);
  NB_LAUNCHED();
  return NB_OK;
}

nb_status train_dispatch(int W, const TrainJob& J, hipStream_t s) {
  switch (W) {
    case 32: return train_w<32>(J, s);
    case 64: return train_w<64>(J, s);
    case 128: return train_w<128>(J, s);
    case 256: return train_w<256>(J, s);
    default: break;
  }
  nb_set_error("bfloat16 training has no kernel for width %d", W);
  return NB_ERR_UNSUPPORTED;
}

}  // namespace

BF16TrainPlan bf16_train_plan(int64_t n, int max_wg) {
  BF16TrainPlan p;
  p.n_wg = (int)std::min<int64_t>(std::max(1, std::min(256, max_wg)), (n + 63) / 64);
  const int64_t per = (n + p.n_wg - 1) / p.n_wg;
  p.chunk = (per + 63) / 64 * 64;
  p.n_wg = (int)((n + p.chunk - 1) / p.chunk);
  p.padded = p.chunk * p.n_wg;
  return p;
}

bool bf16_train_supported(int in_dim, int n_hidden, int width) {
  return in_dim >= 1 && in_dim <= 8 && n_hidden >= 2 && n_hidden <= 8 &&
         (width == 32 || width == 64 || width == 128 || width == 256);
}

int64_t bf16_packt_elems(int n_hidden, int width) {
  const int RB = width / 16, KS = width / 32;
  return (int64_t)(n_hidden - 1) * RB * KS * 64 * 8;
}

nb_status bf16_pack_t(const nb_bound* b, hipStream_t s) {
  const int64_t total = b->pack16t_elems;
  if (total == 0) return NB_OK;
  k_pack_bf16_t<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(b->theta, b->in_dim, b->width, b->n_hidden,
                                                                b->pack16t, total, bf16_uses_fused(b));
  NB_LAUNCHED();
  return NB_OK;
}

bool bf16_uses_fused(const nb_bound* b) {
  return b->precision == NB_BF16 && b->train_kernel == NB_TRAIN_AUTO &&
         bf16_fused_supported(b->in_dim, b->n_hidden, b->width);
}

nb_status bf16_train_partials(const nb_bound* b, const float* q, const uint8_t* y, int64_t n, float alpha,
                              float beta, float tau, const BF16TrainPlan& plan, hipStream_t s) {
  if (bf16_uses_fused(b)) {
    FusedJob F;
    F.in_dim = b->in_dim;
    F.NH = b->n_hidden;
    F.W = b->width;
    F.n = n;
    F.plan = plan;
    F.q = q;
    F.y = y;
    F.theta = b->theta;
    F.pack = reinterpret_cast<const bf16x8*>(b->pack16);
    F.packT = reinterpret_cast<const bf16x8*>(b->pack16t);
    F.partial = b->partial;
    F.aux = b->aux;
    F.alpha = alpha;
    F.beta = beta;
    F.inv_n = (float)(1.0 / (double)n);
    F.tau = tau;
    F.T = TrObjs{nullptr, nullptr, nullptr, nullptr, 0, 0, 0, b->n_params, nullptr};
    return bf16_fused_train(F, s);
  }
  TrainJob J;
  J.in_dim = b->in_dim;
  J.NH = b->n_hidden;
  J.members = 1;
  J.n = n;
  J.plan = plan;
  J.q = q;
  J.y = y;
  J.theta = b->theta;
  J.pack = reinterpret_cast<const bf16x8*>(b->pack16);
  J.packT = reinterpret_cast<const bf16x8*>(b->pack16t);
  J.act = b->tr_act;
  J.every = b->recompute;
  J.stream_fwd = b->train_kernel == NB_TRAIN_AUTO;
  J.grad = b->tr_grad;
  J.partial = b->partial;
  J.aux = b->aux;
  J.alpha = alpha;
  J.beta = beta;
  J.inv_n = (float)(1.0 / (double)n);
  J.tau = tau;
  J.T = TrObjs{nullptr, nullptr, nullptr, nullptr, 0, 0, 0, b->n_params, nullptr};
  return train_dispatch(b->width, J, s);
}

nb_status bf16_group_train_class(const nb_group* gr, int width, const int* d_members, int n_members,
                                 const float* q, const uint8_t* y, int64_t per_obj, float alpha,
                                 const float* alpha_obj, float beta,
                                 float tau, const BF16TrainPlan& plan, uint16_t* act, uint16_t* grad,
                                 hipStream_t s) {
  if (bf16_fused_supported(gr->in_dim, gr->n_hidden, width)) {
    FusedJob F;
    F.in_dim = gr->in_dim;
    F.NH = gr->n_hidden;
    F.W = width;
    F.members = n_members;
    F.n = per_obj;
    F.plan = plan;
    F.q = q;
    F.y = y;
    F.theta = gr->theta;
    F.pack = reinterpret_cast<const bf16x8*>(gr->pack16);
    F.packT = reinterpret_cast<const bf16x8*>(gr->pack16t);
    F.partial = gr->partial;
    F.aux = gr->aux;
    F.alpha = alpha;
    F.beta = beta;
    F.inv_n = (float)(1.0 / (double)per_obj);
    F.tau = tau;
    F.T = TrObjs{d_members, gr->d_poff, gr->d_pkoff, gr->d_ptoff, per_obj, 0, 0, 0, alpha_obj};
    return bf16_fused_train(F, s);
  }
  TrainJob J;
  J.in_dim = gr->in_dim;
  J.NH = gr->n_hidden;
  J.members = n_members;
  J.n = per_obj;
  J.plan = plan;
  J.q = q;
  J.y = y;
  J.theta = gr->theta;
  J.pack = reinterpret_cast<const bf16x8*>(gr->pack16);
  J.packT = reinterpret_cast<const bf16x8*>(gr->pack16t);
  J.act = act;
  J.grad = grad;
  J.partial = gr->partial;
  J.aux = gr->aux;
  J.alpha = alpha;
  J.beta = beta;
  J.inv_n = (float)(1.0 / (double)per_obj);
  J.tau = tau;
  const int64_t per_a = (int64_t)(gr->n_hidden - 1) * plan.padded * width;
  const int64_t per_d = (int64_t)2 * plan.padded * width;
  J.T = TrObjs{d_members, gr->d_poff, gr->d_pkoff, gr->d_ptoff, per_obj, per_a, per_d, 0, alpha_obj};
  return train_dispatch(width, J, s);
}

int bf16_act_slots(int n_hidden, int every) { return act_slots(n_hidden, every).count(); }
