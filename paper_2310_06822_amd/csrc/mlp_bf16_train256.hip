// Training kernels for 256-wide bfloat16 bounds (Alg. 1 steps 4-5,
// gradient of Eq. 1) that replace groups of the layer-wise kernels.
//
// k_tr_stream: the forward half of a step in one launch, in place of the
// first-layer, hidden-layer and head kernels.  A 256-wide layer does not fit
// next to a second one in LDS, so, as in the streamed forward, every hidden
// layer streams through two 64 KiB LDS buffers in half-layer chunks (row
// blocks 0..7, then 8..15), copied straight from global memory into the idle
// buffer while the waves multiply the other one; the first layer's fragments
// and all biases stay resident.  One workgroup of 8 waves (two per SIMD)
// takes one chunk of the batch in tiles of 256 queries, two blocks of 16 per
// wave, so every streamed chunk serves 256 queries.  What the backward reads
// goes to HBM: the activation rows A_l that are kept (all of them, or the
// checkpoints and the last segment when the backward recomputes the rest),
// in the operand order of the layer-wise kernels, and D_{NH-1} = dL/dz w_out
// [a > 0].  The output layer's gradient, the loss and the confusion counts
// of the chunk go to the chunk's partial.
//
// k_tr_back: one layer of the backward pass, in place of the data- and
// weight-gradient kernels, so that D_l and A_{l-1} are read from HBM once:
//   D_{l-1} = (W_l^T D_l) [A_{l-1} > 0],  dW_l = sum_q D_l[q] A_{l-1}[q]^T,
//   db_l = sum_q D_l[q].
// One workgroup of eight waves per CU (two per SIMD) takes one chunk of the
// batch in steps of 32 queries: W_l^T's fragments stay in registers (each
// wave's two row blocks), the steps' D_l and A_{l-1} rows stream into a four-step LDS ring
// three steps ahead (direct-to-LDS loads), and the step's rows are written
// once more transposed ([neuron][query] tiles) for the weight gradient,
// which needs the queries on the MFMA's K dimension.
//
// Rounding points and the order of every product are those of the
// layer-wise kernels (bias first, K steps in order; the output logit summed
// over row blocks in order; weight-gradient tiles summed over the same
// 32-query slabs in the same order), so activations, logits, D_l and dW_l
// are bit-identical to theirs.  The output-weight and bias sums go through
// other fixed orders: deterministic, float32 rounding apart.
#include <algorithm>

#include "nb_bf16_train.h"

namespace {

template <int NH>
struct TrStream {
  static constexpr int W = 256, RB = 16, KS = 8, FH = RB * KS, HALF = FH / 2;
  static constexpr int NB = 2, THREADS = 512, WAVES = THREADS / 64, TILE = WAVES * NB * 16;
  static constexpr int PER = HALF * 64 / THREADS;   // 16-byte fragment slices per thread per chunk
  static constexpr int IN_WAVE = NB * 16 * 8;       // staged input floats per wave (in_dim <= 8)
  static constexpr size_t bias_bytes() { return ((size_t)(NH * W + W + 1) * 4 + 15) / 16 * 16; }
  static constexpr size_t lds_bytes() {
    return (size_t)(RB * 64 + 2 * HALF * 64) * 16 + bias_bytes() + (size_t)WAVES * IN_WAVE * 4;
  }
  static_assert(lds_bytes() <= 160 * 1024, "streamed training forward: LDS of one CU");
};

template <int NH>
__global__ __launch_bounds__(512, 1) void k_tr_stream(const float* __restrict__ q, int64_t n, int in_dim,
                                                      int64_t CH, const bf16x8* __restrict__ pack,
                                                      const float* __restrict__ theta, uint16_t* __restrict__ act,
                                                      int64_t act_stride, StreamSlots slots,
                                                      uint16_t* __restrict__ Dout, const uint8_t* __restrict__ y,
                                                      float alpha, float beta, float inv_n, float tau, int64_t P,
                                                      float* __restrict__ partial, float* __restrict__ aux) {
  using S = TrStream<NH>;
  constexpr int W = S::W, RB = S::RB, KS = S::KS, NB = S::NB, RA = RB / 2;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  // LDS region offsets kept opaque: every access is a region base register
  // plus an immediate below 64 KB
  int obuf = RB * 64 * 16, obias = (RB * 64 + 2 * S::HALF * 64) * 16;
  asm volatile("" : "+s"(obuf), "+s"(obias));
  bf16x8* sfirst = reinterpret_cast<bf16x8*>(smem_raw);
  bf16x8* sbuf = reinterpret_cast<bf16x8*>(smem_raw + obuf);   // [2][HALF * 64]
  float* sbias = reinterpret_cast<float*>(smem_raw + obias);
  const float* swo = sbias + NH * W;
  const int wave_u = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  float* sin = reinterpret_cast<float*>(reinterpret_cast<unsigned char*>(sbias) + S::bias_bytes()) +
               wave_u * S::IN_WAVE;
  const int64_t cbeg = (int64_t)blockIdx.x * CH, cend = cbeg + CH;
  const int64_t vend = cend < n ? cend : n;   // rows of the chunk with inputs and labels
  // a wave's next-tile inputs, copied straight into LDS during the last layer
  auto stage_inputs = [&](int64_t q0s) {
    const int64_t first = q0s * in_dim;
    const int64_t end = (q0s + NB * 16 < vend ? q0s + NB * 16 : vend) * in_dim;
#pragma unroll
    for (int i = 0; i < S::IN_WAVE / 64; ++i) {
      const int64_t e = first + i * 64 + (threadIdx.x & 63);
      if (i * 64 < NB * 16 * in_dim && e < end)
        __builtin_amdgcn_global_load_lds((const void*)(q + e), (__attribute__((address_space(3))) void*)(sin + i * 64),
                                         4, 0, 0);
    }
  };

  for (int i = threadIdx.x; i < RB * 64; i += S::THREADS) sfirst[i] = pack[i];
  for (int i = threadIdx.x; i < NH * W; i += S::THREADS) sbias[i] = theta[nb_b_off(i / W, in_dim, W, NH) + i % W];
  for (int i = threadIdx.x; i < W + 1; i += S::THREADS) sbias[NH * W + i] = theta[nb_w_off(NH, in_dim, W) + i];

  const int nchunk = 2 * (NH - 1);
  const int64_t tiles = (CH + S::TILE - 1) / S::TILE;
  const int64_t total_chunks = tiles * nchunk;
  // chunk k of the stream: layer 1 + (k % nchunk) / 2, half (k % nchunk) % 2
  auto chunk_src = [&](int64_t k) {
    const int c = (int)(k % nchunk), l = 1 + c / 2, h = c % 2;
    return pack + (RB + (l - 1) * S::FH + h * S::HALF) * 64;
  };
  auto prefetch = [&](int64_t kk, bf16x8* dst) {
    const bf16x8* src = chunk_src(kk);
#pragma unroll
    for (int i = 0; i < S::PER; ++i) {
      const int slot = i * S::THREADS + wave_u * 64;
      __builtin_amdgcn_global_load_lds((const void*)(src + slot + (threadIdx.x & 63)),
                                       (__attribute__((address_space(3))) void*)(dst + slot), 16, 0, 0);
    }
  };
  {
    const bf16x8* src = chunk_src(0);
#pragma unroll
    for (int i = 0; i < S::PER; ++i) sbuf[threadIdx.x + i * S::THREADS] = src[threadIdx.x + i * S::THREADS];
  }
  stage_inputs(cbeg + wave_u * NB * 16);
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();

  const int lane = threadIdx.x & 63, c = lane & 15, grp = lane >> 4;
  const bool wide = in_dim > 4;
  const float bo = swo[W];
  float gwo[4] = {0.0f, 0.0f, 0.0f, 0.0f};   // value c + 16 g of the lane's 64, summed over the row's queries
  float gbo = 0.0f, lsum = 0.0f;
  unsigned cnt[4] = {0u, 0u, 0u, 0u};

  // one half-layer's products from LDS buffer buf into acc (row blocks
  // 8h .. 8h+7), four row blocks at a time, the next K step's fragments
  // loading behind the first row block's products
  auto half_products = [&](const bf16x8* buf, int l, int h, const bf16x8 (&opnd)[NB][KS], floatx4 (&acc)[NB][RA]) {
#pragma unroll
    for (int m4 = 0; m4 < RA; m4 += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float* b = sbias + l * W + 16 * (h * RA + m4 + u) + 4 * grp;
        const floatx4 bi = floatx4{b[0], b[1], b[2], b[3]};
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb][m4 + u] = bi;
      }
      bf16x8 fa[4], fb[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) fa[u] = buf[((m4 + u) * KS + 0) * 64 + lane];
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        bf16x8(&cur)[4] = (ks & 1) ? fb : fa;
        bf16x8(&nxt)[4] = (ks & 1) ? fa : fb;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb][m4] = nb_mfma_bf16(cur[0], opnd[nb][ks], acc[nb][m4]);
        __builtin_amdgcn_sched_barrier(0);
        if (ks + 1 < KS) {
#pragma unroll
          for (int u = 0; u < 4; ++u) nxt[u] = buf[((m4 + u) * KS + ks + 1) * 64 + lane];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 1; u < 4; ++u)
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) acc[nb][m4 + u] = nb_mfma_bf16(cur[u], opnd[nb][ks], acc[nb][m4 + u]);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  };

  int64_t k = 0;
#pragma unroll 1
  for (int64_t t = 0; t < tiles; ++t) {
    const int64_t q0 = cbeg + t * S::TILE + wave_u * NB * 16;
    bf16x8 opnd[NB][KS];   // the current layer's input activations (B operands)
    {
      floatx4 acc[NB][RA];
      bf16x8 xb[NB], xb1[NB];
      {
        float xr[NB][8];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const bool valid = q0 + nb * 16 + c < vend;
#pragma unroll
          for (int j = 0; j < 8; ++j) xr[nb][j] = (valid && j < in_dim) ? sin[(nb * 16 + c) * in_dim + j] : 0.0f;
        }
        nb_first_operands<NB>(xr, grp, wide, xb, xb1);
      }
#pragma unroll
      for (int h0 = 0; h0 < RB; h0 += RA) {
#pragma unroll
        for (int u = 0; u < RA; ++u) {
          const int mo = h0 + u;
          const float* b = sbias + 16 * mo + 4 * grp;
          const floatx4 bi = floatx4{b[0], b[1], b[2], b[3]};
          const bf16x8 a = sfirst[mo * 64 + lane];
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) acc[nb][u] = nb_mfma_bf16(a, xb[nb], bi);
        }
        if (wide) {
          // the second first-layer step's fragments come from global memory (L2)
          typedef const __attribute__((address_space(1))) bf16x8* gpk_t;
          gpk_t pk = (gpk_t)pack;
          asm volatile("" : "+s"(pk));
#pragma unroll
          for (int u = 0; u < RA; ++u) {
            const bf16x8 a = pk[(RB + (NH - 1) * S::FH + h0 + u) * 64 + lane];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) acc[nb][u] = nb_mfma_bf16(a, xb1[nb], acc[nb][u]);
          }
        }
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
          for (int kk = 0; kk < RA / 2; ++kk) {
            float v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = acc[nb][2 * kk + j / 4][j % 4];
            opnd[nb][h0 / 2 + kk] = nb_relu_bf16x8(v);
          }
      }
    }
    // A_{l-1}'s rows go out at the start of layer l, behind that layer's
    // first prefetch: by the end-of-chunk wait (which counts stores too) they
    // have long completed
    auto store_rows = [&](int l) {
      const int sl = slots.s[l];
      if (sl < 0) return;
      // the row base formed here, at the stores (opaque), not held across the tile
      typedef __attribute__((address_space(1))) bf16x8* gact_t;
      gact_t base = (gact_t)(act + (int64_t)sl * act_stride + q0 * W);
      asm volatile("" : "+s"(base));
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        if (q0 + nb * 16 < cend) {   // whole blocks: the chunk is a multiple of 16 rows
#pragma unroll
          for (int ks = 0; ks < KS; ++ks) base[((nb * 16 + c) * W + 32 * ks + 8 * grp) / 8] = opnd[nb][ks];
        }
      }
    };

#pragma unroll 1
    for (int l = 1; l < NH - 1; ++l) {
      bf16x8 nxt[NB][KS];   // the next layer's operands, filled half by half
#pragma unroll
      for (int h = 0; h < 2; ++h, ++k) {
        const bf16x8* buf = sbuf + (k & 1) * S::HALF * 64;
        if (k + 1 < total_chunks) prefetch(k + 1, sbuf + ((k + 1) & 1) * S::HALF * 64);
        if (h == 0) store_rows(l - 1);
        floatx4 acc[NB][RA];
        half_products(buf, l, h, opnd, acc);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
          for (int kk = 0; kk < KS / 2; ++kk) {
            float v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = acc[nb][2 * kk + j / 4][j % 4];
            nxt[nb][h * (KS / 2) + kk] = nb_relu_bf16x8(v);
          }
        if (h == 1) {
#pragma unroll
          for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) opnd[nb][ks] = nxt[nb][ks];
        }
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
      }
    }

    // the last hidden layer, both halves' accumulators kept for the head
    floatx4 acc0[NB][RA], acc1[NB][RA];
#pragma unroll
    for (int h = 0; h < 2; ++h, ++k) {
      const bf16x8* buf = sbuf + (k & 1) * S::HALF * 64;
      if (k + 1 < total_chunks) prefetch(k + 1, sbuf + ((k + 1) & 1) * S::HALF * 64);
      if (h == 0) {
        store_rows(NH - 2);
        if (t + 1 < tiles) stage_inputs(q0 + S::TILE);
        half_products(buf, NH - 1, 0, opnd, acc0);
      } else {
        half_products(buf, NH - 1, 1, opnd, acc1);
      }
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();
    }

    // head: output logit, Eq. 1 and dL/dz, D_{NH-1}, output-layer terms
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      float p = 0.0f;
#pragma unroll
      for (int mo = 0; mo < RB; ++mo)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float a = mo < RA ? acc0[nb][mo][r] : acc1[nb][mo - RA][r];
          p = fmaf(swo[16 * mo + 4 * grp + r], fmaxf(a, 0.0f), p);
        }
      p += __shfl_xor(p, 16);
      p += __shfl_xor(p, 32);
      const float z = p + bo;
      const int64_t qi = q0 + nb * 16 + c;
      const bool valid = qi < vend;
      const bool yv = y[valid ? qi : cbeg] != 0 && valid;   // a load from a valid row, no branch
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
      // D_{NH-1} rows of the chunk (padding rows included: dz = 0 there).
      // The output weights are read again through a fresh base (not held
      // from the logit's loop) and taken before the selects (no branches).
      // Row blocks in pairs: the lanes of rows g and g ^ 1 (same query) swap
      // one row block's values (v_permlane16_swap), so that every lane
      // writes 16 bytes, 8 consecutive neurons of row block 2p (even g) or
      // 2p + 1 (odd g).
      if (q0 + nb * 16 < cend) {
        typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
        typedef __attribute__((address_space(1))) u32x4* gd_t;
        gd_t out = (gd_t)(Dout + (q0 + nb * 16) * W);
        asm volatile("" : "+s"(out));
        typedef const __attribute__((address_space(3))) float* lds_f;
        lds_f wo2 = (lds_f)(swo + 4 * grp);
        asm volatile("" : "+v"(wo2));
        const bool oddrow = grp & 1;
#pragma unroll
        for (int pr = 0; pr < RB / 2; ++pr) {
          uint2 pk[2];
#pragma unroll
          for (int e = 0; e < 2; ++e) {
            const int mo = 2 * pr + e;
            float w4[4], d[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) w4[r] = wo2[16 * mo + r];
            asm volatile("" : "+v"(w4[0]), "+v"(w4[1]), "+v"(w4[2]), "+v"(w4[3]));
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const float a = mo < RA ? acc0[nb][mo][r] : acc1[nb][mo - RA][r];
              d[r] = a > 0.0f ? dz * w4[r] : 0.0f;
            }
            pk[e] = pack4(d[0], d[1], d[2], d[3]);
          }
          const auto sx = __builtin_amdgcn_permlane16_swap(pk[0].x, pk[1].x, false, false);
          const auto sy = __builtin_amdgcn_permlane16_swap(pk[0].y, pk[1].y, false, false);
          const int mo = 2 * pr + (oddrow ? 1 : 0);
          out[(c * W + 16 * mo + 4 * (grp & ~1)) / 8] = u32x4{sx[0], sy[0], sx[1], sy[1]};
        }
      }
      // output-weight terms dz a, summed over the block's 16 queries
#pragma unroll
      for (int g4 = 0; g4 < 4; ++g4) {
        float tv[16], sm[1];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int mo = 4 * g4 + i / 4;
          const float a = mo < RA ? acc0[nb][mo][i % 4] : acc1[nb][mo - RA][i % 4];
          tv[i] = dz * fmaxf(a, 0.0f);
        }
        nb_row_reduce_scatter<16>(tv, c, sm);
        gwo[g4] += sm[0];
      }
    }
  }

  // ---- the chunk's output-layer partial, waves summed in index order
  float* red = reinterpret_cast<float*>(sbuf);   // [WAVES][W], then [WAVES][8]
  float* saux = red + S::WAVES * W;
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) {
    gbo += __shfl_xor(gbo, m);
    lsum += __shfl_xor(lsum, m);
  }
#pragma unroll
  for (int g4 = 0; g4 < 4; ++g4) red[wave_u * W + 16 * (4 * g4 + c / 4) + 4 * grp + c % 4] = gwo[g4];
  if (lane == 0) {
    saux[wave_u * 8 + 0] = lsum;
    saux[wave_u * 8 + 1] = gbo;
    for (int i = 0; i < 4; ++i) saux[wave_u * 8 + 2 + i] = __uint_as_float(cnt[i]);
  }
  __syncthreads();
  float* out = partial + (int64_t)blockIdx.x * P + nb_w_off(NH, in_dim, W);
  if (threadIdx.x < W) {
    float v = red[threadIdx.x];
    for (int w = 1; w < S::WAVES; ++w) v += red[w * W + threadIdx.x];
    out[threadIdx.x] = v;
  }
  if (threadIdx.x == 0) {
    float ls = saux[0], gb = saux[1];
    unsigned cs[4];
    for (int i = 0; i < 4; ++i) cs[i] = __float_as_uint(saux[2 + i]);
    for (int w = 1; w < S::WAVES; ++w) {
      ls += saux[w * 8];
      gb += saux[w * 8 + 1];
      for (int i = 0; i < 4; ++i) cs[i] += __float_as_uint(saux[w * 8 + 2 + i]);
    }
    out[W] = gb;
    aux[blockIdx.x * 8] = ls;
    for (int i = 0; i < 4; ++i) aux[blockIdx.x * 8 + 1 + i] = __uint_as_float(cs[i]);
  }
}

// Recomputation of a segment A_{l0} .. A_{l1} of activation rows from the
// checkpoint A_{l0-1} (width 256), one launch in place of one hidden-layer
// launch per layer: the checkpoint rows are read once and every recomputed
// row written once, the layers streaming through LDS in half-layer chunks
// as in k_tr_stream (same products in the same order: the same bits).
__global__ __launch_bounds__(512, 1) void k_tr_recompute(const uint16_t* __restrict__ ain, int64_t CH, int l0, int l1,
                                                         int in_dim, int NH, const bf16x8* __restrict__ pack,
                                                         const float* __restrict__ theta, uint16_t* __restrict__ act,
                                                         int64_t act_stride, StreamSlots slots) {
  using S = TrStream<6>;   // (the streaming shape; the biases below hold only the segment's layers)
  constexpr int W = S::W, RB = S::RB, KS = S::KS, NB = S::NB, RA = RB / 2;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  int obias = 2 * S::HALF * 64 * 16;
  asm volatile("" : "+s"(obias));
  bf16x8* sbuf = reinterpret_cast<bf16x8*>(smem_raw);   // [2][HALF * 64]
  float* sbias = reinterpret_cast<float*>(smem_raw + obias);   // [l1 - l0 + 1][W]
  const int wave_u = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t cbeg = (int64_t)blockIdx.x * CH, cend = cbeg + CH;
  const int nl = l1 - l0 + 1, nchunk = 2 * nl;
  for (int i = threadIdx.x; i < nl * W; i += S::THREADS) sbias[i] = theta[nb_b_off(l0 + i / W, in_dim, W, NH) + i % W];
  const int64_t tiles = (CH + S::TILE - 1) / S::TILE;
  const int64_t total_chunks = tiles * nchunk;
  auto chunk_src = [&](int64_t k) {
    const int cc = (int)(k % nchunk), l = l0 + cc / 2, h = cc % 2;
    return pack + (RB + (l - 1) * S::FH + h * S::HALF) * 64;
  };
  auto prefetch = [&](int64_t kk, bf16x8* dst) {
    const bf16x8* src = chunk_src(kk);
#pragma unroll
    for (int i = 0; i < S::PER; ++i) {
      const int slot = i * S::THREADS + wave_u * 64;
      __builtin_amdgcn_global_load_lds((const void*)(src + slot + (threadIdx.x & 63)),
                                       (__attribute__((address_space(3))) void*)(dst + slot), 16, 0, 0);
    }
  };
  {
    const bf16x8* src = chunk_src(0);
#pragma unroll
    for (int i = 0; i < S::PER; ++i) sbuf[threadIdx.x + i * S::THREADS] = src[threadIdx.x + i * S::THREADS];
  }
  __syncthreads();

  const int lane = threadIdx.x & 63, c = lane & 15, grp = lane >> 4;
  auto half_products = [&](const bf16x8* buf, int lb, int h, const bf16x8 (&opnd)[NB][KS], floatx4 (&acc)[NB][RA]) {
#pragma unroll
    for (int m4 = 0; m4 < RA; m4 += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float* b = sbias + lb * W + 16 * (h * RA + m4 + u) + 4 * grp;
        const floatx4 bi = floatx4{b[0], b[1], b[2], b[3]};
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb][m4 + u] = bi;
      }
      bf16x8 fa[4], fb[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) fa[u] = buf[((m4 + u) * KS + 0) * 64 + lane];
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        bf16x8(&cur)[4] = (ks & 1) ? fb : fa;
        bf16x8(&nx)[4] = (ks & 1) ? fa : fb;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb][m4] = nb_mfma_bf16(cur[0], opnd[nb][ks], acc[nb][m4]);
        __builtin_amdgcn_sched_barrier(0);
        if (ks + 1 < KS) {
#pragma unroll
          for (int u = 0; u < 4; ++u) nx[u] = buf[((m4 + u) * KS + ks + 1) * 64 + lane];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 1; u < 4; ++u)
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) acc[nb][m4 + u] = nb_mfma_bf16(cur[u], opnd[nb][ks], acc[nb][m4 + u]);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  };

  int64_t k = 0;
#pragma unroll 1
  for (int64_t t = 0; t < tiles; ++t) {
    const int64_t q0 = cbeg + t * S::TILE + wave_u * NB * 16;
    const bool rows = q0 < cend;   // whole blocks: the chunk is a multiple of 32 rows
    bf16x8 opnd[NB][KS];
    {
      typedef const __attribute__((address_space(1))) bf16x8* gin_t;
      gin_t src = (gin_t)(ain + (rows ? q0 : cbeg) * W);
      asm volatile("" : "+s"(src));
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) opnd[nb][ks] = src[((nb * 16 + c) * W + 32 * ks + 8 * grp) / 8];
    }
    auto store_rows = [&](int l) {
      if (!rows) return;
      typedef __attribute__((address_space(1))) bf16x8* gact_t;
      gact_t base = (gact_t)(act + (int64_t)slots.s[l] * act_stride + q0 * W);
      asm volatile("" : "+s"(base));
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) base[((nb * 16 + c) * W + 32 * ks + 8 * grp) / 8] = opnd[nb][ks];
    };
#pragma unroll 1
    for (int l = l0; l <= l1; ++l) {
      bf16x8 nxt[NB][KS];
#pragma unroll
      for (int h = 0; h < 2; ++h, ++k) {
        const bf16x8* buf = sbuf + (k & 1) * S::HALF * 64;
        if (k + 1 < total_chunks) prefetch(k + 1, sbuf + ((k + 1) & 1) * S::HALF * 64);
        if (h == 0 && l > l0) store_rows(l - 1);
        floatx4 acc[NB][RA];
        half_products(buf, l - l0, h, opnd, acc);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
          for (int kk = 0; kk < KS / 2; ++kk) {
            float v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = acc[nb][2 * kk + j / 4][j % 4];
            nxt[nb][h * (KS / 2) + kk] = nb_relu_bf16x8(v);
          }
        if (h == 1) {
#pragma unroll
          for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) opnd[nb][ks] = nxt[nb][ks];
        }
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
      }
    }
    store_rows(l1);
  }
}

template <int NH>
nb_status stream_launch(const StreamJob& J, hipStream_t s) {
  using S = TrStream<NH>;
  NB_TRY(allow_lds(k_tr_stream<NH>, S::lds_bytes()));
  k_tr_stream<NH><<<(unsigned)J.plan.n_wg, S::THREADS, S::lds_bytes(), s>>>(
      J.q, J.n, J.in_dim, J.plan.chunk, J.pack, J.theta, J.act, J.act_stride, J.slots, J.Dout, J.y, J.alpha, J.beta,
      J.inv_n, J.tau, J.P, J.partial, J.aux);
  NB_LAUNCHED();
  return NB_OK;
}

// ------------------------------------------------------------ backward

// LDS of k_tr_back: a ring of four 32-query steps of D_l and A_{l-1} rows
// (16 KiB each, row-major as in HBM but with the 16-byte chunks of row q
// permuted, chunk k at k ^ (q & 7), so that a 16-lane read of one chunk
// from 16 rows hits distinct banks), loaded straight from global memory
// three steps ahead; then the step's [neuron][32 query] transposed tiles.
// W_l^T stays in registers (each wave's 16 / WV row blocks).
struct Back256 {
  static constexpr int W = 256, RB = 16, KS = 8, QS = 32, RING = 4;
  static constexpr int WAVES = 8;   // two per SIMD (measured 379 us per 2^20 samples against 455 with four)
  static constexpr int SLOT = QS * W;                 // bfloat16 elements of one tensor's step
  static constexpr size_t ring_bytes() { return (size_t)RING * 2 * SLOT * 2; }
  static constexpr size_t tile_bytes() { return (size_t)W * QS * 2; }
  static constexpr size_t lds_bytes() { return ring_bytes() + 2 * tile_bytes(); }
};
static_assert(Back256::lds_bytes() <= 160 * 1024, "backward layer: LDS of one CU");

// Workgroup barrier for LDS traffic only: the wave's LDS operations are
// complete (lgkmcnt 0), its global loads and stores stay in flight (a
// __syncthreads would also wait for those).
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Transposed tile: row i (neuron) of 32 queries, 64 bytes in four 16-byte
// chunks of 8 queries; chunk k of row i sits at k ^ ((i >> 1) & 3), so that
// the weight-gradient operand reads (lane c: row 16 b + c, chunk g) of 8
// consecutive lanes hit distinct banks.
__device__ __forceinline__ int tile_off(int row, int q) {
  return row * 32 + (((q >> 3) ^ ((row >> 1) & 3)) << 3) + (q & 7);
}

// Writes the lane's operand (8 values of one query, element j = neuron
// nrn(j)) into a transposed tile, two queries per 32-bit store: the lanes of
// queries c and c ^ 1 swap dword halves (one DPP move, one byte permute);
// the even lane writes neuron nrn(2m), the odd lane nrn(2m + 1), each for
// both queries.  nrn(2m + 1) = nrn(2m) + 1.
template <class NRN>
__device__ __forceinline__ void tile_store(uint16_t* __restrict__ tile, bf16x8 v, int q, NRN nrn) {
  const int odd = q & 1;
  const unsigned sel = odd ? 0x03020706u : 0x05040100u;
  const nb_uint4 u = __builtin_bit_cast(nb_uint4, v);
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const unsigned pu = (unsigned)__builtin_amdgcn_mov_dpp((int)u[m], 0xB1, 0xF, 0xF, false);   // lane c ^ 1
    const unsigned w = __builtin_amdgcn_perm(pu, u[m], sel);
    const int row = nrn(2 * m) + odd;
    *reinterpret_cast<unsigned*>(tile + tile_off(row, q & ~1)) = w;
  }
}

// s_waitcnt vmcnt(n) for a wave-uniform n in 0 .. 31.
__device__ __forceinline__ void wait_vm(int n) {
  switch (n) {
    case 0: asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); break;
    case 1: asm volatile("s_waitcnt vmcnt(1)" ::: "memory"); break;
    case 2: asm volatile("s_waitcnt vmcnt(2)" ::: "memory"); break;
    case 3: asm volatile("s_waitcnt vmcnt(3)" ::: "memory"); break;
    case 4: asm volatile("s_waitcnt vmcnt(4)" ::: "memory"); break;
    case 5: asm volatile("s_waitcnt vmcnt(5)" ::: "memory"); break;
    case 6: asm volatile("s_waitcnt vmcnt(6)" ::: "memory"); break;
    case 7: asm volatile("s_waitcnt vmcnt(7)" ::: "memory"); break;
    case 8: asm volatile("s_waitcnt vmcnt(8)" ::: "memory"); break;
    case 9: asm volatile("s_waitcnt vmcnt(9)" ::: "memory"); break;
    case 10: asm volatile("s_waitcnt vmcnt(10)" ::: "memory"); break;
    case 11: asm volatile("s_waitcnt vmcnt(11)" ::: "memory"); break;
    case 12: asm volatile("s_waitcnt vmcnt(12)" ::: "memory"); break;
    case 13: asm volatile("s_waitcnt vmcnt(13)" ::: "memory"); break;
    case 14: asm volatile("s_waitcnt vmcnt(14)" ::: "memory"); break;
    case 15: asm volatile("s_waitcnt vmcnt(15)" ::: "memory"); break;
    case 16: asm volatile("s_waitcnt vmcnt(16)" ::: "memory"); break;
    case 17: asm volatile("s_waitcnt vmcnt(17)" ::: "memory"); break;
    case 18: asm volatile("s_waitcnt vmcnt(18)" ::: "memory"); break;
    case 19: asm volatile("s_waitcnt vmcnt(19)" ::: "memory"); break;
    case 20: asm volatile("s_waitcnt vmcnt(20)" ::: "memory"); break;
    case 21: asm volatile("s_waitcnt vmcnt(21)" ::: "memory"); break;
    case 22: asm volatile("s_waitcnt vmcnt(22)" ::: "memory"); break;
    case 23: asm volatile("s_waitcnt vmcnt(23)" ::: "memory"); break;
    case 24: asm volatile("s_waitcnt vmcnt(24)" ::: "memory"); break;
    case 25: asm volatile("s_waitcnt vmcnt(25)" ::: "memory"); break;
    case 26: asm volatile("s_waitcnt vmcnt(26)" ::: "memory"); break;
    case 27: asm volatile("s_waitcnt vmcnt(27)" ::: "memory"); break;
    case 28: asm volatile("s_waitcnt vmcnt(28)" ::: "memory"); break;
    case 29: asm volatile("s_waitcnt vmcnt(29)" ::: "memory"); break;
    case 30: asm volatile("s_waitcnt vmcnt(30)" ::: "memory"); break;
    default: asm volatile("s_waitcnt vmcnt(31)" ::: "memory"); break;
  }
}

// One backward layer over one chunk of the batch (CH queries, a multiple of
// 32) per workgroup of WV waves (8: two per SIMD, 256 registers each; 4:
// one per SIMD).  Wave w owns RPW = 16 / WV row blocks RPW w ..: their data
// gradient for both 16-query blocks of every step (W_l^T's fragments of
// those rows in registers), their weight-gradient tiles against all 16
// column blocks, and their bias rows (a fragment of ones as the MFMA's B
// operand).  Per step every wave issues 32 / WV ring loads (three steps
// ahead, after the step's first barrier) and 16 / WV stores of D_{l-1}, and
// nothing else that counts in vmcnt, so the loads of a step are complete
// once no more than the stores and loads issued after them remain.
template <int WV>
__global__ __launch_bounds__(64 * WV, 1) void k_tr_back(const uint16_t* __restrict__ Dl,
                                                    const uint16_t* __restrict__ Aprev, int64_t CH, int l,
                                                    int in_dim, int NH, const bf16x8* __restrict__ packT,
                                                    uint16_t* __restrict__ Dprev, int64_t P,
                                                    float* __restrict__ partial) {
  using B = Back256;
  constexpr int W = B::W, KS = B::KS;
  constexpr int RPW = B::RB / WV;    // row blocks per wave (data gradient, weight-gradient rows)
  constexpr int H = RPW / 2;         // A_{l-1} pieces per query block (two row blocks each)
  constexpr int LI = 16 / WV;        // ring load instructions per tensor and step
  constexpr int KPW = KS / WV;       // D_l K steps a wave transposes
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  int otile = (int)B::ring_bytes();
  asm volatile("" : "+s"(otile));
  uint16_t* ring = reinterpret_cast<uint16_t*>(smem_raw);   // [RING][D slot, A slot]
  uint16_t* sDT = reinterpret_cast<uint16_t*>(smem_raw + otile);
  uint16_t* sAT = sDT + W * B::QS;
  const int lane = threadIdx.x & 63, c0 = lane & 15, grp0 = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t cbeg = (int64_t)blockIdx.x * CH;
  const int nst = (int)(CH / B::QS);

  // the step's rows into ring slot (st & 3): 32 rows x 512 bytes per tensor
  // are 1024 sixteen-byte units; wave w, instruction i fills units
  // 64 (4 i + w) + lane, unit u = row q, chunk position p holding the row's
  // chunk p ^ (q & 7)
  // (the bases are opaque and the lane offsets formed here, so that no
  // per-lane address is held across the loop)
  auto load_step = [&](int st) {
    const int64_t r0 = cbeg + (int64_t)st * B::QS;
    uint16_t* slot = ring + (st & 3) * 2 * B::SLOT;
    int ln = lane;
    asm volatile("" : "+v"(ln));
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const uint16_t* src = (t == 0 ? Dl : Aprev) + r0 * W;
      asm volatile("" : "+s"(src));
#pragma unroll
      for (int i = 0; i < LI; ++i) {
        const int u0 = 64 * (WV * i + wave);              // wave-uniform first unit
        const int u = u0 + ln, qq = u >> 5, p = u & 31;
        __builtin_amdgcn_global_load_lds((const void*)(src + qq * W + 8 * (p ^ (qq & 7))),
                                         (__attribute__((address_space(3))) void*)(slot + t * B::SLOT + 8 * u0),
                                         16, 0, 0);
      }
    }
  };
  // 16-byte chunk k of row q of a ring tensor
  auto ring_chunk = [&](const uint16_t* base, int q, int k) {
    return *reinterpret_cast<const bf16x8*>(base + q * W + 8 * (k ^ (q & 7)));
  };

  for (int st = 0; st < 3 && st < nst; ++st) load_step(st);

  // W_l^T fragments of the wave's row blocks (natural K order)
  bf16x8 wt[RPW][KS];
  {
    const bf16x8* src = packT + (int64_t)(l - 1) * B::RB * KS * 64 + lane;
#pragma unroll
    for (int u = 0; u < RPW; ++u)
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) wt[u][ks] = src[((RPW * wave + u) * KS + ks) * 64];
  }
  floatx4 dw[RPW][16], db[RPW];
  const floatx4 zero4 = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int a = 0; a < RPW; ++a) {
    db[a] = zero4;
#pragma unroll
    for (int b = 0; b < 16; ++b) dw[a][b] = zero4;
  }
  nb_uint4 onesu;
#pragma unroll
  for (int i = 0; i < 4; ++i) onesu[i] = 0x3F803F80u;
  const bf16x8 ones = __builtin_bit_cast(bf16x8, onesu);
  // lane offset of the weight-gradient operand reads (row 16 b + c, chunk grp)

#pragma unroll 1
  for (int st = 0; st < nst; ++st) {
    // lane coordinates made opaque per step: the LDS addresses built from
    // them are formed where they are used, not held across the loop
    int c = c0, grp = grp0;
    asm volatile("" : "+v"(c), "+v"(grp));
    const int64_t r0 = cbeg + (int64_t)st * B::QS;
    const uint16_t* sD = ring + (st & 3) * 2 * B::SLOT;
    const uint16_t* sA = sD + B::SLOT;
    // this step's rows have landed once at most the stores of the three
    // steps before (2H each) and the loads of the two after (2LI each) are
    // outstanding
    wait_vm(2 * H * (st < 3 ? st : 3) + 2 * LI * (nst - 1 - st < 2 ? nst - 1 - st : 2));
    lds_barrier();   // the step's rows are in LDS; every wave is done with step st - 1 (its slot, the tiles)
    if (st + 3 < nst) load_step(st + 3);
    asm volatile("" ::: "memory");   // the loads issue before this step's stores (the counts above)
    // D_{l-1} = (W_l^T D_l) [A_{l-1} > 0], the wave's row blocks, both query
    // blocks.  The chunks the wave reads for it also fill its share of the
    // transposed tiles: D_l's K steps KPW w .. and the A_{l-1} mask pieces
    // (K steps H w .. of the operand-order rows).
    {
      floatx4 acc[2][RPW];
#pragma unroll
      for (int nb = 0; nb < 2; ++nb)
#pragma unroll
        for (int u = 0; u < RPW; ++u) acc[nb][u] = zero4;
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const bf16x8 b0 = ring_chunk(sD, c, 4 * ks + grp), b1 = ring_chunk(sD, 16 + c, 4 * ks + grp);
        if (ks / KPW == wave) {
          tile_store(sDT, b0, c, [&](int j) { return 32 * ks + 8 * grp + j; });
          tile_store(sDT, b1, 16 + c, [&](int j) { return 32 * ks + 8 * grp + j; });
        }
#pragma unroll
        for (int u = 0; u < RPW; ++u) {
          acc[0][u] = nb_mfma_bf16(wt[u][ks], b0, acc[0][u]);
          acc[1][u] = nb_mfma_bf16(wt[u][ks], b1, acc[1][u]);
        }
      }
      // stores: the lanes of rows g and g ^ 1 (same query) swap one row
      // block's values (v_permlane16_swap), so that every lane writes 16
      // bytes: 8 consecutive neurons of row block RPW w + 2h (even g) or
      // RPW w + 2h + 1 (odd g)
      typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
      typedef __attribute__((address_space(1))) u32x4* gst_t;
      gst_t out = (gst_t)(Dprev + r0 * W);
      asm volatile("" : "+s"(out));
      const bool oddrow = grp & 1;
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) {
        const int q = 16 * nb + c;
#pragma unroll
        for (int h = 0; h < H; ++h) {   // row blocks RPW w + 2h, + 1: one 16-byte piece of A_{l-1}
          const int kp = H * wave + h;
          const bf16x8 av = ring_chunk(sA, q, 4 * kp + grp);
          tile_store(sAT, av, q, [&](int j) { return 16 * (2 * kp + j / 4) + 4 * grp + (j & 3); });
          const nb_uint4 au = __builtin_bit_cast(nb_uint4, av);
          uint2 pk[2];
#pragma unroll
          for (int e = 0; e < 2; ++e) {
            const int u = 2 * h + e;
            float a[4];
            unpack4(e ? uint2{au[2], au[3]} : uint2{au[0], au[1]}, a);
            pk[e] = pack4(a[0] > 0.0f ? acc[nb][u][0] : 0.0f, a[1] > 0.0f ? acc[nb][u][1] : 0.0f,
                          a[2] > 0.0f ? acc[nb][u][2] : 0.0f, a[3] > 0.0f ? acc[nb][u][3] : 0.0f);
          }
          const auto sx = __builtin_amdgcn_permlane16_swap(pk[0].x, pk[1].x, false, false);
          const auto sy = __builtin_amdgcn_permlane16_swap(pk[0].y, pk[1].y, false, false);
          const int mo = RPW * wave + 2 * h + (oddrow ? 1 : 0);
          out[((int64_t)q * W + 16 * mo + 4 * (grp & ~1)) / 8] = u32x4{sx[0], sy[0], sx[1], sy[1]};
        }
      }
    }
    lds_barrier();   // the transposed tiles are complete
    // dW_l += D_l A_{l-1}^T, db_l += D_l 1 over the 32 queries (K)
    {
      typedef const __attribute__((address_space(3))) bf16x8* lop_t;
      const int rd_off = c * 32 + ((grp ^ ((c >> 1) & 3)) << 3);   // row 16 b + c, chunk grp
      lop_t dt = (lop_t)(sDT + rd_off);
      lop_t at = (lop_t)(sAT + rd_off);
      bf16x8 af[RPW];
#pragma unroll
      for (int a = 0; a < RPW; ++a) af[a] = dt[(16 * (RPW * wave + a)) * 32 / 8];
#pragma unroll
      for (int b = 0; b < 16; ++b) {
        const bf16x8 bf = at[(16 * b) * 32 / 8];
#pragma unroll
        for (int a = 0; a < RPW; ++a) dw[a][b] = nb_mfma_bf16(af[a], bf, dw[a][b]);
      }
#pragma unroll
      for (int a = 0; a < RPW; ++a) db[a] = nb_mfma_bf16(af[a], ones, db[a]);
    }
  }

  // the chunk's partial: the wave's weight-gradient tiles and bias rows
  const int c = c0, grp = grp0;
  float* out = partial + (int64_t)blockIdx.x * P;
  const int64_t wo = nb_w_off(l, in_dim, W);
#pragma unroll
  for (int a = 0; a < RPW; ++a)
#pragma unroll
    for (int b = 0; b < 16; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        out[wo + (int64_t)(16 * (RPW * wave + a) + 4 * grp + r) * W + 16 * b + c] = dw[a][b][r];
  if (c == 0) {
    const int64_t bo = nb_b_off(l, in_dim, W, NH);
#pragma unroll
    for (int a = 0; a < RPW; ++a)
#pragma unroll
      for (int r = 0; r < 4; ++r) out[bo + 16 * (RPW * wave + a) + 4 * grp + r] = db[a][r];
  }
}
}  // namespace

// Up to six hidden layers: the biases of seven or eight no longer fit the
// LDS beside the two streamed half-layers, the first layer and the inputs.
bool bf16_stream_forward_supported(int in_dim, int n_hidden, int width) {
  return width == 256 && in_dim >= 1 && in_dim <= 8 && n_hidden >= 2 && n_hidden <= 6;
}

nb_status bf16_back256(const Back256Job& J, hipStream_t s) {
  if (J.plan.chunk % Back256::QS != 0) {
    nb_set_error("backward layer kernel: chunk of %lld queries is not a multiple of 32", (long long)J.plan.chunk);
    return NB_ERR_UNSUPPORTED;
  }
  constexpr int WV = Back256::WAVES;
  NB_TRY(allow_lds(k_tr_back<WV>, Back256::lds_bytes()));
  k_tr_back<WV><<<(unsigned)J.plan.n_wg, 64 * WV, Back256::lds_bytes(), s>>>(
      J.Dl, J.Aprev, J.plan.chunk, J.l, J.in_dim, J.NH, J.packT, J.Dprev, J.P, J.partial);
  NB_LAUNCHED();
  return NB_OK;
}

nb_status bf16_recompute256(const RecomputeJob& J, hipStream_t s) {
  using S = TrStream<6>;
  const int nl = J.l1 - J.l0 + 1;
  if (J.l0 < 1 || nl < 1 || J.l1 > J.NH - 2 || J.plan.chunk % 32 != 0) {
    nb_set_error("recomputation kernel: unsupported segment %d .. %d", J.l0, J.l1);
    return NB_ERR_UNSUPPORTED;
  }
  const size_t lds = (size_t)2 * S::HALF * 64 * 16 + (size_t)nl * 256 * 4;
  if (lds > 160 * 1024) {
    nb_set_error("recomputation kernel: a segment of %d layers does not fit the LDS", nl);
    return NB_ERR_UNSUPPORTED;
  }
  NB_TRY(allow_lds(k_tr_recompute, 160 * 1024));
  k_tr_recompute<<<(unsigned)J.plan.n_wg, S::THREADS, lds, s>>>(J.ain, J.plan.chunk, J.l0, J.l1, J.in_dim, J.NH,
                                                              J.pack, J.theta, J.act, J.act_stride, J.slots);
  NB_LAUNCHED();
  return NB_OK;
}

nb_status bf16_stream_forward(const StreamJob& J, hipStream_t s) {
  if (!bf16_stream_forward_supported(J.in_dim, J.NH, 256) || J.plan.chunk % 16 != 0) {
    nb_set_error("streamed training forward: unsupported shape (in_dim %d, %d hidden layers)", J.in_dim, J.NH);
    return NB_ERR_UNSUPPORTED;
  }
  switch (J.NH) {
    case 2: return stream_launch<2>(J, s);
    case 3: return stream_launch<3>(J, s);
    case 4: return stream_launch<4>(J, s);
    case 5: return stream_launch<5>(J, s);
    default: return stream_launch<6>(J, s);
  }
}
