// Forward half of a bfloat16 training step for 256-wide bounds (Alg. 1
// step 4 and Eq. 1), one launch in place of the layer-wise first-layer,
// hidden-layer and head kernels.
//
// A 256-wide layer does not fit next to a second one in LDS, so, as in the
// streamed forward, every hidden layer streams through two 64 KiB LDS
// buffers in half-layer chunks (row blocks 0..7, then 8..15), copied straight
// from global memory into the idle buffer while the waves multiply the other
// one; the first layer's fragments and all biases stay resident.  One
// workgroup of 8 waves (two per SIMD) takes one chunk of the batch in tiles
// of 256 queries, two blocks of 16 per wave, so every streamed chunk serves
// 256 queries.
//
// What the backward kernels read goes to HBM: the activation rows A_l that
// are kept (all of them, or the checkpoints and the last segment when the
// backward recomputes the rest), in the same operand order and with the
// same bits as the layer-wise kernels write them, and D_{NH-1} = dL/dz w_out
// [a > 0] of the last hidden layer.  The output layer's gradient (w_out,
// b_out), the loss and the confusion counts of the chunk go to the chunk's
// partial; everything else of a tile stays on the chip.
//
// Rounding points and the order of every product are those of the
// layer-wise kernels (bias first, K steps in order; the output logit summed
// over row blocks in order), so the activations, the logits and D_{NH-1} are
// bit-identical to theirs.  The output-weight sums go through a per-block
// reduce-scatter over the 16 queries of a row and then the waves in order:
// deterministic, but summed in another order than the layer-wise head.
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
      if (q0 + nb * 16 < cend) {
        typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
        typedef __attribute__((address_space(1))) u32x2* gd_t;
        gd_t out = (gd_t)(Dout + (q0 + nb * 16) * W);
        asm volatile("" : "+s"(out));
        typedef const __attribute__((address_space(3))) float* lds_f;
        lds_f wo2 = (lds_f)(swo + 4 * grp);
        asm volatile("" : "+v"(wo2));
#pragma unroll
        for (int mo = 0; mo < RB; ++mo) {
          float w4[4], d[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) w4[r] = wo2[16 * mo + r];
          asm volatile("" : "+v"(w4[0]), "+v"(w4[1]), "+v"(w4[2]), "+v"(w4[3]));
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const float a = mo < RA ? acc0[nb][mo][r] : acc1[nb][mo - RA][r];
            d[r] = a > 0.0f ? dz * w4[r] : 0.0f;
          }
          const uint2 pk = pack4(d[0], d[1], d[2], d[3]);
          out[(c * W + 16 * mo + 4 * grp) / 4] = u32x2{pk.x, pk.y};
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

}  // namespace

// Up to six hidden layers: the biases of seven or eight no longer fit the
// LDS beside the two streamed half-layers, the first layer and the inputs.
bool bf16_stream_forward_supported(int in_dim, int n_hidden, int width) {
  return width == 256 && in_dim >= 1 && in_dim <= 8 && n_hidden >= 2 && n_hidden <= 6;
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
