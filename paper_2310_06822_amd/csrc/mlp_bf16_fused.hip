// Fused bfloat16 training step (Alg. 1 steps 4-5: forward, Eq. 1 and its
// gradient, backward) for widths 32..128 and 2..4 hidden layers.  One
// workgroup of four waves takes one chunk of the batch, in tiles of 128
// queries (two blocks of 16 per wave), and keeps everything of a tile on
// the chip: activations and back-propagated gradients stay in registers,
// only the inputs and labels are read from HBM and one gradient partial per
// chunk is written.
//
// The rounding points are those of the layer-wise kernels: first layer at
// float32 accuracy (three bfloat16 pieces per value), bfloat16 hidden
// activations A_l and gradients D_l, float32 output layer and loss.
//
// Weights.  The layers' fragments stream through two LDS buffers, one
// layer per stage, the next stage's copied straight from global memory
// (L2) into the idle buffer while the current one computes.  Stages of a
// tile: forward layers 1 .. NH-1 (the last one with the output layer and
// Eq. 1), then the transposed layers NH-1 .. 1 for the data gradient
//   D_{l-1} = (W_l^T D_l) [A_{l-1} > 0],
// whose fragments are packed with the reduction over W_l's outputs in
// "operand order" (nb_op_neuron), the order in which a lane already holds
// D_l after the previous products.
//
// Weight gradients dW_l = sum_q D_l[q] A_{l-1}[q]^T need the queries on the
// MFMA's K dimension: each backward stage writes D_l and A_{l-1} of the
// tile's 128 queries transposed into LDS ([neuron][query] rows), and after
// a barrier every wave multiplies its share of the 16 x 16 output tiles
// (whole row blocks), K = 128 queries, accumulating in float32.  Bias
// gradients come from the same D_l fragments times a fragment of ones; the
// first layer's dW_0 from D_0 times the three bfloat16 pieces of every
// input (and a row of ones for db_0), summed piece by piece at the end.
// Up to 64 accumulator registers per lane the weight-gradient tiles stay in
// registers for the whole chunk; beyond that (width 128 with 3 or 4 hidden
// layers) each wave adds its tiles into the chunk's partial buffer once per
// tile of queries -- in tile order while the chunk runs, in parameter
// order on the last tile (a wave's row blocks cover the same addresses in
// both orders) -- so that only the wave that owns them ever touches them.
//
// Every sum has a fixed order (queries within a tile by the MFMA, tiles in
// sequence, waves in index order), so a step is bit-reproducible.
#include <algorithm>

#include "nb_bf16_train.h"

namespace {

// Waves per workgroup (WV): eight single-block waves or four two-block
// waves; a tile is 128 queries either way.
template <int W>
constexpr int fz_waves() { return W >= 128 ? 8 : 4; }

template <int W, int NH, int WV>
struct Fz {
  static constexpr int RB = W / 16, KS = W / 32, FH = RB * KS;
  // width 128: eight waves of one block of 16 queries (two waves per SIMD,
  // 256 registers each); narrower: four waves of two blocks, two or more
  // workgroups per CU.  A tile is 128 queries either way.
  static constexpr int WAVES = WV, NB = 8 / WV, THREADS = 64 * WAVES;
  static constexpr int Q = 16 * NB * WAVES;   // queries per tile
  static constexpr int GW = (RB * 4 + 15) / 16;   // output-weight gradient values per lane
  static constexpr int KQ = Q / 32;           // K = 32 steps over a tile's queries
  static constexpr int QP = Q + 8;            // LDS row stride (bfloat16) of the transposed tiles
  static constexpr int TILES = RB * RB, TPW = TILES / WAVES;   // 16 x 16 weight-gradient tiles per wave
  // hidden layers whose weight-gradient tiles stay in registers for the
  // whole chunk: all of them if they fit 64 accumulator registers, otherwise
  // as many as fit beside one layer's tiles in flight from the chunk's
  // partial (the others' go through the partial once per tile)
  static constexpr int NREG = TPW * 4 * (NH - 1) <= 64 ? NH - 1 : (64 - TPW * 4) / (TPW * 4);
  static constexpr int RW = TPW >= RB ? TPW / RB : 1;          // row blocks per wave (whole rows if TPW >= RB)
  static constexpr int R0 = (RB + WAVES - 1) / WAVES;          // first-layer gradient row blocks per wave
  static constexpr int XROWS = 32;   // input-piece rows: 3 in_dim + 1 <= 25, read as two 16-row B tiles
  static constexpr int NBIAS = NH * W + W + 1;
  // LDS: two streamed-layer buffers | biases, output weights | D^T | A^T |
  // first-layer fragments (both steps) | input pieces and ones (x^T)
  static constexpr size_t OFF_B = (size_t)2 * FH * 64 * 16;
  static constexpr size_t OFF_DT = (OFF_B + (size_t)NBIAS * 4 + 15) / 16 * 16;
  static constexpr size_t OFF_AT = OFF_DT + (size_t)W * QP * 2;
  static constexpr size_t OFF_F1 = OFF_AT + (size_t)W * QP * 2;
  static constexpr size_t OFF_X = OFF_F1 + (size_t)2 * RB * 64 * 16;
  static constexpr size_t LDS = OFF_X + (size_t)XROWS * QP * 2;
  static_assert(TILES % WAVES == 0, "weight-gradient tiles must split evenly over the waves");
  static_assert(TPW < RB ? TPW == 1 : TPW % RB == 0, "a wave owns one tile or whole row blocks");
  // the end-of-chunk reduction reuses the transposed tiles' LDS
  static_assert(((size_t)(W + 8) + WAVES * 8 + (size_t)W * 32) * 4 <= OFF_F1 - OFF_DT, "reduction scratch");
  static_assert(LDS <= 160 * 1024, "fused training exceeds the CU's LDS");
  static_assert(WV == 4 || WV == 8, "four or eight waves");
};

// Eight float32 values rounded to bfloat16 (nearest even), as an operand.
__device__ __forceinline__ bf16x8 to_bf16x8(const float (&v)[8]) {
  nb_uint4 u;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const nb_float2 f = {v[2 * p], v[2 * p + 1]};
    u[p] = __builtin_bit_cast(unsigned, __builtin_convertvector(f, nb_bf16x2));
  }
  return __builtin_bit_cast(bf16x8, u);
}

__device__ __forceinline__ uint16_t elem_bits(bf16x8 v, int j) {
  const nb_uint4 u = __builtin_bit_cast(nb_uint4, v);
  return (uint16_t)(u[j >> 1] >> (16 * (j & 1)));
}

// Writes the operands op[nb][ks] of the wave's query blocks into a
// [neuron][query] tile: element j of operand ks is neuron
// nb_op_neuron(32 ks + 8 g + j), the lane's query column c of block nb.
//
// Dword m of an operand holds elements 2m and 2m + 1 (two neurons) of the
// lane's query; the lanes of queries c and c ^ 1 swap halves (one DPP move
// and one byte permute) so that the even lane writes neuron 2m and the odd
// lane neuron 2m + 1, each for both queries, as one 32-bit store.
template <int NB, int KS, int QP>
__device__ __forceinline__ void store_transposed(uint16_t* __restrict__ dst, const bf16x8 (&op)[NB][KS], int col0,
                                                 int grp, int c) {
  const int odd = c & 1;
  // one per-lane base (opaque, so that every store is base + immediate):
  // row 4 g (+ 1 for the odd lane, its neuron 2m + 1), columns c & ~1, c | 1
  int lb = ((4 * grp + odd) * QP + col0 + (c & ~1)) * 2;
  asm volatile("" : "+v"(lb));
  unsigned char* b = reinterpret_cast<unsigned char*>(dst) + lb;
  // v_perm_b32 selectors: even lane (own low half, partner's low half),
  // odd lane (partner's high half, own high half)
  const unsigned sel = odd ? 0x03020706u : 0x05040100u;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const nb_uint4 u = __builtin_bit_cast(nb_uint4, op[nb][ks]);
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const unsigned pu = (unsigned)__builtin_amdgcn_mov_dpp((int)u[m], 0xB1, 0xF, 0xF, false);   // lane c ^ 1
        const unsigned w = __builtin_amdgcn_perm(pu, u[m], sel);
        // elements 2m, 2m + 1: neurons 32 ks + 16 (m / 2) + 4 g + 2 (m % 2) (+ 1)
        *reinterpret_cast<unsigned*>(b + ((32 * ks + 16 * (m >> 1) + 2 * (m & 1)) * QP + nb * 16) * 2) = w;
      }
    }
}

__device__ __forceinline__ bf16x8 lds16(const uint16_t* p) { return *reinterpret_cast<const bf16x8*>(p); }

// acc[nb][mo] += sum_ks W(mo, ks) op[nb][ks] over one layer's fragments fw
// (lane offset included): row blocks in groups of up to four with the K
// steps outermost, so that every group keeps four (x NB) independent
// accumulation chains in flight, and two fragment slots, so that the next K
// step's fragments load while the current one's products issue.  `between`
// runs after each group (work to interleave with the products).
template <int RB, int KS, int NB, class Between>
__device__ __forceinline__ void layer_products(const bf16x8* __restrict__ fw, const bf16x8 (&op)[NB][KS],
                                               floatx4 (&acc)[NB][RB], Between&& between) {
  constexpr int G = RB < 4 ? RB : 4;
#pragma unroll
  for (int m0 = 0; m0 < RB; m0 += G) {
    bf16x8 fa[G], fb[G];
#pragma unroll
    for (int u = 0; u < G; ++u) fa[u] = fw[((m0 + u) * KS) * 64];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      bf16x8(&cur)[G] = (ks & 1) ? fb : fa;
      bf16x8(&nxt)[G] = (ks & 1) ? fa : fb;
      if (ks + 1 < KS) {
#pragma unroll
        for (int u = 0; u < G; ++u) nxt[u] = fw[((m0 + u) * KS + ks + 1) * 64];
      }
#pragma unroll
      for (int u = 0; u < G; ++u)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb][m0 + u] = nb_mfma_bf16(cur[u], op[nb][ks], acc[nb][m0 + u]);
    }
    between(m0 / G);
    __builtin_amdgcn_sched_barrier(0);
  }
}

// A wave-uniform global-memory pointer the compiler cannot see through:
// addresses formed from it are computed where they are used instead of
// being hoisted out of the tile loop and held in registers.  (Returned in
// the global address space, so that accesses stay global, not flat.)
template <class T>
using gptr = __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ gptr<T> opaque(T* p) {
  gptr<T> g = (gptr<T>)p;
  asm volatile("" : "+s"(g));
  return g;
}

template <int W, int NH, int WV>
__global__ __launch_bounds__(64 * WV, (WV == 8 || W >= 128 ? 1 : 2)) void k_tr_fused(
    const float* __restrict__ q, const uint8_t* __restrict__ y, int64_t n, int64_t CH, int in_dim,
    const bf16x8* __restrict__ pack, const bf16x8* __restrict__ packT, const float* __restrict__ theta, float alpha,
    float beta, float inv_n, float tau, float* __restrict__ partial, float* __restrict__ aux, TrObjs TO) {
  using F = Fz<W, NH, WV>;
  constexpr int RB = F::RB, KS = F::KS, FH = F::FH, NB = F::NB, WAVES = F::WAVES, Q = F::Q, QP = F::QP;
  constexpr int TPW = F::TPW, RW = F::RW, R0 = F::R0, KQ = F::KQ, GW = F::GW;
  constexpr int NREG = F::NREG;
  auto in_regs = [](int l) { return l - 1 < NREG; };   // layer l's tiles in registers
  const TrObj ob = tr_obj(TO);
  const int64_t P = ob.P;
  pack += TO.pkoff ? TO.pkoff[ob.o] : 0;
  packT += TO.ptoff ? TO.ptoff[ob.o] : 0;
  theta += ob.poff;
  q += ob.o * TO.q_stride * in_dim;
  y += ob.o * TO.q_stride;
  if (TO.alpha) alpha = TO.alpha[ob.o];
  partial += (int64_t)gridDim.x * ob.poff;
  aux += (int64_t)ob.o * gridDim.x * 8;
  float* out = partial + (int64_t)blockIdx.x * P;

  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  // region offsets the compiler cannot fold into the constant part of an
  // access: every LDS access is then a region base register plus an
  // immediate below 64 KB (the instruction's offset field), instead of one
  // address register per distinct offset
  int obias = (int)F::OFF_B, odt = (int)F::OFF_DT, oat = (int)F::OFF_AT, of1 = (int)F::OFF_F1, ox = (int)F::OFF_X;
  asm volatile("" : "+s"(obias), "+s"(odt), "+s"(oat), "+s"(of1), "+s"(ox));
  bf16x8* sW = reinterpret_cast<bf16x8*>(smem_raw);
  float* sb = reinterpret_cast<float*>(smem_raw + obias);
  uint16_t* sDt = reinterpret_cast<uint16_t*>(smem_raw + odt);
  uint16_t* sAt = reinterpret_cast<uint16_t*>(smem_raw + oat);
  bf16x8* sF1 = reinterpret_cast<bf16x8*>(smem_raw + of1);
  uint16_t* sX = reinterpret_cast<uint16_t*>(smem_raw + ox);
  const float* swo = sb + NH * W;

  const int lane = threadIdx.x & 63, c = lane & 15, grp = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform: scalar registers
  const bool wide = in_dim > 4;
  const int64_t base = (int64_t)blockIdx.x * CH;
  const int64_t vend = base + CH < n ? base + CH : n;   // rows of this chunk that are queries
  const int iters = (int)((CH + Q - 1) / Q);
  constexpr int NST = 2 * (NH - 1);

  // stage s of a tile (0 .. NST-1): forward layer s + 1 for s < NH - 1, then
  // the transposed layers NH - 1 .. 1; stage s computes from buffer s % 2
  // (NST is even, so the parity holds across tiles)
  auto stage_src = [&](int s) -> const bf16x8* {
    return s < NH - 1 ? pack + (int64_t)(RB + s * FH) * 64 : packT + (int64_t)(NST - 1 - s) * FH * 64;
  };
  // global_load_lds: lane i of a wave fills the i-th 16-byte slot after the
  // wave-uniform LDS base; waited for before the end-of-stage barrier.  The
  // stage's source is made opaque so that its per-slot addresses are formed
  // here and not kept in registers across the loop.
  auto prefetch = [&](int s) {
    const gptr<const bf16x8> src = opaque(stage_src(s)) + lane;
    bf16x8* dst = sW + (s & 1) * FH * 64;
    constexpr int SL = FH * 64;
#pragma unroll
    for (int i = 0; i < (SL + F::THREADS - 1) / F::THREADS; ++i) {
      const int slot = i * F::THREADS + wave * 64;
      if (SL % F::THREADS == 0 || slot < SL)
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(src + slot),
                                         (__attribute__((address_space(3))) void*)(dst + slot), 16, 0, 0);
    }
  };
  {
    const bf16x8* src = stage_src(0);
    for (int i = threadIdx.x; i < FH * 64; i += F::THREADS) sW[i] = src[i];
    for (int i = threadIdx.x; i < NH * W; i += F::THREADS) sb[i] = theta[nb_b_off(i / W, in_dim, W, NH) + i % W];
    for (int i = threadIdx.x; i < W + 1; i += F::THREADS) sb[NH * W + i] = theta[nb_w_off(NH, in_dim, W) + i];
    // first layer: step 0, then (in_dim > 4) step 1, which follows the hidden layers in the pack
    for (int i = threadIdx.x; i < RB * 64; i += F::THREADS) {
      sF1[i] = pack[i];
      if (wide) sF1[RB * 64 + i] = pack[(RB + (NH - 1) * FH) * 64 + i];
    }
    for (int i = threadIdx.x; i < Q; i += F::THREADS) sX[3 * in_dim * QP + i] = 0x3F80;   // 1.0: db_0
  }
  __syncthreads();

  const floatx4 zero4 = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
  const bf16x8 ones = __builtin_bit_cast(bf16x8, nb_uint4{0x3F803F80u, 0x3F803F80u, 0x3F803F80u, 0x3F803F80u});
  // output-weight gradient: lane c keeps the values i = c + 16 k (i = 4 mo + r:
  // neuron 16 mo + 4 g + r) of every tile's row sums
  float gwo[GW];
#pragma unroll
  for (int k = 0; k < GW; ++k) gwo[k] = 0.0f;
  float gbo = 0.0f, lsum = 0.0f;
  unsigned cnt[4] = {0u, 0u, 0u, 0u};
  floatx4 dbh[NH - 1][RW];                        // hidden-layer bias gradients of the wave's row blocks
  floatx4 dwr[NREG > 0 ? NREG : 1][TPW];         // weight gradients kept in registers (layers 1 .. NREG)
  floatx4 dw0[R0][2];                            // first-layer gradient tiles
#pragma unroll
  for (int l = 0; l < NH - 1; ++l)
#pragma unroll
    for (int i = 0; i < RW; ++i) dbh[l][i] = zero4;
#pragma unroll
  for (int l = 0; l < (NREG > 0 ? NREG : 1); ++l)
#pragma unroll
    for (int t = 0; t < TPW; ++t) dwr[l][t] = zero4;
#pragma unroll
  for (int i = 0; i < R0; ++i) dw0[i][0] = dw0[i][1] = zero4;

  const int col0 = wave * NB * 16;   // the wave's first query column in a tile
  // a tile's inputs and labels, loaded one tile ahead (during the previous
  // tile's backward pass) as they are: rows past the chunk's queries read
  // the chunk's last query (every load in bounds, none under a branch) and
  // are zeroed where the tile uses them, so that no instruction waits for
  // the loads before then
  float xraw[NB][8];
  uint8_t yraw[NB];
  auto load_inputs = [&](int tile) {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int64_t qi = base + (int64_t)tile * Q + col0 + nb * 16 + c;
      const int64_t qr = qi < vend ? qi : vend - 1;
#pragma unroll
      for (int j = 0; j < 8; ++j) xraw[nb][j] = q[qr * in_dim + (j < in_dim ? j : in_dim - 1)];
      yraw[nb] = y[qr];
    }
  };
  load_inputs(0);
  for (int it = 0; it < iters; ++it) {
    const int64_t q0 = base + (int64_t)it * Q + col0;
    const bool last_tile = it + 1 == iters;
    float xr[NB][8];
    int ylab[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const bool valid = q0 + nb * 16 + c < vend;
#pragma unroll
      for (int j = 0; j < 8; ++j) xr[nb][j] = (valid && j < in_dim) ? xraw[nb][j] : 0.0f;
      ylab[nb] = valid ? (int)yraw[nb] : 0;
    }
    bf16x8 act[NH - 1][NB][KS];   // A_0 .. A_{NH-2}
    bf16x8 dop[NB][KS];           // D_l as the B operand of the next products
    floatx4 acc[NB][RB];
    // ---- first layer
    {
      bf16x8 xb[NB], xb1[NB];
      nb_first_operands<NB>(xr, grp, wide, xb, xb1);
#pragma unroll
      for (int mo = 0; mo < RB; ++mo) {
        const floatx4 bi = *reinterpret_cast<const floatx4*>(sb + 16 * mo + 4 * grp);
        const bf16x8 a = sF1[mo * 64 + lane];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb][mo] = nb_mfma_bf16(a, xb[nb], bi);
      }
      if (wide) {
#pragma unroll
        for (int mo = 0; mo < RB; ++mo) {
          const bf16x8 a = sF1[(RB + mo) * 64 + lane];
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) acc[nb][mo] = nb_mfma_bf16(a, xb1[nb], acc[nb][mo]);
        }
      }
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          float v[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) v[j] = acc[nb][2 * ks + j / 4][j % 4];
          act[0][nb][ks] = nb_relu_bf16x8(v);
        }
    }
    // ---- forward stages: hidden layers 1 .. NH-1, the last with the head
#pragma unroll
    for (int l = 1; l < NH; ++l) {
      const int st = l - 1;
      prefetch(st + 1);
      const bf16x8* fw = sW + (st & 1) * FH * 64 + lane;
#pragma unroll
      for (int mo = 0; mo < RB; ++mo) {
        const floatx4 bi = *reinterpret_cast<const floatx4*>(sb + l * W + 16 * mo + 4 * grp);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb][mo] = bi;
      }
      layer_products<RB, KS, NB>(fw, act[l - 1], acc, [](int) {});
      if (l < NH - 1) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
          for (int ks = 0; ks < KS; ++ks) {
            float v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = acc[nb][2 * ks + j / 4][j % 4];
            act[l][nb][ks] = nb_relu_bf16x8(v);
          }
      } else {
        // output layer, Eq. 1 and dL/dz; D_{NH-1} = dz w_out [a > 0]
        float gt[RB * 4];   // this tile's dz relu(a) per lane, summed over the wave's blocks
#pragma unroll
        for (int i = 0; i < RB * 4; ++i) gt[i] = 0.0f;
        // the lane's output weights, read once (a read under the ReLU select
        // below would become a branch around each LDS load)
        floatx4 wo4[RB];
#pragma unroll
        for (int mo = 0; mo < RB; ++mo) wo4[mo] = *reinterpret_cast<const floatx4*>(swo + 16 * mo + 4 * grp);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          float p = 0.0f;
#pragma unroll
          for (int mo = 0; mo < RB; ++mo)
#pragma unroll
            for (int r = 0; r < 4; ++r) p = fmaf(wo4[mo][r], nb_relu(acc[nb][mo][r]), p);
          p += __shfl_xor(p, 16);
          p += __shfl_xor(p, 32);
          const float z = p + swo[W];
          const int64_t qi = q0 + nb * 16 + c;
          const bool valid = qi < vend;
          const bool yv = ylab[nb] != 0;
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
#pragma unroll
          for (int ks = 0; ks < KS; ++ks) {
            float d[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
              const int mo = 2 * ks + j / 4, r = j % 4;
              const float a = fmaxf(acc[nb][mo][r], 0.0f);
              gt[mo * 4 + r] = fmaf(dz, a, gt[mo * 4 + r]);
              const float dw = dz * wo4[mo][r];
              d[j] = acc[nb][mo][r] > 0.0f ? dw : 0.0f;
            }
            dop[nb][ks] = to_bf16x8(d);
          }
        }
        {
          constexpr int V = RB * 4 < 16 ? 16 : RB * 4;
          float gv[V], sums[V / 16];
#pragma unroll
          for (int i = 0; i < V; ++i) gv[i] = i < RB * 4 ? gt[i] : 0.0f;
          nb_row_reduce_scatter<V>(gv, c, sums);
#pragma unroll
          for (int k = 0; k < GW; ++k) gwo[k] += sums[k];
        }
      }
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();
      if (l == 1) {
        // x^T for dW_0: the three pieces of every input (rows 3 f .. 3 f + 2);
        // the previous tile's readers of these rows have all passed the
        // barrier above
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const int col = col0 + nb * 16 + c;
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int f = grp + 4 * h;
            if (f < in_dim) {
              const float x = xr[nb][f];
              const float x1 = __uint_as_float(__float_as_uint(x) & 0xFFFF0000u);
              const float rr = x - x1;
              const float x2 = __uint_as_float(__float_as_uint(rr) & 0xFFFF0000u);
              const float x3 = rr - x2;
              sX[(3 * f) * QP + col] = nb_hi16(x1);
              sX[(3 * f + 1) * QP + col] = nb_hi16(x2);
              sX[(3 * f + 2) * QP + col] = nb_hi16(x3);
            }
          }
        }
      }
    }
    // ---- backward stages: layers NH-1 .. 1
#pragma unroll
    for (int l = NH - 1; l >= 1; --l) {
      const int st = NST - l;
      if (st + 1 < NST) prefetch(st + 1);
      else if (!last_tile) prefetch(0);
      if (l == NH - 1 && !last_tile) load_inputs(it + 1);   // this tile's inputs and labels are used up
      const bf16x8* fw = sW + (st & 1) * FH * 64 + lane;
      // partials of this layer's weight-gradient tiles (kept in memory):
      // loaded here so that the transposes and the data gradient cover
      // their latency
      floatx4 dwm[TPW];
      const gptr<float> R = opaque(out + nb_w_off(l, in_dim, W));
      const int lr = in_regs(l) ? l - 1 : 0;   // (l is a constant here: the loop is unrolled)
      if (!in_regs(l)) {
        if (it == 0) {
#pragma unroll
          for (int t = 0; t < TPW; ++t) dwm[t] = zero4;
        } else {
#pragma unroll
          for (int t = 0; t < TPW; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) dwm[t][r] = R[(int64_t)(wave * TPW + t) * 256 + lane * 4 + r];
        }
      }
      // D_{l-1} = (W_l^T D_l) [A_{l-1} > 0]; the transposes of D_l and
      // A_{l-1} for the weight gradient are written between the row-block
      // groups' products (the LDS stores issue while the products run)
#pragma unroll
      for (int mo = 0; mo < RB; ++mo)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb][mo] = zero4;
      {
        constexpr int NGRP = RB < 4 ? 1 : RB / 4;
        layer_products<RB, KS, NB>(fw, dop, acc, [&](int gi) {
          if (NGRP == 1) {
            store_transposed<NB, KS, QP>(sDt, dop, col0, grp, c);
            store_transposed<NB, KS, QP>(sAt, act[l - 1], col0, grp, c);
          } else if (gi == 0) {
            store_transposed<NB, KS, QP>(sDt, dop, col0, grp, c);
          } else if (gi == 1) {
            store_transposed<NB, KS, QP>(sAt, act[l - 1], col0, grp, c);
          }
        });
      }
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          float d[8];
#pragma unroll
          for (int j = 0; j < 8; ++j)
            d[j] = (int16_t)elem_bits(act[l - 1][nb][ks], j) > 0 ? acc[nb][2 * ks + j / 4][j % 4] : 0.0f;
          dop[nb][ks] = to_bf16x8(d);
        }
      __syncthreads();
      // dW_l += D_l A_{l-1}^T and db_l += D_l 1 over the tile's queries
      {
        floatx4 dw[TPW];
#pragma unroll
        for (int t = 0; t < TPW; ++t) dw[t] = in_regs(l) ? dwr[lr][t] : dwm[t];
#pragma unroll
        for (int s = 0; s < KQ; ++s) {
          if constexpr (TPW >= RB) {
            bf16x8 a[RW];
#pragma unroll
            for (int i = 0; i < RW; ++i) a[i] = lds16(sDt + (16 * (wave * RW + i) + c) * QP + 32 * s + 8 * grp);
            // the column blocks' B fragments in groups of four (fewer live registers)
            constexpr int KG = RB >= 4 ? 4 : RB;
#pragma unroll
            for (int k0 = 0; k0 < RB; k0 += KG) {
              bf16x8 b[KG];
#pragma unroll
              for (int k = 0; k < KG; ++k) b[k] = lds16(sAt + (16 * (k0 + k) + c) * QP + 32 * s + 8 * grp);
#pragma unroll
              for (int i = 0; i < RW; ++i)
#pragma unroll
                for (int k = 0; k < KG; ++k) dw[i * RB + k0 + k] = nb_mfma_bf16(a[i], b[k], dw[i * RB + k0 + k]);
            }
#pragma unroll
            for (int i = 0; i < RW; ++i) dbh[l - 1][i] = nb_mfma_bf16(a[i], ones, dbh[l - 1][i]);
          } else {
            const int no = wave / RB, ko = wave % RB;
            const bf16x8 a = lds16(sDt + (16 * no + c) * QP + 32 * s + 8 * grp);
            const bf16x8 b = lds16(sAt + (16 * ko + c) * QP + 32 * s + 8 * grp);
            dw[0] = nb_mfma_bf16(a, b, dw[0]);
            if (ko == 0) dbh[l - 1][0] = nb_mfma_bf16(a, ones, dbh[l - 1][0]);
          }
          __builtin_amdgcn_sched_barrier(0);
        }
        if (in_regs(l)) {
#pragma unroll
          for (int t = 0; t < TPW; ++t) dwr[lr][t] = dw[t];
        } else {
          if (last_tile) {
#pragma unroll
            for (int t = 0; t < TPW; ++t) {
              const int T = wave * TPW + t, no = T / RB, ko = T % RB;
#pragma unroll
              for (int r = 0; r < 4; ++r) R[(int64_t)(16 * no + 4 * grp + r) * W + 16 * ko + c] = dw[t][r];
            }
          } else {
#pragma unroll
            for (int t = 0; t < TPW; ++t)
#pragma unroll
              for (int r = 0; r < 4; ++r) R[(int64_t)(wave * TPW + t) * 256 + lane * 4 + r] = dw[t][r];
          }
        }
      }
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();
    }
    // ---- first layer: dW_0 and db_0 from D_0 and the input pieces
    {
      store_transposed<NB, KS, QP>(sDt, dop, col0, grp, c);
      __syncthreads();
      const bool two = 3 * in_dim + 1 > 16;
#pragma unroll
      for (int s = 0; s < KQ; ++s) {
        const bf16x8 b0 = lds16(sX + c * QP + 32 * s + 8 * grp);
        const bf16x8 b1 = lds16(sX + (16 + c) * QP + 32 * s + 8 * grp);
#pragma unroll
        for (int i = 0; i < R0; ++i) {
          const int no = wave + i * WAVES;
          if (no < RB) {
            const bf16x8 a = lds16(sDt + (16 * no + c) * QP + 32 * s + 8 * grp);
            dw0[i][0] = nb_mfma_bf16(a, b0, dw0[i][0]);
            if (two) dw0[i][1] = nb_mfma_bf16(a, b1, dw0[i][1]);
          }
        }
      }
    }
  }
  __syncthreads();

  // ---- end of the chunk: fixed-order workgroup reductions, one partial
  float* red = reinterpret_cast<float*>(sDt);                      // [W + 1] output layer
  float* saux = red + W + 8;                                      // [WAVES][8] loss and counts
  float* red0 = saux + WAVES * 8;                                 // [W][32] first-layer tiles
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) {
    gbo += __shfl_xor(gbo, m);
    lsum += __shfl_xor(lsum, m);
  }
#pragma unroll
  for (int i = 0; i < R0; ++i) {
    const int no = wave + i * WAVES;
    if (no < RB)
#pragma unroll
      for (int t0 = 0; t0 < 2; ++t0)
#pragma unroll
        for (int r = 0; r < 4; ++r) red0[(16 * no + 4 * grp + r) * 32 + 16 * t0 + c] = dw0[i][t0][r];
  }
  for (int w = 0; w < WAVES; ++w) {
    if (wave == w) {
#pragma unroll
      for (int k = 0; k < GW; ++k) {
        const int i = c + 16 * k;
        if (i < RB * 4) {
          const int nrn = 16 * (i >> 2) + 4 * grp + (i & 3);
          red[nrn] = w == 0 ? gwo[k] : red[nrn] + gwo[k];
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
  for (int i = threadIdx.x; i < W + 1; i += F::THREADS) out[nb_w_off(NH, in_dim, W) + i] = red[i];
  if (threadIdx.x == 0) {
    float ls = 0.0f;
    unsigned cs[4] = {0u, 0u, 0u, 0u};
    for (int w = 0; w < WAVES; ++w) {
      ls += saux[w * 8];
      for (int i = 0; i < 4; ++i) cs[i] += __float_as_uint(saux[w * 8 + 1 + i]);
    }
    aux[blockIdx.x * 8] = ls;
    for (int i = 0; i < 4; ++i) aux[blockIdx.x * 8 + 1 + i] = __uint_as_float(cs[i]);
  }
  // dW_0[n][f] = the three piece columns of input f summed in order; db_0 the ones column
  for (int i = threadIdx.x; i < W * (in_dim + 1); i += F::THREADS) {
    const int nrn = i / (in_dim + 1), f = i % (in_dim + 1);
    const float* rw = red0 + nrn * 32;
    if (f < in_dim)
      out[(int64_t)nrn * in_dim + f] = (rw[3 * f] + rw[3 * f + 1]) + rw[3 * f + 2];
    else
      out[nb_b_off(0, in_dim, W, NH) + nrn] = rw[3 * in_dim];
  }
  // hidden layers: bias gradients (column 0 of the ones products) and the
  // weight gradients kept in registers
#pragma unroll
  for (int l = 1; l < NH; ++l) {
    if (c == 0) {
#pragma unroll
      for (int i = 0; i < RW; ++i) {
        const int no = TPW >= RB ? wave * RW + i : wave / RB;
        if (TPW >= RB || wave % RB == 0)
#pragma unroll
          for (int r = 0; r < 4; ++r) out[nb_b_off(l, in_dim, W, NH) + 16 * no + 4 * grp + r] = dbh[l - 1][i][r];
      }
    }
    if (in_regs(l)) {
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
        const int T = wave * TPW + t, no = T / RB, ko = T % RB;
#pragma unroll
        for (int r = 0; r < 4; ++r)
          out[nb_w_off(l, in_dim, W) + (int64_t)(16 * no + 4 * grp + r) * W + 16 * ko + c] =
              dwr[in_regs(l) ? l - 1 : 0][t][r];
      }
    }
  }
}

template <int W, int NH, int WV = fz_waves<W>()>
nb_status fused_launch(const FusedJob& J, hipStream_t s) {
  using F = Fz<W, NH, WV>;
  NB_TRY(allow_lds(k_tr_fused<W, NH, WV>, F::LDS));
  const dim3 grid((unsigned)J.plan.n_wg, (unsigned)J.members);
  k_tr_fused<W, NH, WV><<<grid, F::THREADS, F::LDS, s>>>(J.q, J.y, J.n, J.plan.chunk, J.in_dim, J.pack, J.packT,
                                                     J.theta, J.alpha, J.beta, J.inv_n, J.tau, J.partial, J.aux,
                                                     J.T);
  NB_LAUNCHED();
  return NB_OK;
}

template <int W>
nb_status fused_w(const FusedJob& J, hipStream_t s) {
  switch (J.NH) {
    case 2: return fused_launch<W, 2>(J, s);
    case 3: return fused_launch<W, 3>(J, s);
    case 4: return fused_launch<W, 4>(J, s);
    default: break;
  }
  nb_set_error("fused bfloat16 training has no kernel for %d hidden layers", J.NH);
  return NB_ERR_UNSUPPORTED;
}

}  // namespace

bool bf16_fused_supported(int in_dim, int n_hidden, int width) { return nb_bf16_fused_shape(in_dim, n_hidden, width); }

nb_status bf16_fused_train(const FusedJob& J, hipStream_t s) {
  if (!bf16_fused_supported(J.in_dim, J.NH, J.W)) {
    nb_set_error("fused bfloat16 training has no kernel for %d x %d^%d", J.in_dim, J.W, J.NH);
    return NB_ERR_UNSUPPORTED;
  }
  switch (J.W) {
    case 32: return fused_w<32>(J, s);
    case 64: return fused_w<64>(J, s);
    default: return fused_w<128>(J, s);
  }
}
