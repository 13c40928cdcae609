// The bound h_theta as a bfloat16 MLP on the matrix cores (Sec. 3.4,
// "Architecture"; ReLU hidden layers), v_mfma_f32_16x16x32_bf16 with float32
// accumulation.
//
// Rounding points (the paper states no precision; bfloat16 operands with
// float32 accumulation where the work is, the small first and last layers
// at float32 accuracy):
//   first layer   each float32 weight and input cut exactly into three
//                 bfloat16 pieces; the six piece products that matter go
//                 through one K = 32 MFMA step (input dimension <= 4) or two
//                 (5..8); layout in nb_mlp.h.
//   hidden layers weights and input activations rounded to bfloat16.
//   output layer  float32 dot product of float32 activations.
//
// Register layout (as in the float32 kernel): neurons are MFMA rows, queries
// MFMA columns; after a layer, lane l holds neurons 16*mo + 4*(l/16) + r of
// query l % 16.  A K = 32 step of the next layer takes the 8 values of row
// blocks 2*ks and 2*ks + 1 that a lane already holds; the weight fragments
// are packed in that K order, one 16-byte slice per lane.
//
// Each wave works on NB blocks of 16 queries at once so that one 1 KiB weight
// fragment read from LDS feeds NB matrix-core instructions.
#include <algorithm>

#include "nb_internal.h"
#include "nb_mlp.h"
#include "nb_bf16_fwd.h"

namespace {

// ------------------------------------------------------------------ packing

// Forward fragment pack (layout in nb_bf16_pack_elem).
__global__ void k_pack_bf16(const float* __restrict__ theta, int in_dim, int W, int NH, uint16_t* __restrict__ pack,
                            int64_t total) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  pack[idx] = nb_bf16_pack_elem(theta, in_dim, W, NH, idx);
}

// ------------------------------------------------------------------ forward

template <int W, int NH, int NB, int THREADS>
__global__ __launch_bounds__(THREADS) void k_fwd_bf16(const float* __restrict__ q, int64_t n, int in_dim,
                                                  const bf16x8* __restrict__ pack, const float* __restrict__ theta,
                                                  float tau, float* __restrict__ logits, uint8_t* __restrict__ hout,
                                                  const uint8_t* __restrict__ g, unsigned long long* __restrict__ counts,
                                                  const unsigned long long* __restrict__ n_dev) {
  using N = B16<W, NH>;
  if (n_dev && (int64_t)*n_dev < n) n = (int64_t)*n_dev;   // rows counted on the device
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  bf16x8* swt = reinterpret_cast<bf16x8*>(smem_raw);
  float* sbias = reinterpret_cast<float*>(smem_raw + (size_t)N::NALL * 64 * 16);

  for (int i = threadIdx.x; i < N::NALL * 64; i += blockDim.x) swt[i] = pack[i];
  for (int i = threadIdx.x; i < NH * W; i += blockDim.x) sbias[i] = theta[nb_b_off(i / W, in_dim, W, NH) + i % W];
  for (int i = threadIdx.x; i < W + 1; i += blockDim.x) sbias[NH * W + i] = theta[nb_w_off(NH, in_dim, W) + i];
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int waves = blockDim.x >> 6;
  unsigned cnt[4] = {0u, 0u, 0u, 0u};
  const int64_t tiles = (n + NB * 16 - 1) / (NB * 16);
  // The first layer on the float32 matrix cores (16x16x4): lane group g
  // supplies features g and g + 4 of its query column, so a lane loads two
  // inputs per block and holds its slice of W_1 (rows 16 mo + c, columns g
  // and g + 4) in registers; the hidden layers and the output follow
  // bf16_fwd_rest.  Padding queries read the last row (no predicated loads)
  // and are zeroed.
  constexpr int RB = W / 16;
  const int c = lane & 15, grp = lane >> 4;
  const bool wide = in_dim > 4;
  float w1[RB][2];
#pragma unroll
  for (int mo = 0; mo < RB; ++mo)
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int k = grp + 4 * t;
      w1[mo][t] = k < in_dim ? theta[(int64_t)(16 * mo + c) * in_dim + k] : 0.0f;
    }
  const int f0 = grp < in_dim ? grp : in_dim - 1, f1 = grp + 4 < in_dim ? grp + 4 : in_dim - 1;
  for (int64_t tile = (int64_t)blockIdx.x * waves + (threadIdx.x >> 6); tile < tiles;
       tile += (int64_t)gridDim.x * waves) {
    const int64_t q0 = tile * NB * 16;
    float x[NB][2];
    bool bad[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int64_t qi = q0 + nb * 16 + c;
      const bool valid = qi < n;
      const float* row = q + (valid ? qi : n - 1) * in_dim;
      const float u0 = row[f0], u1 = row[f1];
      x[nb][0] = valid && grp < in_dim ? u0 : 0.0f;
      x[nb][1] = valid && grp + 4 < in_dim ? u1 : 0.0f;
      const unsigned long long m = __ballot(!isfinite(x[nb][0]) || !isfinite(x[nb][1]));
      bad[nb] = ((m | (m >> 16) | (m >> 32) | (m >> 48)) >> c) & 1ull;
    }
    floatx4 acc[NB][RB];
#pragma unroll
    for (int mo = 0; mo < RB; ++mo) {
      const floatx4 bi = *reinterpret_cast<const floatx4*>(sbias + 16 * mo + 4 * grp);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        acc[nb][mo] = __builtin_amdgcn_mfma_f32_16x16x4f32(w1[mo][0], x[nb][0], bi, 0, 0, 0);
    }
    if (wide) {
#pragma unroll
      for (int mo = 0; mo < RB; ++mo)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          acc[nb][mo] = __builtin_amdgcn_mfma_f32_16x16x4f32(w1[mo][1], x[nb][1], acc[nb][mo], 0, 0, 0);
    }
    bf16_fwd_rest<W, NH, NB>(acc, bad, swt, sbias, n, q0, tau, logits, hout, g, counts, cnt);
  }
  if (counts && lane == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (cnt[i]) atomicAdd(&counts[i], (unsigned long long)cnt[i]);
  }
}

template <int W, int NH, int NB, int THREADS>
nb_status fwd_launch(const nb_bound* b, const float* q, int64_t n, float tau, float* logits, uint8_t* h,
                     const uint8_t* g, unsigned long long* counts, const unsigned long long* n_dev, hipStream_t s) {
  using N = B16<W, NH>;
  const size_t lds = N::lds_bytes();
  static bool attr_set[64] = {false};
  int dev = 0;
  NB_HIP(hipGetDevice(&dev));
  if (dev >= 0 && dev < 64 && !attr_set[dev]) {
    NB_HIP(hipFuncSetAttribute((const void*)k_fwd_bf16<W, NH, NB, THREADS>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds));
    attr_set[dev] = true;
  }
  const int64_t tiles = (n + NB * 16 - 1) / (NB * 16);
  const int64_t want = (tiles + THREADS / 64 - 1) / (THREADS / 64);
  const int64_t per_cu = std::max<int64_t>(1, std::min<int64_t>(4, (160 * 1024) / (int64_t)lds));
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(want, per_cu * nb_cu_count()));
  k_fwd_bf16<W, NH, NB, THREADS><<<grid, THREADS, lds, s>>>(q, n, b->in_dim, reinterpret_cast<const bf16x8*>(b->pack16),
                                                    b->theta, tau, logits, h, g, counts, n_dev);
  NB_LAUNCHED();
  return NB_OK;
}

// (W, NH) instances with every hidden layer resident in LDS.
#define NB_BF16_CASES(X) \
  X(32, 1) X(32, 2) X(32, 3) X(32, 4) X(32, 5) X(32, 6) \
  X(64, 1) X(64, 2) X(64, 3) X(64, 4) X(64, 5) X(64, 6) \
  X(128, 1) X(128, 2) X(128, 3) X(128, 4) X(128, 5)

}  // namespace

bool bf16_supported(int in_dim, int n_hidden, int width) {
  if (in_dim < 1 || in_dim > 8) return false;
  if (width == 256) return n_hidden >= 2 && n_hidden <= 8;
#define X(WW, H) \
  if (width == WW && n_hidden == H) return true;
  NB_BF16_CASES(X)
#undef X
  return false;
}

int64_t bf16_pack_elems(int in_dim, int n_hidden, int width) {
  (void)in_dim;
  return nb_bf16_fwd_slices(width, n_hidden) * 8;
}

nb_status bf16_pack(const nb_bound* b, hipStream_t s) {
  const int64_t total = b->pack16_elems;
  k_pack_bf16<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(b->theta, b->in_dim, b->width, b->n_hidden,
                                                              b->pack16, total);
  NB_LAUNCHED();
  return NB_OK;
}

// ------------------------------------------------- width 256: streamed weights
//
// A 256-wide hidden layer is 128 KiB of bfloat16 fragments, so the layers
// stream through LDS in 64 KiB half-layer chunks (row blocks 0..7, then
// 8..15), double-buffered: while the waves multiply chunk c, chunk c + 1
// copies from global memory straight into the other buffer.  One workgroup
// per CU takes WAVES * NB * 16 queries per pass (4 waves x 3 blocks, or 8
// waves x 2 blocks: two waves per SIMD, each chunk serving 256 queries); the
// first-layer fragments and biases stay resident.
template <int NH, int NB_, int THREADS_>
struct Stream256 {
  static constexpr int W = 256, RB = 16, KS = 8, FH = RB * KS, HALF = FH / 2;
  static constexpr int NB = NB_, THREADS = THREADS_, WAVES = THREADS / 64;
  static constexpr int PER = HALF * 64 / THREADS;    // 16-byte fragment slices per thread per chunk
  static constexpr int IN_WAVE = NB * 16 * 8;        // staged input floats per wave (in_dim <= 8)
  static constexpr size_t bias_bytes() { return ((size_t)(NH * W + W + 1) * 4 + 15) / 16 * 16; }
  static constexpr size_t lds_bytes() {
    return (size_t)(RB * 64 + 2 * HALF * 64) * 16 + bias_bytes() + (size_t)WAVES * IN_WAVE * 4;
  }
};

// SPLIT: row blocks (of four) whose products precede the next K step's
// fragment loads; (NB, THREADS): blocks of 16 queries per wave and threads
// of the one workgroup per CU; HALVES: each half-layer's accumulators are
// rounded into the next layer's operands (or summed into the output logit)
// as soon as that half is done, before the chunk's barrier -- one half of
// the accumulators is live instead of the whole layer (tuning variants; all
// give identical results).
template <int NH, int SPLIT, int NB_, int THREADS_, bool HALVES = false>
__global__ __launch_bounds__(THREADS_, 1) void k_fwd_bf16_stream(const float* __restrict__ q, int64_t n, int in_dim,
                                                          const bf16x8* __restrict__ pack,
                                                          const float* __restrict__ theta, float tau,
                                                          float* __restrict__ logits, uint8_t* __restrict__ hout,
                                                          const uint8_t* __restrict__ g,
                                                          unsigned long long* __restrict__ counts,
                                                          const unsigned long long* __restrict__ n_dev) {
  using S = Stream256<NH, NB_, THREADS_>;
  if (n_dev && (int64_t)*n_dev < n) n = (int64_t)*n_dev;   // rows counted on the device
  constexpr int W = S::W, RB = S::RB, KS = S::KS, NB = S::NB;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  // LDS region offsets kept opaque (HALVES variants): every access is then a
  // region base register plus an immediate below 64 KB, not one address
  // register per distinct offset above 64 KB
  int obuf = RB * 64 * 16, obias = (RB * 64 + 2 * S::HALF * 64) * 16;
  if constexpr (HALVES) asm volatile("" : "+s"(obuf), "+s"(obias));
  bf16x8* sfirst = reinterpret_cast<bf16x8*>(smem_raw);
  bf16x8* sbuf = reinterpret_cast<bf16x8*>(smem_raw + obuf);              // [2][HALF * 64]
  float* sbias = reinterpret_cast<float*>(smem_raw + obias);
  const float* swo = sbias + NH * W;
  // each wave's next-tile inputs, copied straight into LDS during the last
  // layer of the current tile (no registers held across the layers)
  const int wave_u = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  float* sin = reinterpret_cast<float*>(reinterpret_cast<unsigned char*>(sbias) + S::bias_bytes()) +
               (HALVES ? wave_u : (int)(threadIdx.x >> 6)) * S::IN_WAVE;
  auto stage_inputs = [&](int64_t q0s) {
    const int64_t first = q0s * in_dim;
    const int64_t end = (q0s + NB * 16 < n ? q0s + NB * 16 : n) * in_dim;   // floats of valid queries
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
  const int64_t tiles = (n + S::WAVES * NB * 16 - 1) / (S::WAVES * NB * 16);
  const int64_t my_tiles = blockIdx.x < tiles ? (tiles - 1 - blockIdx.x) / gridDim.x + 1 : 0;
  const int64_t total_chunks = my_tiles * nchunk;
  // chunk k of this workgroup's stream: layer 1 + (k % nchunk) / 2, half (k % nchunk) % 2
  auto chunk_src = [&](int64_t k) {
    const int c = (int)(k % nchunk), l = 1 + c / 2, h = c % 2;
    return pack + (RB + (l - 1) * S::FH + h * S::HALF) * 64;
  };
  // chunk k + 1 goes straight from global memory into the idle LDS buffer
  // (global_load_lds: lane i of a wave fills the i-th 16-byte slot after the
  // wave-uniform LDS base), waited for before the end-of-chunk barrier.
  auto prefetch = [&](int64_t kk, bf16x8* dst) {
    const bf16x8* src = chunk_src(kk);
#pragma unroll
    for (int i = 0; i < S::PER; ++i) {
      const int slot = i * S::THREADS + (HALVES ? wave_u * 64 : (int)(threadIdx.x & ~63));
      __builtin_amdgcn_global_load_lds((const void*)(src + slot + (threadIdx.x & 63)),
                                       (__attribute__((address_space(3))) void*)(dst + slot), 16, 0, 0);
    }
  };
  if (total_chunks > 0) {
    const bf16x8* src = chunk_src(0);
#pragma unroll
    for (int i = 0; i < S::PER; ++i) sbuf[threadIdx.x + i * S::THREADS] = src[threadIdx.x + i * S::THREADS];
  }
  stage_inputs(((int64_t)blockIdx.x * S::WAVES + (threadIdx.x >> 6)) * NB * 16);
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();

  const int lane = threadIdx.x & 63, c = lane & 15, grp = lane >> 4, wave = threadIdx.x >> 6;
  const bool wide = in_dim > 4;
  const float bo = swo[W];
  unsigned cnt[4] = {0u, 0u, 0u, 0u};
  int64_t k = 0;
  for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int64_t q0 = (tile * S::WAVES + wave) * NB * 16;
    constexpr int RA = HALVES ? RB / 2 : RB;   // row blocks of accumulators held at a time
    floatx4 acc[NB][RA];
    bf16x8 act[NB][KS];
    bool bad[NB];   // rows with a non-finite value
    {
      bf16x8 xb[NB], xb1[NB];
      {
        float xr[NB][8];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const bool valid = q0 + nb * 16 + c < n;
          bad[nb] = false;
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            xr[nb][j] = (valid && j < in_dim) ? sin[(nb * 16 + c) * in_dim + j] : 0.0f;
            bad[nb] = bad[nb] || !isfinite(xr[nb][j]);
          }
        }
        nb_first_operands<NB>(xr, grp, wide, xb, xb1);
      }
#pragma unroll
      for (int h0 = 0; h0 < RB; h0 += RA) {   // the whole layer, or two halves
#pragma unroll
        for (int u = 0; u < RA; ++u) {
          const int mo = h0 + u;
          const float* b = sbias + 16 * mo + 4 * grp;
          const floatx4 bi = floatx4{b[0], b[1], b[2], b[3]};
          const bf16x8 a = sfirst[mo * 64 + lane];
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) acc[nb][u] = mfma32(a, xb[nb], bi);
        }
        if (wide) {
          // the second first-layer step's fragments come from global memory
          // (L2): the LDS holds two streamed half-layers beside the first step.
          // HALVES: the base is made opaque here so that the per-fragment
          // addresses are formed at the loads, not held across the tile loop
          typedef const __attribute__((address_space(1))) bf16x8* gpk_t;
          gpk_t pk = (gpk_t)pack;
          if constexpr (HALVES) asm volatile("" : "+s"(pk));
#pragma unroll
          for (int u = 0; u < RA; ++u) {
            const bf16x8 a = pk[(RB + (NH - 1) * S::FH + h0 + u) * 64 + lane];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) acc[nb][u] = mfma32(a, xb1[nb], acc[nb][u]);
          }
        }
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
          for (int k = 0; k < RA / 2; ++k) {
            float v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = acc[nb][2 * k + j / 4][j % 4];
            act[nb][h0 / 2 + k] = nb_relu_bf16x8(v);
          }
      }
    }
    float pout[NB];   // output-layer partial sums (HALVES: accumulated half by half)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) pout[nb] = 0.0f;

#pragma unroll 1
    for (int l = 1; l < NH; ++l) {
      bf16x8 actn[NB][KS];   // HALVES: the next layer's operands, filled half by half
#pragma unroll
      for (int h = 0; h < 2; ++h, ++k) {
        const bf16x8* buf = sbuf + (k & 1) * S::HALF * 64;
        const bool more = k + 1 < total_chunks;
        if (more) prefetch(k + 1, sbuf + ((k + 1) & 1) * S::HALF * 64);
        if (l == NH - 1 && h == 0 && tile + gridDim.x < tiles)
          stage_inputs(((tile + gridDim.x) * S::WAVES + wave) * NB * 16);
        // four row blocks at a time: 4 x NB independent accumulation chains per K step
#pragma unroll
        for (int m4 = 0; m4 < RB / 2; m4 += 4) {
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int mo = h * (RB / 2) + m4 + u;
            const int ma = HALVES ? m4 + u : mo;
            const float* b = sbias + l * W + 16 * mo + 4 * grp;
            const floatx4 bi = floatx4{b[0], b[1], b[2], b[3]};
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) acc[nb][ma] = bi;
          }
          // two fragment slots: K step ks + 1's fragments load while ks computes
          bf16x8 fa[4], fb[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) fa[u] = buf[((m4 + u) * KS + 0) * 64 + lane];
#pragma unroll
          for (int ks = 0; ks < KS; ++ks) {
            bf16x8(&cur)[4] = (ks & 1) ? fb : fa;
            bf16x8(&nxt)[4] = (ks & 1) ? fa : fb;
            // SPLIT of the four row blocks' products, then the next step's
            // loads, then the rest: the loads land behind the remaining products
#pragma unroll
            for (int u = 0; u < SPLIT; ++u)
#pragma unroll
              for (int nb = 0; nb < NB; ++nb) {
                const int ma = HALVES ? m4 + u : h * (RB / 2) + m4 + u;
                acc[nb][ma] = mfma32(cur[u], act[nb][ks], acc[nb][ma]);
              }
            __builtin_amdgcn_sched_barrier(0);
            if (ks + 1 < KS) {
#pragma unroll
              for (int u = 0; u < 4; ++u) nxt[u] = buf[((m4 + u) * KS + ks + 1) * 64 + lane];
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = SPLIT; u < 4; ++u)
#pragma unroll
              for (int nb = 0; nb < NB; ++nb) {
                const int ma = HALVES ? m4 + u : h * (RB / 2) + m4 + u;
                acc[nb][ma] = mfma32(cur[u], act[nb][ks], acc[nb][ma]);
              }
            __builtin_amdgcn_sched_barrier(0);
          }
        }
        if constexpr (HALVES) {
          // this half's row blocks are done: round them into the next
          // layer's operands, or (last layer) add their output terms
          if (l < NH - 1) {
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
#pragma unroll
              for (int kk = 0; kk < KS / 2; ++kk) {
                float v[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) v[j] = acc[nb][2 * kk + j / 4][j % 4];
                actn[nb][h * (KS / 2) + kk] = nb_relu_bf16x8(v);
              }
            if (h == 1) {
#pragma unroll
              for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) act[nb][ks] = actn[nb][ks];
            }
          } else {
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
#pragma unroll
              for (int u = 0; u < RA; ++u)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                  pout[nb] = fmaf(swo[16 * (h * RA + u) + 4 * grp + r], nb_relu(acc[nb][u][r]), pout[nb]);
          }
        } else if (h == 1 && l < NH - 1) {
#pragma unroll
          for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
              float v[8];
#pragma unroll
              for (int j = 0; j < 8; ++j) v[j] = acc[nb][2 * ks + j / 4][j % 4];
              act[nb][ks] = nb_relu_bf16x8(v);
            }
        }
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
      }
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      float p = pout[nb];
      if constexpr (!HALVES) {
#pragma unroll
        for (int mo = 0; mo < RA; ++mo)
#pragma unroll
          for (int r = 0; r < 4; ++r) p = fmaf(swo[16 * mo + 4 * grp + r], nb_relu(acc[nb][mo][r]), p);
      }
      p += __shfl_xor(p, 16);
      p += __shfl_xor(p, 32);
      const float z = bad[nb] ? __builtin_nanf("") : p + bo;   // non-finite row: NaN, decided positive
      const int64_t qi = q0 + nb * 16 + c;
      const bool own = grp == 0 && qi < n;
      const bool pos = !(z < tau);
      if (own) {
        if (logits) logits[qi] = z;
        if (hout) hout[qi] = pos;
      }
      if (counts) {
        const bool gv = own && g[qi] != 0;
        cnt[0] += __popcll(__ballot(own && pos && gv));
        cnt[1] += __popcll(__ballot(own && pos && !gv));
        cnt[2] += __popcll(__ballot(own && !pos && !gv));
        cnt[3] += __popcll(__ballot(own && !pos && gv));
      }
    }
  }
  if (counts && lane == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (cnt[i]) atomicAdd(&counts[i], (unsigned long long)cnt[i]);
  }
}

template <int NH, int SPLIT, int NB, int THREADS, bool HALVES = false>
nb_status stream_launch(const nb_bound* b, const float* q, int64_t n, float tau, float* logits, uint8_t* h,
                        const uint8_t* g, unsigned long long* counts, const unsigned long long* n_dev,
                        hipStream_t s) {
  using S = Stream256<NH, NB, THREADS>;
  static_assert(S::lds_bytes() <= 160 * 1024, "streamed forward exceeds the CU's LDS");
  const size_t lds = S::lds_bytes();
  static bool attr_set[64] = {false};
  int dev = 0;
  NB_HIP(hipGetDevice(&dev));
  if (dev >= 0 && dev < 64 && !attr_set[dev]) {
    NB_HIP(hipFuncSetAttribute((const void*)k_fwd_bf16_stream<NH, SPLIT, NB, THREADS, HALVES>,
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds));
    attr_set[dev] = true;
  }
  const int64_t tiles = (n + S::WAVES * S::NB * 16 - 1) / (S::WAVES * S::NB * 16);
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(tiles, nb_cu_count()));
  k_fwd_bf16_stream<NH, SPLIT, NB, THREADS, HALVES><<<grid, S::THREADS, lds, s>>>(q, n, b->in_dim, reinterpret_cast<const bf16x8*>(b->pack16),
                                                      b->theta, tau, logits, h, g, counts, n_dev);
  NB_LAUNCHED();
  return NB_OK;
}

int bf16_variants() { return 6; }
int bf16_variants_for(int width, int n_hidden) { return width == 256 ? (n_hidden <= 6 ? 7 : 3) : 6; }

// Variant v: (query blocks per wave, threads per workgroup) =
//   0: (2, 768)   1: (2, 512)   2: (3, 512)   3: (1, 1024)   4: (4, 256)   5: (2, 256)
// Variant 0 (three waves per SIMD) measured fastest for widths 32..128.
// Width 256 (streamed): (SPLIT, blocks per wave, threads) =
//   0: (2, 3, 256)   1: (1, 3, 256)   2: (3, 3, 256)   3: (2, 2, 512)   4: (1, 2, 512)
//   5, 6: variants 3 and 4 with half-layer accumulators (HALVES)
// (variants 3 to 6 up to 6 hidden layers).
template <int NH>
nb_status stream_nh(const nb_bound* b, const float* q, int64_t n, float tau, float* logits, uint8_t* h,
                    const uint8_t* g, unsigned long long* counts, const unsigned long long* n_dev, hipStream_t s) {
  switch (b->variant) {
    case 1: return stream_launch<NH, 1, 3, 256>(b, q, n, tau, logits, h, g, counts, n_dev, s);
    case 2: return stream_launch<NH, 3, 3, 256>(b, q, n, tau, logits, h, g, counts, n_dev, s);
    case 3:
    case 4:
    case 5:
    case 6:
      // eight waves fit the CU's LDS up to six hidden layers (the biases grow with depth)
      if constexpr (Stream256<NH, 2, 512>::lds_bytes() <= 160 * 1024) {
        switch (b->variant) {
          case 3: return stream_launch<NH, 2, 2, 512>(b, q, n, tau, logits, h, g, counts, n_dev, s);
          case 4: return stream_launch<NH, 1, 2, 512>(b, q, n, tau, logits, h, g, counts, n_dev, s);
          case 5: return stream_launch<NH, 2, 2, 512, true>(b, q, n, tau, logits, h, g, counts, n_dev, s);
          default: return stream_launch<NH, 1, 2, 512, true>(b, q, n, tau, logits, h, g, counts, n_dev, s);
        }
      } else {
        nb_set_error("streamed variant %d needs at most 6 hidden layers", b->variant);
        return NB_ERR_UNSUPPORTED;
      }
    default: return stream_launch<NH, 2, 3, 256>(b, q, n, tau, logits, h, g, counts, n_dev, s);
  }
}

nb_status bf16_forward(const nb_bound* b, const float* q, int64_t n, float tau, float* logits, uint8_t* h,
                       const uint8_t* g, unsigned long long* counts, hipStream_t s, const unsigned long long* n_dev) {
  if (b->width == 256) {
    switch (b->n_hidden) {
      case 2: return stream_nh<2>(b, q, n, tau, logits, h, g, counts, n_dev, s);
      case 3: return stream_nh<3>(b, q, n, tau, logits, h, g, counts, n_dev, s);
      case 4: return stream_nh<4>(b, q, n, tau, logits, h, g, counts, n_dev, s);
      case 5: return stream_nh<5>(b, q, n, tau, logits, h, g, counts, n_dev, s);
      case 6: return stream_nh<6>(b, q, n, tau, logits, h, g, counts, n_dev, s);
      case 7: return stream_nh<7>(b, q, n, tau, logits, h, g, counts, n_dev, s);
      case 8: return stream_nh<8>(b, q, n, tau, logits, h, g, counts, n_dev, s);
      default: break;
    }
  }
#define X(WW, H)                                                                  \
  if (b->width == WW && b->n_hidden == H) {                                       \
    switch (b->variant) {                                                         \
      case 1: return fwd_launch<WW, H, 2, 512>(b, q, n, tau, logits, h, g, counts, n_dev, s);  \
      case 2: return fwd_launch<WW, H, 3, 512>(b, q, n, tau, logits, h, g, counts, n_dev, s);  \
      case 3: return fwd_launch<WW, H, 1, 1024>(b, q, n, tau, logits, h, g, counts, n_dev, s); \
      case 4: return fwd_launch<WW, H, 4, 256>(b, q, n, tau, logits, h, g, counts, n_dev, s);  \
      case 5: return fwd_launch<WW, H, 2, 256>(b, q, n, tau, logits, h, g, counts, n_dev, s);  \
      default: return fwd_launch<WW, H, 2, 768>(b, q, n, tau, logits, h, g, counts, n_dev, s); \
    }                                                                             \
  }
  NB_BF16_CASES(X)
#undef X
  nb_set_error("bfloat16 bound %d x %d^%d has no kernel", b->in_dim, b->width, b->n_hidden);
  return NB_ERR_UNSUPPORTED;
}
