// The bound h_theta as a float32 MLP on the matrix cores (Sec. 3.4,
// "Architecture": an MLP whose output logit goes through a sigmoid and is
// rounded to {0,1}; ReLU hidden layers, or the paper's sinusoidal ones).
//
// Matrix-core mapping (v_mfma_f32_16x16x4f32, one wave of 64 lanes):
//   neurons are MFMA rows, queries are MFMA columns.  A wave takes 16
//   queries at a time; lane l owns query column c = l % 16 and, after every
//   layer, the four neurons 16*mo + 4*(l/16) + r (r = 0..3) of each 16-row
//   block mo.  Those four values are exactly the B operand the next layer
//   needs if the next layer's reduction index is visited in the order
//   (block mi, r) with lane group l/16 supplying neuron 16*mi + 4*(l/16) + r,
//   so activations never leave registers; the weights are pre-arranged
//   ("packed") in that order, one 64-float fragment per MFMA, so each
//   fragment load is one coalesced 256-byte read.
//   The first layer (in_dim <= 8 inputs) is the same product with the inputs
//   as B operand (zero-padded to a multiple of 4).  The last layer (width ->
//   1) is a per-lane dot product plus two cross-lane adds.
//
// Training (Alg. 1 steps 4-5, Eq. 1): one fused kernel runs forward, loss,
// dL/dz and backward for the queries of a workgroup:
//   delta_{l-1} = (W_l^T delta_l) * [a_{l-1} > 0]   (MFMA, transposed packs)
//   dW_l += delta_l a_{l-1}^T                          (MFMA over queries; the
//            operands go through workgroup-wide LDS tiles, every 16 x 16
//            output tile owned by one wave)
// and writes one partial gradient per workgroup; a second kernel sums the
// partials in a fixed order (deterministic), applies Adam and writes the
// updated weights into their packed fragments.
#include <algorithm>

#include "nb_internal.h"
#include "nb_mlp.h"

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ floatx4 mfma4(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// sin x by Cody and Waite's argument reduction (Cody & Waite,
// "Software Manual for the Elementary Functions", 1980): x = k pi/2 + r with
// k = rint(x 2/pi) and r = x - k pi/2, pi/2 split into a float32 head and
// tail so that two fused multiply-adds leave r accurate to float32 rounding
// for |x| <= 2^16 (the dropped remainder of pi/2 is below 2e-15).  Then the
// Taylor series of sin and cos on |r| <= pi/4 (truncation below 2e-9) and the
// quadrant k mod 4 picks +-sin r or +-cos r.  Larger or non-finite arguments
// take the library's sinf (cosf).  The forward's and the training kernel's sine
// activations use it, and the training kernel its cosine for the derivative.
constexpr float kPio2Hi = 0x1.921fb6p+0f;    // float32 nearest to pi/2
constexpr float kPio2Lo = -0x1.777a5cp-25f;  // float32 nearest to pi/2 - kPio2Hi
constexpr float kTwoOverPi = 0x1.45f306p-1f;
__device__ __forceinline__ void sin_cos_poly(float x, float& sp, float& cp, int& q) {
  const float k = rintf(x * kTwoOverPi);
  float r = fmaf(-k, kPio2Hi, x);
  r = fmaf(-k, kPio2Lo, r);
  q = (int)k & 3;   // k mod 4 (two's complement keeps it right for k < 0)
  const float r2 = r * r;
  sp = fmaf(r2 * r, fmaf(r2, fmaf(r2, fmaf(r2, 1.0f / 362880, -1.0f / 5040), 1.0f / 120), -1.0f / 6), r);
  cp = fmaf(r2, fmaf(r2, fmaf(r2, fmaf(r2, fmaf(r2, -1.0f / 3628800, 1.0f / 40320), -1.0f / 720), 1.0f / 24),
                 -0.5f),
            1.0f);
}
__device__ __forceinline__ float nb_sin(float x) {
  if (!(fabsf(x) <= 65536.0f)) return sinf(x);
  float sp, cp;
  int q;
  sin_cos_poly(x, sp, cp, q);
  const float v = (q & 1) ? cp : sp;   // sin(k pi/2 + r) = sin r, cos r, -sin r, -cos r
  return (q & 2) ? -v : v;
}
// cos x by the same reduction: cos(k pi/2 + r) = cos r, -sin r, -cos r, sin r.
__device__ __forceinline__ float nb_cos(float x) {
  if (!(fabsf(x) <= 65536.0f)) return cosf(x);
  float sp, cp;
  int q;
  sin_cos_poly(x, sp, cp, q);
  const float v = (q & 1) ? sp : cp;
  return ((q + 1) & 2) ? -v : v;
}

// Hidden activation ACT: 0 ReLU, 1 sine (sin z; the paper's choice).  The
// training kernel keeps per layer the value the backward pass needs: the
// ReLU output itself (its sign is the derivative), or the pre-activation z
// for sine (value sin z, derivative cos z).
template <int ACT>
__device__ __forceinline__ float act_apply(float z) {
  // ReLU as the median of (z, 0, FLT_MAX): max(z, 0) in one instruction for
  // every finite z (+inf becomes FLT_MAX)
  return ACT == 0 ? __builtin_amdgcn_fmed3f(z, 0.0f, 3.40282347e38f) : nb_sin(z);
}
template <int ACT>
__device__ __forceinline__ float act_store(float z) { return ACT == 0 ? fmaxf(z, 0.0f) : z; }
// The training kernel evaluates sin and cos with the same reduction and
// polynomials as the forward.
template <int ACT>
__device__ __forceinline__ float act_value(float kept) { return ACT == 0 ? kept : nb_sin(kept); }
template <int ACT>
__device__ __forceinline__ float act_grad(float kept, float g) {
  return ACT == 0 ? (kept > 0.0f ? g : 0.0f) : g * nb_cos(kept);
}

// Geometry of an in_dim -> W^NH -> 1 network with KIN 4-wide input steps.
template <int KIN, int W, int NH>
struct Net {
  static constexpr int RB = W / 16;             // 16-row blocks per layer
  static constexpr int F1 = RB * KIN;           // first-layer fragments
  static constexpr int FH = RB * RB * 4;        // fragments of one W x W layer
  static constexpr int NFWD = F1 + (NH - 1) * FH;
  static constexpr int NPACK = NFWD + (NH - 1) * FH;  // + transposed copies
};

// ------------------------------------------------------------------ packing

// pack[f*64 + lane]:
//   f < F1            first layer, block mo = f / KIN, step s = f % KIN:
//                     W0[16mo + c][4s + g]   (0 beyond in_dim)
//   f < NFWD          hidden layer l (1-based), fragment (mo, mi, r):
//                     W_l[16mo + c][16mi + 4g + r]
//   else              transposed copy of hidden layer l, fragment (mo, mi, r):
//                     W_l[16mi + 4g + r][16mo + c]
// with c = lane % 16, g = lane / 16.
__global__ void k_pack(const float* __restrict__ theta, int in_dim, int W, int NH, float* __restrict__ pack,
                       int64_t total) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int f = (int)(idx >> 6), lane = (int)(idx & 63), c = lane & 15, g = lane >> 4;
  const int RB = W / 16, KIN = (in_dim + 3) / 4, F1 = RB * KIN, FH = RB * RB * 4;
  const int NFWD = F1 + (NH - 1) * FH;
  float v;
  if (f < F1) {
    const int mo = f / KIN, s = f % KIN, k = 4 * s + g;
    v = k < in_dim ? theta[(int64_t)(16 * mo + c) * in_dim + k] : 0.0f;
  } else {
    const bool tr = f >= NFWD;
    const int t = f - (tr ? NFWD : F1);
    const int l = 1 + t / FH, rem = t % FH;
    const int mo = rem / (RB * 4), mi = (rem / 4) % RB, r = rem % 4;
    const float* Wl = theta + nb_w_off(l, in_dim, W);
    v = tr ? Wl[(int64_t)(16 * mi + 4 * g + r) * W + 16 * mo + c] : Wl[(int64_t)(16 * mo + c) * W + 16 * mi + 4 * g + r];
  }
  pack[idx] = v;
}

// ------------------------------------------------------------------ forward

// Waves per SIMD the forward asks the register allocator for: two while the
// weights held in registers leave room (all but the widest, deepest nets).
// Networks 64 or more wide read their hidden weights from LDS (one 16-byte
// read per lane feeds four products), which frees the registers for four
// waves per SIMD; narrower ones keep them in registers.
template <int W>
constexpr bool fwd_lds_weights() { return W >= 64; }
template <int W, int NH, int ACT>
constexpr int fwd_waves() {
  return fwd_lds_weights<W>() ? 4 : (W * W * (NH - 1) > 64 * 64 * (ACT == 0 ? 2 : 1) ? 1 : 2);
}

template <int KIN, int W, int NH, int ACT>
__global__ __launch_bounds__(256, (fwd_waves<W, NH, ACT>())) void k_fwd(const float* __restrict__ q, int64_t n,
                                                                   int in_dim,
                                             const float* __restrict__ pack, const float* __restrict__ theta,
                                             float tau, float* __restrict__ logits, uint8_t* __restrict__ hout,
                                             const uint8_t* __restrict__ g, unsigned long long* __restrict__ counts,
                                             const unsigned long long* __restrict__ n_dev) {
  using N = Net<KIN, W, NH>;
  if (n_dev && (int64_t)*n_dev < n) n = (int64_t)*n_dev;   // rows counted on the device
  constexpr int RB = N::RB;
  const int lane = threadIdx.x & 63, c = lane & 15, grp = lane >> 4;

  float w1[N::F1];
#pragma unroll
  for (int f = 0; f < N::F1; ++f) w1[f] = pack[f * 64 + lane];
  constexpr bool kLdsW = fwd_lds_weights<W>();
  constexpr int NWH = (!kLdsW && (NH - 1) * N::FH > 0) ? (NH - 1) * N::FH : 1;
  float wh[NWH];
  if constexpr (!kLdsW) {
#pragma unroll
    for (int f = 0; f < (NH - 1) * N::FH; ++f) wh[f] = pack[(N::F1 + f) * 64 + lane];
  }
  // LDS copy of the hidden weights: entry ((l-1) RB^2 + mo RB + mi) * 64 + lane
  // holds fragments r = 0..3 of (layer l, row block mo, column block mi)
  constexpr int NW4 = (kLdsW && NH > 1) ? (NH - 1) * RB * RB * 64 : 1;
  __shared__ floatx4 swh[NW4];
  if constexpr (kLdsW) {
    for (int i = threadIdx.x; i < (NH - 1) * RB * RB * 64; i += blockDim.x) {
      const int f0 = N::F1 + (i >> 6) * 4, ln = i & 63;
      swh[i] = floatx4{pack[f0 * 64 + ln], pack[(f0 + 1) * 64 + ln], pack[(f0 + 2) * 64 + ln],
                       pack[(f0 + 3) * 64 + ln]};
    }
  }
  float wo[RB * 4];
#pragma unroll
  for (int mo = 0; mo < RB; ++mo)
#pragma unroll
    for (int r = 0; r < 4; ++r) wo[mo * 4 + r] = theta[nb_w_off(NH, in_dim, W) + 16 * mo + 4 * grp + r];
  const float bo = theta[nb_b_off(NH, in_dim, W, NH)];

  // hidden biases in LDS: read there, they do not queue behind the input
  // prefetch in the vector-memory counter
  __shared__ float sb[NH * W];
  for (int i = threadIdx.x; i < NH * W; i += blockDim.x) sb[i] = theta[nb_b_off(i / W, in_dim, W, NH) + i % W];
  __syncthreads();

  unsigned cnt[4] = {0u, 0u, 0u, 0u};
  const int64_t nblk = (n + 15) / 16;
  const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
  // Raw inputs of a block: the load is always in bounds (row and input
  // clamped); values outside the rows or inputs are zeroed where they are
  // used.
  auto load_raw = [&](int64_t blk, float* raw) {
    const int64_t qi = std::min<int64_t>(blk * 16 + c, n - 1);
#pragma unroll
    for (int s = 0; s < KIN; ++s) raw[s] = q[qi * in_dim + std::min(4 * s + grp, in_dim - 1)];
  };
  auto process = [&](int64_t blk, const float* raw) {
    const int64_t qi = blk * 16 + c;
    const bool valid = qi < n;
    float xs[KIN];
    int bad = 0;   // a non-finite input value in this lane's share of the row
#pragma unroll
    for (int s = 0; s < KIN; ++s) {
      const bool use = valid && 4 * s + grp < in_dim;
      xs[s] = use ? raw[s] : 0.0f;
      bad |= use && !isfinite(raw[s]);
    }
    float a[RB * 4];
    {
      const float* b0 = sb;
      floatx4 acc[RB];
#pragma unroll
      for (int mo = 0; mo < RB; ++mo)
        acc[mo] = floatx4{b0[16 * mo + 4 * grp], b0[16 * mo + 4 * grp + 1], b0[16 * mo + 4 * grp + 2],
                          b0[16 * mo + 4 * grp + 3]};
#pragma unroll
      for (int s = 0; s < KIN; ++s) {
#pragma unroll
        for (int mo = 0; mo < RB; ++mo) acc[mo] = mfma4(w1[mo * KIN + s], xs[s], acc[mo]);
      }
#pragma unroll
      for (int mo = 0; mo < RB; ++mo)
#pragma unroll
        for (int r = 0; r < 4; ++r) a[mo * 4 + r] = act_apply<ACT>(acc[mo][r]);
    }
#pragma unroll
    for (int l = 1; l < NH; ++l) {
      const float* bl = sb + l * W;
      floatx4 acc[RB];
#pragma unroll
      for (int mo = 0; mo < RB; ++mo)
        acc[mo] = floatx4{bl[16 * mo + 4 * grp], bl[16 * mo + 4 * grp + 1], bl[16 * mo + 4 * grp + 2],
                          bl[16 * mo + 4 * grp + 3]};
      // every acc[mo] takes its products in (mi, r) order either way; the
      // wave's issue priority is raised over its products so that a wave
      // feeding the matrix core wins issue over waves in their VALU work
      __builtin_amdgcn_s_setprio(1);
      if constexpr (kLdsW) {
#pragma unroll
        for (int mi = 0; mi < RB; ++mi) {
          floatx4 w4[RB];
#pragma unroll
          for (int mo = 0; mo < RB; ++mo) w4[mo] = swh[((l - 1) * RB * RB + mo * RB + mi) * 64 + lane];
#pragma unroll
          for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int mo = 0; mo < RB; ++mo) acc[mo] = mfma4(w4[mo][r], a[mi * 4 + r], acc[mo]);
        }
      } else {
#pragma unroll
        for (int mi = 0; mi < RB; ++mi)
#pragma unroll
          for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int mo = 0; mo < RB; ++mo)
              acc[mo] = mfma4(wh[(l - 1) * N::FH + (mo * RB + mi) * 4 + r], a[mi * 4 + r], acc[mo]);
      }
      __builtin_amdgcn_s_setprio(0);
#pragma unroll
      for (int mo = 0; mo < RB; ++mo)
#pragma unroll
        for (int r = 0; r < 4; ++r) a[mo * 4 + r] = act_apply<ACT>(acc[mo][r]);
    }
    float p = 0.0f;
#pragma unroll
    for (int i = 0; i < RB * 4; ++i) p = fmaf(wo[i], a[i], p);
    p += __shfl_xor(p, 16);
    p += __shfl_xor(p, 32);
    bad |= __shfl_xor(bad, 16);
    bad |= __shfl_xor(bad, 32);
    // a row with a non-finite value gets logit NaN, hence a positive decision
    const float z = bad ? __builtin_nanf("") : p + bo;
    const bool pos = !(z < tau);
    const bool own = grp == 0 && valid;
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
  };
  // the block index is the same on every lane of the wave: keep it scalar
  int64_t blk = (int64_t)blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t last = nblk - 1;
  float rnext[KIN];
  if (blk < nblk) load_raw(blk, rnext);
  for (; blk < nblk; blk += nwaves) {
    float raw[KIN];
#pragma unroll
    for (int s = 0; s < KIN; ++s) raw[s] = rnext[s];
    load_raw(std::min(blk + nwaves, last), rnext);   // the next block's inputs load while this one computes
    __builtin_amdgcn_sched_barrier(0);               // keep the load issued ahead of the products
    process(blk, raw);
  }
  if (counts && lane == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (cnt[i]) atomicAdd(&counts[i], (unsigned long long)cnt[i]);
  }
}

// ------------------------------------------------------------------ training

// Training with the weight-gradient tiles shared by the workgroup's waves.
// Every wave runs the forward, Eq. 1 and the data gradients of its own block
// of 16 queries in registers, as k_train does, and writes each layer's
// delta and activation columns into workgroup-wide [neuron][query] tiles in
// LDS; after a barrier every 16 x 16 weight-gradient tile is accumulated by
// one wave (tiles dealt round robin), with K = the 16 * WV queries of the
// iteration.  Bias and output-weight gradients are summed over the 16 lanes
// of a row once per block (reduce-scatter: two or three registers per lane
// instead of one per neuron) and over the waves, in order, at the end.  A
// wave then holds a fraction of the weight-gradient accumulators, so eight
// waves (two per SIMD) fit where the LDS allows, against one per SIMD.
// Row stride of the shared tiles: 16 WV + 2 floats, so that the operand
// reads (lane: row c, column g of a K step) hit distinct banks.
template <int KIN, int W, int NH, int WV>
struct TrainShared {
  using N = Net<KIN, W, NH>;
  static constexpr int RB = N::RB, V = RB * 4, V16 = (V + 15) / 16 * 16, GW = V16 / 16;
  static constexpr int QT = 16 * WV, S = QT + 2, ROWS = W > 16 ? W : 16;
  static constexpr int TILES = RB * RB, TPW = (TILES + WV - 1) / WV, R0 = (RB + WV - 1) / WV;
  static constexpr int kBias = NH * W + W + 1;
  // parameters: in_dim W + W, then (NH - 1) (W^2 + W), then W + 1
  __host__ __device__ static constexpr int64_t P(int in_dim) {
    return (int64_t)W * in_dim + W + (int64_t)(NH - 1) * ((int64_t)W * W + W) + W + 1;
  }
  __host__ __device__ static constexpr int64_t head(int in_dim) {
    return (int64_t)N::NPACK * 64 > P(in_dim) ? (int64_t)N::NPACK * 64 : P(in_dim);
  }
  __host__ __device__ static constexpr int64_t floats(int in_dim) {
    return head(in_dim) + kBias + 2 * (int64_t)ROWS * S + WV * 8;
  }
  static_assert((int64_t)WV * (NH + 1) * W <= (int64_t)ROWS * S, "per-wave bias sums fit the delta tile");
};
// Eight waves where the LDS allows (for every input size the network takes);
// four (one per SIMD, 512 registers each) for the 80-wide sine networks with
// two hidden layers, whose activations, sines and cosines need more than the
// 256 registers of two waves per SIMD.
template <int KIN, int W, int NH, int ACT>
constexpr int train_waves() {
  if (ACT == 1 && W >= 80 && NH >= 2) return 4;
  return TrainShared<KIN, W, NH, 8>::floats(4 * KIN) * 4 <= 160 * 1024 ? 8 : 4;
}

template <int KIN, int W, int NH, int ACT, int WV>
__global__ __launch_bounds__(64 * WV, 1) void k_train_s(const float* __restrict__ q, const uint8_t* __restrict__ y,
                                                         int64_t n, int in_dim, int bpw,
                                                         const float* __restrict__ pack,
                                                         const float* __restrict__ theta, float alpha, float beta,
                                                         float inv_n, float tau, float* __restrict__ partial,
                                                         float* __restrict__ aux) {
  using N = Net<KIN, W, NH>;
  using T = TrainShared<KIN, W, NH, WV>;
  constexpr int RB = N::RB, S = T::S, ROWS = T::ROWS, V16 = T::V16, GW = T::GW;
  constexpr int TILES = T::TILES, TPW = T::TPW, R0 = T::R0;
  extern __shared__ float smem[];
  const int64_t P = T::P(in_dim);
  float* spack = smem;                        // packed weights; later the reduction buffer
  float* sbias = smem + T::head(in_dim);      // [NH][W] biases, [W] output weights, output bias
  float* dT = sbias + T::kBias;               // [ROWS][S]: deltas of the iteration's queries
  float* aT = dT + ROWS * S;                  // [ROWS][S]: activations (inputs for the first layer)
  float* saux = aT + ROWS * S;                // [WV][8] per-wave loss / counts

  for (int i = threadIdx.x; i < N::NPACK * 64; i += blockDim.x) spack[i] = pack[i];
  for (int i = threadIdx.x; i < NH * W; i += blockDim.x) sbias[i] = theta[nb_b_off(i / W, in_dim, W, NH) + i % W];
  for (int i = threadIdx.x; i < W + 1; i += blockDim.x) sbias[NH * W + i] = theta[nb_w_off(NH, in_dim, W) + i];
  __syncthreads();

  const int lane = threadIdx.x & 63, c = lane & 15, grp = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const float* swo = sbias + NH * W;
  const float bo = swo[W];
  float wo[RB * 4];   // the lane's output weights (read once: under the ReLU select a read would branch)
#pragma unroll
  for (int mo = 0; mo < RB; ++mo)
#pragma unroll
    for (int r = 0; r < 4; ++r) wo[mo * 4 + r] = swo[16 * mo + 4 * grp + r];

  floatx4 gW0[R0];
  floatx4 gWh[NH > 1 ? NH - 1 : 1][TPW];
  float gb[NH][GW], gwo[GW];
  float gbo = 0.0f, lsum = 0.0f;
  unsigned cnt[4] = {0u, 0u, 0u, 0u};
#pragma unroll
  for (int i = 0; i < R0; ++i) gW0[i] = floatx4{0, 0, 0, 0};
#pragma unroll
  for (int l = 0; l < (NH > 1 ? NH - 1 : 1); ++l)
#pragma unroll
    for (int t = 0; t < TPW; ++t) gWh[l][t] = floatx4{0, 0, 0, 0};
#pragma unroll
  for (int k = 0; k < GW; ++k) {
    gwo[k] = 0.0f;
#pragma unroll
    for (int l = 0; l < NH; ++l) gb[l][k] = 0.0f;
  }
  // sum over the 16 lanes of a row of RB*4 per-lane values, scattered: lane
  // c keeps the sums of values c + 16 k
  auto row_sums = [&](const float (&v)[RB * 4], float (&acc)[GW]) {
    float x[V16], sm[GW];
#pragma unroll
    for (int i = 0; i < V16; ++i) x[i] = i < RB * 4 ? v[i] : 0.0f;
    nb_row_reduce_scatter<V16>(x, c, sm);
#pragma unroll
    for (int k = 0; k < GW; ++k) acc[k] += sm[k];
  };

  const int64_t nblk = (n + 15) / 16;
  const int64_t blk0 = (int64_t)blockIdx.x * bpw;
  const int64_t blk1 = blk0 + bpw < nblk ? blk0 + bpw : nblk;
  const int iters = (bpw + WV - 1) / WV;
  const int col = 16 * wave + c;   // the lane's query column in the shared tiles
  for (int it = 0; it < iters; ++it) {
    const int64_t blk = blk0 + (int64_t)it * WV + wave;
    const int64_t qi = blk * 16 + c;
    const bool valid = blk < blk1 && qi < n;
    float xin[KIN];
#pragma unroll
    for (int s = 0; s < KIN; ++s) {
      const int k = 4 * s + grp;
      xin[s] = (valid && k < in_dim) ? q[qi * in_dim + k] : 0.0f;
    }
    // forward, keeping every layer's activations
    float act[NH][RB * 4];
    {
      floatx4 acc[RB];
#pragma unroll
      for (int mo = 0; mo < RB; ++mo) {
        const float* b = sbias + 16 * mo + 4 * grp;
        acc[mo] = floatx4{b[0], b[1], b[2], b[3]};
      }
#pragma unroll
      for (int s = 0; s < KIN; ++s)
#pragma unroll
        for (int mo = 0; mo < RB; ++mo) acc[mo] = mfma4(spack[(mo * KIN + s) * 64 + lane], xin[s], acc[mo]);
#pragma unroll
      for (int mo = 0; mo < RB; ++mo)
#pragma unroll
        for (int r = 0; r < 4; ++r) act[0][mo * 4 + r] = act_store<ACT>(acc[mo][r]);
    }
#pragma unroll
    for (int l = 1; l < NH; ++l) {
      floatx4 acc[RB];
#pragma unroll
      for (int mo = 0; mo < RB; ++mo) {
        const float* b = sbias + l * W + 16 * mo + 4 * grp;
        acc[mo] = floatx4{b[0], b[1], b[2], b[3]};
      }
      const float* fr = spack + (N::F1 + (l - 1) * N::FH) * 64 + lane;
      float av[RB * 4];
#pragma unroll
      for (int i = 0; i < RB * 4; ++i) av[i] = act_value<ACT>(act[l - 1][i]);
#pragma unroll
      for (int mi = 0; mi < RB; ++mi)
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int mo = 0; mo < RB; ++mo) acc[mo] = mfma4(fr[((mo * RB + mi) * 4 + r) * 64], av[mi * 4 + r], acc[mo]);
#pragma unroll
      for (int mo = 0; mo < RB; ++mo)
#pragma unroll
        for (int r = 0; r < 4; ++r) act[l][mo * 4 + r] = act_store<ACT>(acc[mo][r]);
    }
    float alast[RB * 4];
#pragma unroll
    for (int i = 0; i < RB * 4; ++i) alast[i] = act_value<ACT>(act[NH - 1][i]);
    float p = 0.0f;
#pragma unroll
    for (int i = 0; i < RB * 4; ++i) p = fmaf(wo[i], alast[i], p);
    p += __shfl_xor(p, 16);
    p += __shfl_xor(p, 32);
    const float z = p + bo;

    // Eq. 1 on logits: alpha y softplus(-z) + beta (1 - y) softplus(z);
    // dl/dz = beta (1 - y) sigmoid(z) - alpha y (1 - sigmoid(z)).
    const bool yv = valid && y[qi] != 0;
    const float e = expf(-fabsf(z));
    const float inv1pe = 1.0f / (1.0f + e);
    const float sig = z >= 0.0f ? inv1pe : e * inv1pe;        // sigmoid(z)
    const float sigm = z >= 0.0f ? e * inv1pe : inv1pe;       // 1 - sigmoid(z)
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

    float d[RB * 4];
    {
      float t[RB * 4];
#pragma unroll
      for (int i = 0; i < RB * 4; ++i) {
        t[i] = dz * alast[i];
        d[i] = act_grad<ACT>(act[NH - 1][i], dz * wo[i]);
      }
      row_sums(t, gwo);
    }

#pragma unroll
    for (int l = NH - 1; l >= 1; --l) {
      row_sums(d, gb[l]);
#pragma unroll
      for (int mo = 0; mo < RB; ++mo)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          dT[(16 * mo + 4 * grp + r) * S + col] = d[mo * 4 + r];
          aT[(16 * mo + 4 * grp + r) * S + col] = act_value<ACT>(act[l - 1][mo * 4 + r]);
        }
      floatx4 acc[RB];
#pragma unroll
      for (int mo = 0; mo < RB; ++mo) acc[mo] = floatx4{0, 0, 0, 0};
      const float* fr = spack + (N::NFWD + (l - 1) * N::FH) * 64 + lane;
#pragma unroll
      for (int mi = 0; mi < RB; ++mi)
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int mo = 0; mo < RB; ++mo) acc[mo] = mfma4(fr[((mo * RB + mi) * 4 + r) * 64], d[mi * 4 + r], acc[mo]);
#pragma unroll
      for (int mo = 0; mo < RB; ++mo)
#pragma unroll
        for (int r = 0; r < 4; ++r) d[mo * 4 + r] = act_grad<ACT>(act[l - 1][mo * 4 + r], acc[mo][r]);
      __syncthreads();
      // dW_l += delta_l a_{l-1}^T over the iteration's queries, the wave's tiles
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
        const int Tt = wave + t * WV;
        if (Tt < TILES) {
          const int no = Tt / RB, ko = Tt % RB;
          const float* ra = dT + (16 * no + c) * S + grp;
          const float* rb = aT + (16 * ko + c) * S + grp;
#pragma unroll 8
          for (int s = 0; s < 4 * WV; ++s) gWh[l - 1][t] = mfma4(ra[4 * s], rb[4 * s], gWh[l - 1][t]);
        }
      }
      __syncthreads();
    }

    // first layer: dW0 += delta_0 x^T (inputs as 16 rows, zero-padded)
    row_sums(d, gb[0]);
#pragma unroll
    for (int mo = 0; mo < RB; ++mo)
#pragma unroll
      for (int r = 0; r < 4; ++r) dT[(16 * mo + 4 * grp + r) * S + col] = d[mo * 4 + r];
#pragma unroll
    for (int s = 0; s < 4; ++s) aT[(4 * s + grp) * S + col] = s < KIN ? xin[s < KIN ? s : 0] : 0.0f;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < R0; ++i) {
      const int no = wave + i * WV;
      if (no < RB) {
        const float* ra = dT + (16 * no + c) * S + grp;
        const float* rb = aT + c * S + grp;
#pragma unroll 8
        for (int s = 0; s < 4 * WV; ++s) gW0[i] = mfma4(ra[4 * s], rb[4 * s], gW0[i]);
      }
    }
    __syncthreads();
  }

  // ---- partial of the chunk: weight-gradient tiles from their owners;
  // bias and output-weight sums over the waves in order
  float* red = smem;
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) {
    gbo += __shfl_xor(gbo, m);
    lsum += __shfl_xor(lsum, m);
  }
  float* wsum = dT;   // [WV][NH + 1][W]: per wave, bias gradients of each layer then the output weights
#pragma unroll
  for (int k = 0; k < GW; ++k) {
    const int i = c + 16 * k;
    if (i < RB * 4) {
      const int nrn = 16 * (i >> 2) + 4 * grp + (i & 3);
#pragma unroll
      for (int l = 0; l < NH; ++l) wsum[(wave * (NH + 1) + l) * W + nrn] = gb[l][k];
      wsum[(wave * (NH + 1) + NH) * W + nrn] = gwo[k];
    }
  }
  if (lane == 0) {
    saux[wave * 8 + 0] = lsum;
    saux[wave * 8 + 1] = gbo;
    for (int i = 0; i < 4; ++i) saux[wave * 8 + 2 + i] = __uint_as_float(cnt[i]);
  }
#pragma unroll
  for (int i = 0; i < R0; ++i) {
    const int no = wave + i * WV;
    if (no < RB && c < in_dim)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[(int64_t)(16 * no + 4 * grp + r) * in_dim + c] = gW0[i][r];
  }
#pragma unroll
  for (int l = 1; l < NH; ++l)
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int Tt = wave + t * WV;
      if (Tt < TILES) {
        const int no = Tt / RB, ko = Tt % RB;
#pragma unroll
        for (int r = 0; r < 4; ++r)
          red[nb_w_off(l, in_dim, W) + (int64_t)(16 * no + 4 * grp + r) * W + 16 * ko + c] = gWh[l - 1][t][r];
      }
    }
  __syncthreads();
  for (int i = threadIdx.x; i < (NH + 1) * W; i += blockDim.x) {
    const int l = i / W, nrn = i % W;
    float v = 0.0f;
    for (int w = 0; w < WV; ++w) v += wsum[(w * (NH + 1) + l) * W + nrn];
    red[l < NH ? nb_b_off(l, in_dim, W, NH) + nrn : nb_w_off(NH, in_dim, W) + nrn] = v;
  }
  if (threadIdx.x == 0) {
    float ls = 0.0f, gbs = 0.0f;
    unsigned cs[4] = {0u, 0u, 0u, 0u};
    for (int w = 0; w < WV; ++w) {
      ls += saux[w * 8];
      gbs += saux[w * 8 + 1];
      for (int i = 0; i < 4; ++i) cs[i] += __float_as_uint(saux[w * 8 + 2 + i]);
    }
    red[nb_b_off(NH, in_dim, W, NH)] = gbs;
    aux[blockIdx.x * 8] = ls;
    for (int i = 0; i < 4; ++i) aux[blockIdx.x * 8 + 1 + i] = __uint_as_float(cs[i]);
  }
  __syncthreads();
  float* out = partial + (int64_t)blockIdx.x * P;
  for (int64_t i = threadIdx.x; i < P; i += blockDim.x) out[i] = red[i];
}

// ---------------------------------------------------------------- dispatch

constexpr int kMaxWG = 256;

template <int KIN, int W, int NH, int ACT>
nb_status fwd_launch(const nb_bound* b, const float* q, int64_t n, float tau, float* logits, uint8_t* h,
                     const uint8_t* g, unsigned long long* counts, const unsigned long long* n_dev, hipStream_t s) {
  const int64_t nblk = (n + 15) / 16;
  const int64_t want = (nblk + 3) / 4;
  const int64_t cap = (int64_t)nb_cu_count() * std::max(2, fwd_waves<W, NH, ACT>());
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min(want, cap));
  k_fwd<KIN, W, NH, ACT><<<grid, 256, 0, s>>>(q, n, b->in_dim, b->pack, b->theta, tau, logits, h, g, counts, n_dev);
  NB_LAUNCHED();
  return NB_OK;
}

template <int KIN, int W, int NH, int ACT>
nb_status train_launch(const nb_bound* b, const float* q, const uint8_t* y, int64_t n, float alpha, float beta,
                       float tau, int* n_wg, hipStream_t s) {
  constexpr int WV = train_waves<KIN, W, NH, ACT>();
  using L = TrainShared<KIN, W, NH, WV>;
  const int64_t nblk = (n + 15) / 16;
  const int bpw = (int)((nblk + kMaxWG - 1) / kMaxWG);
  const int grid = (int)((nblk + bpw - 1) / bpw);
  const size_t lds = (size_t)L::floats(b->in_dim) * sizeof(float);
  static bool attr_set[64] = {false};
  int dev = 0;
  NB_HIP(hipGetDevice(&dev));
  if (dev >= 0 && dev < 64 && !attr_set[dev]) {
    NB_HIP(hipFuncSetAttribute((const void*)k_train_s<KIN, W, NH, ACT, WV>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    attr_set[dev] = true;
  }
  k_train_s<KIN, W, NH, ACT, WV><<<grid, 64 * WV, lds, s>>>(q, y, n, b->in_dim, bpw, b->pack, b->theta, alpha,
                                                           beta, (float)(1.0 / (double)n), tau, b->partial,
                                                           b->aux);
  NB_LAUNCHED();
  *n_wg = grid;
  return NB_OK;
}

// (KIN, W, NH) instances: inputs 1..8, widths 16/32/64 with 1..4 hidden
// layers, width 80 (the paper's 75-wide networks, zero-padded) with 1..2.
#define NB_F32_CASES(X) \
  X(1, 16, 1) X(1, 16, 2) X(1, 16, 3) X(1, 16, 4) \
  X(1, 32, 1) X(1, 32, 2) X(1, 32, 3) X(1, 32, 4) \
  X(1, 64, 1) X(1, 64, 2) X(1, 64, 3) X(1, 64, 4) \
  X(1, 80, 1) X(1, 80, 2)                         \
  X(2, 16, 1) X(2, 16, 2) X(2, 16, 3) X(2, 16, 4) \
  X(2, 32, 1) X(2, 32, 2) X(2, 32, 3) X(2, 32, 4) \
  X(2, 64, 1) X(2, 64, 2) X(2, 64, 3) X(2, 64, 4) \
  X(2, 80, 1) X(2, 80, 2)

// Sine instances (the paper's own architectures: the neurons of a 25-, 50-
// or 75-wide layer zero-padded to 32, 64 or 80; 1..3 hidden layers, 1..2 at
// width 80).
#define NB_F32_SINE_CASES(X) \
  X(1, 32, 1) X(1, 32, 2) X(1, 32, 3) X(1, 64, 1) X(1, 64, 2) X(1, 64, 3) X(1, 80, 1) X(1, 80, 2) \
  X(2, 32, 1) X(2, 32, 2) X(2, 32, 3) X(2, 64, 1) X(2, 64, 2) X(2, 64, 3) X(2, 80, 1) X(2, 80, 2)

inline int kin_of(int in_dim) { return (in_dim + 3) / 4; }

}  // namespace

bool f32_sine_supported(int in_dim, int n_hidden, int width) {
  return in_dim >= 1 && in_dim <= 8 && n_hidden >= 1 &&
         (((width == 32 || width == 64) && n_hidden <= 3) || (width == 80 && n_hidden <= 2));
}

bool f32_supported(int in_dim, int n_hidden, int width) {
  return in_dim >= 1 && in_dim <= 8 && n_hidden >= 1 &&
         (((width == 16 || width == 32 || width == 64) && n_hidden <= 4) || (width == 80 && n_hidden <= 2));
}

int64_t f32_pack_floats(int in_dim, int n_hidden, int width) {
  const int RB = width / 16, F1 = RB * kin_of(in_dim), FH = RB * RB * 4;
  return (int64_t)(F1 + 2 * (n_hidden - 1) * FH) * 64;
}

int f32_max_workgroups() { return kMaxWG; }

nb_status f32_pack(const nb_bound* b, hipStream_t s) {
  const int64_t total = b->pack_floats;
  k_pack<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(b->theta, b->in_dim, b->width, b->n_hidden, b->pack, total);
  NB_LAUNCHED();
  return NB_OK;
}

nb_status f32_forward(const nb_bound* b, const float* q, int64_t n, float tau, float* logits, uint8_t* h,
                      const uint8_t* g, unsigned long long* counts, hipStream_t s, const unsigned long long* n_dev) {
  const int kin = kin_of(b->in_dim);
  if (b->activation == NB_ACT_SINE) {
#define X(K, WW, H)                                                                  \
  if (kin == K && b->width == WW && b->n_hidden == H)                                \
    return fwd_launch<K, WW, H, 1>(b, q, n, tau, logits, h, g, counts, n_dev, s);
    NB_F32_SINE_CASES(X)
#undef X
  } else {
#define X(K, WW, H)                                                                  \
  if (kin == K && b->width == WW && b->n_hidden == H)                                \
    return fwd_launch<K, WW, H, 0>(b, q, n, tau, logits, h, g, counts, n_dev, s);
    NB_F32_CASES(X)
#undef X
  }
  nb_set_error("float32 bound %d x %d^%d has no kernel", b->in_dim, b->width, b->n_hidden);
  return NB_ERR_UNSUPPORTED;
}

nb_status f32_train_partials(const nb_bound* b, const float* q, const uint8_t* y, int64_t n, float alpha,
                             float beta, float tau, int* n_wg, hipStream_t s) {
  const int kin = kin_of(b->in_dim);
  if (b->activation == NB_ACT_SINE) {
#define X(K, WW, H)                                                  \
  if (kin == K && b->width == WW && b->n_hidden == H)                \
    return train_launch<K, WW, H, 1>(b, q, y, n, alpha, beta, tau, n_wg, s);
    NB_F32_SINE_CASES(X)
#undef X
  } else {
#define X(K, WW, H)                                                  \
  if (kin == K && b->width == WW && b->n_hidden == H)                \
    return train_launch<K, WW, H, 0>(b, q, y, n, alpha, beta, tau, n_wg, s);
    NB_F32_CASES(X)
#undef X
  }
  nb_set_error("float32 bound %d x %d^%d has no kernel", b->in_dim, b->width, b->n_hidden);
  return NB_ERR_UNSUPPORTED;
}
