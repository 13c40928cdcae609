// The bfloat16 forward pass of one wave over NB blocks of 16 queries after
// the first layer, shared by the single-bound and grouped kernels (weights
// already in LDS).
//
// Rounding points: the first layer at float32 accuracy (the resident
// single-bound and grouped kernels on the float32 matrix cores; the
// streamed and training kernels cut each float32 weight and input exactly
// into three bfloat16 pieces and run the six significant piece products on
// the bfloat16 matrix cores, layout in nb_mlp.h); hidden layers bfloat16
// weights and activations; output layer a float32 dot product.  Lane l
// holds neurons 16*mo + 4*(l/16) + r of query l % 16 after every layer; a
// K = 32 step of the next layer takes the 8 values of row blocks 2*ks and
// 2*ks + 1 that the lane already holds.
#pragma once

#include "nb_mlp.h"

typedef nb_bf16x8 bf16x8;
typedef nb_floatx4 floatx4;

__device__ __forceinline__ floatx4 mfma32(bf16x8 a, bf16x8 b, floatx4 c) { return nb_mfma_bf16(a, b, c); }

template <int W, int NH>
struct B16 {
  static constexpr int RB = W / 16;
  static constexpr int KS = W / 32;
  static constexpr int FH = RB * KS;
  static constexpr int NFWD = RB + (NH - 1) * FH;   // first-layer step 0 and the hidden layers
  static constexpr int NALL = NFWD + RB;             // then first-layer step 1
  static constexpr int kBias = NH * W + W + 1;   // hidden biases, output weights, output bias
  static constexpr size_t lds_bytes() { return (size_t)NALL * 64 * 16 + (size_t)kBias * 4; }
};

// The hidden layers, output layer and decision of one wave's NB blocks of 16
// queries starting at q0 (queries >= n are padding), from the first layer's
// accumulators (bias included, before the ReLU); hidden-layer fragments and
// biases in LDS.  bad[nb]: the block's query column has a non-finite input
// (logit NaN, decided positive).  Writes logits / decisions of the valid
// queries and adds their confusion counts against g to cnt (when counts is
// non-null).
template <int W, int NH, int NB>
__device__ __forceinline__ void bf16_fwd_rest(floatx4 (&acc)[NB][W / 16], const bool (&bad)[NB],
                                              const bf16x8* __restrict__ swt, const float* __restrict__ sbias,
                                              int64_t n, int64_t q0, float tau, float* __restrict__ logits,
                                              uint8_t* __restrict__ hout, const uint8_t* __restrict__ g,
                                              const unsigned long long* counts, unsigned (&cnt)[4]) {
  using N = B16<W, NH>;
  constexpr int RB = N::RB, KS = N::KS;
  const int lane = threadIdx.x & 63, c = lane & 15, grp = lane >> 4;
  const float* swo = sbias + NH * W;
  const float bo = swo[W];
#pragma unroll
  for (int l = 1; l < NH; ++l) {
    bf16x8 act[NB][KS];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        float v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = acc[nb][2 * ks + j / 4][j % 4];
        act[nb][ks] = nb_relu_bf16x8(v);
      }
    const bf16x8* fr = swt + (RB + (l - 1) * N::FH) * 64 + lane;
    // row block mo's bias quad (16-byte aligned: sbias is, W is a multiple of 4)
    const floatx4* sb4 = reinterpret_cast<const floatx4*>(sbias + l * W) + grp;
    // two slots of fragments and bias: row block mo + 1's load while mo
    // computes, issued after mo's first K step so that the remaining K
    // steps' products cover their latency (all of them when KS = 1)
    constexpr int SPLITK = KS > 1 ? 1 : 0;
    bf16x8 fa[KS], fb[KS];
    floatx4 ba, bb;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) fa[ks] = fr[ks * 64];
    ba = sb4[0];
#pragma unroll
    for (int mo = 0; mo < RB; ++mo) {
      bf16x8(&cur)[KS] = (mo & 1) ? fb : fa;
      bf16x8(&nxt)[KS] = (mo & 1) ? fa : fb;
      floatx4& bcur = (mo & 1) ? bb : ba;
      floatx4& bnxt = (mo & 1) ? ba : bb;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[nb][mo] = bcur;
#pragma unroll
      for (int ks = 0; ks < SPLITK; ++ks)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb][mo] = mfma32(cur[ks], act[nb][ks], acc[nb][mo]);
      __builtin_amdgcn_sched_barrier(0);
      if (mo + 1 < RB) {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) nxt[ks] = fr[((mo + 1) * KS + ks) * 64];
        bnxt = sb4[4 * (mo + 1)];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int ks = SPLITK; ks < KS; ++ks)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb][mo] = mfma32(cur[ks], act[nb][ks], acc[nb][mo]);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    float p = 0.0f;
#pragma unroll
    for (int mo = 0; mo < RB; ++mo)
#pragma unroll
      for (int r = 0; r < 4; ++r) p = fmaf(swo[16 * mo + 4 * grp + r], nb_relu(acc[nb][mo][r]), p);
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
