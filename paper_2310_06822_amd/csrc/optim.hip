// Gradient reduction and Adam (Sec. 3.4, "Training": Adam at learning rate
// 1e-3; Kingma & Ba 2014, Algorithm 1, with beta1 0.9, beta2 0.999,
// epsilon 1e-8 unless the caller says otherwise).
//
// The training kernel leaves one partial gradient per workgroup.  The sum
// over workgroups is taken here in a fixed order (8 interleaved strided
// partial sums per parameter, then added 0..7), so a given batch size always
// gives bit-identical gradients.  Optional L1 + L2 regularisation of the
// weight matrices (supplemental "Regularization") adds
// lam1 sign(W) + 2 lam2 W to their gradient.
#include "nb_internal.h"
#include "nb_adam.h"
#include "nb_mlp.h"

namespace {

constexpr int kParamsPerBlock = 32;
constexpr int kParts = 8;

__device__ __forceinline__ void adam_update(int64_t p, float g, float* __restrict__ theta, float* __restrict__ m,
                                            float* __restrict__ v, const AdamArgs& a, int in_dim, int width,
                                            int n_hidden) {
  nb_adam_update(p, g, theta, m, v, a, nb_is_weight(p, in_dim, width, n_hidden) != 0);
}

__global__ __launch_bounds__(256) void k_reduce(const float* __restrict__ partial, const float* __restrict__ aux,
                                                int n_wg, int64_t P, float* __restrict__ grad,
                                                float* __restrict__ theta, float* __restrict__ m,
                                                float* __restrict__ v, AdamArgs adam, int in_dim, int width,
                                                int n_hidden, float* __restrict__ loss, float loss_scale,
                                                unsigned long long* __restrict__ counts,
                                                unsigned* __restrict__ nonfinite, float* __restrict__ pack) {
  __shared__ float part[kParts][kParamsPerBlock];
  const int t = threadIdx.x, j = t % kParamsPerBlock, k = t / kParamsPerBlock;
  const int64_t p = (int64_t)blockIdx.x * kParamsPerBlock + j;
  float s = 0.0f;
  if (p < P) {
    // partials k, k + 8, k + 16, ... added in that order; eight loads are in
    // flight at a time instead of one per add
    const float* src = partial + p;
    int w = k;
    for (; w + 7 * kParts < n_wg; w += 8 * kParts) {
      float x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) x[u] = src[(int64_t)(w + u * kParts) * P];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += x[u];
    }
    for (; w < n_wg; w += kParts) s += src[(int64_t)w * P];
  }
  part[k][j] = s;
  __syncthreads();
  if (t < kParamsPerBlock && p < P) {
    float tot = part[0][t];
#pragma unroll
    for (int i = 1; i < kParts; ++i) tot += part[i][t];
    if (grad) grad[p] = tot;
    if (!isfinite(tot)) *nonfinite = 1u;
    if (adam.enabled) {
      adam_update(p, tot, theta, m, v, adam, in_dim, width, n_hidden);
      // float32 bounds: the updated weight goes straight to its packed slots
      if (pack) nb_f32_pack_put(p, theta[p], pack, in_dim, width, n_hidden);
    }
  }
  // loss and counts: the last block's first wave, lanes strided over workgroups
  if (blockIdx.x == gridDim.x - 1 && t < 64) {
    float ls = 0.0f;
    unsigned long long cs[4] = {0, 0, 0, 0};
    for (int w = t; w < n_wg; w += 64) {
      ls += aux[w * 8];
      for (int i = 0; i < 4; ++i) cs[i] += __float_as_uint(aux[w * 8 + 1 + i]);
    }
    for (int msk = 1; msk < 64; msk <<= 1) {
      ls += __shfl_xor(ls, msk);
      for (int i = 0; i < 4; ++i) cs[i] += __shfl_xor(cs[i], msk);
    }
    if (t == 0) {
      if (!isfinite(ls)) *nonfinite = 1u;
      if (loss) *loss = ls * loss_scale;
      if (counts)
        for (int i = 0; i < 4; ++i) counts[i] = cs[i];
    }
  }
}

__global__ void k_adam(const float* __restrict__ grad, int64_t P, float* __restrict__ theta, float* __restrict__ m,
                       float* __restrict__ v, AdamArgs adam, int in_dim, int width, int n_hidden) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < P) adam_update(p, grad[p], theta, m, v, adam, in_dim, width, n_hidden);
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

}  // namespace

nb_status launch_reduce(const nb_bound* b, int n_wg, float* grad, float* loss, float loss_scale,
                        unsigned long long* counts, const AdamArgs& adam, hipStream_t s, bool pack_f32) {
  const int64_t P = b->n_params;
  const unsigned grid = (unsigned)((P + kParamsPerBlock - 1) / kParamsPerBlock);
  float* pack = pack_f32 && adam.enabled && b->precision == NB_F32 ? b->pack : nullptr;
  k_reduce<<<grid, 256, 0, s>>>(b->partial, b->aux, n_wg, P, grad, b->theta, b->m, b->v, adam, b->in_dim,
                                b->width, b->n_hidden, loss, loss_scale, counts, b->d_nonfinite, pack);
  NB_LAUNCHED();
  return NB_OK;
}

nb_status launch_adam(const nb_bound* b, const float* grad, const AdamArgs& adam, hipStream_t s) {
  const int64_t P = b->n_params;
  k_adam<<<(unsigned)((P + 255) / 256), 256, 0, s>>>(grad, P, b->theta, b->m, b->v, adam, b->in_dim, b->width,
                                                     b->n_hidden);
  NB_LAUNCHED();
  return NB_OK;
}

nb_status launch_zero_u64(unsigned long long* p, int n, hipStream_t s) {
  if (n <= 0) return NB_OK;
  k_zero_u64<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n);
  NB_LAUNCHED();
  return NB_OK;
}
