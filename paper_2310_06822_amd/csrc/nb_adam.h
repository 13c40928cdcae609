// One Adam step on one parameter (Kingma & Ba 2014, Algorithm 1), shared by
// the single-bound and grouped optimisers.  Weight-matrix entries also get
// the L1 + L2 regularisation gradient lam1 sign(w) + 2 lam2 w.
#pragma once

#include "nb_internal.h"

__device__ __forceinline__ void nb_adam_update(int64_t p, float g, float* __restrict__ theta, float* __restrict__ m,
                                               float* __restrict__ v, const AdamArgs& a, bool is_weight) {
  const float th = theta[p];
  if ((a.lam1 != 0.0f || a.lam2 != 0.0f) && is_weight) {
    const float sg = th > 0.0f ? 1.0f : (th < 0.0f ? -1.0f : 0.0f);
    g = g + (a.lam1 * sg + 2.0f * a.lam2 * th);
  }
  const float mm = a.b1 * m[p] + (1.0f - a.b1) * g;
  const float vv = a.b2 * v[p] + (1.0f - a.b2) * (g * g);
  m[p] = mm;
  v[p] = vv;
  const float mhat = mm / a.bc1;
  const float vhat = vv / a.bc2;
  theta[p] = th - a.lr * mhat / (sqrtf(vhat) + a.eps);
}
