// k-DOP bounds optimised with the asymmetric loss (Sec. 4.1, "Methods": the
// paper's k-DOP planes trained with its loss; supplemental: k = 4).
//
// Parameters theta = [n_1 .. n_k (d each), lo_1 .. lo_k, hi_1 .. hi_k, s].
// A region's projection onto direction j is [u_j, v_j] (a point: n.x; a box
// with centre c and half extents e: n.c -+ sum |n_i| e_i; a segment
// o + t w, t in [0, 4]: min / max of n.o and n.(o + 4w)).  The logit is
// z = s min_j min(hi_j - u_j, v_j - lo_j); z >= 0 iff the projection meets
// every slab, a necessary condition for meeting the k-DOP, so a k-DOP that
// contains the indicator's support bounds every query kind conservatively.
// Decision and loss are the network's (Eq. 1, h = !(z < tau)).  Float32, one
// IEEE operation at a time in the written order.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "nb_internal.h"
#include "nb_adam.h"
#include "nb_mlp.h"

constexpr int kKdopMaxK = 8;
constexpr int kKdopThreads = 256;
constexpr int kKdopMaxWG = 256;

struct nb_kdop {
  int d = 0, k = 0, device = 0;
  int64_t P = 0, adam_t = 0;
  float* theta = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  float* partial = nullptr;   // [kKdopMaxWG][P]
  float* aux = nullptr;       // [kKdopMaxWG][8]: loss, TP, FP, TN, FN
  unsigned* nonfinite = nullptr;   // device flag: a training step met a non-finite loss or gradient
  float* batch_q = nullptr;
  uint8_t* batch_y = nullptr;
  int64_t batch_cap = 0;
};

namespace {

constexpr float kTmax = 4.0f;

// Parameters of one k-DOP, read from theta by every thread.
template <int D>
struct KdopParams {
  float n[kKdopMaxK][D];
  float lo[kKdopMaxK], hi[kKdopMaxK];
  float s;
  __device__ void load(const float* __restrict__ th, int k) {
#pragma unroll
    for (int j = 0; j < kKdopMaxK; ++j) {
#pragma unroll
      for (int i = 0; i < D; ++i) n[j][i] = j < k ? th[j * D + i] : 0.0f;
      lo[j] = j < k ? th[k * D + j] : 0.0f;
      hi[j] = j < k ? th[k * D + k + j] : 0.0f;
    }
    s = th[k * D + 2 * k];
  }
};

template <int D>
__device__ __forceinline__ float dot(const float (&a)[D], const float* b) {
  float p = a[0] * b[0];
#pragma unroll
  for (int i = 1; i < D; ++i) p = p + a[i] * b[i];
  return p;
}

// Projection interval of query row r on direction j.
template <int D, int KIND>
__device__ __forceinline__ void interval(const KdopParams<D>& P, int j, const float* r, float& u, float& v) {
  if (KIND == NB_QUERY_POINT) {
    u = v = dot<D>(P.n[j], r);
  } else if (KIND == NB_QUERY_BOX) {
    float c[D], e[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      c[i] = 0.5f * (r[i] + r[D + i]);
      e[i] = 0.5f * (r[D + i] - r[i]);
    }
    const float mid = dot<D>(P.n[j], c);
    float rad = fabsf(P.n[j][0]) * e[0];
#pragma unroll
    for (int i = 1; i < D; ++i) rad = rad + fabsf(P.n[j][i]) * e[i];
    u = mid - rad;
    v = mid + rad;
  } else {
    float f[D];
#pragma unroll
    for (int i = 0; i < D; ++i) f[i] = r[i] + kTmax * r[D + i];
    const float p0 = dot<D>(P.n[j], r), p1 = dot<D>(P.n[j], f);
    u = fminf(p0, p1);
    v = fmaxf(p0, p1);
  }
}

// Margin, arg-min direction (first on ties) and side (hi on ties).
template <int D, int KIND>
__device__ __forceinline__ float margin(const KdopParams<D>& P, int k, const float* r, int& jb, bool& side_hi) {
  float best = INFINITY;
  jb = 0;
  side_hi = true;
#pragma unroll
  for (int j = 0; j < kKdopMaxK; ++j) {
    if (j < k) {
      float u, v;
      interval<D, KIND>(P, j, r, u, v);
      const float up = P.hi[j] - u, dn = v - P.lo[j];
      const float mj = fminf(up, dn);
      if (mj < best) {
        best = mj;
        jb = j;
        side_hi = up <= dn;
      }
    }
  }
  return best;
}

constexpr int row_len(int D, int KIND) { return KIND == NB_QUERY_POINT ? D : 2 * D; }

template <int D, int KIND>
__global__ __launch_bounds__(kKdopThreads) void k_kdop_fwd(const float* __restrict__ theta, int k,
                                                           const float* __restrict__ q, int64_t n, float tau,
                                                           float* __restrict__ logits, uint8_t* __restrict__ hout,
                                                           const uint8_t* __restrict__ g,
                                                           unsigned long long* __restrict__ counts) {
  KdopParams<D> P;
  P.load(theta, k);
  constexpr int R = row_len(D, KIND);
  unsigned cnt[4] = {0u, 0u, 0u, 0u};
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t n_pad = (n + 63) / 64 * 64;   // whole waves, for the ballots
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_pad; i += stride) {
    const bool valid = i < n;
    float r[R];
    bool bad = false;
#pragma unroll
    for (int t = 0; t < R; ++t) {
      r[t] = valid ? q[i * R + t] : 0.0f;
      bad = bad || !isfinite(r[t]);
    }
    int jb;
    bool sh;
    const float m = P.s * margin<D, KIND>(P, k, r, jb, sh);
    const float z = bad ? __builtin_nanf("") : m;   // non-finite row: NaN, decided positive
    const bool pos = !(z < tau);
    if (valid) {
      if (logits) logits[i] = z;
      if (hout) hout[i] = pos;
    }
    if (counts) {
      const bool gv = valid && g[i] != 0;
      cnt[0] += __popcll(__ballot(valid && pos && gv));
      cnt[1] += __popcll(__ballot(valid && pos && !gv));
      cnt[2] += __popcll(__ballot(valid && !pos && !gv));
      cnt[3] += __popcll(__ballot(valid && !pos && gv));
    }
  }
  if (counts && (threadIdx.x & 63) == 0)
    for (int c = 0; c < 4; ++c)
      if (cnt[c]) atomicAdd(&counts[c], (unsigned long long)cnt[c]);
}

// One workgroup per chunk of the batch: Eq. 1, dL/dz and the gradient of z,
// summed per thread, then over the workgroup in a fixed order (butterfly in
// the wave, waves in order) into partial[blockIdx.x].
template <int D, int KIND>
__global__ __launch_bounds__(kKdopThreads) void k_kdop_train(const float* __restrict__ theta, int k,
                                                             const float* __restrict__ q,
                                                             const uint8_t* __restrict__ y, int64_t n, int64_t chunk,
                                                             float alpha, float beta, float inv_n, float tau,
                                                             float* __restrict__ partial, float* __restrict__ aux) {
  KdopParams<D> P;
  P.load(theta, k);
  constexpr int R = row_len(D, KIND);
  constexpr int G = kKdopMaxK * D + 2 * kKdopMaxK + 1;   // gradient slots (only k of each used)
  float gr[G];
#pragma unroll
  for (int t = 0; t < G; ++t) gr[t] = 0.0f;
  float lsum = 0.0f;
  unsigned cnt[4] = {0u, 0u, 0u, 0u};
  const int64_t first = (int64_t)blockIdx.x * chunk;
  const int64_t last = first + chunk < n ? first + chunk : n;
  for (int64_t i0 = first; i0 < last; i0 += blockDim.x) {
    const int64_t i = i0 + threadIdx.x;
    const bool valid = i < last;
    float r[R];
#pragma unroll
    for (int t = 0; t < R; ++t) r[t] = valid ? q[i * R + t] : 0.0f;
    int jb;
    bool sh;
    const float mg = margin<D, KIND>(P, k, r, jb, sh);
    const float z = P.s * mg;
    const bool yv = valid && y[i] != 0;
    const float e = expf(-fabsf(z));
    const float inv1pe = 1.0f / (1.0f + e);
    const float sig = z >= 0.0f ? inv1pe : e * inv1pe;
    const float sigm = z >= 0.0f ? e * inv1pe : inv1pe;
    const float dz = valid ? inv_n * (yv ? -alpha * sigm : beta * sig) : 0.0f;
    if (valid) {
      const float sp = log1pf(e);
      lsum += yv ? alpha * (fmaxf(-z, 0.0f) + sp) : beta * (fmaxf(z, 0.0f) + sp);
    }
    const bool pos = !(z < tau);
    cnt[0] += __popcll(__ballot(valid && pos && yv));
    cnt[1] += __popcll(__ballot(valid && pos && !yv));
    cnt[2] += __popcll(__ballot(valid && !pos && !yv));
    cnt[3] += __popcll(__ballot(valid && !pos && yv));
    // d u / d n and d v / d n of the active direction
    float du[D], dv[D];
    if (KIND == NB_QUERY_POINT) {
#pragma unroll
      for (int t = 0; t < D; ++t) du[t] = dv[t] = r[t];
    } else if (KIND == NB_QUERY_BOX) {
#pragma unroll
      for (int t = 0; t < D; ++t) {
        float nt = 0.0f;
#pragma unroll
        for (int j = 0; j < kKdopMaxK; ++j) nt = j == jb ? P.n[j][t] : nt;
        const float c = 0.5f * (r[t] + r[D + t]), ex = 0.5f * (r[D + t] - r[t]);
        const float sg = nt > 0.0f ? 1.0f : (nt < 0.0f ? -1.0f : 0.0f);
        du[t] = c - sg * ex;
        dv[t] = c + sg * ex;
      }
    } else {
      float nj[D], f[D];
#pragma unroll
      for (int t = 0; t < D; ++t) {
        float nt = 0.0f;
#pragma unroll
        for (int j = 0; j < kKdopMaxK; ++j) nt = j == jb ? P.n[j][t] : nt;
        nj[t] = nt;
        f[t] = r[t] + kTmax * r[D + t];
      }
      const bool first_low = dot<D>(nj, r) <= dot<D>(nj, f);
#pragma unroll
      for (int t = 0; t < D; ++t) {
        du[t] = first_low ? r[t] : f[t];
        dv[t] = first_low ? f[t] : r[t];
      }
    }
    const float ds = dz * P.s;
#pragma unroll
    for (int j = 0; j < kKdopMaxK; ++j) {
      if (j == jb && valid) {
        if (sh) {
          gr[kKdopMaxK * D + kKdopMaxK + j] += ds;
#pragma unroll
          for (int t = 0; t < D; ++t) gr[j * D + t] -= ds * du[t];
        } else {
          gr[kKdopMaxK * D + j] -= ds;
#pragma unroll
          for (int t = 0; t < D; ++t) gr[j * D + t] += ds * dv[t];
        }
      }
    }
    gr[G - 1] += valid ? dz * mg : 0.0f;
  }
  // fixed-order reduction: butterfly within the wave, then waves in order
  __shared__ float red[kKdopThreads / 64][G + 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int t = 0; t < G; ++t)
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) gr[t] += __shfl_xor(gr[t], m);
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) lsum += __shfl_xor(lsum, m);
  if (lane == 0) {
#pragma unroll
    for (int t = 0; t < G; ++t) red[wave][t] = gr[t];
    red[wave][G] = lsum;
  }
  __shared__ unsigned scnt[kKdopThreads / 64][4];
  if (lane == 0)
    for (int c = 0; c < 4; ++c) scnt[wave][c] = cnt[c];
  __syncthreads();
  const int P_all = k * D + 2 * k + 1;
  for (int p = threadIdx.x; p < P_all; p += blockDim.x) {
    // parameter p -> its slot in the padded gradient layout
    int slot;
    if (p < k * D) slot = (p / D) * D + p % D;
    else if (p < k * D + k) slot = kKdopMaxK * D + (p - k * D);
    else if (p < k * D + 2 * k) slot = kKdopMaxK * D + kKdopMaxK + (p - k * D - k);
    else slot = G - 1;
    float tot = red[0][slot];
    for (int w = 1; w < kKdopThreads / 64; ++w) tot += red[w][slot];
    partial[(int64_t)blockIdx.x * P_all + p] = tot;
  }
  if (threadIdx.x == 0) {
    float ls = red[0][G];
    unsigned cs[4] = {scnt[0][0], scnt[0][1], scnt[0][2], scnt[0][3]};
    for (int w = 1; w < kKdopThreads / 64; ++w) {
      ls += red[w][G];
      for (int c = 0; c < 4; ++c) cs[c] += scnt[w][c];
    }
    aux[blockIdx.x * 8] = ls;
    for (int c = 0; c < 4; ++c) aux[blockIdx.x * 8 + 1 + c] = __uint_as_float(cs[c]);
  }
}

// One block per parameter (and a last block for the loss and counts): the
// workgroup partials are summed by a fixed pairwise tree (deterministic), then
// Adam.
constexpr int kReduceThreads = 256;
static_assert(kKdopMaxWG <= kReduceThreads, "one reduction thread per training workgroup");

__global__ __launch_bounds__(kReduceThreads) void k_kdop_reduce(
    const float* __restrict__ partial, const float* __restrict__ aux, int n_wg, int P, float* __restrict__ theta,
    float* __restrict__ m, float* __restrict__ v, AdamArgs adam, float* __restrict__ loss, float loss_scale,
    unsigned long long* __restrict__ counts, unsigned* __restrict__ nonfinite) {
  __shared__ float sf[kReduceThreads];
  __shared__ unsigned long long sc[4][kReduceThreads];
  const int t = threadIdx.x, p = blockIdx.x;
  if (p < P) {
    sf[t] = t < n_wg ? partial[(int64_t)t * P + p] : 0.0f;
  } else {
    sf[t] = t < n_wg ? aux[t * 8] : 0.0f;
#pragma unroll
    for (int c = 0; c < 4; ++c) sc[c][t] = t < n_wg ? (unsigned long long)__float_as_uint(aux[t * 8 + 1 + c]) : 0ull;
  }
  __syncthreads();
  for (int h = kReduceThreads / 2; h > 0; h >>= 1) {
    if (t < h) {
      sf[t] += sf[t + h];
      if (p == P)
#pragma unroll
        for (int c = 0; c < 4; ++c) sc[c][t] += sc[c][t + h];
    }
    __syncthreads();
  }
  if (t != 0) return;
  if (!isfinite(sf[0])) *nonfinite = 1u;
  if (p < P) {
    nb_adam_update(p, sf[0], theta, m, v, adam, false);
  } else {
    if (loss) *loss = sf[0] * loss_scale;
    if (counts)
#pragma unroll
      for (int c = 0; c < 4; ++c) counts[c] = sc[c][0];
  }
}

unsigned fwd_grid(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + kKdopThreads - 1) / kKdopThreads, 4 * nb_cu_count()));
}

template <class F>
nb_status kdop_dispatch(int d, int kind, F&& f) {
  if (kind == NB_QUERY_POINT) {
    if (d == 2) return f(std::integral_constant<int, 2>(), std::integral_constant<int, NB_QUERY_POINT>());
    if (d == 3) return f(std::integral_constant<int, 3>(), std::integral_constant<int, NB_QUERY_POINT>());
    if (d == 4) return f(std::integral_constant<int, 4>(), std::integral_constant<int, NB_QUERY_POINT>());
  } else if (d == 3 && kind == NB_QUERY_BOX) {
    return f(std::integral_constant<int, 3>(), std::integral_constant<int, NB_QUERY_BOX>());
  } else if (d == 3 && kind == NB_QUERY_RAY) {
    return f(std::integral_constant<int, 3>(), std::integral_constant<int, NB_QUERY_RAY>());
  }
  nb_set_error("k-DOP bounds take points in 2-4 D and boxes or rays in 3-D (got kind %d in %d-D)", kind, d);
  return NB_ERR_UNSUPPORTED;
}

float tau_of(float eps) { return (float)std::log((0.5 - (double)eps) / (0.5 + (double)eps)); }

}  // namespace

extern "C" {

nb_status nb_kdop_destroy(nb_kdop* b) {
  if (!b) return NB_OK;
  for (float* p : {b->theta, b->m, b->v, b->partial, b->aux, b->batch_q})
    if (p) (void)hipFree(p);
  if (b->batch_y) (void)hipFree(b->batch_y);
  if (b->nonfinite) (void)hipFree(b->nonfinite);
  delete b;
  return NB_OK;
}

nb_status nb_kdop_create(int dim, int k, nb_kdop** out) {
  NB_REQUIRE(out, "NULL argument");
  *out = nullptr;
  NB_REQUIRE(dim >= 2 && dim <= 4, "dimension must be 2, 3 or 4");
  NB_REQUIRE(k >= 1 && k <= kKdopMaxK, "k must be in 1..%d", kKdopMaxK);
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    nb_set_error("no HIP device is visible");
    return NB_ERR_NO_DEVICE;
  }
  auto* b = new nb_kdop();
  b->d = dim;
  b->k = k;
  b->P = (int64_t)k * dim + 2 * k + 1;
  hipGetDevice(&b->device);
  bool ok = hipMalloc((void**)&b->theta, b->P * 4) == hipSuccess && hipMalloc((void**)&b->m, b->P * 4) == hipSuccess &&
            hipMalloc((void**)&b->v, b->P * 4) == hipSuccess &&
            hipMalloc((void**)&b->partial, (size_t)kKdopMaxWG * b->P * 4) == hipSuccess &&
            hipMalloc((void**)&b->aux, (size_t)kKdopMaxWG * 8 * 4) == hipSuccess &&
            hipMalloc((void**)&b->nonfinite, sizeof(unsigned)) == hipSuccess;
  ok = ok && hipMemset(b->theta, 0, b->P * 4) == hipSuccess && hipMemset(b->m, 0, b->P * 4) == hipSuccess &&
       hipMemset(b->v, 0, b->P * 4) == hipSuccess && hipMemset(b->nonfinite, 0, sizeof(unsigned)) == hipSuccess;
  if (!ok) {
    nb_set_error("allocating the k-DOP state failed");
    nb_kdop_destroy(b);
    return NB_ERR_OOM;
  }
  *out = b;
  return NB_OK;
}

nb_status nb_kdop_num_params(const nb_kdop* b, int64_t* n_params) {
  NB_REQUIRE(b && n_params, "NULL argument");
  *n_params = b->P;
  return NB_OK;
}

nb_status nb_kdop_set_params(nb_kdop* b, const float* theta, int64_t n_params, void* stream) {
  NB_REQUIRE(b && theta, "NULL argument");
  NB_REQUIRE(n_params == b->P, "the k-DOP has %lld parameters, got %lld", (long long)b->P, (long long)n_params);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  NB_HIP(hipMemcpyAsync(b->theta, theta, n_params * 4, hipMemcpyDeviceToDevice, s));
  NB_HIP(hipMemsetAsync(b->m, 0, n_params * 4, s));
  NB_HIP(hipMemsetAsync(b->v, 0, n_params * 4, s));
  b->adam_t = 0;
  return NB_OK;
}

nb_status nb_kdop_get_params(const nb_kdop* b, float* theta, int64_t n_params, void* stream) {
  NB_REQUIRE(b && theta, "NULL argument");
  NB_REQUIRE(n_params == b->P, "parameter count mismatch");
  NB_HIP(hipMemcpyAsync(theta, b->theta, n_params * 4, hipMemcpyDeviceToDevice, reinterpret_cast<hipStream_t>(stream)));
  return NB_OK;
}

nb_status nb_kdop_forward(const nb_kdop* b, int kind, const float* q, int64_t n, float eps, float* logits, uint8_t* h,
                          const uint8_t* g, uint64_t* counts, void* stream) {
  NB_REQUIRE(b && q, "NULL argument");
  NB_REQUIRE(logits || h || (g && counts), "nothing to compute");
  NB_REQUIRE(!counts || g, "counts need the exact answers g");
  NB_REQUIRE(n > 0, "n must be positive");
  NB_REQUIRE(eps >= 0.0f && eps < 0.5f, "eps must be in [0, 0.5)");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  auto* cnt = reinterpret_cast<unsigned long long*>(counts);
  if (cnt) NB_TRY(launch_zero_u64(cnt, 4, s));
  const float tau = tau_of(eps);
  return kdop_dispatch(b->d, kind, [&](auto dd, auto kk) -> nb_status {
    constexpr int D = decltype(dd)::value, KIND = decltype(kk)::value;
    k_kdop_fwd<D, KIND><<<fwd_grid(n), kKdopThreads, 0, s>>>(b->theta, b->k, q, n, tau, logits, h,
                                                              cnt ? g : nullptr, cnt);
    NB_LAUNCHED();
    return NB_OK;
  });
}

nb_status nb_kdop_train_step(nb_kdop* b, const nb_indicator* ind, int kind, uint64_t seed, uint64_t step,
                             int64_t batch, float alpha, float beta, float lr, float* loss, uint64_t* counts,
                             void* stream) {
  NB_REQUIRE(b && ind, "NULL argument");
  NB_REQUIRE(batch > 0 && batch <= (int64_t(1) << 30), "batch must be in 1..2^30");
  NB_REQUIRE(lr > 0 && std::isfinite(alpha) && std::isfinite(beta) && alpha >= 0 && beta >= 0,
             "invalid learning rate or loss weights");
  NB_REQUIRE(ind->dim == b->d, "the indicator is %d-D, the k-DOP %d-D", ind->dim, b->d);
  NB_REQUIRE(kind == NB_QUERY_POINT || (b->d == 3 && (kind == NB_QUERY_BOX || kind == NB_QUERY_RAY)),
             "k-DOP bounds take points in 2-4 D and boxes or rays in 3-D (got kind %d in %d-D)", kind, b->d);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (b->batch_cap < batch) {
    NB_HIP(hipStreamSynchronize(s));
    if (b->batch_q) (void)hipFree(b->batch_q);
    if (b->batch_y) (void)hipFree(b->batch_y);
    b->batch_q = nullptr;
    b->batch_y = nullptr;
    b->batch_cap = 0;
    NB_HIP(hipMalloc((void**)&b->batch_q, (size_t)batch * 8 * 4));
    NB_HIP(hipMalloc((void**)&b->batch_y, (size_t)batch));
    b->batch_cap = batch;
  }
  NB_TRY(launch_sample(kind, ind->dim, seed, step, batch, b->batch_q, s));
  NB_TRY(launch_query_exact(ind, kind, b->batch_q, batch, b->batch_y, s));
  const int n_wg = (int)std::min<int64_t>(kKdopMaxWG, (batch + kKdopThreads - 1) / kKdopThreads);
  const int64_t chunk = (batch + n_wg - 1) / n_wg;
  const float tau = tau_of(1e-5f);
  const float inv_n = (float)(1.0 / (double)batch);
  NB_TRY(kdop_dispatch(b->d, kind, [&](auto dd, auto kk) -> nb_status {
    constexpr int D = decltype(dd)::value, KIND = decltype(kk)::value;
    k_kdop_train<D, KIND><<<n_wg, kKdopThreads, 0, s>>>(b->theta, b->k, b->batch_q, b->batch_y, batch, chunk, alpha,
                                                         beta, inv_n, tau, b->partial, b->aux);
    NB_LAUNCHED();
    return NB_OK;
  }));
  b->adam_t += 1;
  AdamArgs a{};
  a.enabled = 1;
  a.lr = lr;
  a.b1 = 0.9f;
  a.b2 = 0.999f;
  a.eps = 1e-8f;
  a.bc1 = (float)(1.0 - std::pow((double)a.b1, (double)b->adam_t));
  a.bc2 = (float)(1.0 - std::pow((double)a.b2, (double)b->adam_t));
  k_kdop_reduce<<<(unsigned)b->P + 1, kReduceThreads, 0, s>>>(b->partial, b->aux, n_wg, (int)b->P, b->theta, b->m,
                                                               b->v, a, loss, inv_n,
                                                               reinterpret_cast<unsigned long long*>(counts),
                                                               b->nonfinite);
  NB_LAUNCHED();
  return NB_OK;
}

nb_status nb_kdop_sync(nb_kdop* b, void* stream) {
  NB_REQUIRE(b, "k-DOP is NULL");
  NB_HIP(hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)));
  unsigned flag = 0;
  NB_HIP(hipMemcpy(&flag, b->nonfinite, sizeof(flag), hipMemcpyDeviceToHost));
  if (flag) {
    NB_HIP(hipMemset(b->nonfinite, 0, sizeof(unsigned)));
    nb_set_error("a k-DOP training step since the last check met a non-finite loss or gradient");
    return NB_ERR_NONFINITE;
  }
  return NB_OK;
}

}  // extern "C"
