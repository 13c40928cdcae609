// Region sampling for training batches (Alg. 1, "Uniform").
//
// Counter-based: every query is an independent function of (seed, query
// index, step), so a batch is reproducible and any slice of it can be drawn
// by any thread.  The generator is Philox4x32-10 (Salmon, Moraes, Dror,
// Shaw, SC'11), written from its published definition.  The draw rules
// (streams, attempts, transforms) are stated in nbound.h beside
// nb_sample_queries; every float operation is one IEEE float32 operation
// (this file is compiled without floating-point contraction).
#include "nb_internal.h"

namespace {

struct U4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
  constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const uint32_t hi0 = __umulhi(M0, c.x), lo0 = M0 * c.x;
    const uint32_t hi1 = __umulhi(M1, c.z), lo1 = M1 * c.z;
    c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
  }
  return c;
}

__device__ __forceinline__ float u01(uint32_t w) { return (float)(w >> 8) * 0x1.0p-24f; }

struct Draw {
  float a, b, c, d;
};

__device__ __forceinline__ Draw uniforms(uint64_t seed, uint32_t i, uint32_t step, uint32_t stream,
                                         uint32_t attempt) {
  const U4 w = philox4x32_10(U4{i, step, stream, attempt}, (uint32_t)seed, (uint32_t)(seed >> 32));
  return Draw{u01(w.x), u01(w.y), u01(w.z), u01(w.w)};
}

constexpr int kMaxAttempts = 64;

// Origin uniform in the radius-2 ball: 4u - 2, first accepted attempt.
__device__ void ball2(uint64_t seed, uint32_t i, uint32_t step, uint32_t stream, float o[3]) {
  o[0] = o[1] = o[2] = 0.0f;
  for (int a = 0; a < kMaxAttempts; ++a) {
    const Draw u = uniforms(seed, i, step, stream, a);
    const float x = 4.0f * u.a - 2.0f, y = 4.0f * u.b - 2.0f, z = 4.0f * u.c - 2.0f;
    const float r2 = (x * x + y * y) + z * z;
    if (r2 <= 4.0f) {
      o[0] = x;
      o[1] = y;
      o[2] = z;
      return;
    }
  }
}

// Unit vector uniform on the sphere: normalised rejection from the unit ball.
__device__ void unit_dir(uint64_t seed, uint32_t i, uint32_t step, uint32_t stream, float d[3]) {
  d[0] = 0.0f;
  d[1] = 0.0f;
  d[2] = 1.0f;
  for (int a = 0; a < kMaxAttempts; ++a) {
    const Draw u = uniforms(seed, i, step, stream, a);
    const float x = 2.0f * u.a - 1.0f, y = 2.0f * u.b - 1.0f, z = 2.0f * u.c - 1.0f;
    const float r2 = (x * x + y * y) + z * z;
    if (r2 <= 1.0f && r2 > 1e-6f) {
      const float r = sqrtf(r2);
      d[0] = x / r;
      d[1] = y / r;
      d[2] = z / r;
      return;
    }
  }
}

__global__ void k_sample_points(uint64_t seed, uint32_t step, int64_t n, int dim, float* __restrict__ q) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Draw u = uniforms(seed, (uint32_t)i, step, 0, 0);
  float* out = q + i * dim;
  out[0] = 2.0f * u.a - 1.0f;
  out[1] = 2.0f * u.b - 1.0f;
  if (dim >= 3) out[2] = 2.0f * u.c - 1.0f;
  if (dim == 4) out[3] = u.d;
}

__global__ void k_sample_rays(uint64_t seed, uint32_t step, int64_t n, float* __restrict__ q) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float o[3], d[3];
  ball2(seed, (uint32_t)i, step, 1, o);
  unit_dir(seed, (uint32_t)i, step, 2, d);
  float* out = q + i * 6;
  out[0] = o[0];
  out[1] = o[1];
  out[2] = o[2];
  out[3] = d[0];
  out[4] = d[1];
  out[5] = d[2];
}

__global__ void k_sample_boxes(uint64_t seed, uint32_t step, int64_t n, float* __restrict__ q) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Draw uc = uniforms(seed, (uint32_t)i, step, 3, 0);
  const Draw uh = uniforms(seed, (uint32_t)i, step, 4, 0);
  const float c[3] = {2.0f * uc.a - 1.0f, 2.0f * uc.b - 1.0f, 2.0f * uc.c - 1.0f};
  const float h[3] = {0.19f * uh.a + 0.01f, 0.19f * uh.b + 0.01f, 0.19f * uh.c + 0.01f};
  float* out = q + i * 6;
  for (int a = 0; a < 3; ++a) {
    out[a] = c[a] - h[a];
    out[3 + a] = c[a] + h[a];
  }
}

__global__ void k_sample_planes(uint64_t seed, uint32_t step, int64_t n, float* __restrict__ q) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Draw u = uniforms(seed, (uint32_t)i, step, 5, 0);
  float d[3];
  unit_dir(seed, (uint32_t)i, step, 6, d);
  float* out = q + i * 6;
  out[0] = 2.0f * u.a - 1.0f;
  out[1] = 2.0f * u.b - 1.0f;
  out[2] = 2.0f * u.c - 1.0f;
  out[3] = d[0];
  out[4] = d[1];
  out[5] = d[2];
}

}  // namespace

nb_status launch_sample(int kind, int dim, uint64_t seed, uint64_t step, int64_t n, float* q, hipStream_t s) {
  NB_REQUIRE(q != nullptr, "q is NULL");
  NB_REQUIRE(n > 0 && n <= (int64_t(1) << 32), "n must be in 1..2^32 (query index is a 32-bit counter word)");
  NB_REQUIRE(step <= 0xFFFFFFFFull, "step must fit in 32 bits");
  const int threads = 256;
  const unsigned blocks = (unsigned)((n + threads - 1) / threads);
  switch (kind) {
    case NB_QUERY_POINT:
      NB_REQUIRE(dim >= 2 && dim <= 4, "point dimension must be 2, 3 or 4");
      k_sample_points<<<blocks, threads, 0, s>>>(seed, (uint32_t)step, n, dim, q);
      break;
    case NB_QUERY_RAY:
      k_sample_rays<<<blocks, threads, 0, s>>>(seed, (uint32_t)step, n, q);
      break;
    case NB_QUERY_BOX:
      k_sample_boxes<<<blocks, threads, 0, s>>>(seed, (uint32_t)step, n, q);
      break;
    case NB_QUERY_PLANE:
      k_sample_planes<<<blocks, threads, 0, s>>>(seed, (uint32_t)step, n, q);
      break;
    default:
      NB_REQUIRE(false, "unknown query kind %d", kind);
  }
  NB_LAUNCHED();
  return NB_OK;
}
