// Neural early-out (Sec. 3, "Neural Early-out"): the queries a small bound
// reports positive are gathered into a dense batch for the larger bound,
// whose decisions are scattered back.  The compaction is the cascade's.
#include "nb_internal.h"

namespace {

constexpr int kThreads = 256;

// qc[t] = q[idx[t]] (rows of d floats) for t < *count.
__global__ void k_gather_rows(const float* __restrict__ q, int d, const int32_t* __restrict__ idx,
                              const unsigned long long* __restrict__ count, float* __restrict__ qc) {
  const int64_t m = (int64_t)*count * d;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = e / d;
    qc[e] = q[(int64_t)idx[t] * d + (e - t * d)];
  }
}

// h[idx[t]] = hc[t] for t < *count.
__global__ void k_scatter_u8(const uint8_t* __restrict__ hc, const int32_t* __restrict__ idx,
                             const unsigned long long* __restrict__ count, uint8_t* __restrict__ h) {
  const int64_t m = (int64_t)*count;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m; t += (int64_t)gridDim.x * blockDim.x)
    h[idx[t]] = hc[t];
}

unsigned grid_for(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + kThreads - 1) / kThreads, 8192)); }

}  // namespace

nb_status launch_gather_rows(const float* q, int d, const int32_t* idx, const unsigned long long* count, int64_t n_max,
                             float* qc, hipStream_t s) {
  k_gather_rows<<<grid_for(n_max * d), kThreads, 0, s>>>(q, d, idx, count, qc);
  NB_LAUNCHED();
  return NB_OK;
}

nb_status launch_scatter_u8(const uint8_t* hc, const int32_t* idx, const unsigned long long* count, int64_t n_max,
                            uint8_t* h, hipStream_t s) {
  k_scatter_u8<<<grid_for(n_max), kThreads, 0, s>>>(hc, idx, count, h);
  NB_LAUNCHED();
  return NB_OK;
}
