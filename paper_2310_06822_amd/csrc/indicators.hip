// Indicators f and exact region queries g (Sec. 3.1; Sec. 4.2 "Query types":
// g is any() of the indicator over the region).
//
// All geometry is float32, one IEEE operation at a time in the order written
// (this file is compiled without floating-point contraction, with correctly
// rounded division and square root), so the 0/1 answers are reproducible bit
// for bit by any implementation that follows the same expressions.
//
// Voxel grids cover [-1, 1]^3, x fastest (index (k*n + j)*n + i).  A
// coordinate p in [-1, 1] lies in cell floor((p + 1) * (n/2)), clamped to
// n - 1 at p = 1; a point with a coordinate outside the cube (or NaN) has
// f = 0.
#include <algorithm>

#include "nb_internal.h"
#include "nb_voxel.h"

namespace {

constexpr int kThreads = 256;

// Everything an exact query needs, passed to kernels by value.
struct IndView {
  int type, k, n;
  float iso;
  const float* params;
  const uint8_t* grid;
  const float* ray_t;
  const int32_t* occupied;
  const int64_t* occupied_count;
};

IndView view_of(const nb_indicator* ind) {
  return IndView{ind->type, ind->k, ind->n, ind->iso, ind->params, ind->grid, ind->ray_t, ind->occupied,
                 ind->occupied_count};
}

// ------------------------------------------------------------------- points

// f = OR_b ((x - cx)^2 + (y - cy)^2 <= r^2).
__device__ __forceinline__ uint8_t discs2d_at(const float* __restrict__ row, const float* __restrict__ discs, int k) {
  const float x = row[0], y = row[1];
  uint8_t hit = 0;
  for (int b = 0; b < k; ++b) {
    const float dx = x - discs[3 * b], dy = y - discs[3 * b + 1], r = discs[3 * b + 2];
    const float d2 = dx * dx + dy * dy;
    hit |= (d2 <= r * r);
  }
  return hit;
}

// f = 1 iff sum_b R_b^2 / |x - (a_b + t d_b)|^2 >= iso.
__device__ __forceinline__ uint8_t metaballs4d_at(const float* __restrict__ row, const float* __restrict__ prm, int k,
                                                  float iso) {
  const float x = row[0], y = row[1], z = row[2], t = row[3];
  const float* a = prm;           // [k][3] path starts
  const float* d = prm + 3 * k;   // [k][3] b - a
  const float* r = prm + 6 * k;   // [k] radii
  float acc = 0.0f;
  for (int b = 0; b < k; ++b) {
    const float dx = x - (a[3 * b] + t * d[3 * b]);
    const float dy = y - (a[3 * b + 1] + t * d[3 * b + 1]);
    const float dz = z - (a[3 * b + 2] + t * d[3 * b + 2]);
    const float d2 = (dx * dx + dy * dy) + dz * dz;
    acc = acc + (r[b] * r[b]) / d2;
  }
  return acc >= iso;
}

// ------------------------------------------------------------------- planes

// g = 1 iff an occupied cell (centre c, half width 1/n) meets the plane:
// |n.(c - p0)| <= (1/n) (|n_x| + |n_y| + |n_z|), dot product summed x, y, z.
__device__ __forceinline__ uint8_t voxel_plane_at(const float* __restrict__ row, const int32_t* __restrict__ occ,
                                                  const int64_t* __restrict__ n_occ, int gn) {
  const float px = row[0], py = row[1], pz = row[2], nx = row[3], ny = row[4], nz = row[5];
  const float h = (float)(1.0 / (double)gn);
  const float rad = h * ((fabsf(nx) + fabsf(ny)) + fabsf(nz));
  const int64_t m = *n_occ;
  for (int64_t c = 0; c < m; ++c) {
    const int32_t idx = occ[c];
    const int ix = idx % gn, jy = (idx / gn) % gn, kz = idx / (gn * gn);
    const float cx = (float)((2.0 * ix + 1.0) / gn - 1.0);
    const float cy = (float)((2.0 * jy + 1.0) / gn - 1.0);
    const float cz = (float)((2.0 * kz + 1.0) / gn - 1.0);
    const float e = (nx * (cx - px) + ny * (cy - py)) + nz * (cz - pz);
    if (fabsf(e) <= rad) return 1;
  }
  return 0;
}

// ------------------------------------------------------------- dispatch

template <int KIND>
__device__ __forceinline__ uint8_t exact_at(const IndView& v, const float* __restrict__ q, int64_t i) {
  if (KIND == NB_QUERY_POINT) {
    if (v.type == IND_DISCS2D) return discs2d_at(q + 2 * i, v.params, v.k);
    if (v.type == IND_METABALLS4D) return metaballs4d_at(q + 4 * i, v.params, v.k, v.iso);
    const float* r = q + 3 * i;
    return voxel_at(v.grid, v.n, (float)v.n * 0.5f, r[0], r[1], r[2]);
  }
  if (KIND == NB_QUERY_RAY) return voxel_ray_at(q + 6 * i, v.grid, v.n, v.ray_t);
  if (KIND == NB_QUERY_BOX) return voxel_box_at(q + 6 * i, v.grid, v.n);
  return voxel_plane_at(q + 6 * i, v.occupied, v.occupied_count, v.n);
}

template <int KIND>
__global__ void k_exact(IndView v, const float* __restrict__ q, int64_t n, uint8_t* __restrict__ g) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  g[i] = exact_at<KIND>(v, q, i);
}

// ------------------------------------------------------------- cascade

// Indices of the queries the bound calls positive.  Each block takes 4096
// queries, builds its list with wave ballots and an LDS prefix, and reserves
// its slice of the output with a single atomic (order between blocks is
// arbitrary; every positive appears once).
constexpr int kCompactPer = 16;   // queries per thread

__global__ __launch_bounds__(256) void k_compact_positive(const uint8_t* __restrict__ h, int64_t n,
                                                          int32_t* __restrict__ idx,
                                                          unsigned long long* __restrict__ count) {
  __shared__ int wave_tot[4];
  __shared__ unsigned long long block_base;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t base = (int64_t)blockIdx.x * 256 * kCompactPer;
  unsigned long long masks[kCompactPer];
  int tot = 0;
#pragma unroll
  for (int k = 0; k < kCompactPer; ++k) {
    const int64_t i = base + (int64_t)k * 256 + threadIdx.x;
    masks[k] = __ballot(i < n && h[i] != 0);
    tot += __popcll(masks[k]);
  }
  if (lane == 0) wave_tot[wave] = tot;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int all = wave_tot[0] + wave_tot[1] + wave_tot[2] + wave_tot[3];
    block_base = all ? atomicAdd(count, (unsigned long long)all) : 0ull;
  }
  __syncthreads();
  unsigned long long off = block_base;
  for (int w = 0; w < wave; ++w) off += wave_tot[w];
  const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
  for (int k = 0; k < kCompactPer; ++k) {
    if (masks[k] >> lane & 1ull) idx[off + __popcll(masks[k] & below)] = (int32_t)(base + (int64_t)k * 256 + threadIdx.x);
    off += __popcll(masks[k]);
  }
}

// answer[idx[t]] = g(q[idx[t]]) for every listed positive (grid-stride).
template <int KIND>
__global__ void k_cascade_exact(IndView v, const float* __restrict__ q, const int32_t* __restrict__ idx,
                                const unsigned long long* __restrict__ count, uint8_t* __restrict__ answer) {
  const int64_t m = (int64_t)*count;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx[t];
    answer[i] = exact_at<KIND>(v, q, i);
  }
}

// ----------------------------------------------------------- voxelisation

// grid[(k*n + j)*n + i] = 1 iff sum_b R_b^2 / |c - c_b|^2 >= iso at the cell
// centre c = (2i + 1)/n - 1 (computed in double, rounded once).
__global__ void k_voxelize(const float* __restrict__ prm, int k, float iso, int gn, uint8_t* __restrict__ grid) {
  const int64_t cells = (int64_t)gn * gn * gn;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= cells) return;
  const int ix = (int)(idx % gn), jy = (int)((idx / gn) % gn), kz = (int)(idx / ((int64_t)gn * gn));
  const float x = (float)((2.0 * ix + 1.0) / gn - 1.0);
  const float y = (float)((2.0 * jy + 1.0) / gn - 1.0);
  const float z = (float)((2.0 * kz + 1.0) / gn - 1.0);
  const float* c = prm;          // [k][3]
  const float* r = prm + 3 * k;  // [k]
  float acc = 0.0f;
  for (int b = 0; b < k; ++b) {
    const float dx = x - c[3 * b], dy = y - c[3 * b + 1], dz = z - c[3 * b + 2];
    const float d2 = (dx * dx + dy * dy) + dz * dz;
    acc = acc + (r[b] * r[b]) / d2;
  }
  grid[idx] = acc >= iso;
}

// Occupied-cell list in increasing index order (one block per 256 cells,
// a block-wide prefix over a ballot; blocks appended in order by a serial
// second pass would cost a launch, so the list is built by a single block).
__global__ void k_collect_occupied(const uint8_t* __restrict__ grid, int64_t cells, int32_t* __restrict__ out,
                                   int64_t* __restrict__ count) {
  __shared__ int64_t base;
  __shared__ int wave_cnt[kThreads / 64];
  if (threadIdx.x == 0) base = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t start = 0; start < cells; start += kThreads) {
    const int64_t idx = start + threadIdx.x;
    const bool occ = idx < cells && grid[idx] != 0;
    const unsigned long long m = __ballot(occ);
    if (lane == 0) wave_cnt[wave] = __popcll(m);
    __syncthreads();
    int64_t off = base;
    for (int w = 0; w < wave; ++w) off += wave_cnt[w];
    if (occ) out[off + __popcll(m & ((1ull << lane) - 1ull))] = (int32_t)idx;
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t t = 0;
      for (int w = 0; w < kThreads / 64; ++w) t += wave_cnt[w];
      base += t;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *count = base;
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

}  // namespace

nb_status launch_query_exact(const nb_indicator* ind, int kind, const float* q, int64_t n, uint8_t* g,
                             hipStream_t s) {
  NB_REQUIRE(ind != nullptr, "indicator is NULL");
  NB_REQUIRE(q != nullptr && g != nullptr, "q and g must be non-NULL");
  NB_REQUIRE(n > 0, "n must be positive");
  NB_REQUIRE(n <= (int64_t(1) << 40), "n too large");
  NB_REQUIRE(kind == NB_QUERY_POINT || ind->type == IND_VOXELS, "ray, box and plane queries need a voxel indicator");
  const unsigned blocks = blocks_for(n);
  const IndView v = view_of(ind);
  switch (kind) {
    case NB_QUERY_POINT: k_exact<NB_QUERY_POINT><<<blocks, kThreads, 0, s>>>(v, q, n, g); break;
    case NB_QUERY_RAY: k_exact<NB_QUERY_RAY><<<blocks, kThreads, 0, s>>>(v, q, n, g); break;
    case NB_QUERY_BOX: k_exact<NB_QUERY_BOX><<<blocks, kThreads, 0, s>>>(v, q, n, g); break;
    case NB_QUERY_PLANE: k_exact<NB_QUERY_PLANE><<<blocks, kThreads, 0, s>>>(v, q, n, g); break;
    default: NB_REQUIRE(false, "unknown query kind %d", kind);
  }
  NB_LAUNCHED();
  return NB_OK;
}

nb_status launch_compact_positive(const uint8_t* h, int64_t n, int32_t* idx, unsigned long long* count, hipStream_t s) {
  k_compact_positive<<<(unsigned)((n + 256 * kCompactPer - 1) / (256 * kCompactPer)), 256, 0, s>>>(h, n, idx, count);
  NB_LAUNCHED();
  return NB_OK;
}

nb_status launch_cascade_exact(const nb_indicator* ind, int kind, const float* q, const uint8_t* h, int64_t n,
                               int32_t* idx, unsigned long long* count, uint8_t* answer, hipStream_t s) {
  NB_REQUIRE(kind == NB_QUERY_POINT || ind->type == IND_VOXELS, "ray, box and plane queries need a voxel indicator");
  NB_REQUIRE(n <= (int64_t)0x7FFFFFFF, "cascade handles at most 2^31 - 1 queries per call");
  k_compact_positive<<<(unsigned)((n + 256 * kCompactPer - 1) / (256 * kCompactPer)), 256, 0, s>>>(h, n, idx, count);
  NB_LAUNCHED();
  const IndView v = view_of(ind);
  const unsigned blocks = (unsigned)std::min<int64_t>(blocks_for(n), 4096);
  switch (kind) {
    case NB_QUERY_POINT: k_cascade_exact<NB_QUERY_POINT><<<blocks, kThreads, 0, s>>>(v, q, idx, count, answer); break;
    case NB_QUERY_RAY: k_cascade_exact<NB_QUERY_RAY><<<blocks, kThreads, 0, s>>>(v, q, idx, count, answer); break;
    case NB_QUERY_BOX: k_cascade_exact<NB_QUERY_BOX><<<blocks, kThreads, 0, s>>>(v, q, idx, count, answer); break;
    case NB_QUERY_PLANE: k_cascade_exact<NB_QUERY_PLANE><<<blocks, kThreads, 0, s>>>(v, q, idx, count, answer); break;
    default: NB_REQUIRE(false, "unknown query kind %d", kind);
  }
  NB_LAUNCHED();
  return NB_OK;
}

nb_status launch_voxelize(const float* params_dev, int k, float iso, int n, uint8_t* grid, hipStream_t s) {
  const int64_t cells = (int64_t)n * n * n;
  k_voxelize<<<blocks_for(cells), kThreads, 0, s>>>(params_dev, k, iso, n, grid);
  NB_LAUNCHED();
  return NB_OK;
}

nb_status launch_collect_occupied(const uint8_t* grid, int64_t cells, int32_t* out, int64_t* count_dev,
                                  hipStream_t s) {
  k_collect_occupied<<<1, kThreads, 0, s>>>(grid, cells, out, count_dev);
  NB_LAUNCHED();
  return NB_OK;
}
