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
#include "nb_internal.h"

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ bool cell_of(float p, int n, float half_n, int& c) {
  if (!(p >= -1.0f && p <= 1.0f)) return false;
  const float s = (p + 1.0f) * half_n;   // in [0, n]
  const int i = (int)s;                  // s >= 0: truncation is floor
  c = i < n - 1 ? i : n - 1;
  return true;
}

__device__ __forceinline__ uint8_t voxel_at(const uint8_t* __restrict__ grid, int n, float half_n, float x,
                                            float y, float z) {
  int i, j, k;
  if (!cell_of(x, n, half_n, i) || !cell_of(y, n, half_n, j) || !cell_of(z, n, half_n, k)) return 0;
  return grid[((int64_t)k * n + j) * n + i] != 0;
}

// ------------------------------------------------------------------- points

__global__ void k_discs2d(const float* __restrict__ q, int64_t n, const float* __restrict__ discs, int k,
                          uint8_t* __restrict__ g) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float x = q[2 * i], y = q[2 * i + 1];
  uint8_t hit = 0;
  for (int b = 0; b < k; ++b) {
    const float dx = x - discs[3 * b], dy = y - discs[3 * b + 1], r = discs[3 * b + 2];
    const float d2 = dx * dx + dy * dy;
    hit |= (d2 <= r * r);
  }
  g[i] = hit;
}

__global__ void k_voxel_points(const float* __restrict__ q, int64_t n, const uint8_t* __restrict__ grid, int gn,
                               uint8_t* __restrict__ g) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  g[i] = voxel_at(grid, gn, (float)gn * 0.5f, q[3 * i], q[3 * i + 1], q[3 * i + 2]);
}

__global__ void k_metaballs4d(const float* __restrict__ q, int64_t n, const float* __restrict__ prm, int k,
                              float iso, uint8_t* __restrict__ g) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float x = q[4 * i], y = q[4 * i + 1], z = q[4 * i + 2], t = q[4 * i + 3];
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
  g[i] = acc >= iso;
}

// --------------------------------------------------------------------- rays

// g = max_j f(o + t_j d) over the sample table; stops at the first hit.
__global__ void k_voxel_rays(const float* __restrict__ q, int64_t n, const uint8_t* __restrict__ grid, int gn,
                             const float* __restrict__ ray_t, uint8_t* __restrict__ g) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float ox = q[6 * i], oy = q[6 * i + 1], oz = q[6 * i + 2];
  const float dx = q[6 * i + 3], dy = q[6 * i + 4], dz = q[6 * i + 5];
  const float half_n = (float)gn * 0.5f;
  uint8_t hit = 0;
  for (int j = 0; j < 256 && !hit; ++j) {
    const float t = ray_t[j];
    hit = voxel_at(grid, gn, half_n, ox + t * dx, oy + t * dy, oz + t * dz);
  }
  g[i] = hit;
}

// -------------------------------------------------------------------- boxes

// g = OR over cells cell(max(lo,-1)) .. cell(min(hi,1)) per axis; a box
// with hi < -1, lo > 1 or lo > hi on some axis is empty.
__global__ void k_voxel_boxes(const float* __restrict__ q, int64_t n, const uint8_t* __restrict__ grid, int gn,
                              uint8_t* __restrict__ g) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float half_n = (float)gn * 0.5f;
  int a[3], b[3];
  bool empty = false;
  for (int ax = 0; ax < 3; ++ax) {
    const float lo = q[6 * i + ax], hi = q[6 * i + 3 + ax];
    if (!(hi >= -1.0f && lo <= 1.0f && lo <= hi)) {
      empty = true;
      break;
    }
    cell_of(fmaxf(lo, -1.0f), gn, half_n, a[ax]);
    cell_of(fminf(hi, 1.0f), gn, half_n, b[ax]);
  }
  uint8_t hit = 0;
  if (!empty) {
    for (int kz = a[2]; kz <= b[2] && !hit; ++kz)
      for (int jy = a[1]; jy <= b[1] && !hit; ++jy) {
        const uint8_t* row = grid + ((int64_t)kz * gn + jy) * gn;
        for (int ix = a[0]; ix <= b[0]; ++ix)
          if (row[ix]) {
            hit = 1;
            break;
          }
      }
  }
  g[i] = hit;
}

// ------------------------------------------------------------------- planes

// g = 1 iff an occupied cell (centre c, half width 1/n) meets the plane:
// |n.(c - p0)| <= (1/n) (|n_x| + |n_y| + |n_z|), dot product summed x, y, z.
__global__ void k_voxel_planes(const float* __restrict__ q, int64_t n, const int32_t* __restrict__ occ,
                               const int64_t* __restrict__ n_occ, int gn, uint8_t* __restrict__ g) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float px = q[6 * i], py = q[6 * i + 1], pz = q[6 * i + 2];
  const float nx = q[6 * i + 3], ny = q[6 * i + 4], nz = q[6 * i + 5];
  const float h = (float)(1.0 / (double)gn);
  const float rad = h * ((fabsf(nx) + fabsf(ny)) + fabsf(nz));
  const int64_t m = *n_occ;
  uint8_t hit = 0;
  for (int64_t c = 0; c < m && !hit; ++c) {
    const int32_t idx = occ[c];
    const int ix = idx % gn, jy = (idx / gn) % gn, kz = idx / (gn * gn);
    const float cx = (float)((2.0 * ix + 1.0) / gn - 1.0);
    const float cy = (float)((2.0 * jy + 1.0) / gn - 1.0);
    const float cz = (float)((2.0 * kz + 1.0) / gn - 1.0);
    const float e = (nx * (cx - px) + ny * (cy - py)) + nz * (cz - pz);
    hit = fabsf(e) <= rad;
  }
  g[i] = hit;
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
  const unsigned blocks = blocks_for(n);
  if (kind == NB_QUERY_POINT) {
    switch (ind->type) {
      case IND_DISCS2D:
        k_discs2d<<<blocks, kThreads, 0, s>>>(q, n, ind->params, ind->k, g);
        break;
      case IND_VOXELS:
        k_voxel_points<<<blocks, kThreads, 0, s>>>(q, n, ind->grid, ind->n, g);
        break;
      case IND_METABALLS4D:
        k_metaballs4d<<<blocks, kThreads, 0, s>>>(q, n, ind->params, ind->k, ind->iso, g);
        break;
      default:
        NB_REQUIRE(false, "unknown indicator type");
    }
  } else {
    NB_REQUIRE(ind->type == IND_VOXELS, "ray, box and plane queries need a voxel indicator");
    switch (kind) {
      case NB_QUERY_RAY:
        k_voxel_rays<<<blocks, kThreads, 0, s>>>(q, n, ind->grid, ind->n, ind->ray_t, g);
        break;
      case NB_QUERY_BOX:
        k_voxel_boxes<<<blocks, kThreads, 0, s>>>(q, n, ind->grid, ind->n, g);
        break;
      case NB_QUERY_PLANE:
        NB_REQUIRE(ind->occupied != nullptr, "plane query: occupied-cell list missing");
        k_voxel_planes<<<blocks, kThreads, 0, s>>>(q, n, ind->occupied, ind->occupied_count,
                                                   ind->n, g);
        break;
      default:
        NB_REQUIRE(false, "unknown query kind %d", kind);
    }
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
