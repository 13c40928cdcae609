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
#include <mutex>

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
  const float* centre;
  const uint64_t* colmask;
  int mask_words;
  const uint64_t* coarse_mask;
  int coarse_n, coarse_words;
};

IndView view_of(const nb_indicator* ind) {
  return IndView{ind->type,     ind->k,        ind->n,          ind->iso,      ind->params,
                 ind->grid,     ind->ray_t,    ind->occupied,   ind->occupied_count,
                 ind->centre,   ind->colmask,  ind->mask_words, ind->coarse_mask, ind->coarse_n,
                 ind->coarse_words};
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

// The definition: g = 1 iff an occupied cell (centre c, half width h = 1/n)
// meets the plane through p0 with normal m, i.e.
//   |m.(c - p0)| <= h (|m_x| + |m_y| + |m_z|)
// (the plane / axis-aligned box overlap test), the dot product summed x, y, z
// in float32 and the centres c = (2i + 1)/n - 1 rounded once from double.
//
// Evaluating that over every occupied cell costs O(n^3).  The query below
// is O(n^2) and gives the same answer bit for bit: along the dominant axis a
// of m (|m_a| = max), each column of cells (fixed coordinates on the two
// other axes) meets the slab |m.(c - p0)| <= rad in an interval of at most
// about four cells.  For every column the interval is computed in double,
// widened by a bound on the float32 rounding error of the predicate (so it
// holds every cell for which the float32 predicate can be true) and by one
// cell; its occupied cells come from the column's occupancy bits, and each
// is then tested with the float32 predicate itself.  A coarse level in front
// does the same for columns of 8 x 8 cells against blocks of 8 x 8 x 8 cells:
// the union of the fine intervals of a coarse column, widened by one more
// cell, is tested against the coarse occupancy bits, and only the coarse
// columns that pass are searched cell column by cell column, so a plane that
// misses the object is usually rejected after n^2/4096 coarse tests.  One
// wave takes one plane (64 coarse columns, then the 64 cell columns of one
// coarse column, per pass) and stops at the first hit.  Planes with a
// non-finite value or a normal
// whose largest component is outside [2^-60, 2^60] (where the error bound
// would not hold) take the plain loop over the occupied-cell list instead.

struct PlaneRow {
  float px, py, pz, mx, my, mz, rad;
};

__device__ __forceinline__ bool plane_meets(const PlaneRow& r, const float* __restrict__ centre, int ix, int jy,
                                            int kz) {
  const float cx = centre[ix], cy = centre[jy], cz = centre[kz];
  const float e = (r.mx * (cx - r.px) + r.my * (cy - r.py)) + r.mz * (cz - r.pz);
  return fabsf(e) <= r.rad;
}

__device__ __forceinline__ float pick3(int a, float x, float y, float z) { return a == 0 ? x : (a == 1 ? y : z); }

// The definition over the occupied-cell list, one wave per plane.
__device__ uint8_t plane_wave_list(const IndView& v, const PlaneRow& r, int lane) {
  const int gn = v.n;
  const int64_t m = *v.occupied_count;
  for (int64_t base = 0; base < m; base += 64) {
    const int64_t c = base + lane;
    bool hit = false;
    if (c < m) {
      const int32_t idx = v.occupied[c];
      hit = plane_meets(r, v.centre, idx % gn, (idx / gn) % gn, idx / (gn * gn));
    }
    if (__ballot(hit)) return 1;
  }
  return 0;
}

// Bits lo .. hi (absolute positions) of word w of a bit row.
__device__ __forceinline__ uint64_t word_range(uint64_t bits, int w, int lo, int hi) {
  const int b0 = w * 64;
  if (lo > b0) bits &= ~0ull << (lo - b0);
  if (hi - b0 < 63) bits &= (2ull << (hi - b0)) - 1ull;
  return bits;
}

// Any of the bits lo .. hi of a bit row set?
__device__ __forceinline__ bool any_bits(const uint64_t* __restrict__ row, int lo, int hi) {
  for (int w = lo >> 6; w <= (hi >> 6); ++w)
    if (word_range(row[w], w, lo, hi)) return true;
  return false;
}

__device__ uint8_t plane_wave(const IndView& v, const float* __restrict__ row, int lane) {
  PlaneRow r;
  r.px = row[0];
  r.py = row[1];
  r.pz = row[2];
  r.mx = row[3];
  r.my = row[4];
  r.mz = row[5];
  const int gn = v.n;
  const float h = (float)(1.0 / (double)gn);
  r.rad = h * ((fabsf(r.mx) + fabsf(r.my)) + fabsf(r.mz));
  const float ax = fabsf(r.mx), ay = fabsf(r.my), az = fabsf(r.mz);
  const int a = (az > ax && az > ay) ? 2 : (ay > ax ? 1 : 0);   // dominant axis (lowest on ties)
  const float amax = pick3(a, ax, ay, az);
  const bool regular = amax >= 0x1p-60f && amax <= 0x1p60f && isfinite(r.px) && isfinite(r.py) &&
                       isfinite(r.pz) && isfinite(r.mx) && isfinite(r.my) && isfinite(r.mz);
  if (!regular) return plane_wave_list(v, r, lane);

  const int sa = a == 0 ? 1 : 0, ta = a == 2 ? 1 : 2;   // the two other axes, increasing
  const double u = 0x1p-24;
  const double S = (double)ax * (1.0 + fabs((double)r.px)) + (double)ay * (1.0 + fabs((double)r.py)) +
                   (double)az * (1.0 + fabs((double)r.pz));
  // |float32 e - exact e| <= 5 u S (+ subnormal terms); 16 u S + 2^-140 covers it
  const double err = 16.0 * u * S + 0x1p-140;
  const double N = (double)gn;
  const double ma = pick3(a, r.mx, r.my, r.mz), ms = pick3(sa, r.mx, r.my, r.mz), mt = pick3(ta, r.mx, r.my, r.mz);
  const double pa = pick3(a, r.px, r.py, r.pz), ps = pick3(sa, r.px, r.py, r.pz), pt = pick3(ta, r.px, r.py, r.pz);
  // centre of the interval, in cell units along a, as K0 + s Ks + t Kt
  const double Ks = -ms / ma, Kt = -mt / ma;
  const double K0 = ((pa + 1.0) * N - 1.0) * 0.5 - (N / (2.0 * ma)) * (ms * (1.0 / N - 1.0 - ps) +
                                                                         mt * (1.0 / N - 1.0 - pt));
  const double Kw = ((double)r.rad + err) * N / (2.0 * fabs(ma)) + 1.0;

  const uint64_t* mask_a = v.colmask + (size_t)a * gn * gn * v.mask_words;
  const int C = v.coarse_n;
  const int ccols = C * C;
  const uint64_t* cmask_a = v.coarse_mask + (size_t)a * ccols * v.coarse_words;
  for (int base = 0; base < ccols; base += 64) {
    const int cc = base + lane;
    bool flag = false;
    if (cc < ccols) {
      // coarse column (cs, ct): cells s in [8 cs, 8 cs + 7], t in [8 ct, 8 ct + 7]
      const int ct = cc / C, cs = cc - ct * C;
      const double s0 = 8.0 * cs, s1 = fmin(s0 + 7.0, N - 1.0), t0 = 8.0 * ct, t1 = fmin(t0 + 7.0, N - 1.0);
      const double kmin = K0 + fmin(s0 * Ks, s1 * Ks) + fmin(t0 * Kt, t1 * Kt);
      const double kmax = K0 + fmax(s0 * Ks, s1 * Ks) + fmax(t0 * Kt, t1 * Kt);
      const double lo_d = fmax(floor(kmin - Kw) - 1.0, 0.0), hi_d = fmin(ceil(kmax + Kw) + 1.0, N - 1.0);
      if (lo_d <= hi_d) {
        const int lo = (int)lo_d >> 3, hi = (int)hi_d >> 3;
        flag = any_bits(cmask_a + (size_t)cc * v.coarse_words, lo, hi);
      }
    }
    uint64_t todo = __ballot(flag);   // the same on every lane
    while (todo) {
      const int cc2 = base + __builtin_ctzll(todo);
      todo &= todo - 1ull;
      const int ct = cc2 / C, cs = cc2 - ct * C;
      const int s = 8 * cs + (lane & 7), t = 8 * ct + (lane >> 3);
      bool hit = false;
      if (s < gn && t < gn) {
        const double kc = fma((double)t, Kt, fma((double)s, Ks, K0));
        const double lo_d = fmax(floor(kc - Kw), 0.0), hi_d = fmin(ceil(kc + Kw), N - 1.0);
        if (lo_d <= hi_d) {
          const int lo = (int)lo_d, hi = (int)hi_d;
          const uint64_t* colbits = mask_a + ((size_t)t * gn + s) * v.mask_words;
          for (int w = lo >> 6; w <= (hi >> 6) && !hit; ++w) {
            uint64_t bits = word_range(colbits[w], w, lo, hi);
            while (bits && !hit) {
              const int k = w * 64 + __builtin_ctzll(bits);
              bits &= bits - 1ull;
              const int ix = a == 0 ? k : s;
              const int jy = a == 1 ? k : (a == 0 ? s : t);
              const int kz = a == 2 ? k : t;
              hit = plane_meets(r, v.centre, ix, jy, kz);
            }
          }
        }
      }
      if (__ballot(hit)) return 1;
    }
  }
  return 0;
}

// g[i] (or answer[idx[t]] for a listed subset) for plane queries, one wave
// per plane, grid-stride over planes.
template <bool LISTED>
__global__ __launch_bounds__(256) void k_plane_exact(IndView v, const float* __restrict__ q, int64_t n,
                                                     const int32_t* __restrict__ idx,
                                                     const unsigned long long* __restrict__ count,
                                                     uint8_t* __restrict__ g) {
  const int lane = threadIdx.x & 63;
  const int64_t m = LISTED ? (int64_t)*count : n;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; t < m; t += waves) {
    const int64_t i = LISTED ? (int64_t)idx[t] : t;
    const uint8_t hit = plane_wave(v, q + 6 * i, lane);
    if (lane == 0) g[i] = hit;
  }
}

// Column occupancy bits for the plane query (layout in nb_indicator).
__global__ void k_column_masks(const uint8_t* __restrict__ grid, int gn, int words, uint64_t* __restrict__ mask) {
  const int64_t total = 3ll * gn * gn * words;
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= total) return;
  const int w = (int)(id % words);
  const int64_t col = id / words;
  const int s = (int)(col % gn), t = (int)((col / gn) % gn), a = (int)(col / ((int64_t)gn * gn));
  uint64_t bits = 0;
  for (int b = 0; b < 64; ++b) {
    const int c = 64 * w + b;
    if (c >= gn) break;
    const int i = a == 0 ? c : s;
    const int j = a == 0 ? s : (a == 1 ? c : t);
    const int k = a == 2 ? c : t;
    if (grid[((int64_t)k * gn + j) * gn + i]) bits |= 1ull << b;
  }
  mask[id] = bits;
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
  static_assert(KIND != NB_QUERY_PLANE, "plane queries run one wave per plane (k_plane_exact)");
  if (KIND == NB_QUERY_RAY) return voxel_ray_at(q + 6 * i, v.grid, v.n, v.ray_t);
  return voxel_box_at(q + 6 * i, v.grid, v.n);
}

template <int KIND>
__global__ void k_exact(IndView v, const float* __restrict__ q, int64_t n, uint8_t* __restrict__ g) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  g[i] = exact_at<KIND>(v, q, i);
}

// Rays with L lanes each: lane s of a ray's group takes samples j0 + s,
// j0 + s + L, ... of the clipped range; after every round of L samples a wave
// ballot tells the group whether any of its lanes hit, and the group stops
// at the first such round.  The answer is the OR over the same samples with
// the same arithmetic as the one-lane test; only where it stops differs.
// Small batches (training labels) get L times the threads.
template <int L>
__global__ __launch_bounds__(256) void k_exact_ray_split(IndView v, const float* __restrict__ q, int64_t n,
                                                         uint8_t* __restrict__ g) {
  static_assert(L == 2 || L == 4 || L == 8, "lanes per ray");
  const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / L;
  if (i >= n) return;   // whole groups: blockDim is a multiple of L
  const int sub = threadIdx.x & (L - 1), gbase = (threadIdx.x & 63) & ~(L - 1);
  const float* row = q + 6 * i;
  int j0, j1;
  bool found = false;
  if (ray_sample_range(row, j0, j1)) {   // the same range on every lane of the group
    const float ox = row[0], oy = row[1], oz = row[2], dx = row[3], dy = row[4], dz = row[5];
    const float half_n = (float)v.n * 0.5f;
    for (int jb = j0; jb <= j1; jb += L) {
      const int j = jb + sub;
      bool hit = false;
      if (j <= j1) {
        const float t = v.ray_t[j];
        hit = voxel_at(v.grid, v.n, half_n, ox + t * dx, oy + t * dy, oz + t * dz) != 0;
      }
      if ((__ballot(hit) >> gbase) & ((1ull << L) - 1)) {
        found = true;
        break;
      }
    }
  }
  if (sub == 0) g[i] = found;
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

// Coarse occupancy bits: for each axis and column of 8 x 8 cells (coarse
// coordinates of the two other axes, the higher one outer), bit K of word
// w is set iff a cell of the column with coordinate 8 (64 w + K) .. +7 along
// the axis is occupied.  Built from the cell column bits.
__global__ void k_coarse_masks(const uint64_t* __restrict__ mask, int gn, int words, int C, int cwords,
                               uint64_t* __restrict__ cmask) {
  const int64_t total = 3ll * C * C * cwords;
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= total) return;
  const int wc = (int)(id % cwords);
  const int64_t col = id / cwords;
  const int cs = (int)(col % C), ct = (int)((col / C) % C), a = (int)(col / ((int64_t)C * C));
  uint64_t bits = 0;
  for (int dt = 0; dt < 8; ++dt) {
    const int t = 8 * ct + dt;
    if (t >= gn) break;
    for (int ds = 0; ds < 8; ++ds) {
      const int s = 8 * cs + ds;
      if (s >= gn) break;
      const uint64_t* fine = mask + (((int64_t)a * gn + t) * gn + s) * words;
      for (int K = 0; K < 64; ++K) {
        const int kc = 64 * wc + K;
        if (kc >= C) break;
        const int f = 8 * kc;
        if ((fine[f >> 6] >> (f & 63)) & 0xFFull) bits |= 1ull << K;
      }
    }
  }
  cmask[id] = bits;
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
constexpr int64_t kRaySplitMax = int64_t(1) << 21;

// one wave per plane, grid-stride beyond 2^16 blocks (2^18 waves)
inline unsigned plane_blocks(int64_t n) {
  return (unsigned)std::min<int64_t>((n + kThreads / 64 - 1) / (kThreads / 64), 65536);
}

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
    case NB_QUERY_RAY:
      if (n <= (int64_t(1) << 19))
        k_exact_ray_split<8><<<blocks_for(8 * n), kThreads, 0, s>>>(v, q, n, g);
      else if (n <= kRaySplitMax)   // four lanes per ray up to 2^21 rays
        k_exact_ray_split<4><<<blocks_for(4 * n), kThreads, 0, s>>>(v, q, n, g);
      else
        k_exact<NB_QUERY_RAY><<<blocks, kThreads, 0, s>>>(v, q, n, g);
      break;
    case NB_QUERY_BOX: k_exact<NB_QUERY_BOX><<<blocks, kThreads, 0, s>>>(v, q, n, g); break;
    case NB_QUERY_PLANE:
      k_plane_exact<false><<<plane_blocks(n), kThreads, 0, s>>>(v, q, n, nullptr, nullptr, g);
      break;
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
    case NB_QUERY_PLANE:
      k_plane_exact<true><<<plane_blocks(n), kThreads, 0, s>>>(v, q, n, idx, count, answer);
      break;
    default: NB_REQUIRE(false, "unknown query kind %d", kind);
  }
  NB_LAUNCHED();
  return NB_OK;
}

// Index list of the allocation-free cascade (nb_cascade_noalloc): a
// file-scope device array, one copy per GPU, held until the process ends.
// Host code never passes the array's name to a kernel: it looks up the
// array's device address once per device (hipGetSymbolAddress) and passes
// that.
static __device__ __align__(256) int32_t scratch[NB_CASCADE_NOALLOC_MAX];

nb_status cascade_scratch(int32_t** out) {
  static std::mutex mu;
  static int32_t* ptr[kMaxDevices] = {};
  int dev = 0;
  NB_HIP(hipGetDevice(&dev));
  NB_REQUIRE(dev >= 0 && dev < kMaxDevices, "device %d beyond the %d the library tracks", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    NB_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    ptr[dev] = static_cast<int32_t*>(p);
  }
  *out = ptr[dev];
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

nb_status launch_column_masks(const uint8_t* grid, int n, int words, uint64_t* mask, int coarse_n, int coarse_words,
                              uint64_t* coarse_mask, hipStream_t s) {
  k_column_masks<<<blocks_for(3ll * n * n * words), kThreads, 0, s>>>(grid, n, words, mask);
  NB_LAUNCHED();
  k_coarse_masks<<<blocks_for(3ll * coarse_n * coarse_n * coarse_words), kThreads, 0, s>>>(
      mask, n, words, coarse_n, coarse_words, coarse_mask);
  NB_LAUNCHED();
  return NB_OK;
}
