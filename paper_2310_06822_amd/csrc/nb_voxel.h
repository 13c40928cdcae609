// Voxel-grid indicator and region queries as per-query device functions,
// shared by the single-indicator and grouped kernels.
//
// Grids cover [-1, 1]^3, x fastest (index (k*n + j)*n + i).  A coordinate
// p in [-1, 1] lies in cell floor((p + 1) * (n/2)), clamped to n - 1 at
// p = 1; a point with a coordinate outside the cube (or NaN) has f = 0.
// Every float operation is one IEEE float32 operation in the order written
// (the files including this are compiled without contraction).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

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

// --------------------------------------------------------------------- rays

// Sample index range [j0, j1] that can reach the cube [-1, 1]^3: the slab
// interval of the segment o + t d, widened by one sample on each side and by
// 1e-4 in t, so every sample inside the cube is kept (float rounding of the
// sample positions moves them by far less than the 4/255 sample spacing).
// Returns false if no sample can be inside.
__device__ __forceinline__ bool ray_sample_range(const float* __restrict__ row, int& j0, int& j1) {
  float tlo = 0.0f, thi = 4.0f;
  for (int a = 0; a < 3; ++a) {
    const float o = row[a], d = row[3 + a];
    if (fabsf(d) < 1e-30f) {
      if (!(o >= -1.0f && o <= 1.0f)) return false;   // parallel to the slab and outside (or NaN)
      continue;
    }
    const float t1 = (-1.0f - o) / d, t2 = (1.0f - o) / d;
    tlo = fmaxf(tlo, fminf(t1, t2));
    thi = fminf(thi, fmaxf(t1, t2));
  }
  if (!(tlo <= thi + 1e-4f)) return false;
  const float scale = 255.0f / 4.0f;
  j0 = max(0, (int)floorf((tlo - 1e-4f) * scale) - 1);
  j1 = min(255, (int)ceilf((thi + 1e-4f) * scale) + 1);
  return j0 <= j1;
}

// g = max_j f(o + t_j d) over the sample table; stops at the first hit.
// Only samples in the clipped range are evaluated; the others lie outside
// the cube, where f = 0.
__device__ __forceinline__ uint8_t voxel_ray_at(const float* __restrict__ row, const uint8_t* __restrict__ grid, int gn,
                                                const float* __restrict__ ray_t) {
  const float ox = row[0], oy = row[1], oz = row[2], dx = row[3], dy = row[4], dz = row[5];
  int j0, j1;
  if (!ray_sample_range(row, j0, j1)) return 0;
  const float half_n = (float)gn * 0.5f;
  uint8_t hit = 0;
  for (int j = j0; j <= j1 && !hit; ++j) {
    const float t = ray_t[j];
    hit = voxel_at(grid, gn, half_n, ox + t * dx, oy + t * dy, oz + t * dz);
  }
  return hit;
}

// -------------------------------------------------------------------- boxes

// Cells a[ax] .. b[ax] per axis that meet the closed box [lo, hi]:
// cell(max(lo,-1)) .. cell(min(hi,1)); false for a box with hi < -1,
// lo > 1 or lo > hi on some axis (it meets no cell).
__device__ __forceinline__ bool box_cell_range(const float* __restrict__ row, int gn, int (&a)[3], int (&b)[3]) {
  const float half_n = (float)gn * 0.5f;
  for (int ax = 0; ax < 3; ++ax) {
    const float lo = row[ax], hi = row[3 + ax];
    if (!(hi >= -1.0f && lo <= 1.0f && lo <= hi)) return false;
    cell_of(fmaxf(lo, -1.0f), gn, half_n, a[ax]);
    cell_of(fminf(hi, 1.0f), gn, half_n, b[ax]);
  }
  return true;
}

// g = OR over the box's cells, scanned row by row with an early exit.
__device__ __forceinline__ uint8_t voxel_box_at(const float* __restrict__ row, const uint8_t* __restrict__ grid, int gn) {
  int a[3], b[3];
  if (!box_cell_range(row, gn, a, b)) return 0;
  for (int kz = a[2]; kz <= b[2]; ++kz)
    for (int jy = a[1]; jy <= b[1]; ++jy) {
      const uint8_t* r = grid + ((int64_t)kz * gn + jy) * gn;
      for (int ix = a[0]; ix <= b[0]; ++ix)
        if (r[ix]) return 1;
    }
  return 0;
}

// Occupied-cell count table of a grid: S[(k*(n+1) + j)*(n+1) + i] is the
// number of occupied cells with z < k, y < j, x < i.  The box's OR is then
// "count over its cell range > 0", an integer inclusion-exclusion over the
// range's 8 corners: the same answer as the scan, in constant time.
__device__ __forceinline__ uint8_t voxel_box_table_at(const float* __restrict__ row,
                                                      const int32_t* __restrict__ S, int gn) {
  int a[3], b[3];
  if (!box_cell_range(row, gn, a, b)) return 0;
  const int64_t m = gn + 1;
  const int64_t x0 = a[0], x1 = b[0] + 1, y0 = a[1] * m, y1 = (b[1] + 1) * m, z0 = a[2] * m * m,
                z1 = (int64_t)(b[2] + 1) * m * m;
  const int32_t cnt = S[z1 + y1 + x1] - S[z0 + y1 + x1] - S[z1 + y0 + x1] - S[z1 + y1 + x0] + S[z0 + y0 + x1] +
                      S[z0 + y1 + x0] + S[z1 + y0 + x0] - S[z0 + y0 + x0];
  return cnt > 0;
}

// Point, ray or box query on one grid (query kinds as in nbound.h: 0 point,
// 1 ray, 2 box); q holds rows of 3 (points) or 6 floats.
__device__ __forceinline__ uint8_t nb_voxel_query(int kind, const float* __restrict__ q, int64_t i,
                                                  const uint8_t* __restrict__ grid, int gn,
                                                  const float* __restrict__ ray_t) {
  if (kind == 0) {
    const float* r = q + 3 * i;
    return voxel_at(grid, gn, (float)gn * 0.5f, r[0], r[1], r[2]);
  }
  if (kind == 1) return voxel_ray_at(q + 6 * i, grid, gn, ray_t);
  return voxel_box_at(q + 6 * i, grid, gn);
}
