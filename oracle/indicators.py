"""Indicators f and region queries g (test infrastructure; see oracle/__init__).

Sec. 3.1 defines the indicator f(x) in {0,1} (1 inside the object and on its
surface) and the query g(r) = 1 iff f is 1 somewhere in the region r; for a
point query g = f.  Sec. 4.2 ("Query types") computes g as any() over the
indicator across the region.  The synthetic indicators below stand in for
the paper's images, voxelised meshes and animations.

Arithmetic rule: every geometric quantity is a float32 expression evaluated
one IEEE operation at a time in the order written (no fused multiply-add,
correctly rounded division and square root), so the integer results are
defined bit for bit.  Numpy float32 array arithmetic does exactly that.

Conventions
  * Voxel grid: uint8[n^3] over the cube [-1, 1]^3, x fastest:
    index (k*n + j)*n + i.  Cell centre c_i = (2i + 1)/n - 1 (exact).
  * Cell of a coordinate p in [-1, 1]: floor((p + 1) * (n/2)), with p = 1
    mapped to n - 1.  A point with any coordinate outside [-1, 1] (or NaN)
    lies outside the grid and has f = 0.
  * Metaball field F(x) = sum_b R_b^2 / |x - c_b|^2, summed over b in order;
    inside iff F >= iso.  A single ball gives exactly the sphere |x - c| <= R.
"""

from __future__ import annotations

import numpy as np

F = np.float32


# --------------------------------------------------------------- 2-D discs

def discs2d(q: np.ndarray, discs: np.ndarray) -> np.ndarray:
    """Point in a union of discs.  q [n,2], discs [k,3] rows (cx, cy, r).
    f = OR_b ((x-cx)^2 + (y-cy)^2 <= r^2)."""
    q = np.asarray(q, dtype=np.float32)
    x, y = q[:, 0], q[:, 1]
    out = np.zeros(q.shape[0], dtype=bool)
    for cx, cy, r in np.asarray(discs, dtype=np.float32):
        dx = x - F(cx)
        dy = y - F(cy)
        d2 = dx * dx + dy * dy
        out |= d2 <= F(r) * F(r)
    return out.astype(np.uint8)


# ---------------------------------------------------------- metaball field

def metaball_field(p: np.ndarray, centres: np.ndarray, radii: np.ndarray) -> np.ndarray:
    """F(p) in float32, p [n,3]."""
    p = np.asarray(p, dtype=np.float32)
    acc = np.zeros(p.shape[0], dtype=np.float32)
    with np.errstate(divide="ignore", invalid="ignore"):
        for c, r in zip(np.asarray(centres, dtype=np.float32), np.asarray(radii, dtype=np.float32)):
            dx = p[:, 0] - c[0]
            dy = p[:, 1] - c[1]
            dz = p[:, 2] - c[2]
            d2 = (dx * dx + dy * dy) + dz * dz
            acc = acc + (r * r) / d2
    return acc


def voxelize_metaballs(centres, radii, n: int, iso: float = 1.0) -> np.ndarray:
    """uint8[n^3]: cell value = 1 iff the field at the cell centre is >= iso."""
    c = ((2.0 * np.arange(n) + 1.0) / n - 1.0).astype(np.float32)   # exact
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    p = np.stack([c[i.ravel()], c[j.ravel()], c[k.ravel()]], axis=1)
    return (metaball_field(p, centres, radii) >= F(iso)).astype(np.uint8)


# ------------------------------------------------------------- voxel grid

def cell_index(p: np.ndarray, n: int):
    """(cell index int64, inside bool) for float32 coordinates p."""
    p = np.asarray(p, dtype=np.float32)
    inside = (p >= F(-1)) & (p <= F(1))
    with np.errstate(invalid="ignore"):
        s = (p + F(1)) * F(n / 2)
        s = np.where(inside, s, F(0))
    i = np.minimum(np.floor(s).astype(np.int64), n - 1)
    return i, inside


def voxel_points(q: np.ndarray, grid: np.ndarray, n: int) -> np.ndarray:
    """Point query on a voxel grid: f(x) = grid[cell(x)], 0 outside [-1,1]^3."""
    q = np.asarray(q, dtype=np.float32)
    ijk, ins = cell_index(q[:, :3], n)
    inside = ins.all(axis=1)
    idx = (ijk[:, 2] * n + ijk[:, 1]) * n + ijk[:, 0]
    return np.where(inside, grid[idx], 0).astype(np.uint8)


def ray_t_table(samples: int = 256, t_max: float = 4.0) -> np.ndarray:
    """Sample parameters t_j = t_max * j / (samples - 1), rounded once to float32
    from double, so t_0 = 0 and t_last = t_max exactly."""
    j = np.arange(samples, dtype=np.float64)
    return (t_max * j / (samples - 1)).astype(np.float32)


def voxel_rays(q: np.ndarray, grid: np.ndarray, n: int, t: np.ndarray | None = None) -> np.ndarray:
    """Ray (segment) query: g = max_j f(o + t_j * d) over the sample table t.
    q [m,6] rows (o, d); p_j = o + (t_j * d) per component."""
    q = np.asarray(q, dtype=np.float32)
    t = ray_t_table() if t is None else np.asarray(t, dtype=np.float32)
    o, d = q[:, :3], q[:, 3:6]
    out = np.zeros(q.shape[0], dtype=np.uint8)
    for tj in t:
        out |= voxel_points(o + F(tj) * d, grid, n)
    return out


def voxel_boxes(q: np.ndarray, grid: np.ndarray, n: int) -> np.ndarray:
    """Box query: g = OR of grid over every cell that meets the closed box
    [lo, hi], i.e. cells cell(max(lo,-1)) .. cell(min(hi,1)) per axis.
    A box with hi < -1 or lo > 1 on some axis (or lo > hi) is empty: g = 0."""
    q = np.asarray(q, dtype=np.float32)
    lo, hi = q[:, :3], q[:, 3:6]
    g3 = np.asarray(grid).reshape(n, n, n)          # [k][j][i]
    empty = ~((hi >= F(-1)) & (lo <= F(1)) & (lo <= hi)).all(axis=1)
    a, _ = cell_index(np.maximum(lo, F(-1)), n)
    b, _ = cell_index(np.minimum(hi, F(1)), n)
    out = np.zeros(q.shape[0], dtype=np.uint8)
    for r in np.nonzero(~empty)[0]:
        out[r] = g3[a[r, 2]:b[r, 2] + 1, a[r, 1]:b[r, 1] + 1, a[r, 0]:b[r, 0] + 1].any()
    return out


def _occupied_cells(grid, n):
    idx = np.nonzero(np.asarray(grid))[0]
    i = idx % n
    j = (idx // n) % n
    k = idx // (n * n)
    c = ((2.0 * np.arange(n) + 1.0) / n - 1.0).astype(np.float32)
    return c[i], c[j], c[k]


def voxel_planes(q: np.ndarray, grid: np.ndarray, n: int) -> np.ndarray:
    """Plane query: g = 1 iff some occupied cell meets the plane through p0
    with normal nrm.  A cell with centre c and half width h = 1/n meets it iff
    |nrm . (c - p0)| <= h * (|n_x| + |n_y| + |n_z|) (the plane / axis-aligned
    box overlap test), with the dot product summed x, y, z in order."""
    q = np.asarray(q, dtype=np.float32)
    cx, cy, cz = _occupied_cells(grid, n)
    h = F(1.0 / n)
    out = np.zeros(q.shape[0], dtype=np.uint8)
    if cx.size == 0:
        return out
    for r in range(q.shape[0]):
        px, py, pz, nx, ny, nz = q[r]
        e = (nx * (cx - px) + ny * (cy - py)) + nz * (cz - pz)
        rad = h * ((np.abs(nx) + np.abs(ny)) + np.abs(nz))
        out[r] = (np.abs(e) <= rad).any()
    return out


# ------------------------------------------------------ 4-D moving metaballs

def metaballs4d(q: np.ndarray, a: np.ndarray, b: np.ndarray, radii: np.ndarray,
                iso: float = 1.0) -> np.ndarray:
    """4-D point query (x, y, z, t): balls move on straight paths,
    c_b(t) = a_b + t * (b_b - a_b) per component; f = 1 iff
    sum_b R_b^2 / |x - c_b(t)|^2 >= iso (summed over b in order)."""
    q = np.asarray(q, dtype=np.float32)
    t = q[:, 3]
    acc = np.zeros(q.shape[0], dtype=np.float32)
    a = np.asarray(a, dtype=np.float32)
    d = (np.asarray(b, dtype=np.float32) - a).astype(np.float32)
    with np.errstate(divide="ignore", invalid="ignore"):
        for ab, db, r in zip(a, d, np.asarray(radii, dtype=np.float32)):
            dx = q[:, 0] - (ab[0] + t * db[0])
            dy = q[:, 1] - (ab[1] + t * db[1])
            dz = q[:, 2] - (ab[2] + t * db[2])
            d2 = (dx * dx + dy * dy) + dz * dz
            acc = acc + (r * r) / d2
    return (acc >= F(iso)).astype(np.uint8)
