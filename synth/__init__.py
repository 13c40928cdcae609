"""Seeded synthetic inputs for Neural Bounding workloads.

This module draws random numbers and nothing else: scene parameters, query
batches and initial weights.  It holds none of the method's arithmetic (no
indicator, no network, no loss), so both the GPU path and the CPU oracle can
take their inputs from here without sharing any computation.

Every generator takes an explicit integer seed and returns float32 (or uint8)
numpy arrays.  Draws are made in float64 and rounded once to float32.

Workloads (synthetic stand-ins for the paper's image / voxel / animation
data, Sec. 4.2 "Indicators"):
  * 2-D: a union of discs, centres U[-0.7,0.7]^2, radii U[0.05,0.3].
  * 3-D: metaballs, centres U[-0.7,0.7]^3, radii U[0.05,0.25].
  * 4-D: metaballs moving on straight paths a -> b over t in [0,1],
    endpoints U[-0.7,0.7]^3, radii U[0.05,0.2].
Query encodings follow the supplemental "Parameterization" paragraph: rays
as (origin, direction), boxes as (min corner, max corner), planes as
(point p0, normal).
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "rng", "discs2d", "metaballs3d", "metaballs4d", "random_grid",
    "points", "points4d", "rays", "boxes", "planes", "init_params",
    "layer_shapes", "num_params", "seed_for", "object_set", "kdop_init", "pad_params",
]

# Seed bases per stream: scene / training stream / held-out eval / init.
SEED_SCENE, SEED_TRAIN, SEED_EVAL, SEED_INIT = 1000, 2000, 3000, 4000


def seed_for(stream: int, config: int) -> int:
    """Seed of one stream (SEED_* base) for a workload number."""
    return int(stream) + int(config)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


# ----------------------------------------------------------------- scenes

def discs2d(seed: int, k: int = 8) -> np.ndarray:
    """[k, 3] float32 rows (cx, cy, r)."""
    g = rng(seed)
    c = g.uniform(-0.7, 0.7, size=(k, 2))
    r = g.uniform(0.05, 0.3, size=(k, 1))
    return np.ascontiguousarray(np.concatenate([c, r], axis=1).astype(np.float32))


def metaballs3d(seed: int, k: int = 16, rlo: float = 0.05, rhi: float = 0.25):
    """(centres [k,3] float32, radii [k] float32)."""
    g = rng(seed)
    c = g.uniform(-0.7, 0.7, size=(k, 3)).astype(np.float32)
    r = g.uniform(rlo, rhi, size=(k,)).astype(np.float32)
    return np.ascontiguousarray(c), np.ascontiguousarray(r)


def metaballs4d(seed: int, k: int = 24, rlo: float = 0.05, rhi: float = 0.2):
    """(path starts a [k,3], path ends b [k,3], radii [k]), all float32."""
    g = rng(seed)
    a = g.uniform(-0.7, 0.7, size=(k, 3)).astype(np.float32)
    b = g.uniform(-0.7, 0.7, size=(k, 3)).astype(np.float32)
    r = g.uniform(rlo, rhi, size=(k,)).astype(np.float32)
    return np.ascontiguousarray(a), np.ascontiguousarray(b), np.ascontiguousarray(r)


def object_set(seed: int, n_obj: int, grid_sizes=(32, 64, 128), widths=(32, 64, 128), k_range=(4, 32),
               rlo: float = 0.05, rhi: float = 0.25):
    """Per-object draws of a batch of bounds: a list of dicts with the
    object's grid size n, hidden width w, and metaball scene (centres,
    radii; k balls with k uniform in k_range inclusive)."""
    g = rng(seed)
    out = []
    for o in range(n_obj):
        n = int(g.choice(grid_sizes))
        w = int(g.choice(widths))
        k = int(g.integers(k_range[0], k_range[1] + 1))
        c, r = metaballs3d(int(seed) * 1000 + o, k=k, rlo=rlo, rhi=rhi)
        out.append({"n": n, "width": w, "k": k, "centres": c, "radii": r})
    return out


def lattice_objects(seed: int, lattice: int, k_range=(2, 5), rlo: float = 0.03, rhi: float = 0.08,
                    spread: float = 0.5):
    """One small metaball cluster per cell of a lattice^3 arrangement of
    [-1, 1]^3 (cells x fastest): k balls (k uniform in k_range inclusive)
    with centres uniform within `spread` of the cell's half width around the
    cell centre and radii uniform in [rlo, rhi].  List of (centres [k,3]
    float32, radii [k] float32)."""
    g = rng(seed)
    half = 1.0 / lattice
    out = []
    for cz in range(lattice):
        for cy in range(lattice):
            for cx in range(lattice):
                mid = np.array([-1.0 + (2 * cx + 1) * half, -1.0 + (2 * cy + 1) * half, -1.0 + (2 * cz + 1) * half])
                k = int(g.integers(k_range[0], k_range[1] + 1))
                c = mid + g.uniform(-spread * half, spread * half, size=(k, 3))
                r = g.uniform(rlo, rhi, size=(k,))
                out.append((np.ascontiguousarray(c.astype(np.float32)), np.ascontiguousarray(r.astype(np.float32))))
    return out


def random_grid(seed: int, n: int, density: float = 0.1) -> np.ndarray:
    """Random occupancy grid uint8[n*n*n], x fastest (index (k*n + j)*n + i)."""
    g = rng(seed)
    return np.ascontiguousarray((g.random(n * n * n) < density).astype(np.uint8))


# ---------------------------------------------------------------- queries

def points(seed: int, n: int, dim: int) -> np.ndarray:
    """[n, dim] float32, uniform in [-1, 1]^dim."""
    g = rng(seed)
    return np.ascontiguousarray(g.uniform(-1.0, 1.0, size=(n, dim)).astype(np.float32))


def points4d(seed: int, n: int) -> np.ndarray:
    """[n, 4] float32 rows (x, y, z, t): xyz uniform in [-1,1]^3, t in [0,1]."""
    g = rng(seed)
    xyz = g.uniform(-1.0, 1.0, size=(n, 3))
    t = g.uniform(0.0, 1.0, size=(n, 1))
    return np.ascontiguousarray(np.concatenate([xyz, t], axis=1).astype(np.float32))


def _in_ball(g: np.random.Generator, n: int, radius: float) -> np.ndarray:
    """n points uniform in a 3-D ball, by rejection from the bounding cube."""
    out = np.empty((0, 3))
    while out.shape[0] < n:
        m = max(2 * (n - out.shape[0]), 64)
        v = g.uniform(-radius, radius, size=(m, 3))
        ok = np.einsum("ij,ij->i", v, v) <= radius * radius
        out = np.concatenate([out, v[ok]], axis=0)
    return out[:n]


def _on_sphere(g: np.random.Generator, n: int) -> np.ndarray:
    """n unit vectors uniform on S^2 (normalised rejection from the ball)."""
    out = np.empty((0, 3))
    while out.shape[0] < n:
        m = max(2 * (n - out.shape[0]), 64)
        v = g.uniform(-1.0, 1.0, size=(m, 3))
        r2 = np.einsum("ij,ij->i", v, v)
        ok = (r2 <= 1.0) & (r2 > 1e-6)
        out = np.concatenate([out, v[ok] / np.sqrt(r2[ok])[:, None]], axis=0)
    return out[:n]


def rays(seed: int, n: int, origin_radius: float = 2.0) -> np.ndarray:
    """[n, 6] float32 rows (ox, oy, oz, dx, dy, dz): origin uniform in a ball
    of the given radius, direction uniform on the unit sphere."""
    g = rng(seed)
    o = _in_ball(g, n, origin_radius)
    d = _on_sphere(g, n)
    return np.ascontiguousarray(np.concatenate([o, d], axis=1).astype(np.float32))


def boxes(seed: int, n: int, hlo: float = 0.01, hhi: float = 0.2) -> np.ndarray:
    """[n, 6] float32 rows (lo_x, lo_y, lo_z, hi_x, hi_y, hi_z): centre
    uniform in [-1,1]^3, half-extent per axis uniform in [hlo, hhi]."""
    g = rng(seed)
    c = g.uniform(-1.0, 1.0, size=(n, 3))
    h = g.uniform(hlo, hhi, size=(n, 3))
    return np.ascontiguousarray(np.concatenate([c - h, c + h], axis=1).astype(np.float32))


def planes(seed: int, n: int) -> np.ndarray:
    """[n, 6] float32 rows (p0_x, p0_y, p0_z, n_x, n_y, n_z): p0 uniform in
    [-1,1]^3, unit normal uniform on S^2."""
    g = rng(seed)
    p = g.uniform(-1.0, 1.0, size=(n, 3))
    nrm = _on_sphere(g, n)
    return np.ascontiguousarray(np.concatenate([p, nrm], axis=1).astype(np.float32))


# ---------------------------------------------------------------- weights

def layer_shapes(in_dim: int, widths) -> list:
    """[(out, in)] of every linear layer of in_dim -> widths... -> 1."""
    dims = [int(in_dim)] + [int(w) for w in widths] + [1]
    return [(dims[i + 1], dims[i]) for i in range(len(dims) - 1)]


def num_params(in_dim: int, widths) -> int:
    return sum(o * i + o for o, i in layer_shapes(in_dim, widths))


def init_params(seed: int, in_dim: int, widths) -> np.ndarray:
    """Flat float32 parameter vector: for each layer W[out, in] (row-major)
    then b[out], layers in order.  W and b are drawn U(-1/sqrt(fan_in),
    +1/sqrt(fan_in)), the usual default for a linear layer."""
    g = rng(seed)
    parts = []
    for o, i in layer_shapes(in_dim, widths):
        bound = 1.0 / np.sqrt(i)
        parts.append(g.uniform(-bound, bound, size=(o * i,)))
        parts.append(g.uniform(-bound, bound, size=(o,)))
    return np.ascontiguousarray(np.concatenate(parts).astype(np.float32))


def kdop_init(d: int, k: int, scale: float = 10.0, seed: int | None = None) -> np.ndarray:
    """Initial k-DOP parameters [n_1..n_k, lo, hi, s]: the d axes first, then
    unit diagonals (sign patterns of the first axes), optionally jittered by
    a seeded draw; slabs start at the projection of the cube [-1, 1]^d, so
    the initial k-DOP contains every query domain."""
    dirs = [np.eye(d)[i] for i in range(d)]
    signs = [np.array([1.0] + [(1.0 if (m >> i) & 1 == 0 else -1.0) for i in range(d - 1)]) for m in range(2 ** (d - 1))]
    dirs += [sg / np.sqrt(d) for sg in signs]
    if k > len(dirs):
        raise ValueError(f"at most {len(dirs)} directions in {d}-D")
    N = np.array(dirs[:k], dtype=np.float64)
    if seed is not None:
        N = N + 0.05 * rng(seed).standard_normal(N.shape)
        N /= np.linalg.norm(N, axis=1, keepdims=True)
    ext = np.abs(N).sum(axis=1)
    theta = np.concatenate([N.ravel(), -ext, ext, [scale]])
    return np.ascontiguousarray(theta.astype(np.float32))


def pad_params(theta, in_dim: int, widths, padded_widths) -> np.ndarray:
    """Embed a network's flat parameters into a wider one of the same depth,
    the extra neurons' weights and biases zero (a layout copy, no arithmetic)."""
    src = layer_shapes(in_dim, widths)
    dst = layer_shapes(in_dim, padded_widths)
    out, off = [], 0
    for (o, i), (po, pi) in zip(src, dst):
        W = np.zeros((po, pi), dtype=np.asarray(theta).dtype)
        b = np.zeros(po, dtype=W.dtype)
        W[:o, :i] = np.asarray(theta[off:off + o * i]).reshape(o, i)
        off += o * i
        b[:o] = theta[off:off + o]
        off += o
        out += [W.ravel(), b]
    return np.ascontiguousarray(np.concatenate(out))
