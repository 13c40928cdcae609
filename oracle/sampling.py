"""Region sampling for training batches (test infrastructure; see oracle/__init__).

Alg. 1 starts every loss evaluation by drawing a region r uniformly
("Uniform").  Training batches are drawn from Philox4x32-10 so that any
implementation can reproduce them bit for bit.  This module states the draw
rules; every float operation is a single float32 operation in the order
written (no fused multiply-add).

Key = (seed mod 2^32, seed >> 32).  Counter = (query index i, training step,
stream, attempt).  A uint32 word w gives u = (w >> 8) * 2^-24 in [0, 1).

  point (dim 2 or 3)  stream 0, attempt 0: p_c = 2 u_c - 1 (exact in float32).
  point 4-D           stream 0, attempt 0: xyz = 2 u_c - 1, t = u_3.
  ray                 origin, stream 1: o = 4 u - 2, accepted on the first
                      attempt with (ox*ox + oy*oy) + oz*oz <= 4 (a ball of
                      radius 2); direction, stream 2: v = 2 u - 1, accepted
                      when 1e-6 < |v|^2 <= 1, then d = v / sqrt(|v|^2).  At
                      most 64 attempts each; if none is accepted the origin
                      is 0 and the direction (0, 0, 1).
  box                 centre, stream 3: c = 2 u - 1; half extent, stream 4:
                      h = 0.01 + 0.19 u; (lo, hi) = (c - h, c + h).
  plane               point, stream 5: p0 = 2 u - 1; normal, stream 6: as the
                      ray direction.
"""

from __future__ import annotations

import numpy as np

from .philox import philox4x32, u01

F = np.float32
MAX_ATTEMPTS = 64


def _key(seed: int):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & 0xFFFFFFFF, seed >> 32


def _uniforms(seed, step, stream, attempt, n):
    k0, k1 = _key(seed)
    i = np.arange(n, dtype=np.uint64)
    w = philox4x32(i, np.uint64(step), np.uint64(stream), np.uint64(attempt), k0, k1)
    return [u01(x) for x in w]


def _rejection(seed, step, stream, n, scale, shift, accept):
    """First accepted attempt per query of v = scale*u - shift (float32)."""
    out = np.zeros((n, 3), dtype=np.float32)
    done = np.zeros(n, dtype=bool)
    for a in range(MAX_ATTEMPTS):
        u = _uniforms(seed, step, stream, a, n)
        v = np.stack([F(scale) * u[c] - F(shift) for c in range(3)], axis=1).astype(np.float32)
        r2 = (v[:, 0] * v[:, 0] + v[:, 1] * v[:, 1]) + v[:, 2] * v[:, 2]
        ok = accept(r2) & ~done
        out[ok] = v[ok]
        done |= ok
        if done.all():
            break
    return out, done


def sample_points(seed: int, step: int, n: int, dim: int) -> np.ndarray:
    u = _uniforms(seed, step, 0, 0, n)
    cols = [F(2) * u[c] - F(1) for c in range(min(dim, 3))]
    if dim == 4:
        cols.append(u[3])
    elif dim != len(cols):
        raise ValueError("point dimension must be 2, 3 or 4")
    return np.ascontiguousarray(np.stack(cols, axis=1).astype(np.float32))


def _unit_dirs(seed, step, stream, n):
    v, done = _rejection(seed, step, stream, n, 2, 1,
                         lambda r2: (r2 <= F(1)) & (r2 > F(1e-6)))
    r2 = (v[:, 0] * v[:, 0] + v[:, 1] * v[:, 1]) + v[:, 2] * v[:, 2]
    with np.errstate(invalid="ignore", divide="ignore"):
        d = v / np.sqrt(r2)[:, None]
    d[~done] = np.array([0, 0, 1], dtype=np.float32)
    return d.astype(np.float32)


def sample_rays(seed: int, step: int, n: int) -> np.ndarray:
    o, _ = _rejection(seed, step, 1, n, 4, 2, lambda r2: r2 <= F(4))
    d = _unit_dirs(seed, step, 2, n)
    return np.ascontiguousarray(np.concatenate([o, d], axis=1))


def sample_boxes(seed: int, step: int, n: int) -> np.ndarray:
    uc = _uniforms(seed, step, 3, 0, n)
    uh = _uniforms(seed, step, 4, 0, n)
    c = np.stack([F(2) * uc[i] - F(1) for i in range(3)], axis=1)
    h = np.stack([F(0.19) * uh[i] + F(0.01) for i in range(3)], axis=1)
    return np.ascontiguousarray(np.concatenate([c - h, c + h], axis=1).astype(np.float32))


def sample_planes(seed: int, step: int, n: int) -> np.ndarray:
    u = _uniforms(seed, step, 5, 0, n)
    p = np.stack([F(2) * u[i] - F(1) for i in range(3)], axis=1).astype(np.float32)
    nrm = _unit_dirs(seed, step, 6, n)
    return np.ascontiguousarray(np.concatenate([p, nrm], axis=1))


def sample(kind: str, seed: int, step: int, n: int, dim: int = 3) -> np.ndarray:
    if kind == "point":
        return sample_points(seed, step, n, dim)
    if kind == "ray":
        return sample_rays(seed, step, n)
    if kind == "box":
        return sample_boxes(seed, step, n)
    if kind == "plane":
        return sample_planes(seed, step, n)
    raise ValueError(kind)
