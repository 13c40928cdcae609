"""k-DOP bound trained with the asymmetric loss (test infrastructure; see
oracle/__init__).

Sec. 4.1 ("Methods"): besides networks, the paper optimises the planes of a
k-DOP (k discretely oriented slabs) with its asymmetric loss; the
supplemental uses k = 4 directions.  The paper gives no formula for the
k-DOP's logit; the reading used here:

  parameters  theta = [n_1 .. n_k (d each), lo_1 .. lo_k, hi_1 .. hi_k, s]
  region r    per direction j the interval [u_j, v_j] of n_j . x over r:
                point x:               u = v = n . x
                box [a, b]:            n . c -+ sum_i |n_i| e_i,
                                       c = (a + b)/2, e = (b - a)/2
                segment o + t w,       u, v = min, max of n . o and
                t in [0, 4]:           n . (o + 4 w)
  margin      m_j = min(hi_j - u_j, v_j - lo_j),  m = min_j m_j
  logit       z = s m   (the decision and Eq. 1 are the network's)

m >= 0 iff the region's projection meets every slab, a necessary condition
for the region to meet the k-DOP, so a k-DOP that contains the indicator's
support is a conservative bound for every query kind.  The gradient of z
goes to the arg-min direction (lowest j on ties) and side (hi on ties).
Everything here is float64.
"""

from __future__ import annotations

import numpy as np

T_MAX = 4.0   # segment length parameter of ray queries (as the ray indicator)


def num_params(d: int, k: int) -> int:
    return k * d + 2 * k + 1


def unpack(theta, d: int, k: int):
    theta = np.asarray(theta, dtype=np.float64)
    if theta.size != num_params(d, k):
        raise ValueError("parameter count mismatch")
    N = theta[:k * d].reshape(k, d)
    lo = theta[k * d:k * d + k]
    hi = theta[k * d + k:k * d + 2 * k]
    return N, lo, hi, float(theta[-1])


def intervals(theta, d: int, k: int, kind: str, q):
    """Per-direction projection intervals (u, v), each [n_queries, k]."""
    N, _, _, _ = unpack(theta, d, k)
    q = np.asarray(q, dtype=np.float64)
    if kind == "point":
        p = q @ N.T
        return p, p.copy()
    if kind == "box":
        a, b = q[:, :d], q[:, d:2 * d]
        c, e = 0.5 * (a + b), 0.5 * (b - a)
        mid = c @ N.T
        rad = e @ np.abs(N).T
        return mid - rad, mid + rad
    if kind == "ray":
        o, w = q[:, :d], q[:, d:2 * d]
        p0 = o @ N.T
        p1 = (o + T_MAX * w) @ N.T
        return np.minimum(p0, p1), np.maximum(p0, p1)
    raise ValueError(kind)


def margins(theta, d: int, k: int, kind: str, q):
    _, lo, hi, _ = unpack(theta, d, k)
    u, v = intervals(theta, d, k, kind, q)
    return np.minimum(hi[None, :] - u, v - lo[None, :])


def forward(theta, d: int, k: int, kind: str, q):
    """Logits z = s min_j m_j, float64[n]."""
    s = unpack(theta, d, k)[3]
    with np.errstate(invalid="ignore"):
        z = s * margins(theta, d, k, kind, q).min(axis=1)
    # a region with a non-finite parameter: NaN, decided positive
    return np.where(np.all(np.isfinite(np.asarray(q, dtype=np.float64)), axis=1), z, np.nan)


def backward(theta, d: int, k: int, kind: str, q, dz):
    """sum_i dz_i dz_i/dtheta for upstream gradients dz (float64[n])."""
    N, lo, hi, s = unpack(theta, d, k)
    q = np.asarray(q, dtype=np.float64)
    u, v = intervals(theta, d, k, kind, q)
    up = hi[None, :] - u
    dn = v - lo[None, :]
    m = np.minimum(up, dn)
    j = np.argmin(m, axis=1)                     # first index on ties
    rows = np.arange(q.shape[0])
    side_hi = up[rows, j] <= dn[rows, j]         # hi side on ties
    gN = np.zeros_like(N)
    glo = np.zeros(k)
    ghi = np.zeros(k)
    gs = float(np.sum(dz * m[rows, j]))
    # d u / d n_j and d v / d n_j per query for its active direction
    Nj = N[j]
    if kind == "point":
        du = dv = q[:, :d]
    elif kind == "box":
        a, b = q[:, :d], q[:, d:2 * d]
        c, e = 0.5 * (a + b), 0.5 * (b - a)
        sg = np.sign(Nj)
        du, dv = c - sg * e, c + sg * e
    else:
        o, w = q[:, :d], q[:, d:2 * d]
        far = o + T_MAX * w
        first_low = (o * Nj).sum(1) <= (far * Nj).sum(1)
        du = np.where(first_low[:, None], o, far)
        dv = np.where(first_low[:, None], far, o)
    for i in range(q.shape[0]):
        jj = j[i]
        if side_hi[i]:
            ghi[jj] += dz[i] * s
            gN[jj] -= dz[i] * s * du[i]
        else:
            glo[jj] -= dz[i] * s
            gN[jj] += dz[i] * s * dv[i]
    return np.concatenate([gN.ravel(), glo, ghi, [gs]])
