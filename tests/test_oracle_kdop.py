"""Pins of the k-DOP bound's oracle: membership by explicit constraints,
projection intervals by brute force over box corners and dense segment
samples, gradients by central differences, and conservativeness."""

import itertools

import numpy as np
import pytest

import synth
from oracle import kdop


def _theta(d, k, seed):
    th = synth.kdop_init(d, k, seed=seed).astype(np.float64)
    g = np.random.default_rng(seed)
    th[k * d:k * d + 2 * k] *= g.uniform(0.3, 0.8, 2 * k)   # slabs inside the cube
    th[k * d:k * d + 2 * k] += g.uniform(-0.05, 0.05, 2 * k)
    return th


@pytest.mark.parametrize("d,k", [(2, 4), (3, 4), (4, 4), (3, 7)])
def test_point_membership(d, k):
    th = _theta(d, k, 1)
    N, lo, hi, s = kdop.unpack(th, d, k)
    x = np.random.default_rng(2).uniform(-1, 1, (3000, d))
    inside = np.ones(len(x), bool)
    for j in range(k):
        p = x @ N[j]
        inside &= (p >= lo[j]) & (p <= hi[j])
    z = kdop.forward(th, d, k, "point", x)
    assert np.array_equal(z >= 0, inside)
    assert 0 < inside.sum() < len(x)


@pytest.mark.parametrize("d", [2, 3])
def test_box_intervals_brute_force(d):
    k = 4
    th = _theta(d, k, 3)
    N = kdop.unpack(th, d, k)[0]
    g = np.random.default_rng(4)
    c = g.uniform(-1, 1, (200, d))
    e = g.uniform(0.01, 0.3, (200, d))
    boxes = np.concatenate([c - e, c + e], axis=1)
    u, v = kdop.intervals(th, d, k, "box", boxes)
    for i in range(len(boxes)):
        corners = np.array([[boxes[i, a + d * bit] for a, bit in enumerate(bits)]
                            for bits in itertools.product([0, 1], repeat=d)])
        p = corners @ N.T
        assert np.allclose(u[i], p.min(0), atol=1e-12) and np.allclose(v[i], p.max(0), atol=1e-12)


def test_ray_intervals_dense_samples():
    d, k = 3, 4
    th = _theta(d, k, 5)
    N = kdop.unpack(th, d, k)[0]
    rays = synth.rays(6, 100).astype(np.float64)
    u, v = kdop.intervals(th, d, k, "ray", rays)
    t = np.linspace(0.0, 4.0, 4001)
    for i in range(len(rays)):
        pts = rays[i, :3][None, :] + t[:, None] * rays[i, 3:][None, :]
        p = pts @ N.T
        assert np.allclose(u[i], p.min(0), atol=1e-12) and np.allclose(v[i], p.max(0), atol=1e-12)


@pytest.mark.parametrize("kind,d", [("point", 2), ("point", 4), ("box", 3), ("ray", 3)])
def test_gradient_central_differences(kind, d):
    k = 4
    th = _theta(d, k, 7)
    g = np.random.default_rng(8)
    if kind == "point":
        q = g.uniform(-1, 1, (64, d))
    elif kind == "box":
        c, e = g.uniform(-1, 1, (64, d)), g.uniform(0.01, 0.2, (64, d))
        q = np.concatenate([c - e, c + e], axis=1)
    else:
        q = synth.rays(9, 64).astype(np.float64)
    dz = g.standard_normal(len(q))
    grad = kdop.backward(th, d, k, kind, q, dz)
    h = 1e-6
    num = np.zeros_like(th)
    for p in range(th.size):
        tp, tm = th.copy(), th.copy()
        tp[p] += h
        tm[p] -= h
        num[p] = (np.dot(dz, kdop.forward(tp, d, k, kind, q)) - np.dot(dz, kdop.forward(tm, d, k, kind, q))) / (2 * h)
    assert np.allclose(grad, num, rtol=1e-5, atol=1e-6)


def test_conservative_for_regions_meeting_the_kdop():
    """Boxes and segments through a point inside the k-DOP have m >= 0."""
    d, k = 3, 4
    th = _theta(d, k, 10)
    g = np.random.default_rng(11)
    x = g.uniform(-1, 1, (20000, d))
    x = x[kdop.forward(th, d, k, "point", x) >= 0][:500]
    e = g.uniform(0.0, 0.3, x.shape)
    lo = x - e * g.uniform(0, 1, x.shape)
    boxes = np.concatenate([lo, lo + e], axis=1)
    assert np.all(kdop.forward(th, d, k, "box", boxes) >= 0)
    w = g.standard_normal(x.shape)
    w /= np.linalg.norm(w, axis=1, keepdims=True)
    t = g.uniform(0, 4, (len(x), 1))
    rays = np.concatenate([x - t * w, w], axis=1)
    assert np.all(kdop.forward(th, d, k, "ray", rays) >= -1e-9)


def test_kdop_nonfinite_rows_are_nan():
    th = synth.kdop_init(3, 4, seed=3)
    q = synth.points(4, 20, 3)
    q[5, 1] = np.nan
    q[7, 0] = -np.inf
    z = kdop.forward(th, 3, 4, "point", q)
    assert np.isnan(z[5]) and np.isnan(z[7])
    ok = np.ones(20, bool)
    ok[[5, 7]] = False
    assert np.array_equal(z[ok], kdop.forward(th, 3, 4, "point", q[ok]))
