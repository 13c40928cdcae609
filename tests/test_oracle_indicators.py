"""Pins for the oracle's indicators and region queries: closed forms,
brute-force enumeration on tiny grids, and an independent summed-volume
algorithm for boxes."""

import math

import numpy as np
import pytest

import synth
from oracle import indicators as I


# ------------------------------------------------------------------ discs

def test_single_disc_closed_form():
    disc = np.array([[0.1, -0.2, 0.3]], dtype=np.float32)
    ang = np.linspace(0, 2 * np.pi, 97)
    for scale, want in [(0.99, 1), (1.01, 0), (0.0, 1), (0.5, 1), (2.0, 0)]:
        q = np.stack([0.1 + scale * 0.3 * np.cos(ang), -0.2 + scale * 0.3 * np.sin(ang)], 1)
        assert np.all(I.discs2d(q.astype(np.float32), disc) == want)


def test_discs_union_matches_float64():
    discs = synth.discs2d(11)
    q = synth.points(12, 20000, 2)
    got = I.discs2d(q, discs)
    q64 = q.astype(np.float64)
    d2 = ((q64[:, None, :] - discs[None, :, :2].astype(np.float64)) ** 2).sum(-1)
    r2 = discs[None, :, 2].astype(np.float64) ** 2
    ref = (d2 <= r2).any(1)
    near = (np.abs(d2 - r2) < 1e-5).any(1)
    assert np.array_equal(got.astype(bool)[~near], ref[~near])
    assert 0.05 < got.mean() < 0.95


# -------------------------------------------------------------- metaballs

def test_single_metaball_is_a_sphere():
    c = np.array([[0.2, -0.1, 0.3]], dtype=np.float32)
    r = np.array([0.25], dtype=np.float32)
    rng = np.random.default_rng(0)
    v = rng.normal(size=(500, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    for s, want in [(0.98, 1), (1.02, 0), (0.0, 1)]:
        p = (c.astype(np.float64) + s * 0.25 * v).astype(np.float32)
        assert np.all((I.metaball_field(p, c, r) >= 1.0) == bool(want))


def test_metaball_field_two_balls_sum():
    c = np.array([[-0.5, 0, 0], [0.5, 0, 0]], dtype=np.float32)
    r = np.array([0.2, 0.3], dtype=np.float32)
    p = np.array([[0.0, 0.0, 0.0], [0.0, 0.4, 0.0]], dtype=np.float32)
    want = [0.04 / 0.25 + 0.09 / 0.25, 0.04 / 0.41 + 0.09 / 0.41]
    assert np.allclose(I.metaball_field(p, c, r), want, rtol=1e-6)


@pytest.mark.parametrize("n", [4, 8])
def test_voxelize_brute_force(n):
    c, r = synth.metaballs3d(21, k=5, rlo=0.2, rhi=0.5)
    grid = I.voxelize_metaballs(c, r, n)
    for k in range(n):
        for j in range(n):
            for i in range(n):
                p = [(2 * i + 1) / n - 1, (2 * j + 1) / n - 1, (2 * k + 1) / n - 1]
                f = 0.0
                for cb, rb in zip(c.tolist(), r.tolist()):
                    d2 = sum((p[a] - cb[a]) ** 2 for a in range(3))
                    f += rb * rb / d2 if d2 > 0 else math.inf
                if abs(f - 1.0) > 1e-5:
                    assert grid[(k * n + j) * n + i] == (1 if f >= 1.0 else 0), (i, j, k, f)


def test_voxelize_single_ball_volume():
    n = 64
    c = np.zeros((1, 3), dtype=np.float32)
    r = np.array([0.5], dtype=np.float32)
    vol = I.voxelize_metaballs(c, r, n).sum() * (2.0 / n) ** 3
    assert abs(vol - 4.0 / 3.0 * np.pi * 0.125) / (4.0 / 3.0 * np.pi * 0.125) < 0.02


# ------------------------------------------------------------- voxel grid

def test_cell_index_edges():
    n = 8
    p = np.array([-1.0, 1.0, -0.75, -0.7499999, 0.0, np.nextafter(np.float32(1), np.float32(0)),
                  1.0001, -1.0001, np.nan], dtype=np.float32)
    i, ins = I.cell_index(p, n)
    assert i[:6].tolist() == [0, 7, 1, 1, 4, 7]
    assert ins.tolist() == [True] * 6 + [False] * 3


def test_voxel_points_brute_force():
    n = 8
    grid = synth.random_grid(3, n, 0.4)
    q = synth.points(4, 5000, 3) * np.float32(1.05)
    got = I.voxel_points(q, grid, n)
    for row, gv in zip(q.astype(np.float64), got):
        if np.any(np.abs(row) > 1.0):
            assert gv == 0
            continue
        s = (row + 1.0) * n / 2.0
        if np.any(np.abs(s - np.round(s)) < 1e-5):
            continue                       # on a cell boundary: float32 rounding decides
        i, j, k = [min(int(math.floor(v)), n - 1) for v in s]
        assert gv == grid[(k * n + j) * n + i]


def _segment_hits_cells(o, d, n, grid, t_max=4.0, m=20000):
    """Dense float64 sampling of the segment: the set of occupied cells hit."""
    t = np.linspace(0.0, t_max, m)
    p = o[None, :] + t[:, None] * d[None, :]
    ok = np.all(np.abs(p) <= 1.0, axis=1)
    s = np.minimum(np.floor((p[ok] + 1.0) * n / 2.0).astype(int), n - 1)
    idx = (s[:, 2] * n + s[:, 1]) * n + s[:, 0]
    return bool(grid[idx].any()) if idx.size else False


def test_ray_special_cases_and_dense_bound():
    n = 4
    grid = synth.random_grid(8, n, 0.3)
    q = synth.rays(9, 400)
    got = I.voxel_rays(q, grid, n)
    # the 256 samples lie on the segment, so sampled any() <= dense any();
    # with 4^3 cells (width 0.5) and spacing 4/255 they agree but for grazing rays
    dense = np.array([_segment_hits_cells(r[:3].astype(np.float64), r[3:].astype(np.float64), n, grid)
                      for r in q])
    assert np.all(got.astype(bool) <= dense)
    assert (got.astype(bool) == dense).mean() > 0.97
    # d = 0: the query reduces to the point test at the origin
    q0 = q.copy()
    q0[:, :3] = synth.points(10, 400, 3)
    q0[:, 3:] = 0
    assert np.array_equal(I.voxel_rays(q0, grid, n), I.voxel_points(q0[:, :3], grid, n))
    # a segment that stays outside the cube never hits
    far = np.array([[3.0, 3.0, 3.0, 0.0, 0.0, 1.0]], dtype=np.float32)
    assert I.voxel_rays(far, np.ones(n ** 3, np.uint8), n)[0] == 0


def test_ray_t_table():
    t = I.ray_t_table()
    assert t.dtype == np.float32 and t.size == 256
    assert t[0] == 0.0 and t[-1] == 4.0 and np.all(np.diff(t) > 0)


def _sat(grid, n):
    g = grid.reshape(n, n, n).astype(np.int64)
    s = np.zeros((n + 1, n + 1, n + 1), dtype=np.int64)
    s[1:, 1:, 1:] = g.cumsum(0).cumsum(1).cumsum(2)
    return s


def test_boxes_vs_summed_volume_table():
    n = 16
    grid = synth.random_grid(5, n, 0.02)
    q = synth.boxes(6, 3000, 0.01, 0.3)
    got = I.voxel_boxes(q, grid, n)
    s = _sat(grid, n)
    for row, gv in zip(q.astype(np.float64), got):
        lo, hi = np.maximum(row[:3], -1.0), np.minimum(row[3:], 1.0)
        if np.any(hi < lo):
            assert gv == 0
            continue
        a = np.minimum(np.floor((lo + 1) * n / 2).astype(int), n - 1)
        b = np.minimum(np.floor((hi + 1) * n / 2).astype(int), n - 1) + 1
        cnt = (s[b[2], b[1], b[0]] - s[a[2], b[1], b[0]] - s[b[2], a[1], b[0]] - s[b[2], b[1], a[0]]
               + s[a[2], a[1], b[0]] + s[a[2], b[1], a[0]] + s[b[2], a[1], a[0]] - s[a[2], a[1], a[0]])
        assert gv == (1 if cnt > 0 else 0)
    assert 0.05 < got.mean() < 0.95


def test_boxes_degenerate_and_full():
    n = 8
    grid = synth.random_grid(1, n, 0.3)
    p = synth.points(2, 500, 3)
    q = np.concatenate([p, p], axis=1)
    assert np.array_equal(I.voxel_boxes(q, grid, n), I.voxel_points(p, grid, n))
    full = np.array([[-2, -2, -2, 2, 2, 2]], dtype=np.float32)
    assert I.voxel_boxes(full, grid, n)[0] == grid.any()
    out = np.array([[1.5, -0.5, -0.5, 2.0, 0.5, 0.5]], dtype=np.float32)
    assert I.voxel_boxes(out, np.ones(n ** 3, np.uint8), n)[0] == 0


def test_plane_axis_aligned_layers():
    n = 8
    grid = synth.random_grid(4, n, 0.05)
    g3 = grid.reshape(n, n, n)
    for z0 in [-0.9, -0.5, -0.3, 0.1, 0.26, 0.75, 0.99]:
        q = np.array([[0.3, -0.2, z0, 0, 0, 1]], dtype=np.float32)
        # cells whose closed z-extent [-1 + 2k/n, -1 + 2(k+1)/n] contains z0
        ks = [k for k in range(n) if -1 + 2 * k / n <= z0 <= -1 + 2 * (k + 1) / n]
        want = any(g3[k].any() for k in ks)
        assert I.voxel_planes(q, grid, n)[0] == want


def test_plane_oblique_vs_float64():
    n = 8
    grid = synth.random_grid(2, n, 0.03)
    q = synth.planes(3, 300)
    got = I.voxel_planes(q, grid, n)
    idx = np.nonzero(grid)[0]
    c = np.stack([(2 * (idx % n) + 1) / n - 1, (2 * ((idx // n) % n) + 1) / n - 1,
                  (2 * (idx // (n * n)) + 1) / n - 1], 1)
    for row, gv in zip(q.astype(np.float64), got):
        e = (c - row[:3]) @ row[3:]
        rad = np.abs(row[3:]).sum() / n
        margin = np.abs(np.abs(e) - rad)
        if np.any(margin < 1e-5):
            continue
        assert gv == (np.abs(e) <= rad).any()


# ------------------------------------------------------------ 4-D balls

def test_metaballs4d_static_and_endpoints():
    a, b, r = synth.metaballs4d(31, k=6)
    p = synth.points(32, 3000, 3)
    t = synth.points4d(33, 3000)[:, 3:]
    q = np.concatenate([p, t], 1)
    # static paths (b = a): the 4-D indicator is the 3-D metaball field
    assert np.array_equal(I.metaballs4d(q, a, a, r), (I.metaball_field(p, a, r) >= 1).astype(np.uint8))
    # at t = 0 the balls sit at a
    q0 = np.concatenate([p, np.zeros((3000, 1), np.float32)], 1)
    assert np.array_equal(I.metaballs4d(q0, a, b, r), (I.metaball_field(p, a, r) >= 1).astype(np.uint8))
    # at t = 1 they sit at b (up to one rounding of a + (b - a))
    q1 = np.concatenate([p, np.ones((3000, 1), np.float32)], 1)
    f1 = I.metaball_field(p, b, r)
    ok = np.abs(f1 - 1) > 1e-4
    assert np.array_equal(I.metaballs4d(q1, a, b, r)[ok], (f1 >= 1).astype(np.uint8)[ok])


def test_metaballs4d_vs_float64():
    a, b, r = synth.metaballs4d(41)
    q = synth.points4d(42, 20000)
    got = I.metaballs4d(q, a, b, r)
    q64 = q.astype(np.float64)
    c = a.astype(np.float64)[None] + q64[:, 3:4, None] * (b.astype(np.float64) - a)[None]
    d2 = ((q64[:, None, :3] - c) ** 2).sum(-1)
    f = (r.astype(np.float64) ** 2 / d2).sum(1)
    ok = np.abs(f - 1) > 1e-4
    assert np.array_equal(got[ok].astype(bool), (f >= 1)[ok])
    assert 0.01 < got.mean() < 0.9
