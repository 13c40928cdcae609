"""Pins for the oracle's counter-based generator and training-batch sampler."""

import os

import numpy as np
import pytest

from oracle import philox, sampling

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat_rows():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append([int(x, 16) for x in line.split()])
    return rows


@pytest.mark.parametrize("row", _kat_rows())
def test_philox_known_answers(row):
    out = philox.philox4x32(*row[:4], *row[4:6])
    assert [int(v) for v in out] == row[6:]


def test_philox_vectorised_matches_scalar():
    i = np.arange(17, dtype=np.uint64)
    vec = philox.philox4x32(i, 3, 5, 7, 11, 13)
    for n in range(17):
        sc = philox.philox4x32(n, 3, 5, 7, 11, 13)
        assert [int(v[n]) for v in vec] == [int(s) for s in sc]


def test_u01_exact_and_in_range():
    w = np.array([0, 255, 256, 0xFFFFFFFF, 0x80000000], dtype=np.uint32)
    u = philox.u01(w)
    assert u.dtype == np.float32
    assert u[0] == 0.0 and u[1] == 0.0
    assert u[2] == np.float32(2.0 ** -24)
    assert u[3] == np.float32(1.0 - 2.0 ** -24)
    assert u[4] == np.float32(0.5)


def test_points_range_grid_and_moments():
    p = sampling.sample_points(7, 0, 1 << 16, 3)
    assert p.dtype == np.float32 and p.shape == (1 << 16, 3)
    assert p.min() >= -1.0 and p.max() < 1.0
    # every value is a multiple of 2^-23 (2u - 1 is exact in float32)
    k = p.astype(np.float64) * 2.0 ** 23
    assert np.all(k == np.round(k))
    assert abs(p.mean()) < 0.01 and abs(p.var() - 1.0 / 3.0) < 0.01
    # a different step gives a different batch; same step, same batch
    assert not np.array_equal(p, sampling.sample_points(7, 1, 1 << 16, 3))
    assert np.array_equal(p, sampling.sample_points(7, 0, 1 << 16, 3))


def test_points4d_time_in_unit_interval():
    p = sampling.sample_points(1, 2, 4096, 4)
    assert p[:, 3].min() >= 0.0 and p[:, 3].max() < 1.0
    assert p[:, :3].min() >= -1.0


def test_rays_distribution():
    r = sampling.sample_rays(3, 0, 1 << 15)
    o, d = r[:, :3].astype(np.float64), r[:, 3:].astype(np.float64)
    ro = np.linalg.norm(o, axis=1)
    assert ro.max() <= 2.0 + 1e-6
    # uniform in a ball of radius 2: P(|o| <= 1) = 1/8
    assert abs((ro <= 1.0).mean() - 0.125) < 0.01
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-6)
    # uniform on the sphere: each component has mean 0 and variance 1/3
    assert np.all(np.abs(d.mean(axis=0)) < 0.02)
    assert np.all(np.abs(d.var(axis=0) - 1.0 / 3.0) < 0.02)


def test_boxes_extent():
    b = sampling.sample_boxes(5, 1, 1 << 14)
    lo, hi = b[:, :3].astype(np.float64), b[:, 3:].astype(np.float64)
    w = hi - lo
    assert w.min() >= 0.02 - 1e-6 and w.max() <= 0.4 + 1e-6
    c = 0.5 * (lo + hi)
    assert c.min() >= -1.0 - 1e-6 and c.max() <= 1.0 + 1e-6
    assert abs(w.mean() - 0.21) < 0.01


def test_planes_unit_normals():
    p = sampling.sample_planes(9, 0, 4096)
    assert np.allclose(np.linalg.norm(p[:, 3:].astype(np.float64), axis=1), 1.0, atol=1e-6)
    assert p[:, :3].min() >= -1.0 and p[:, :3].max() < 1.0
