"""Pins of the radiodensity-aware dual sampling reference (oracle/rads_ref.py)
against closed forms: a linear ramp (every crossing lies on the level plane,
one per row of x-edges), a distance field (crossings on the sphere within
the linear-interpolation error), weighted draws with known weights, the key
subsample, and the nearest-neighbour scale of a regular grid.  CPU only."""
import numpy as np
import pytest

from oracle import rads_ref


def test_ramp_crossings_lie_on_the_level_plane():
    nz, ny, nx = 5, 6, 9
    x = np.arange(nx, dtype=np.float32)
    hu = np.broadcast_to(10.0 * x - 3.0, (nz, ny, nx)).astype(np.float32)
    iso = rads_ref.iso_level(hu)
    assert iso == np.float32((-3.0 + 77.0) * 0.5)
    pts, ids = rads_ref.crossings(hu, iso, (0.5, 1.0, 2.0), (1.0, -2.0, 3.0))
    assert len(pts) == ny * nz  # one x-edge per row crosses, no y- or z-edge
    assert np.all(ids % 3 == 0) and np.all(np.diff(ids) > 0)
    x_level = (float(iso) + 3.0) / 10.0  # voxel coordinate where the ramp meets the level
    np.testing.assert_allclose(pts[:, 0], 1.0 + 0.5 * x_level, rtol=0, atol=1e-12)
    ys, zs = np.meshgrid(np.arange(ny), np.arange(nz))
    np.testing.assert_allclose(np.sort(pts[:, 1]), np.sort(-2.0 + ys.ravel().astype(float)), atol=1e-12)
    np.testing.assert_allclose(np.sort(pts[:, 2]), np.sort(3.0 + 2.0 * zs.ravel().astype(float)), atol=1e-12)


def test_distance_field_crossings_lie_on_the_sphere():
    """Distance field |p - c| at level r: crossings lie on the sphere up to the
    chord error of linear interpolation (below h^2 / (2 r) for unit voxels)."""
    n, r = 40, 12.0
    g = np.arange(n) + 0.0
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    c = np.array([19.0, 20.0, 18.0])  # a voxel centre: the minimum is 0
    d = np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2).astype(np.float32)
    hu = np.minimum(d, np.float32(2 * r))  # min 0 at the centre, max 2r: level r
    iso = rads_ref.iso_level(hu)
    assert iso == np.float32(r)
    pts, _ = rads_ref.crossings(hu, iso, (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))
    dist = np.linalg.norm(pts - c, axis=1)
    assert len(pts) > 4 * np.pi * r * r  # at least the sphere's area in unit faces
    assert np.abs(dist - r).max() < 1.0 / (2 * r) + 1e-6


def test_weighted_draws_follow_the_weights():
    """Three voxels above the minimum: weights 65535, floor(0.5 * 65535) and
    floor(0.25 * 65535); a draw picks the first voxel whose running sum
    exceeds it."""
    hu = np.zeros((2, 3, 4), np.float32)
    hu[0, 1, 2] = 4.0   # max: index 6
    hu[1, 0, 0] = 2.0   # index 12
    hu[1, 2, 3] = 1.0   # index 23
    w = rads_ref.weights(hu)
    assert w[6] == 65535 and w[12] == 32767 and w[23] == 16383 and w.sum() == 65535 + 32767 + 16383
    draws = np.array([0, 65534, 65535, 65535 + 32766, 65535 + 32767, w.sum() - 1], np.uint64)
    pts, idx = rads_ref.weighted_draws(hu, draws, (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))
    assert idx.tolist() == [6, 6, 12, 12, 23, 23]
    np.testing.assert_array_equal(pts[0], [2.0, 1.0, 0.0])
    np.testing.assert_array_equal(pts[-1], [3.0, 2.0, 1.0])


def test_grid_nearest_neighbour_scale():
    """On a regular grid of spacing h every point has at least three
    neighbours at distance h, so every log-scale is log h."""
    h = 0.7
    g = np.arange(4) * h
    P = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    np.testing.assert_allclose(rads_ref.knn_log_scale(P), np.log(h), rtol=0, atol=1e-12)
    # coincident points clamp at 1e-7 mm^2
    assert rads_ref.knn_log_scale(np.zeros((5, 3))) == pytest.approx(0.5 * np.log(1e-7))


def test_rads_sets_and_subsample():
    """Keys in reverse edge order keep the last n1 crossings, reversed; the
    isotropic set is P^mc plus the first half of P^dw."""
    rng = np.random.default_rng(1)
    hu = rng.normal(size=(6, 7, 8)).astype(np.float32)
    pmc, _ = rads_ref.crossings(hu, rads_ref.iso_level(hu), (1, 1, 1), (0, 0, 0))
    M = len(pmc)
    keys = np.arange(M, 0, -1, dtype=np.uint32)
    W = int(rads_ref.weights(hu).astype(np.uint64).sum())
    draws = rng.integers(0, W, 9).astype(np.uint64)
    pts, n_iso, ls = rads_ref.rads(hu, (1, 1, 1), (0, 0, 0), 5, keys, draws)
    np.testing.assert_array_equal(pts[:5], pmc[::-1][:5])
    assert n_iso == 5 + 4 and len(pts) == 14 and ls.shape == (14,)
