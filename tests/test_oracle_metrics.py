"""Pins of the accuracy-metric oracle (Sec. IV-A metric definitions).

Every expected value here follows from the geometry of the case, not from the
formulas of ``oracle/metrics.py``: grids of points at dyadic spacing (exact in
fp32 and fp64) so that nearest distances are known in closed form.
"""
import math

import numpy as np
import pytest

from oracle import metrics

S = 0.25      # grid spacing (dyadic: exact)


def plane(n=16, z=0.0):
    """An n x n grid of points on the plane z, spacing S."""
    x, y = np.meshgrid(np.arange(n) * S, np.arange(n) * S, indexing="ij")
    return np.stack([x.ravel(), y.ravel(), np.full(x.size, z)], 1).astype(np.float32)


def cube_surface(n=8):
    """Points of the surface of the cube [0, (n-1) S]^3 on the S grid."""
    g = np.arange(n) * S
    pts = set()
    for a in range(3):
        for fixed in (0.0, g[-1]):
            u, v = np.meshgrid(g, g, indexing="ij")
            p = np.zeros((u.size, 3))
            p[:, a] = fixed
            p[:, (a + 1) % 3] = u.ravel()
            p[:, (a + 2) % 3] = v.ravel()
            pts.update(map(tuple, p))
    return np.array(sorted(pts), np.float32)


@pytest.mark.parametrize("d", [0.0625, 0.09375, 0.015625])
def test_parallel_planes_at_offset(d):
    """A plane against the same grid lifted by d < S: every point's nearest
    partner is its twin, at exactly d (any other point is at sqrt(S^2 + d^2)
    or farther), both ways."""
    gt, pred = plane(), plane(z=d)
    m = metrics.surface_metrics(pred, gt, tolerance=0.1)
    assert m["accuracy"] == d and m["completeness"] == d and m["chamfer_l1"] == d
    inside = 1.0 if d < 0.1 else 0.0
    assert m["precision"] == inside and m["recall"] == inside and m["fscore"] == inside
    assert m["n_pred"] == m["n_gt"] == 256


def test_tolerance_is_strict():
    """Reading A1: a distance equal to the tolerance is not within it."""
    m = metrics.surface_metrics(plane(z=0.125), plane(), tolerance=0.125)
    assert m["recall"] == 0.0 and m["precision"] == 0.0 and m["fscore"] == 0.0
    m = metrics.surface_metrics(plane(z=0.125), plane(), tolerance=0.125 + 2 ** -20)
    assert m["recall"] == 1.0 and m["precision"] == 1.0 and m["fscore"] == 1.0


def test_half_prediction():
    """Prediction = the even x columns of the reference: accuracy 0 (a subset);
    completeness: half the reference points at 0, half at S from the column
    beside them, so S / 2; recall 1/2 below S and 1 above; precision 1;
    F = 2 (1/2) / (3/2) = 2/3 below S."""
    gt = plane()
    pred = gt[(np.round(gt[:, 0] / S).astype(int) % 2) == 0]
    m = metrics.surface_metrics(pred, gt, tolerance=0.2)
    assert m["accuracy"] == 0.0
    assert m["completeness"] == S / 2
    assert m["chamfer_l1"] == S / 4
    assert m["recall"] == 0.5 and m["precision"] == 1.0
    assert m["fscore"] == pytest.approx(2.0 / 3.0, rel=1e-15)
    m = metrics.surface_metrics(pred, gt, tolerance=0.3)
    assert m["recall"] == 1.0 and m["fscore"] == 1.0


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_cube_shifted(axis):
    """The cube's surface grid shifted by d < S / 2 along one axis: for every
    shifted point the source point lies at d, and every reference point at
    least d away (its coordinate along the axis differs from the shifted
    point's by d or by at least S - d), so both means are d, whatever the face
    orientation; the two directions are symmetric."""
    d = 0.078125
    gt = cube_surface()
    pred = gt.copy()
    pred[:, axis] += np.float32(d)
    m = metrics.surface_metrics(pred, gt, tolerance=0.05)
    assert m["accuracy"] == d and m["completeness"] == d
    assert m["recall"] == 0.0
    assert len(gt) == 6 * 8 * 8 - 12 * 8 + 8   # faces - shared edges + corners counted once


def test_far_outlier_counts_fully():
    """Reading A4: no outlier cut. One predicted point 10 m away adds 10 m / n
    to the accuracy."""
    gt = plane()
    pred = np.concatenate([gt, np.array([[0.0, 0.0, 10.0]], np.float32)])
    m = metrics.surface_metrics(pred, gt, tolerance=0.1)
    assert m["accuracy"] == pytest.approx(10.0 / 257, rel=1e-15)
    assert m["completeness"] == 0.0
    assert m["precision"] == 256 / 257 and m["recall"] == 1.0


def test_fscore_zero_when_nothing_within():
    m = metrics.surface_metrics(plane(z=1.0), plane(), tolerance=0.5)
    assert m["precision"] == 0.0 and m["recall"] == 0.0 and m["fscore"] == 0.0


def test_empty_sets_refused():
    with pytest.raises(ValueError):
        metrics.surface_metrics(np.zeros((0, 3), np.float32), plane(), 0.1)
    with pytest.raises(ValueError):
        metrics.surface_metrics(plane(), np.zeros((0, 3), np.float32), 0.1)


def test_single_point_distance():
    """3-4-12 triangle: sqrt(9 + 16 + 144) = 13 (exact)."""
    q = np.array([[1.0, 2.0, 3.0]], np.float32)
    r = np.array([[4.0, 6.0, 15.0], [100.0, 0.0, 0.0]], np.float32)
    assert metrics.nearest_sq_brute(q, r).tolist() == [169.0]
    m = metrics.surface_metrics(q, r, 20.0)
    assert m["accuracy"] == 13.0


def test_tree_path_equals_definition():
    """The k-d tree path (taken for large sets) gives the pairwise minimum bit
    for bit, near-ties included (points on a coarse lattice have many equal
    distances)."""
    rng = np.random.default_rng(7)
    q = (rng.integers(0, 40, size=(3000, 3)) * 0.125).astype(np.float32)
    r = (rng.integers(0, 40, size=(2500, 3)) * 0.125 + 0.0625).astype(np.float32)
    r2 = np.concatenate([r, r[:100]])   # duplicates too
    brute = metrics.nearest_sq_brute(q, r2)
    from scipy.spatial import cKDTree  # noqa: F401  (the path below uses it)
    tree = metrics.nearest_sq(np.repeat(q, 1, 0), np.tile(r2, (2, 1)))   # > 4e6 pairs: the tree path
    assert np.array_equal(brute, tree)
    # and on continuous random clouds
    q = rng.normal(size=(2500, 3)).astype(np.float32)
    r = rng.normal(size=(2000, 3)).astype(np.float32)
    assert np.array_equal(metrics.nearest_sq_brute(q, r), metrics.nearest_sq(q, np.tile(r, (2, 1))))
