"""Reconstruction-accuracy metrics of a predicted point set against a reference
set -- test infrastructure only (tests, smoke check, benchmark CPU leg).

The paper scores a map by nearest-neighbour distances between points sampled
from the zero level of its mesh and the ground-truth points (Sec. IV-A,
"Metrics"):

- Accuracy: the mean distance from each predicted point to its nearest
  ground-truth point;
- Completeness: the mean distance from each ground-truth point to its nearest
  predicted point;
- Chamfer-L1: the mean of the two;
- at a tolerance t, Recall: the share of ground-truth points whose nearest
  predicted point lies within t; Precision: the share of predicted points
  whose nearest ground-truth point lies within t; F-score: their harmonic mean.

Readings (the paper gives the definitions in words only):

A1  "Within t" is strictly closer than t: d^2 < t^2, both in fp64, with
    t^2 = t * t.
A2  A squared distance is ((qx - rx)^2 + (qy - ry)^2) + (qz - rz)^2 in IEEE
    fp64 from fp32 coordinates, one operation at a time in that order; a
    distance is the fp64 square root of it.
A3  The F-score of P = R = 0 is 0.
A4  The means are over all points of the set (no outlier cut); either set
    being empty is an error.

The nearest squared distance is a minimum over all reference points, so it
does not depend on the order in which candidates are visited: the brute-force
definition below and the k-d tree path give the same value bit for bit.
"""
from __future__ import annotations

import numpy as np

__all__ = ["nearest_sq_brute", "nearest_sq", "surface_metrics"]


def _as_f32_points(p) -> np.ndarray:
    p = np.ascontiguousarray(p, dtype=np.float32)
    if p.ndim != 2 or p.shape[1] != 3:
        raise ValueError("points must have shape (n, 3)")
    return p


def _sq(q64: np.ndarray, r64: np.ndarray) -> np.ndarray:
    """Reading A2, for broadcastable fp64 arrays of points (last axis xyz)."""
    dx = q64[..., 0] - r64[..., 0]
    dy = q64[..., 1] - r64[..., 1]
    dz = q64[..., 2] - r64[..., 2]
    return (dx * dx + dy * dy) + dz * dz


def nearest_sq_brute(query, ref, chunk: int = 2048) -> np.ndarray:
    """Per query point: the smallest squared distance to any reference point
    (the definition, every pair evaluated)."""
    q = _as_f32_points(query).astype(np.float64)
    r = _as_f32_points(ref).astype(np.float64)
    if len(r) == 0:
        raise ValueError("empty reference set")
    out = np.empty(len(q), np.float64)
    for i in range(0, len(q), chunk):
        d2 = _sq(q[i:i + chunk, None, :], r[None, :, :])
        out[i:i + chunk] = d2.min(axis=1)
    return out


def nearest_sq(query, ref, k: int = 8) -> np.ndarray:
    """The same minimum through a k-d tree (scipy), for sets too large for the
    pairwise definition: the tree proposes the k nearest candidates in its own
    arithmetic and the minimum of reading A2 over them is taken, so that a
    near-tie the tree's rounding orders differently still yields the exact
    minimum."""
    q = _as_f32_points(query)
    r = _as_f32_points(ref)
    if len(r) == 0:
        raise ValueError("empty reference set")
    if len(q) * len(r) <= 4_000_000:
        return nearest_sq_brute(q, r)
    from scipy.spatial import cKDTree

    r64 = r.astype(np.float64)
    q64 = q.astype(np.float64)
    tree = cKDTree(r64)
    kk = min(k, len(r))
    _, idx = tree.query(q64, k=kk)
    idx = np.asarray(idx).reshape(len(q), kk)
    d2 = _sq(q64[:, None, :], r64[idx])
    return d2.min(axis=1)


def surface_metrics(pred, gt, tolerance: float) -> dict:
    """Accuracy, completeness, Chamfer-L1 (metres) and precision, recall,
    F-score at ``tolerance`` of ``pred`` against ``gt`` (Sec. IV-A)."""
    pred = _as_f32_points(pred)
    gt = _as_f32_points(gt)
    if len(pred) == 0 or len(gt) == 0:
        raise ValueError("both point sets must be non-empty (reading A4)")
    d2_pred = nearest_sq(pred, gt)      # predicted -> ground truth
    d2_gt = nearest_sq(gt, pred)        # ground truth -> predicted
    t = float(tolerance)
    t2 = t * t
    acc = float(np.sqrt(d2_pred).mean())
    comp = float(np.sqrt(d2_gt).mean())
    n_pred_in = int(np.count_nonzero(d2_pred < t2))
    n_gt_in = int(np.count_nonzero(d2_gt < t2))
    precision = n_pred_in / len(pred)
    recall = n_gt_in / len(gt)
    fscore = 0.0 if precision + recall == 0.0 else 2.0 * precision * recall / (precision + recall)
    return {"accuracy": acc, "completeness": comp, "chamfer_l1": 0.5 * (acc + comp),
            "precision": precision, "recall": recall, "fscore": fscore,
            "n_pred": len(pred), "n_gt": len(gt), "n_pred_within": n_pred_in, "n_gt_within": n_gt_in,
            "tolerance": t}
