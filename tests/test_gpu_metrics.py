"""Accuracy metrics on the GPU (Sec. IV-A) against the metric oracle.

Nearest squared distances are compared bit for bit (both sides take the
minimum of the same fp64 expression over the whole reference set); counts
within the tolerance, precision, recall and F-score exactly; the two means to
1e-12 relative (the GPU sums in a different order).
"""
import numpy as np
import pytest

from oracle import mesh as omesh
from oracle import metrics as om
from synth import scene as synth
from tests import parity as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def db():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2509_20081_amd as db
    return db


def dev(a):
    return P.to_device(np.asarray(a, np.float32).reshape(-1, 3))


def clouds():
    rng = np.random.default_rng(11)
    lat_q = (rng.integers(0, 30, size=(4000, 3)) * 0.1).astype(np.float32)
    lat_r = (rng.integers(0, 30, size=(3000, 3)) * 0.1).astype(np.float32)
    plane_q = np.c_[rng.uniform(-5, 5, (2000, 2)), np.zeros(2000)].astype(np.float32)
    plane_r = np.c_[rng.uniform(-5, 5, (1500, 2)), np.full(1500, 0.03)].astype(np.float32)
    far_q = np.concatenate([rng.normal(size=(500, 3)), [[40.0, -30.0, 25.0], [-60.0, 0.0, 0.0]]]).astype(np.float32)
    return {
        "gauss": (rng.normal(size=(5000, 3)).astype(np.float32), rng.normal(size=(4000, 3)).astype(np.float32)),
        "lattice_ties_dups": (lat_q, np.concatenate([lat_r, lat_r[:500]])),
        "flat_plane": (plane_q, plane_r),
        "far_outliers": (far_q, rng.normal(size=(3000, 3)).astype(np.float32)),
        "one_ref": (rng.normal(size=(300, 3)).astype(np.float32), np.array([[0.5, -0.25, 2.0]], np.float32)),
        "ragged_tail": (rng.uniform(-3, 3, (257, 3)).astype(np.float32), rng.uniform(-3, 3, (1025, 3)).astype(np.float32)),
    }


@pytest.mark.parametrize("name", list(clouds().keys()))
def test_nearest_sq_bit_exact(db, name):
    q, r = clouds()[name]
    got = db.nearest_sq(dev(q), dev(r)).cpu().numpy()
    ref = om.nearest_sq_brute(q, r)
    assert got.dtype == np.float64 and got.shape == ref.shape
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64)), \
        f"{np.count_nonzero(got != ref)} of {len(ref)} differ; first {np.argwhere(got != ref)[:3].ravel()}"


@pytest.mark.parametrize("name", ["gauss", "lattice_ties_dups", "flat_plane", "far_outliers"])
@pytest.mark.parametrize("tol", [0.0, 0.05, 0.1, 0.3])
def test_surface_metrics_match_oracle(db, name, tol):
    q, r = clouds()[name]
    got = db.surface_metrics(dev(q), dev(r), tol)
    ref = om.surface_metrics(q, r, tol)
    for k in ("n_pred", "n_gt", "n_pred_within", "n_gt_within", "precision", "recall", "fscore"):
        assert got[k] == ref[k], (k, got[k], ref[k])
    for k in ("accuracy", "completeness", "chamfer_l1"):
        assert got[k] == pytest.approx(ref[k], rel=1e-12, abs=0), (k, got[k], ref[k])


def test_empty_and_bad_inputs(db):
    import torch
    z = torch.zeros((0, 3), dtype=torch.float32, device="cuda")
    r = dev(np.eye(3))
    assert db.nearest_sq(z, r).shape == (0,)
    with pytest.raises(db.DbtsdfError):
        db.nearest_sq(r, z)
    with pytest.raises(db.DbtsdfError):
        db.surface_metrics(z, r, 0.1)
    with pytest.raises(db.DbtsdfError):
        db.surface_metrics(r, r, -1.0)
    bad = dev([[0.0, float("nan"), 0.0]])
    with pytest.raises(db.DbtsdfError):
        db.nearest_sq(bad, r)


def test_metrics_of_fused_map_chain(db):
    """The whole evaluation chain on a small map: the GPU grid (bit-exact with
    the oracle grid), its GPU mesh (equal as a set to the oracle mesh) and its
    point export, each scored on the GPU against the reference points of the
    same rays, and the same numbers from the oracle's own mesh and points
    scored by the oracle."""
    dims, vs, origin = (96, 96, 48), 0.1, (-4.8, -4.8, -0.4)
    o, g, _ = P.make_pair(dims, vs, origin, kernel_size=7, shadow_r2=9, hit_threshold=1)
    m, p = o.new_grid()
    for pose, pts in synth.config_scans(1, scan_ids=[0]):
        o.integrate(m, p, pose, pts)
        g.integrate(pose, P.to_device(pts))
    g.sync()
    gm, gp = P.gpu_planes(g)
    P.assert_grids_equal(gm, gp, m, p, what="planes")
    gt = synth.config_ground_truth(1, scan_ids=[0], cell=0.05)
    lo = np.array(origin) + vs
    hi = np.array(origin) + (np.array(dims) - 1) * vs
    gt = gt[np.all((gt >= lo) & (gt <= hi), axis=1)]
    gt_dev = P.to_device(gt)
    sets = {
        "mesh": (db.mesh_vertices(g.extract_mesh()), omesh.extract_mesh(m, p, origin, vs).reshape(-1, 3)),
        "points": (g.extract_points(), omesh.occupied_points(m, p, origin, vs)),
        "centroids": (db.mesh_centroids(g.extract_mesh()), None),
    }
    res = {}
    rt = omesh.extract_mesh(m, p, origin, vs).reshape(-1, 3, 3)
    rt = rt.astype(np.float64)
    sets["centroids"] = (sets["centroids"][0], ((rt[:, 0] + rt[:, 1] + rt[:, 2]) / 3.0).astype(np.float32))
    for name, (pred_dev, pred_ref) in sets.items():
        got = db.surface_metrics(pred_dev, gt_dev, 0.2)
        ref = om.surface_metrics(pred_ref, gt, 0.2)
        for k in ("n_pred", "n_gt", "n_pred_within", "n_gt_within", "precision", "recall", "fscore"):
            assert got[k] == ref[k], (name, k, got[k], ref[k])
        for k in ("accuracy", "completeness", "chamfer_l1"):
            assert got[k] == pytest.approx(ref[k], rel=1e-12), (name, k, got[k], ref[k])
        res[name] = got
    # the occupied voxels of one noisy scan at 0.1 m lie within a voxel of the
    # surfaces the rays hit, and the mesh covers them; the mesh also closes
    # the shadow region behind each surface against the untouched voxels, so
    # its accuracy is not bounded the same way
    assert res["points"]["accuracy"] < vs, res
    assert res["mesh"]["completeness"] < vs and res["mesh"]["recall"] > 0.9, res
