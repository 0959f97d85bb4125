"""Mesh export on the GPU (Marching Cubes at iso = 0.0) against the mesh oracle, bit for bit.

Triangles come out of the GPU in no fixed order, so both meshes are compared as
canonical sets (each triangle rotated, orientation kept, to start at its least
vertex; rows sorted).
"""
import numpy as np
import pytest

from tests import parity as P
from oracle import mesh
from synth import scene as synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def db():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2509_20081_amd as db
    return db


def same_mesh(gpu_tris, ref_tris):
    a = mesh.canonical(gpu_tris.cpu().numpy())
    b = mesh.canonical(ref_tris)
    return a.shape == b.shape and np.array_equal(a.view(np.uint32), b.view(np.uint32))


@pytest.mark.parametrize("case", [
    dict(K=5, dims=(40, 33, 29), voxel=0.1, origin=(0.0, 0.0, 0.0), shadow_r2=4, hit_threshold=2),
    dict(K=11, dims=(64, 48, 40), voxel=0.05, origin=(-1.2, 0.7, -0.3), shadow_r2=9, hit_threshold=1),
    dict(K=7, dims=(50, 50, 50), voxel=0.1, origin=(0.0, 0.0, 0.0), shadow_r2=6, hit_threshold=3, binning="azel",
         bins_az=8, bins_el=5),
], ids=["K5", "K11", "K7azel"])
def test_mesh_of_fused_scans_matches_oracle(db, case):
    case = dict(case)
    dims, vs, origin, K = case.pop("dims"), case.pop("voxel"), case.pop("origin"), case.pop("K")
    o, g, _ = P.make_pair(dims, vs, origin, kernel_size=K, **case)
    m, p = o.new_grid()
    rng = np.random.default_rng(K)
    centre = np.array(origin) + np.array(dims) * vs / 2
    for _ in range(3):
        pose = synth.random_pose(rng, centre - 0.3, centre + 0.3)
        pts = synth.random_cloud(rng, 1000, -np.array(dims) * vs * 0.45, np.array(dims) * vs * 0.45)
        o.integrate(m, p, pose, pts)
        g.integrate(pose, P.to_device(pts))
    g.sync()
    gm, gp = P.gpu_planes(g)
    P.assert_grids_equal(gm, gp, m, p, what="planes before the mesh")
    ref = mesh.extract_mesh(m, p, origin, vs)
    assert len(ref) > 100
    assert g.count_mesh() == len(ref)
    assert same_mesh(g.extract_mesh(), ref)
    lo, hi = (3, 5, 2), (dims[0] - 4, dims[1] - 2, dims[2] // 2)
    assert same_mesh(g.extract_mesh(lo, hi), mesh.extract_mesh(m, p, origin, vs, lo=lo, hi=hi))


def test_mesh_of_written_fields_with_saddles(db):
    """Random signed fields written into the planes (negative voxels carry a confirmed hit count): many
    saddle faces and loops fanned from their centre; the mesh equals the oracle's."""
    dims, T = (36, 28, 20), 5
    ks = db.KernelSet(kernel_size=5, binning="cube26", shadow_r2=4)
    g = db.Grid(dims, 0.25, (0.5, -1.0, 2.0), ks, hit_threshold=T)
    rng = np.random.default_rng(3)
    d = rng.integers(-6, 7, size=(dims[2], dims[1], dims[0]))
    n = np.minimum(np.abs(d), 32)
    mask = np.where(n >= 32, 0xFFFFFFFF, (1 << n) - 1).astype(np.uint32)
    packed = np.where(d < 0, T, 0x80000000).astype(np.uint32)
    g.write_voxels(mask, packed)
    ref = mesh.extract_mesh(mask, packed, (0.5, -1.0, 2.0), 0.25)
    assert any(c for k in range(256) for _, c in mesh.case_polygons(k))
    assert same_mesh(g.extract_mesh(), ref)


def test_mesh_count_only_overflow_and_empty_boxes(db):
    import torch
    dims = (32, 32, 32)
    o, g, _ = P.make_pair(dims, 0.1, (0.0, 0.0, 0.0), kernel_size=5, shadow_r2=4, hit_threshold=1)
    rng = np.random.default_rng(1)
    pose = synth.random_pose(rng, np.full(3, 1.5), np.full(3, 1.7))
    pts = synth.random_cloud(rng, 800, np.full(3, -1.2), np.full(3, 1.2))
    g.integrate(pose, P.to_device(pts))
    g.sync()
    n = g.count_mesh()
    assert n > 0
    small = torch.zeros((n // 3, 3, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError):
        g.extract_mesh(out=small)
    # the written part of an overflowing call is a subset of the full mesh
    full = {tuple(r) for r in mesh.canonical(g.extract_mesh().cpu().numpy()).view(np.uint32)}
    part = mesh.canonical(small.cpu().numpy()).view(np.uint32)
    assert all(tuple(r) in full for r in part)
    assert g.count_mesh((0, 0, 0), (1, 32, 32)) == 0      # no whole cube in a one-voxel slab
    assert len(g.extract_mesh((5, 5, 5), (7, 6, 9))) == 0
    with pytest.raises(Exception):
        g.count_mesh((0, 0, 0), (33, 32, 32))


def _rows(a):
    a = np.ascontiguousarray(a, np.float32).reshape(-1, 3).view(np.uint32)
    return a[np.lexsort(a.T[::-1])] if len(a) else a


@pytest.mark.parametrize("T", [1, 2])
def test_point_export_matches_oracle(db, T):
    """Occupied contact voxels after a few fused scans, exported as points: the same set of fp32 centres as
    the oracle's, bit for bit, over the whole grid and over a ragged sub-box; count-only agrees."""
    dims, vs, origin = (70, 45, 33), 0.05, (-0.4, 1.1, 0.2)
    o, g, _ = P.make_pair(dims, vs, origin, kernel_size=7, shadow_r2=4, hit_threshold=T)
    m, p = o.new_grid()
    rng = np.random.default_rng(20 + T)
    centre = np.array(origin) + np.array(dims) * vs / 2
    for _ in range(3):
        pose = synth.random_pose(rng, centre - 0.2, centre + 0.2)
        pts = synth.random_cloud(rng, 1500, -np.array(dims) * vs * 0.45, np.array(dims) * vs * 0.45)
        o.integrate(m, p, pose, pts)
        g.integrate(pose, P.to_device(pts))
    g.sync()
    ref = mesh.occupied_points(m, p, origin, vs)
    assert len(ref) > 50
    got = g.extract_points()
    assert np.array_equal(_rows(got.cpu().numpy()), _rows(ref))
    lo, hi = (3, 7, 1), (67, 44, 30)
    sub = g.extract_points(lo, hi)
    assert np.array_equal(_rows(sub.cpu().numpy()), _rows(mesh.occupied_points(m, p, origin, vs, lo=lo, hi=hi)))
    with pytest.raises(Exception):
        g.extract_points((5, 5, 5), (5, 9, 9))   # boxes are non-empty: lo < hi on every axis


def test_point_export_of_written_planes_and_overflow(db):
    """Planes written from the host: every row pattern (x runs longer than a wavefront) exports exactly
    the oracle's points; a buffer too small gets a prefix of valid points and the full count."""
    import ctypes as C
    import torch
    from paper_2509_20081_amd import _lib as L
    dims = (131, 9, 5)
    ks = db.KernelSet(kernel_size=5, binning="cube26", shadow_r2=4)
    g = db.Grid(dims, 0.2, (1.0, -3.0, 0.5), ks, hit_threshold=3)
    rng = np.random.default_rng(4)
    mask = np.where(rng.random(dims[::-1]) < 0.4, 0, 7).astype(np.uint32)
    packed = np.where(rng.random(dims[::-1]) < 0.6, 3, 0x80000001).astype(np.uint32)
    g.write_voxels(mask, packed)
    ref = mesh.occupied_points(mask, packed, (1.0, -3.0, 0.5), 0.2)
    got = g.extract_points().cpu().numpy()
    assert np.array_equal(_rows(got), _rows(ref))
    small = torch.zeros((len(ref) // 2, 3), dtype=torch.float32, device="cuda")
    n = C.c_uint64()
    L.check(L.lib().dbtsdf_extract_points(g._h, None, None, C.c_void_p(small.data_ptr()), small.shape[0],
                                          C.byref(n)), "extract_points")
    assert int(n.value) == len(ref)
    full = {tuple(r) for r in _rows(ref)}
    assert all(tuple(r) in full for r in _rows(small.cpu().numpy()))
    # one pass into a caller's buffer; a buffer too small raises
    buf = torch.full((len(ref) + 5, 3), -1.0, dtype=torch.float32, device="cuda")
    got2 = g.extract_points(out=buf)
    assert np.array_equal(_rows(got2.cpu().numpy()), _rows(ref))
    assert bool((buf[len(ref):] == -1.0).all())
    with pytest.raises(ValueError):
        g.extract_points(out=torch.zeros((len(ref) - 1, 3), dtype=torch.float32, device="cuda"))
