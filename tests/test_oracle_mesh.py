"""Pins of the mesh oracle (Marching Cubes at iso = 0.0, the export of the fused map).

The readings M1-M5 are stated in ``oracle/mesh.py``. These tests fix them with
a hand-worked cube, closed-surface properties (every edge of the mesh shared by
two triangles running it in opposite directions), the enclosed volume and area
of a sphere, and the vertex formula on a linear field.
"""
import math

import numpy as np

from oracle import mesh


def planes_from_distance(d):
    """mask / packed planes whose read-out signed distance is d (|d| <= 32, integer)."""
    d = np.asarray(d, np.int64)
    n = np.minimum(np.abs(d), 32)
    mask = np.where(n >= 32, 0xFFFFFFFF, (1 << n) - 1).astype(np.uint32)
    packed = np.where(d >= 0, 0x80000000, 0).astype(np.uint32)
    return mask, packed


def test_signed_distance_readout():
    d = np.array([[[-3, 0, 5, 32, -32]]])
    m, p = planes_from_distance(d)
    assert mesh.signed_distance(m, p).tolist() == d.tolist()


def test_edge_numbering_and_faces():
    assert len(mesh.EDGES) == 12
    # x edges first (lower corners 0, 2, 4, 6), then y (0, 1, 4, 5), then z (0, 1, 2, 3)
    assert mesh.EDGES[:4] == [(0, 0), (0, 2), (0, 4), (0, 6)]
    assert mesh.EDGES[4:8] == [(1, 0), (1, 1), (1, 4), (1, 5)]
    assert mesh.EDGES[8:] == [(2, 0), (2, 1), (2, 2), (2, 3)]
    # every face cycle runs counter-clockwise about its outward normal
    for ring in mesh.FACES:
        pts = np.array([mesh.corner_offset(c) for c in ring], float)
        centre = pts.mean(0)
        normal = np.cross(pts[1] - pts[0], pts[2] - pts[1])
        outward = centre - 0.5
        assert np.dot(normal, outward) > 0


def test_every_crossed_edge_in_exactly_one_loop():
    for case in range(256):
        inside = [(case >> c) & 1 for c in range(8)]
        crossed = {n for n, (a, c) in enumerate(mesh.EDGES) if inside[c] != inside[c | (1 << a)]}
        loops = mesh.case_loops(case)
        seen = [e for loop in loops for e in loop]
        assert sorted(seen) == sorted(crossed), case
        assert all(len(loop) >= 3 for loop in loops)
        pol = mesh.case_polygons(case)
        assert sum(len(w) if c else len(w) - 2 for w, c in pol) == len(mesh.TABLE[case])
    assert mesh.TABLE[0] == [] and mesh.TABLE[255] == []


def test_hand_worked_single_corner_cube():
    """One cube, corner 0 at d = -1 and the rest at +3, unit voxels from the origin: one triangle on
    the three edges at corner 0, each vertex a quarter of the way (t = -1 / (-1 - 3)), normal along +(1,1,1)."""
    d = np.full((2, 2, 2), 3)
    d[0, 0, 0] = -1
    m, p = planes_from_distance(d)
    tris = mesh.extract_mesh(m, p, (0.0, 0.0, 0.0), 1.0)
    assert tris.shape == (1, 3, 3)
    want = np.array([[0.75, 0.5, 0.5], [0.5, 0.75, 0.5], [0.5, 0.5, 0.75]], np.float32)
    assert np.array_equal(tris[0], want)
    nrm = np.cross(tris[0][1] - tris[0][0], tris[0][2] - tris[0][0])
    assert np.all(nrm > 0)


def test_each_single_inside_corner_gives_one_outward_triangle():
    for c in range(8):
        d = np.full((2, 2, 2), 2)
        cx, cy, cz = mesh.corner_offset(c)
        d[cz, cy, cx] = -2
        m, p = planes_from_distance(d)
        tris = mesh.extract_mesh(m, p, (0.0, 0.0, 0.0), 1.0)
        assert tris.shape == (1, 3, 3)
        nrm = np.cross(tris[0][1] - tris[0][0], tris[0][2] - tris[0][0])
        away = tris[0].mean(0) - (np.array([cx, cy, cz]) + 0.5)
        assert np.dot(nrm, away) > 0, c


def test_linear_field_vertex_formula():
    """d = 3 (z - 2) - 1 over z: the zero level lies a third of the way from z = 2 to z = 3 (M2)."""
    z = np.arange(6)
    d = np.broadcast_to((3 * (z - 2) - 1)[:, None, None], (6, 4, 5)).copy()
    m, p = planes_from_distance(d)
    origin, s = (1.5, -2.0, 0.25), 0.1
    tris = mesh.extract_mesh(m, p, origin, s)
    assert len(tris) == 2 * 3 * 4        # two triangles per cube of the 3 x 4 sheet of cubes
    t = np.float32(np.float32(-1.0) / np.float32(-1.0 - 2.0))
    cz = np.float32(np.float32(0.25) + np.float32(np.float32(2.5) * np.float32(s)))
    want_z = np.float32(cz + np.float32(t * np.float32(s)))
    assert np.all(tris[:, :, 2] == want_z)
    nrm = np.cross(tris[:, 1] - tris[:, 0], tris[:, 2] - tris[:, 0])
    assert np.all(nrm[:, 2] > 0) and np.allclose(nrm[:, :2], 0)


def _edge_balance(tris):
    """Directed edges (by vertex bit patterns) of a triangle soup: {(a, b): count}."""
    v = np.ascontiguousarray(tris, np.float32).reshape(-1, 3).view(np.uint32)
    keys = [tuple(int(x) for x in row) for row in v]
    cnt = {}
    for i in range(0, len(keys), 3):
        tri = keys[i:i + 3]
        for k in range(3):
            e = (tri[k], tri[(k + 1) % 3])
            cnt[e] = cnt.get(e, 0) + 1
    return cnt


def _closed_and_oriented(tris):
    cnt = _edge_balance(tris)
    return all(v == 1 and cnt.get((b, a)) == 1 for (a, b), v in cnt.items())


def test_random_fields_give_closed_oriented_surfaces():
    """Random signs inside a box whose border is outside: every mesh edge is run once in each direction
    by two triangles (no holes, M3; consistent orientation, M4), saddle faces included."""
    rng = np.random.default_rng(5)
    for trial in range(6):
        n = 9
        d = rng.integers(-4, 5, size=(n, n, n))
        d[d == 0] = 1
        d[0], d[-1], d[:, 0], d[:, -1], d[:, :, 0], d[:, :, -1] = 3, 3, 3, 3, 3, 3
        m, p = planes_from_distance(d)
        tris = mesh.extract_mesh(m, p, (0.0, 0.0, 0.0), 1.0)
        assert len(tris) > 0
        assert _closed_and_oriented(tris), trial


def test_sphere_volume_and_area():
    """A sphere of radius 9 voxels: enclosed volume (divergence theorem, positive for outward normals)
    and area within a few per cent of 4/3 pi r^3 and 4 pi r^2."""
    n, r0 = 26, 9.0
    g = np.arange(n) + 0.5
    zz, yy, xx = np.meshgrid(g, g, g, indexing="ij")
    r = np.sqrt((xx - n / 2) ** 2 + (yy - n / 2) ** 2 + (zz - n / 2) ** 2)
    d = np.where(r >= r0, np.ceil(r - r0), -np.ceil(r0 - r)).astype(int)
    d[d == 0] = 1
    m, p = planes_from_distance(d)
    tris = mesh.extract_mesh(m, p, (0.0, 0.0, 0.0), 1.0).astype(np.float64)
    assert _closed_and_oriented(tris.astype(np.float32))
    vol = np.einsum("ij,ij->i", tris[:, 0], np.cross(tris[:, 1], tris[:, 2])).sum() / 6.0
    area = 0.5 * np.linalg.norm(np.cross(tris[:, 1] - tris[:, 0], tris[:, 2] - tris[:, 0]), axis=1).sum()
    assert abs(vol / (4.0 / 3.0 * math.pi * r0 ** 3) - 1.0) < 0.08
    assert abs(area / (4.0 * math.pi * r0 ** 2) - 1.0) < 0.12


def test_box_restricts_cubes():
    rng = np.random.default_rng(9)
    d = rng.integers(-3, 4, size=(7, 8, 9))
    m, p = planes_from_distance(d)
    full = mesh.canonical(mesh.extract_mesh(m, p, (0.0, 0.0, 0.0), 0.5))
    parts = [mesh.extract_mesh(m, p, (0.0, 0.0, 0.0), 0.5, lo=(0, 0, 0), hi=(9, 8, 4)),
             mesh.extract_mesh(m, p, (0.0, 0.0, 0.0), 0.5, lo=(0, 0, 3), hi=(9, 8, 7))]
    both = mesh.canonical(np.concatenate(parts))
    assert np.array_equal(full.view(np.uint32), both.view(np.uint32))
    assert len(mesh.extract_mesh(m, p, (0.0, 0.0, 0.0), 0.5, lo=(2, 2, 2), hi=(3, 8, 7))) == 0


def test_point_export_of_the_hand_worked_scan(golden_dir):
    """The hand-worked single return (T = 1): only its contact voxel has mask 0, and its shadow count
    reached T, so the point export is that voxel's centre alone."""
    import json
    import os
    from oracle.oracle import Oracle
    gold = json.load(open(os.path.join(golden_dir, "hand_worked_scan.json")))
    kw = {k: v for k, v in gold["kernel"].items()}
    o = Oracle(dims=gold["grid"]["dims"], voxel_size=gold["grid"]["voxel_size"], origin=gold["grid"]["origin"], **kw)
    m, p = o.new_grid()
    pose = np.eye(4, dtype=np.float32)
    pose[:3, 3] = gold["pose_translation"]
    o.integrate(m, p, pose, np.array([gold["point"]], np.float32))
    pts = mesh.occupied_points(m, p, gold["grid"]["origin"], gold["grid"]["voxel_size"])
    v = gold["expect"]["voxel"]
    assert pts.tolist() == [[v[0] + 0.5, v[1] + 0.5, v[2] + 0.5]]
    # a hit below the threshold is not yet occupied
    o2 = Oracle(dims=gold["grid"]["dims"], voxel_size=1.0, **dict(kw, hit_threshold=2))
    m2, p2 = o2.new_grid()
    o2.integrate(m2, p2, pose, np.array([gold["point"]], np.float32))
    assert len(mesh.occupied_points(m2, p2, (0.0, 0.0, 0.0), 1.0)) == 0
    o2.integrate(m2, p2, pose, np.array([gold["point"]], np.float32))
    assert len(mesh.occupied_points(m2, p2, (0.0, 0.0, 0.0), 1.0)) == 1


def test_point_export_coordinates_and_box():
    m = np.full((3, 4, 5), 0xFFFFFFFF, np.uint32)
    p = np.full((3, 4, 5), 0x80000000, np.uint32)
    m[2, 1, 3], p[2, 1, 3] = 0, 5          # occupied contact voxel
    m[0, 0, 0], p[0, 0, 0] = 0, 0x80000001  # hit once, still free
    m[1, 3, 4], p[1, 3, 4] = 1, 5          # confirmed but not a contact voxel
    pts = mesh.occupied_points(m, p, (1.0, -2.0, 0.5), 0.1)
    want = [np.float32(np.float32(1.0) + np.float32(3.5) * np.float32(0.1)),
            np.float32(np.float32(-2.0) + np.float32(1.5) * np.float32(0.1)),
            np.float32(np.float32(0.5) + np.float32(2.5) * np.float32(0.1))]
    assert pts.shape == (1, 3) and pts[0].tolist() == [float(w) for w in want]
    assert len(mesh.occupied_points(m, p, (0.0, 0.0, 0.0), 1.0, lo=(0, 0, 0), hi=(3, 4, 3))) == 0

