"""File writers of the map exports: CSV and PCD point clouds, PLY triangle soups (host only)."""
import numpy as np
import pytest

from paper_2509_20081_amd import export


def test_point_cloud_csv_and_pcd_round_trip(tmp_path):
    rng = np.random.default_rng(2)
    pts = rng.normal(size=(37, 3)).astype(np.float32) * np.float32(12.345)
    export.write_point_cloud(str(tmp_path / "a.csv"), pts)
    back = np.loadtxt(tmp_path / "a.csv", delimiter=",", skiprows=1, dtype=np.float64).astype(np.float32)
    assert np.array_equal(back, pts)
    export.write_point_cloud(str(tmp_path / "a.pcd"), pts)
    lines = (tmp_path / "a.pcd").read_text().splitlines()
    head = {ln.split()[0]: ln.split()[1:] for ln in lines[:11] if not ln.startswith("#")}
    assert head["FIELDS"] == ["x", "y", "z"] and head["POINTS"] == ["37"] and head["DATA"] == ["ascii"]
    back = np.array([[float(v) for v in ln.split()] for ln in lines[11:]], np.float64).astype(np.float32)
    assert np.array_equal(back, pts)
    export.write_point_cloud(str(tmp_path / "empty.csv"), np.zeros((0, 3), np.float32))
    assert (tmp_path / "empty.csv").read_text() == "x,y,z\n"
    with pytest.raises(ValueError):
        export.write_point_cloud(str(tmp_path / "a.xyz"), pts)


def test_mesh_ply_round_trip(tmp_path):
    rng = np.random.default_rng(3)
    tris = rng.normal(size=(11, 3, 3)).astype(np.float32)
    export.write_mesh_ply(str(tmp_path / "m.ply"), tris)
    raw = (tmp_path / "m.ply").read_bytes()
    end = raw.index(b"end_header\n") + len(b"end_header\n")
    header = raw[:end].decode("ascii").splitlines()
    assert "element vertex 33" in header and "element face 11" in header
    verts = np.frombuffer(raw[end:end + 33 * 12], dtype="<f4").reshape(11, 3, 3)
    assert np.array_equal(verts, tris)
    faces = np.frombuffer(raw[end + 33 * 12:], dtype=[("k", "u1"), ("v", "<i4", (3,))])
    assert (faces["k"] == 3).all() and np.array_equal(faces["v"].ravel(), np.arange(33))
