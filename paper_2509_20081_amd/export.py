"""File writers for the map exports (the last block of the paper's pipeline figure, Sec. III).

The device kernels produce the data (``Grid.extract_mesh``, ``Grid.extract_points``);
these functions only format it for files:

* point clouds as CSV (``x,y,z`` header) or ASCII PCD v0.7 (the PCL format);
* triangle meshes as binary little-endian PLY, three vertices per face
  (a triangle soup, counter-clockwise about the outward normal).

Floats are written with nine significant digits, enough to round-trip fp32.
"""
from __future__ import annotations

import os

import numpy as np


def _host(a, shape_tail) -> np.ndarray:
    if hasattr(a, "detach"):
        a = a.detach().cpu().numpy()
    a = np.ascontiguousarray(a, dtype=np.float32)
    if a.shape[1:] != shape_tail:
        raise ValueError(f"expected shape (n, {', '.join(map(str, shape_tail))}), got {a.shape}")
    return a


def write_point_cloud(path: str, xyz, fmt: str | None = None) -> None:
    """Write (n, 3) points as CSV or PCD (fmt from the file extension when None)."""
    pts = _host(xyz, (3,))
    fmt = (fmt or os.path.splitext(path)[1].lstrip(".")).lower()
    sep = "," if fmt == "csv" else " "
    rows = "\n".join(f"{x:.9g}{sep}{y:.9g}{sep}{z:.9g}" for x, y, z in pts.tolist())
    with open(path, "w") as f:
        if fmt == "csv":
            f.write("x,y,z\n")
        elif fmt == "pcd":
            n = len(pts)
            f.write("# .PCD v0.7 - Point Cloud Data file format\nVERSION 0.7\nFIELDS x y z\nSIZE 4 4 4\n"
                    "TYPE F F F\nCOUNT 1 1 1\n"
                    f"WIDTH {n}\nHEIGHT 1\nVIEWPOINT 0 0 0 1 0 0 0\nPOINTS {n}\nDATA ascii\n")
        else:
            raise ValueError(f"unknown point cloud format {fmt!r} (csv or pcd)")
        if rows:
            f.write(rows + "\n")


def write_mesh_ply(path: str, tris) -> None:
    """Write (n, 3, 3) triangles as a binary PLY triangle soup (3 n vertices, n faces)."""
    t = _host(tris, (3, 3))
    n = len(t)
    header = ("ply\nformat binary_little_endian 1.0\n"
              f"element vertex {3 * n}\nproperty float x\nproperty float y\nproperty float z\n"
              f"element face {n}\nproperty list uchar int vertex_indices\nend_header\n").encode("ascii")
    faces = np.zeros(n, dtype=[("k", "u1"), ("v", "<i4", (3,))])
    faces["k"] = 3
    faces["v"] = np.arange(3 * n, dtype=np.int32).reshape(n, 3)
    with open(path, "wb") as f:
        f.write(header)
        f.write(t.reshape(-1, 3).astype("<f4").tobytes())
        f.write(faces.tobytes())
