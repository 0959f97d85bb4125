"""Host-side checks of the C ABI library (no GPU needed).

The library must load, export every entry point its header declares, and build
kernel tables that equal, byte for byte, the ones the oracle builds on its own
from the paper's definitions (Sec. III-B, eqs. 2-3).
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle.oracle import Oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dbtsdf.h")


@pytest.fixture(scope="module")
def db():
    import paper_2509_20081_amd as db
    from paper_2509_20081_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2509_20081_amd import build
        build.build()
    return db


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dbtsdf_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(db):
    from paper_2509_20081_amd import _lib
    names = declared_functions()
    assert len(names) >= 30
    h = C.CDLL(_lib.LIB_PATH)
    missing = [n for n in names if not hasattr(h, n)]
    assert not missing
    # and the binding declares a signature for each of them
    assert set(names) <= set(_lib.SIGNATURES)


def test_status_strings(db):
    from paper_2509_20081_amd import _lib
    lib = _lib.lib()
    for s in range(7):
        assert lib.dbtsdf_status_string(s)
    assert lib.dbtsdf_status_string(99) == b"unknown status"


def test_grid_bytes_eq1(db):
    """eq. (1): M = Nx * Ny * Nz * 8 bytes."""
    assert db.grid_bytes((1024, 1024, 256)) == 1024 * 1024 * 256 * 8
    assert db.grid_bytes((2048, 2048, 512)) == 2 ** 31 * 8


@pytest.mark.parametrize("K,binning,r2,metric", [
    (3, "cube26", 1, "l2"), (5, "cube26", 4, "l2"), (11, "cube26", 9, "l2"), (21, "cube26", 16, "l2"),
    (11, "azel", 9, "l2"), (5, "azel", 2, "l1"), (7, "cube26", -1, "l2"), (37, "cube26", 25, "l2"),
])
def test_kernel_tables_match_oracle(db, K, binning, r2, metric):
    ks = db.KernelSet(kernel_size=K, binning=binning, shadow_r2=r2, metric=metric)
    m, s, d = ks.export()
    o = Oracle(dims=(K, K, K), voxel_size=1.0, kernel_size=K, binning=binning, shadow_r2=r2, metric=metric)
    om, osh, od = o.tables()
    assert m.tobytes() == om.tobytes()
    assert s.tobytes() == osh.tobytes()
    assert np.allclose(d, od, rtol=0, atol=1e-15)


@pytest.mark.parametrize("kw", [
    dict(kernel_size=11, binning="cube26", shadow_r2=9, cone_deg=30.0),
    dict(kernel_size=11, binning="cube26", shadow_r2=9, cone_deg=45.0),
    dict(kernel_size=11, binning="cube26", shadow_r2=16, cone_deg=90.0),
    dict(kernel_size=9, binning="azel", bins_az=8, bins_el=5, shadow_r2=9, cone_deg=25.0),
    dict(kernel_size=21, binning="azel", shadow_r2=16, cone_deg=60.0),
], ids=["cube30", "cube45", "cube90", "azel25", "azel40x40_60"])
def test_cone_shadows_match_oracle(db, kw):
    """The conical shadow sets of the library equal the oracle's, boundary cases (45 degrees) included."""
    ks = db.KernelSet(shadow_model="cone", **kw)
    _, s, _ = ks.export()
    K = kw["kernel_size"]
    o = Oracle(dims=(K, K, K), voxel_size=1.0, shadow_model="cone", **kw)
    _, osh, _ = o.tables()
    assert s.tobytes() == osh.tobytes()


def test_host_bins_match_oracle(db):
    rng = np.random.default_rng(4)
    dirs = rng.normal(size=(3000, 3)).astype(np.float32)
    dirs[:50] = np.round(dirs[:50])          # axis-aligned and diagonal cases
    dirs[50:60, :2] = 0
    for binning in ("cube26", "azel"):
        ks = db.KernelSet(kernel_size=5, binning=binning)
        o = Oracle(dims=(5, 5, 5), voxel_size=1.0, kernel_size=5, binning=binning)
        for v in dirs:
            if not np.any(v):
                continue
            assert ks.bin(v) == o.bin(v)


@pytest.mark.parametrize("kw", [
    dict(kernel_size=4), dict(kernel_size=1), dict(kernel_size=39), dict(kernel_size=23, metric="l1"),
    dict(binning="azel", bins_az=41), dict(binning="azel", bins_az=0),
    dict(shadow_model="cone", cone_deg=0.0), dict(shadow_model="cone", cone_deg=91.0),
])
def test_kernel_set_validation(db, kw):
    with pytest.raises(db.DbtsdfError):
        db.KernelSet(**kw)


def test_sweep_constants_match_oracle(db):
    """The library's per-sweep deskew constants (host fp64, rounded to fp32) equal the oracle's bit for bit
    over random pose pairs, small and large turns, both modes; bad arguments are rejected."""
    import math
    from oracle import oracle as O

    def rot(axis, ang):
        a = np.asarray(axis, float)
        a /= np.linalg.norm(a)
        K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
        return np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * (K @ K)

    rng = np.random.default_rng(0)
    for i in range(1500):
        P0 = np.eye(4, dtype=np.float32)
        P0[:3, :3] = rot(rng.normal(size=3), rng.uniform(0, 3.1))
        P0[:3, 3] = rng.normal(size=3)
        P1 = np.eye(4, dtype=np.float32)
        turn = rot(rng.normal(size=3), rng.uniform(0, 0.2) if i % 2 else rng.uniform(0, 3.14))
        P1[:3, :3] = turn @ P0[:3, :3]
        P1[:3, 3] = rng.normal(size=3)
        for mode in ("se3", "yaw"):
            a, b = db.deskew_constants(P0, P1, mode), O.deskew_constants(P0, P1, mode)
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), (i, mode)
    bad = np.eye(4, dtype=np.float32)
    bad[0, 0] = np.nan
    with pytest.raises(db.DbtsdfError):
        db.deskew_constants(bad, np.eye(4))
    with pytest.raises(KeyError):
        db.deskew_constants(np.eye(4), np.eye(4), "roll")


def test_missing_library_fails_loudly(tmp_path):
    """With the HIP library absent every entry point raises: there is no CPU fallback (checked in a child
    process whose binding points at an empty directory)."""
    import subprocess
    import sys
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "from paper_2509_20081_amd import _lib\n"
        "_lib.LIB_PATH = %r\n"
        "import paper_2509_20081_amd as db\n"
        "try:\n"
        "    db.KernelSet(kernel_size=5)\n"
        "except RuntimeError as e:\n"
        "    assert 'is not built' in str(e), e\n"
        "    print('raised')\n"
    ) % (os.path.dirname(os.path.dirname(os.path.abspath(__file__))), str(tmp_path / "libdbtsdf.so"))
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.strip() == "raised", (out.stdout, out.stderr)


def test_checkpoint_refuses_planes_that_do_not_fit_the_header(db, tmp_path):
    """A checkpoint whose planes do not have the header's (Nz, Ny, Nx) uint32 shape is refused before any
    grid is made (a short plane would otherwise be read past its end by the library)."""
    import json

    from paper_2509_20081_amd.checkpoint import FORMAT, load_checkpoint
    header = dict(format=FORMAT, dims=[8, 6, 4], voxel_size=0.1, origin=[0.0, 0.0, 0.0], hit_threshold=5,
                  hit_max=65535, dedup=True, kernel=dict(kernel_size=3, binning="cube26", shadow_r2=1))
    good = np.full((4, 6, 8), 0xFFFFFFFF, np.uint32)
    cases = {"short": (good[:, :, :7], good), "transposed": (good, good.transpose(2, 1, 0).copy()),
             "wrong dtype": (good.astype(np.int64), good)}
    for what, (m, p) in cases.items():
        path = str(tmp_path / f"{what.replace(' ', '_')}.npz")
        with open(path, "wb") as f:
            np.savez(f, header=np.array(json.dumps(header)), mask=m, packed=p)
        with pytest.raises(ValueError):
            load_checkpoint(path)
    bad = dict(header, dims=[8, 6])
    path = str(tmp_path / "bad_dims.npz")
    with open(path, "wb") as f:
        np.savez(f, header=np.array(json.dumps(bad)), mask=good, packed=good)
    with pytest.raises(ValueError):
        load_checkpoint(path)
