"""The allocation-free entry point (dbtsdf_integrate_scan_noalloc) against dbtsdf_integrate_scan.

Two calls in a row on one grid, the second with fewer points, called through
the C ABI; after each call both planes and the statistics must equal those of
the plain entry point on a second grid fed the same scans.
"""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2509_20081_amd as db  # noqa: E402
from paper_2509_20081_amd import _lib as L  # noqa: E402
from synth import scene as synth  # noqa: E402

pytestmark = pytest.mark.gpu

FIELDS = ("n_in", "n_invalid", "n_out_of_bounds", "n_duplicate", "n_integrated", "voxel_updates",
          "shadow_updates", "n_revisit")


def _noalloc(grid, pose, pts):
    pose = np.ascontiguousarray(pose, dtype=np.float32).reshape(16)
    st = L.ScanStats()
    rc = L.lib().dbtsdf_integrate_scan_noalloc(grid._h, pose.ctypes.data_as(C.c_void_p), C.c_void_p(pts.data_ptr()),
                                               int(pts.shape[0]), C.byref(st))
    L.check(rc, "integrate_scan_noalloc")
    return st.as_dict()


def _planes(g):
    return g.mask_tensor.cpu().numpy().view(np.uint32), g.packed_tensor.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("kernel", ["cube26", "azel"])
def test_noalloc_equals_plain_on_two_calls(kernel):
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    kp = dict(kernel_size=11, binning="cube26", shadow_r2=9) if kernel == "cube26" else \
        dict(kernel_size=9, binning="azel", bins_az=16, bins_el=8, shadow_r2=9)
    ks = db.KernelSet(**kp)
    dims, vs = (384, 384, 128), 0.1
    origin = (-19.2, -19.2, -1.4)
    scans = list(synth.config_scans(2, 0, [0, 1]))
    # the second call is smaller than the first
    inputs = [(scans[0][0], scans[0][1]), (scans[1][0], scans[1][1][:20000])]
    print(f"[noalloc] kernel={kernel} dims={dims} n={[len(p) for _, p in inputs]}", flush=True)
    a = db.Grid(dims, vs, origin, ks, planes="torch")
    b = db.Grid(dims, vs, origin, ks, planes="torch")
    b.set_tuning(strategy="atomic")
    for k, (pose, pts) in enumerate(inputs):
        dev = torch.from_numpy(np.ascontiguousarray(pts)).cuda()
        got = _noalloc(a, pose, dev)
        st = b.integrate(pose, dev)
        b.sync()
        want = st.as_dict()
        assert want["n_integrated"] > 1000
        for f in FIELDS:
            assert got[f] == want[f], (k, f, got[f], want[f])
        am, ap = _planes(a)
        bm, bp = _planes(b)
        assert np.array_equal(am, bm), f"call {k}: mask plane differs"
        assert np.array_equal(ap, bp), f"call {k}: packed plane differs"
    a.close()
    b.close()


def test_noalloc_refuses_more_than_its_maximum():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    ks = db.KernelSet(kernel_size=11, binning="cube26", shadow_r2=9)
    g = db.Grid((64, 64, 64), 0.1, (0.0, 0.0, 0.0), ks, planes="torch")
    cap = 131072
    big = torch.zeros((cap + 1, 3), dtype=torch.float32, device="cuda")
    pose = np.eye(4, dtype=np.float32)
    with pytest.raises(db.DbtsdfError):
        _noalloc(g, pose, big)
    # the grid is untouched and still usable
    m, p = _planes(g)
    assert (m == 0xFFFFFFFF).all() and (p == 0x80000000).all()
    st = _noalloc(g, pose, big[:10])
    assert st["n_in"] == 10 and st["n_invalid"] == 10   # zero-range returns
    g.close()
