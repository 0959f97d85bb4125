"""ctypes front of the plain C oracle (test infrastructure only).

Grids are numpy ``uint32`` arrays of shape ``(Nz, Ny, Nx)`` (x fastest): the
distance-mask plane and the packed plane (hit counter in bits 0-15, sign in
bit 31, 1 = free). The oracle follows Section III of the paper; see
``dbtsdf_oracle.c`` for the step-by-step statement and the readings it takes.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

BINNING = {"azel": 0, "cube26": 1}
METRIC = {"l2": 0, "l1": 1}
SHADOW = {"hemisphere": 0, "cone": 1}
DESKEW = {"se3": 0, "yaw": 1}


class _Params(C.Structure):
    _fields_ = [
        ("kernel_size", C.c_uint32), ("binning", C.c_uint32), ("bins_az", C.c_uint32),
        ("bins_el", C.c_uint32), ("shadow_r2", C.c_int32), ("metric", C.c_uint32),
        ("dims", C.c_uint32 * 3), ("voxel_size", C.c_float), ("origin", C.c_float * 3),
        ("hit_threshold", C.c_uint32), ("hit_max", C.c_uint32), ("dedup", C.c_uint32),
        ("shadow_model", C.c_uint32), ("cone_deg", C.c_float),
    ]


class _Stats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in (
        "n_in", "n_invalid", "n_out_of_bounds", "n_duplicate", "n_integrated",
        "voxel_updates", "shadow_updates", "u_mask", "c_mask", "u_shadow")]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        lib = C.CDLL(_LIB_PATH)
        lib.orc_create.restype = C.c_void_p
        lib.orc_create.argtypes = [C.POINTER(_Params)]
        lib.orc_destroy.argtypes = [C.c_void_p]
        lib.orc_n_bins.restype = C.c_uint32
        lib.orc_n_bins.argtypes = [C.c_void_p]
        lib.orc_export.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        lib.orc_bin.restype = C.c_int
        lib.orc_bin.argtypes = [C.c_void_p, C.c_float, C.c_float, C.c_float]
        lib.orc_grid_init.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        lib.orc_front_end.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64,
                                      C.c_void_p, C.c_void_p, C.c_void_p]
        lib.orc_integrate_omp.restype = C.c_int
        lib.orc_integrate_omp.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                          C.c_uint64, C.c_void_p, C.c_void_p]
        lib.orc_integrate.restype = C.c_int
        lib.orc_integrate.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_uint64, C.POINTER(_Stats), C.c_int]
        lib.orc_read_distance.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        lib.orc_deskew_constants.restype = C.c_int
        lib.orc_deskew_constants.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]
        lib.orc_deskew_pose.argtypes = [C.c_void_p, C.c_void_p, C.c_float, C.c_void_p]
        lib.orc_integrate_deskew.restype = C.c_int
        lib.orc_integrate_deskew.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int,
                                             C.c_void_p, C.c_void_p, C.c_uint64, C.POINTER(_Stats), C.c_int]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class Oracle:
    """One grid configuration plus its kernel tables, built from the paper's definitions."""

    def __init__(self, dims, voxel_size, origin=(0.0, 0.0, 0.0), kernel_size=11, binning="cube26",
                 bins_az=40, bins_el=40, shadow_r2=9, metric="l2", hit_threshold=5,
                 hit_max=65535, dedup=True, shadow_model="hemisphere", cone_deg=90.0):
        lib = _load()
        p = _Params()
        p.kernel_size = kernel_size
        p.binning = BINNING[binning]
        p.bins_az = bins_az
        p.bins_el = bins_el
        p.shadow_r2 = shadow_r2
        p.metric = METRIC[metric]
        p.dims[:] = [int(d) for d in dims]
        p.voxel_size = voxel_size
        p.origin[:] = [float(o) for o in origin]
        p.hit_threshold = hit_threshold
        p.hit_max = hit_max
        p.dedup = 1 if dedup else 0
        p.shadow_model = SHADOW[shadow_model]
        p.cone_deg = cone_deg
        self._p = p
        self._ctx = lib.orc_create(C.byref(p))
        if not self._ctx:
            raise ValueError("oracle: invalid parameters")
        self.dims = tuple(int(d) for d in dims)
        self.K = kernel_size
        self.R = (kernel_size - 1) // 2
        self.n_bins = int(lib.orc_n_bins(self._ctx))
        self.hit_threshold = hit_threshold
        self.hit_max = hit_max
        self.binning = binning

    def __del__(self):
        ctx = getattr(self, "_ctx", None)
        if ctx and _lib is not None:
            _lib.orc_destroy(ctx)
            self._ctx = None

    # -- tables --------------------------------------------------------------
    def tables(self):
        """(masks[K,K,K] indexed [dz+R, dy+R, dx+R], shadow[n_bins,K,K,K] u8, dirs[n_bins,3] f64)."""
        K = self.K
        masks = np.zeros((K, K, K), dtype=np.uint32)
        shadow = np.zeros((self.n_bins, K, K, K), dtype=np.uint8)
        dirs = np.zeros((self.n_bins, 3), dtype=np.float64)
        _lib.orc_export(self._ctx, _ptr(masks), _ptr(shadow), _ptr(dirs))
        return masks, shadow, dirs

    def bin(self, d) -> int:
        d = np.asarray(d, dtype=np.float32)
        return int(_lib.orc_bin(self._ctx, C.c_float(d[0]), C.c_float(d[1]), C.c_float(d[2])))

    # -- grid ----------------------------------------------------------------
    def new_grid(self):
        nx, ny, nz = self.dims
        mask = np.empty((nz, ny, nx), dtype=np.uint32)
        packed = np.empty((nz, ny, nx), dtype=np.uint32)
        _lib.orc_grid_init(self._ctx, _ptr(mask), _ptr(packed))
        return mask, packed

    def front_end(self, pose, pts):
        """Per point: voxel (int32[N,3], x y z), bin (int32[N], -1 unless ok), status (0 ok, 1 invalid, 2 out of bounds)."""
        pose = np.ascontiguousarray(pose, dtype=np.float32).reshape(16)
        pts = np.ascontiguousarray(pts, dtype=np.float32).reshape(-1, 3)
        n = pts.shape[0]
        vox = np.zeros((n, 3), dtype=np.int32)
        bins = np.zeros(n, dtype=np.int32)
        status = np.zeros(n, dtype=np.int32)
        _lib.orc_front_end(self._ctx, _ptr(pose), _ptr(pts), n, _ptr(vox), _ptr(bins), _ptr(status))
        return vox, bins, status

    def integrate(self, mask, packed, pose, pts, count_traffic=False) -> dict:
        assert mask.dtype == np.uint32 and packed.dtype == np.uint32
        assert mask.flags.c_contiguous and packed.flags.c_contiguous
        assert mask.size == packed.size == self.dims[0] * self.dims[1] * self.dims[2]
        pose = np.ascontiguousarray(pose, dtype=np.float32).reshape(16)
        pts = np.ascontiguousarray(pts, dtype=np.float32).reshape(-1, 3)
        st = _Stats()
        rc = _lib.orc_integrate(self._ctx, _ptr(mask), _ptr(packed), _ptr(pose), _ptr(pts),
                                pts.shape[0], C.byref(st), 1 if count_traffic else 0)
        if rc != 0:
            raise ValueError("oracle: non-finite pose")
        return {n: int(getattr(st, n)) for n, _ in _Stats._fields_}

    def integrate_parallel(self, mask, packed, pose, pts):
        """``integrate`` on every host core (OpenMP; the all-core CPU timing leg): the same planes bit for
        bit, statistics without the traffic counts. Returns (statistics, threads used)."""
        assert mask.dtype == np.uint32 and packed.dtype == np.uint32
        assert mask.flags.c_contiguous and packed.flags.c_contiguous
        assert mask.size == packed.size == self.dims[0] * self.dims[1] * self.dims[2]
        pose = np.ascontiguousarray(pose, dtype=np.float32).reshape(16)
        pts = np.ascontiguousarray(pts, dtype=np.float32).reshape(-1, 3)
        st = _Stats()
        thr = C.c_int(0)
        rc = _lib.orc_integrate_omp(self._ctx, _ptr(mask), _ptr(packed), _ptr(pose), _ptr(pts), pts.shape[0],
                                    C.byref(st), C.byref(thr))
        if rc == 1:
            raise ValueError("oracle: non-finite pose")
        if rc != 0:
            raise RuntimeError(f"oracle: parallel integration unavailable (code {rc})")
        return {n: int(getattr(st, n)) for n, _ in _Stats._fields_}, int(thr.value)

    def integrate_deskew(self, mask, packed, pose_start, pose_end, pts, times, mode="se3",
                         count_traffic=False) -> dict:
        """One motion-compensated sweep: return i is placed with the pose at time fraction times[i]
        between pose_start and pose_end (see ``deskew_constants``)."""
        assert mask.dtype == np.uint32 and packed.dtype == np.uint32
        assert mask.flags.c_contiguous and packed.flags.c_contiguous
        p0 = np.ascontiguousarray(pose_start, dtype=np.float32).reshape(16)
        p1 = np.ascontiguousarray(pose_end, dtype=np.float32).reshape(16)
        pts = np.ascontiguousarray(pts, dtype=np.float32).reshape(-1, 3)
        times = np.ascontiguousarray(times, dtype=np.float32).reshape(-1)
        assert times.shape[0] == pts.shape[0]
        st = _Stats()
        rc = _lib.orc_integrate_deskew(self._ctx, _ptr(mask), _ptr(packed), _ptr(p0), _ptr(p1), DESKEW[mode],
                                       _ptr(times), _ptr(pts), pts.shape[0], C.byref(st), 1 if count_traffic else 0)
        if rc != 0:
            raise ValueError("oracle: non-finite pose")
        return {n: int(getattr(st, n)) for n, _ in _Stats._fields_}

    def read_distance(self, mask, packed):
        out = np.empty(mask.shape, dtype=np.int8)
        _lib.orc_read_distance(self._ctx, _ptr(np.ascontiguousarray(mask)),
                               _ptr(np.ascontiguousarray(packed)), _ptr(out))
        return out


def deskew_constants(pose_start, pose_end, mode="se3") -> np.ndarray:
    """The sweep's fp32 constants: q (w, x, y, z) of the rotation over the sweep (or its yaw), then t1 - t0."""
    lib = _load()
    p0 = np.ascontiguousarray(pose_start, dtype=np.float32).reshape(16)
    p1 = np.ascontiguousarray(pose_end, dtype=np.float32).reshape(16)
    out = np.zeros(7, np.float32)
    if lib.orc_deskew_constants(_ptr(p0), _ptr(p1), DESKEW[mode], _ptr(out)) != 0:
        raise ValueError("oracle: non-finite pose or unknown mode")
    return out


def deskew_pose(pose_start, constants, tau) -> np.ndarray:
    """The 4 x 4 fp32 pose of a return at time fraction tau."""
    lib = _load()
    p0 = np.ascontiguousarray(pose_start, dtype=np.float32).reshape(16)
    k = np.ascontiguousarray(constants, dtype=np.float32).reshape(7)
    out = np.zeros(16, np.float32)
    lib.orc_deskew_pose(_ptr(p0), _ptr(k), C.c_float(tau), _ptr(out))
    return out.reshape(4, 4)
