"""DB-TSDF scan integration on MI355X (gfx950): Python binding of ``libdbtsdf.so``.

Thin marshalling over the C ABI declared in ``include/dbtsdf.h``; every step of
the integration runs in the library's HIP kernels. PyTorch is used only for
device memory (point clouds, optional grid planes) and for the stream handle.
If the library has not been built, every entry point raises: there is no CPU
fallback.

Example::

    import paper_2509_20081_amd as db
    ks = db.KernelSet(kernel_size=11, binning="cube26", shadow_r2=9)
    g = db.Grid((1024, 1024, 256), 0.05, origin, ks)
    st = g.integrate(pose_4x4, points_cuda_Nx3)   # async
    g.sync(); print(st.as_dict())
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L
from ._lib import DbtsdfError  # noqa: F401

__all__ = ["KernelSet", "Grid", "Batch", "Server", "DbtsdfError", "now_ns", "library_path", "nearest_sq",
           "surface_metrics", "mesh_vertices", "mesh_centroids"]

_BINNING = {"azel": L.BIN_AZEL, "cube26": L.BIN_CUBE26}
_METRIC = {"l2": L.DIST_L2, "l1": L.DIST_L1}
_SHADOW = {"hemisphere": 0, "cone": 1}
_STRATEGY = {"auto": L.STRATEGY_AUTO, "brick": L.STRATEGY_BRICK, "atomic": L.STRATEGY_ATOMIC,
             "sort": L.STRATEGY_SORT, "tile": L.STRATEGY_TILE}
_STRATEGY_NAME = {v: k for k, v in _STRATEGY.items()}


def library_path() -> str:
    return L.LIB_PATH


def now_ns() -> int:
    return int(L.lib().dbtsdf_now_ns())


def _f32(a, shape=None) -> np.ndarray:
    out = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    if shape is not None:
        out = out.reshape(shape)
    return out


def _current_stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _points_arg(points):
    """(pointer, n, on_device, keepalive) for a torch CUDA tensor or host array of N x 3 fp32."""
    try:
        import torch
    except ImportError:  # pragma: no cover
        torch = None
    if torch is not None and isinstance(points, torch.Tensor):
        if points.dtype != torch.float32 or points.dim() != 2 or points.shape[1] != 3:
            raise ValueError("points must be an (N, 3) float32 tensor")
        if not points.is_contiguous():
            points = points.contiguous()
        if points.is_cuda:
            return C.c_void_p(points.data_ptr()), int(points.shape[0]), 1, points
        points = points.numpy()
    arr = _f32(points)
    if arr.ndim != 2 or arr.shape[1] != 3:
        raise ValueError("points must be (N, 3)")
    return arr.ctypes.data_as(C.c_void_p), int(arr.shape[0]), 0, arr


def _times_arg(times, n, on_device):
    """(pointer, keepalive) for n fp32 time fractions on the same side as the points."""
    try:
        import torch
    except ImportError:  # pragma: no cover
        torch = None
    if torch is not None and isinstance(times, torch.Tensor):
        if times.dtype != torch.float32 or times.numel() != n:
            raise ValueError("times must hold one float32 per point")
        times = times.contiguous().reshape(-1)
        if bool(times.is_cuda) != bool(on_device):
            raise ValueError("times must be where the points are")
        if times.is_cuda:
            return C.c_void_p(times.data_ptr()), times
        times = times.numpy()
    if on_device:
        raise ValueError("times must be where the points are")
    arr = _f32(times).reshape(-1)
    if arr.shape[0] != n:
        raise ValueError("times must hold one float32 per point")
    return arr.ctypes.data_as(C.c_void_p), arr


DESKEW = {"se3": 0, "yaw": 1}


def deskew_constants(pose_start, pose_end, mode="se3"):
    """The sweep's fp32 constants the library uses: quaternion (w, x, y, z) of the rotation over the sweep
    (or of its yaw), then the end translation minus the start translation."""
    out = np.zeros(7, np.float32)
    p0, p1 = _f32(pose_start, (16,)), _f32(pose_end, (16,))
    L.check(L.lib().dbtsdf_deskew_constants(p0.ctypes.data_as(C.c_void_p), p1.ctypes.data_as(C.c_void_p),
                                            DESKEW[mode], out.ctypes.data_as(C.c_void_p)), "deskew_constants")
    return out


def _cloud_arg(pts, name):
    import torch
    if not isinstance(pts, torch.Tensor) or not pts.is_cuda or pts.dtype != torch.float32 or pts.dim() != 2 \
            or pts.shape[1] != 3 or not pts.is_contiguous():
        raise ValueError(f"{name} must be a contiguous (n, 3) float32 CUDA tensor")
    return C.c_void_p(pts.data_ptr() if pts.shape[0] else 0), int(pts.shape[0])


def nearest_sq(query, ref):
    """Per query point, the smallest squared distance (fp64, exact) to the reference points: a float64
    CUDA tensor of shape (n_query,)."""
    import torch
    q, nq = _cloud_arg(query, "query")
    r, nr = _cloud_arg(ref, "ref")
    out = torch.empty(nq, dtype=torch.float64, device=query.device)
    torch.cuda.synchronize(query.device)   # the library runs on the device's null stream
    L.check(L.lib().dbtsdf_nearest_sq(query.device.index or 0, q, nq, r, nr,
                                      C.c_void_p(out.data_ptr() if nq else 0)), "nearest_sq")
    return out


def surface_metrics(pred, gt, tolerance: float) -> dict:
    """Accuracy, completeness, Chamfer-L1 (metres), precision, recall and F-score at `tolerance` of the
    predicted points `pred` against the ground truth `gt` (both (n, 3) float32 CUDA tensors)."""
    import torch
    p, n_p = _cloud_arg(pred, "pred")
    g, n_g = _cloud_arg(gt, "gt")
    m = L.Metrics()
    torch.cuda.synchronize(pred.device)
    L.check(L.lib().dbtsdf_surface_metrics(pred.device.index or 0, p, n_p, g, n_g, float(tolerance), C.byref(m)),
            "surface_metrics")
    return {"accuracy": m.accuracy, "completeness": m.completeness, "chamfer_l1": m.chamfer_l1,
            "precision": m.precision, "recall": m.recall, "fscore": m.fscore, "n_pred": int(m.n_pred),
            "n_gt": int(m.n_gt), "n_pred_within": int(m.n_pred_within), "n_gt_within": int(m.n_gt_within),
            "tolerance": float(tolerance)}


def mesh_centroids(tris):
    """The predicted point set the benchmark scores: one point per triangle of a mesh from
    Grid.extract_mesh, its centroid: the three fp32 vertices summed in fp64 (exact for coordinates of
    like magnitude, so the vertex order does not matter), divided by 3 and rounded to fp32 (a (n, 3)
    float32 CUDA tensor)."""
    import torch
    t = tris.reshape(-1, 3, 3).to(torch.float64)
    return ((t[:, 0] + t[:, 1] + t[:, 2]) / 3.0).to(torch.float32).contiguous()


def mesh_vertices(tris):
    """The predicted point set of the accuracy metrics: the three vertices of every triangle of a mesh
    from Grid.extract_mesh (a (n, 9) float32 CUDA tensor), as an (3 n, 3) view."""
    return tris.reshape(-1, 3)


def integrate_batch(items) -> list:
    """items: [(grid, pose, cuda points)] in one launch sequence on the library's own batch context of the
    grids' device; returns the filled Stats (the call waits for the batch)."""
    n = len(items)
    if n == 0:
        return []
    grids = (C.c_void_p * n)(*[g._h for g, _, _ in items])
    poses = np.stack([_f32(p, (16,)) for _, p, _ in items]).astype(np.float32)
    args = [_points_arg(pts) for _, _, pts in items]
    if any(a[2] != 1 for a in args):
        raise ValueError("integrate_batch takes device points")
    ptrs = (C.c_void_p * n)(*[a[0] for a in args])
    counts = (C.c_uint64 * n)(*[a[1] for a in args])
    stats = (L.ScanStats * n)()
    L.check(L.lib().dbtsdf_integrate_batch(n, grids, poses.ctypes.data_as(C.c_void_p), ptrs, counts, stats),
            "integrate_batch")
    out = []
    for i in range(n):
        s = Stats()
        s._c = stats[i]
        out.append(s)
    return out


def _period(enable, every) -> int:
    if not enable:
        return 0
    if int(every) < 1:
        raise ValueError("every must be >= 1")
    return int(every)


def _read_profile(fn, h) -> dict:
    cm, am = C.c_double(), C.c_double()
    cn, an = C.c_uint64(), C.c_uint64()
    L.check(fn(h, C.byref(cm), C.byref(cn), C.byref(am), C.byref(an)), "read_profile")
    return dict(call_ms=cm.value, calls=int(cn.value), apply_ms=am.value, applies=int(an.value))


class Stats:
    """Statistics of one scan; filled when the owning grid / batch is synchronised."""

    def __init__(self):
        self._c = L.ScanStats()

    def as_dict(self) -> dict:
        return self._c.as_dict()

    def __getattr__(self, name):
        if name in L.STAT_FIELDS:
            return int(getattr(self._c, name))
        raise AttributeError(name)

    def __repr__(self):
        return f"Stats({self.as_dict()})"


class KernelSet:
    """Directional kernels (Sec. III-B): eq. 3 masks, per-bin hemispherical shadows."""

    def __init__(self, kernel_size: int = 11, binning: str = "cube26", bins_az: int = 40, bins_el: int = 40,
                 shadow_r2: int = 9, metric: str = "l2", shadow_model: str = "hemisphere", cone_deg: float = 90.0):
        p = L.KernelParams(kernel_size, _BINNING[binning], bins_az, bins_el, shadow_r2, _METRIC[metric],
                           _SHADOW[shadow_model], cone_deg)
        h = C.c_void_p()
        self._lib = L.lib()  # held so that destruction at interpreter exit still finds it
        L.check(self._lib.dbtsdf_kernel_set_create(C.byref(p), C.byref(h)), "kernel_set_create")
        self._h = h
        self.kernel_size = kernel_size
        self.binning = binning
        self.params = dict(kernel_size=int(kernel_size), binning=binning, bins_az=int(bins_az), bins_el=int(bins_el),
                           shadow_r2=int(shadow_r2), metric=metric, shadow_model=shadow_model,
                           cone_deg=float(cone_deg))
        self.n_bins = int(L.lib().dbtsdf_kernel_set_n_bins(h))

    def export(self):
        """(masks[K,K,K] uint32 [dz,dy,dx], shadow[n_bins,K,K,K] uint8, dirs[n_bins,3] float64)."""
        K = self.kernel_size
        masks = np.zeros((K, K, K), np.uint32)
        shadow = np.zeros((self.n_bins, K, K, K), np.uint8)
        dirs = np.zeros((self.n_bins, 3), np.float64)
        nb = C.c_uint32()
        L.check(L.lib().dbtsdf_kernel_set_export(self._h, masks.ctypes.data_as(C.c_void_p),
                                                 shadow.ctypes.data_as(C.c_void_p),
                                                 dirs.ctypes.data_as(C.c_void_p), C.byref(nb)), "kernel_set_export")
        return masks, shadow, dirs

    def bin(self, d) -> int:
        d = _f32(d, (3,))
        return int(L.lib().dbtsdf_kernel_set_bin(self._h, C.c_float(d[0]), C.c_float(d[1]), C.c_float(d[2])))

    def __del__(self):
        h, lib = getattr(self, "_h", None), getattr(self, "_lib", None)
        if h and lib is not None:
            lib.dbtsdf_kernel_set_destroy(h)
            self._h = None


def grid_params(dims, voxel_size, origin=(0.0, 0.0, 0.0), hit_threshold=5, hit_max=65535, dedup=True,
                count_traffic=False) -> L.GridParams:
    p = L.GridParams()
    p.dims[:] = [int(d) for d in dims]
    p.voxel_size = float(voxel_size)
    p.origin[:] = [float(o) for o in origin]
    p.hit_threshold = hit_threshold
    p.hit_max = hit_max
    p.flags = (L.DEDUP_FIRST if dedup else 0) | (L.COUNT_TRAFFIC if count_traffic else 0)
    return p


def grid_bytes(dims) -> int:
    p = grid_params(dims, 1.0)
    return int(L.lib().dbtsdf_grid_bytes(C.byref(p)))


class Grid:
    """A dense DB-TSDF voxel grid resident in GPU memory (Sec. III-A).

    ``planes="torch"`` puts the two planes in torch-owned int32 tensors of shape
    (Nz, Ny, Nx) (``mask_tensor``, ``packed_tensor``; reinterpret as uint32);
    otherwise the library owns them. ``stream`` is a raw hipStream_t value; by
    default torch's current stream.
    """

    def __init__(self, dims, voxel_size, origin, kernel_set: KernelSet, hit_threshold=5, hit_max=65535,
                 dedup=True, count_traffic=False, planes=None, stream=None, _handle=None):
        self.dims = tuple(int(d) for d in dims)
        self.kernel_set = kernel_set
        self.params = grid_params(dims, voxel_size, origin, hit_threshold, hit_max, dedup, count_traffic)
        self._keep = []
        self._pending = []
        self.mask_tensor = self.packed_tensor = None
        self._owned = _handle is None
        self._lib = L.lib()
        if _handle is not None:
            self._h = _handle
            return
        h = C.c_void_p()
        st = _current_stream() if stream is None else C.c_void_p(stream)
        if planes == "torch":
            import torch
            nx, ny, nz = self.dims
            self.mask_tensor = torch.empty((nz, ny, nx), dtype=torch.int32, device="cuda")
            self.packed_tensor = torch.empty((nz, ny, nx), dtype=torch.int32, device="cuda")
            rc = L.lib().dbtsdf_create_grid_on(C.byref(self.params), kernel_set._h, st,
                                               C.c_void_p(self.mask_tensor.data_ptr()),
                                               C.c_void_p(self.packed_tensor.data_ptr()), C.byref(h))
        else:
            rc = L.lib().dbtsdf_create_grid(C.byref(self.params), kernel_set._h, st, C.byref(h))
        L.check(rc, "create_grid")
        self._h = h

    # -- integration --------------------------------------------------------
    def integrate(self, pose, points, every: int = 1, pose_end=None, times=None, deskew="se3") -> Stats:
        """Enqueue one scan (every > 1: only every `every`-th return, in order, the paper's sequential
        downsampling); the returned Stats are filled at the next sync(). With pose_end and times (one time
        fraction in [0, 1] per point, beside the points) the scan is a sweep from pose to pose_end,
        motion-compensated ("se3" or "yaw")."""
        pose = _f32(pose, (16,))
        ptr, n, on_dev, keep = _points_arg(points)
        st = Stats()
        if pose_end is not None:
            if times is None:
                raise ValueError("a deskewed sweep needs times")
            p1 = _f32(pose_end, (16,))
            tptr, tkeep = _times_arg(times, n, on_dev)
            rc = L.lib().dbtsdf_integrate_scan_deskew(self._h, pose.ctypes.data_as(C.c_void_p),
                                                      p1.ctypes.data_as(C.c_void_p), ptr, tptr, n, int(every),
                                                      DESKEW[deskew], on_dev, C.byref(st._c))
            L.check(rc, "integrate_scan_deskew")
            self._pending.append((st, (keep, tkeep) if on_dev else None))
            return st
        if every == 1:
            rc = L.lib().dbtsdf_integrate_scan(self._h, pose.ctypes.data_as(C.c_void_p), ptr, n, on_dev,
                                               C.byref(st._c))
        else:
            rc = L.lib().dbtsdf_integrate_scan_every(self._h, pose.ctypes.data_as(C.c_void_p), ptr, n, int(every),
                                                     on_dev, C.byref(st._c))
        L.check(rc, "integrate_scan")
        self._pending.append((st, keep if on_dev else None))
        return st

    def sync(self) -> None:
        L.check(L.lib().dbtsdf_sync(self._h), "sync")
        self._pending.clear()

    def reset(self) -> None:
        L.check(L.lib().dbtsdf_reset_grid(self._h), "reset_grid")

    # -- device timing ----------------------------------------------------------
    def set_profiling(self, enable=True, every: int = 1) -> None:
        """Time every `every`-th integrate call with HIP events (off when `enable` is false)."""
        L.check(L.lib().dbtsdf_set_profiling(self._h, _period(enable, every)), "set_profiling")

    def read_profile(self) -> dict:
        return _read_profile(L.lib().dbtsdf_read_profile, self._h)

    # -- tuning -----------------------------------------------------------------
    @property
    def tuning(self) -> dict:
        t = L.Tuning()
        L.check(L.lib().dbtsdf_get_tuning(self._h, C.byref(t)), "get_tuning")
        return dict(strategy=_STRATEGY_NAME[t.strategy], brick=tuple(t.brick), block_threads=t.block_threads,
                    apply_blocks=t.apply_blocks, chunk=t.chunk)

    def set_tuning(self, strategy="brick", brick=(32, 16, 8), block_threads=256, apply_blocks=0, chunk=0) -> None:
        t = L.Tuning(_STRATEGY[strategy], (C.c_uint32 * 3)(*brick), block_threads, apply_blocks,
                     0xFFFFFFFF if chunk is None else chunk)
        L.check(L.lib().dbtsdf_set_tuning(self._h, C.byref(t)), "set_tuning")

    def autotune(self, scans, device_points) -> dict:
        """Time candidate tunings on a scratch copy with ``scans`` [(pose, cuda points)], keep the fastest."""
        n = len(scans)
        poses = np.stack([_f32(p, (16,)) for p, _ in scans]).astype(np.float32)
        ptrs = (C.c_void_p * n)(*[C.c_void_p(pts.data_ptr()) for _, pts in scans])
        counts = (C.c_uint64 * n)(*[int(pts.shape[0]) for _, pts in scans])
        best = L.Tuning()
        L.check(L.lib().dbtsdf_autotune(self._h, n, poses.ctypes.data_as(C.c_void_p), ptrs, counts,
                                        C.byref(best)), "autotune")
        return self.tuning

    # -- readout ----------------------------------------------------------------
    def _box(self, lo, hi):
        lo = (0, 0, 0) if lo is None else lo
        hi = self.dims if hi is None else hi
        lo_a = (C.c_uint32 * 3)(*[int(v) for v in lo])
        hi_a = (C.c_uint32 * 3)(*[int(v) for v in hi])
        shape = (int(hi[2]) - int(lo[2]), int(hi[1]) - int(lo[1]), int(hi[0]) - int(lo[0]))
        return lo_a, hi_a, shape

    def read_voxels(self, lo=None, hi=None):
        """(mask, packed) uint32 arrays of shape (z, y, x) for the box [lo, hi)."""
        lo_a, hi_a, shape = self._box(lo, hi)
        mask = np.empty(shape, np.uint32)
        packed = np.empty(shape, np.uint32)
        L.check(L.lib().dbtsdf_read_voxels(self._h, lo_a, hi_a, mask.ctypes.data_as(C.c_void_p),
                                           packed.ctypes.data_as(C.c_void_p)), "read_voxels")
        return mask, packed

    def read_distance(self, lo=None, hi=None):
        lo_a, hi_a, shape = self._box(lo, hi)
        out = np.empty(shape, np.int8)
        L.check(L.lib().dbtsdf_read_distance(self._h, lo_a, hi_a, out.ctypes.data_as(C.c_void_p)),
                "read_distance")
        return out

    def count_mesh(self, lo=None, hi=None) -> int:
        """Number of triangles extract_mesh would return for the box [lo, hi)."""
        lo_a, hi_a, _ = self._box(lo, hi)
        n = C.c_uint64()
        L.check(L.lib().dbtsdf_extract_mesh(self._h, lo_a, hi_a, None, 0, C.byref(n)), "extract_mesh")
        return int(n.value)

    def extract_mesh(self, lo=None, hi=None, out=None):
        """Marching-cubes mesh of the zero level over the box [lo, hi): a (n, 3, 3) float32 CUDA tensor of
        triangles (vertices counter-clockwise about the normal, which points to positive distance), in no
        particular order. `out`, a float32 CUDA tensor of shape (m, 3, 3), is filled instead when given
        and m is enough (a counting pass sizes the result otherwise)."""
        import torch
        lo_a, hi_a, _ = self._box(lo, hi)
        n = C.c_uint64()
        if out is None:
            count = self.count_mesh(lo, hi)
            dev = self.mask_tensor.device if self.mask_tensor is not None else torch.device("cuda")
            out = torch.empty((count, 3, 3), dtype=torch.float32, device=dev)
        if out.dtype != torch.float32 or not out.is_cuda or not out.is_contiguous() or tuple(out.shape[1:]) != (3, 3):
            raise ValueError("out must be a contiguous float32 CUDA tensor of shape (m, 3, 3)")
        ptr = C.c_void_p(out.data_ptr()) if out.shape[0] else None
        L.check(L.lib().dbtsdf_extract_mesh(self._h, lo_a, hi_a, ptr, int(out.shape[0]), C.byref(n)),
                "extract_mesh")
        if int(n.value) > out.shape[0]:
            raise ValueError(f"mesh has {int(n.value)} triangles, out holds {out.shape[0]}")
        return out[: int(n.value)]

    def extract_points(self, lo=None, hi=None, out=None):
        """Centres of the occupied contact voxels (mask 0, sign 0) of the box [lo, hi): a (n, 3) float32 CUDA
        tensor (rows in no fixed order, x order within a row). With `out` (a CUDA float32 (cap, 3) tensor)
        one pass writes into it and returns the filled rows; ValueError if it is too small. See
        write_point_cloud for CSV / PCD files."""
        import torch
        lo_a, hi_a, _ = self._box(lo, hi)
        if out is not None:
            if out.dtype != torch.float32 or not out.is_cuda or out.dim() != 2 or out.shape[1] != 3 \
                    or not out.is_contiguous():
                raise ValueError("out must be a contiguous (cap, 3) float32 CUDA tensor")
            n = C.c_uint64()
            L.check(L.lib().dbtsdf_extract_points(self._h, lo_a, hi_a, C.c_void_p(out.data_ptr()), out.shape[0],
                                                  C.byref(n)), "extract_points")
            if int(n.value) > out.shape[0]:
                raise ValueError(f"the box holds {int(n.value)} points, out holds {out.shape[0]}")
            return out[: int(n.value)]
        n = C.c_uint64()
        L.check(L.lib().dbtsdf_extract_points(self._h, lo_a, hi_a, None, 0, C.byref(n)), "extract_points")
        dev = self.mask_tensor.device if self.mask_tensor is not None else torch.device("cuda")
        out = torch.empty((int(n.value), 3), dtype=torch.float32, device=dev)
        if out.shape[0]:
            m = C.c_uint64()
            L.check(L.lib().dbtsdf_extract_points(self._h, lo_a, hi_a, C.c_void_p(out.data_ptr()), out.shape[0],
                                                  C.byref(m)), "extract_points")
            if int(m.value) != out.shape[0]:
                raise RuntimeError("the grid changed between the counting and the writing pass")
        return out

    def write_voxels(self, mask, packed) -> None:
        """Overwrite the whole grid from (Nz, Ny, Nx) uint32 planes (validated by the library)."""
        shape = (self.dims[2], self.dims[1], self.dims[0])
        for name, a in (("mask", mask), ("packed", packed)):
            if np.shape(a) != shape:
                raise ValueError(f"write_voxels: {name} has shape {np.shape(a)}, the grid needs {shape}")
        m = np.ascontiguousarray(mask, dtype=np.uint32)
        p = np.ascontiguousarray(packed, dtype=np.uint32)
        L.check(L.lib().dbtsdf_write_voxels(self._h, m.ctypes.data_as(C.c_void_p), p.ctypes.data_as(C.c_void_p)),
                "write_voxels")

    def planes(self):
        """Raw device pointers (mask, packed) of the planes."""
        m, p = C.c_void_p(), C.c_void_p()
        L.check(L.lib().dbtsdf_grid_planes(self._h, C.byref(m), C.byref(p)), "grid_planes")
        return m.value, p.value

    def close(self) -> None:
        h, lib = getattr(self, "_h", None), getattr(self, "_lib", None)
        if h and self._owned and lib is not None:
            lib.dbtsdf_destroy_grid(h)
        self._h = None

    def __del__(self):
        self.close()


class Batch:
    """Batched integration: many scans of many grids per launch sequence, optionally graph-replayed."""

    def __init__(self, stream=None, use_graph=True):
        h = C.c_void_p()
        st = C.c_void_p(stream) if stream is not None else C.c_void_p(None)
        self._lib = L.lib()
        L.check(self._lib.dbtsdf_batch_create(st, 1 if use_graph else 0, C.byref(h)), "batch_create")
        self._h = h
        self._keep = []

    def integrate(self, items) -> list:
        """items: [(grid, pose, points)] with points all on the device or all on the host."""
        n = len(items)
        if n == 0:
            return []
        grids = (C.c_void_p * n)(*[g._h for g, _, _ in items])
        poses = np.stack([_f32(p, (16,)) for _, p, _ in items]).astype(np.float32)
        args = [_points_arg(pts) for _, _, pts in items]
        on_dev = {a[2] for a in args}
        if len(on_dev) != 1:
            raise ValueError("batch points must be all on the device or all on the host")
        ptrs = (C.c_void_p * n)(*[a[0] for a in args])
        counts = (C.c_uint64 * n)(*[a[1] for a in args])
        stats = (L.ScanStats * n)()
        L.check(L.lib().dbtsdf_batch_integrate(self._h, n, grids, poses.ctypes.data_as(C.c_void_p), ptrs, counts,
                                               on_dev.pop(), stats), "batch_integrate")
        self._keep.append((stats, [a[3] for a in args]))
        return self._stats_list(stats, n)

    def integrate_sweeps(self, items, deskew="se3") -> list:
        """items: [(grid, pose_start, pose_end, points, times)], motion-compensated sweeps in one launch;
        points (and times beside them) all on the device or all on the host."""
        n = len(items)
        if n == 0:
            return []
        grids = (C.c_void_p * n)(*[it[0]._h for it in items])
        p0 = np.stack([_f32(it[1], (16,)) for it in items]).astype(np.float32)
        p1 = np.stack([_f32(it[2], (16,)) for it in items]).astype(np.float32)
        args = [_points_arg(it[3]) for it in items]
        on_dev = {a[2] for a in args}
        if len(on_dev) != 1:
            raise ValueError("batch points must be all on the device or all on the host")
        on = on_dev.pop()
        targs = [_times_arg(it[4], a[1], on) for it, a in zip(items, args)]
        ptrs = (C.c_void_p * n)(*[a[0] for a in args])
        tptrs = (C.c_void_p * n)(*[t[0] for t in targs])
        counts = (C.c_uint64 * n)(*[a[1] for a in args])
        stats = (L.ScanStats * n)()
        L.check(L.lib().dbtsdf_batch_integrate_deskew(self._h, n, grids, p0.ctypes.data_as(C.c_void_p),
                                                      p1.ctypes.data_as(C.c_void_p), DESKEW[deskew], ptrs, tptrs,
                                                      counts, on, stats), "batch_integrate_deskew")
        self._keep.append((stats, [a[3] for a in args], [t[1] for t in targs]))
        return self._stats_list(stats, n)

    @staticmethod
    def _stats_list(stats, n):
        out = []
        for i in range(n):
            s = Stats()
            s._c = stats[i]
            out.append(s)
        return out

    def sync(self) -> None:
        L.check(L.lib().dbtsdf_batch_sync(self._h), "batch_sync")
        self._keep = self._keep[-4:]

    def set_profiling(self, enable=True, every: int = 1) -> None:
        """Time every `every`-th launch with HIP events (off when `enable` is false)."""
        L.check(L.lib().dbtsdf_batch_set_profiling(self._h, _period(enable, every)), "batch_set_profiling")

    def read_profile(self) -> dict:
        return _read_profile(L.lib().dbtsdf_batch_read_profile, self._h)

    def graph_stats(self):
        c, r = C.c_uint64(), C.c_uint64()
        L.check(L.lib().dbtsdf_batch_graph_stats(self._h, C.byref(c), C.byref(r)), "batch_graph_stats")
        return int(c.value), int(r.value)

    def close(self):
        h, lib = getattr(self, "_h", None), getattr(self, "_lib", None)
        if h and lib is not None:
            lib.dbtsdf_batch_destroy(h)
        self._h = None

    def __del__(self):
        self.close()


from .serve import Server  # noqa: E402,F401
