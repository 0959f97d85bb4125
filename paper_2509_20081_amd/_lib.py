"""ctypes declarations of the C ABI in include/dbtsdf.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdbtsdf.so")

OK = 0
STATUS_NAMES = {0: "OK", 1: "ERR_INVALID_ARG", 2: "ERR_OUT_OF_MEMORY", 3: "ERR_DEVICE",
                4: "ERR_OUT_OF_RANGE", 5: "ERR_POISONED", 6: "ERR_BUSY"}

BIN_AZEL, BIN_CUBE26 = 0, 1
DIST_L2, DIST_L1 = 0, 1
DEDUP_FIRST, COUNT_TRAFFIC = 0x1, 0x2
STRATEGY_AUTO, STRATEGY_BRICK, STRATEGY_ATOMIC, STRATEGY_SORT, STRATEGY_TILE = 0, 1, 2, 3, 4


class KernelParams(C.Structure):
    _fields_ = [("kernel_size", C.c_uint32), ("binning", C.c_uint32), ("bins_az", C.c_uint32),
                ("bins_el", C.c_uint32), ("shadow_r2", C.c_int32), ("metric", C.c_uint32),
                ("shadow_model", C.c_uint32), ("cone_deg", C.c_float)]


class GridParams(C.Structure):
    _fields_ = [("dims", C.c_uint32 * 3), ("voxel_size", C.c_float), ("origin", C.c_float * 3),
                ("hit_threshold", C.c_uint32), ("hit_max", C.c_uint32), ("flags", C.c_uint32)]


STAT_FIELDS = ("n_in", "n_invalid", "n_out_of_bounds", "n_duplicate", "n_integrated",
               "voxel_updates", "shadow_updates", "u_mask", "c_mask", "u_shadow", "n_revisit")


class ScanStats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in STAT_FIELDS]

    def as_dict(self) -> dict:
        return {n: int(getattr(self, n)) for n in STAT_FIELDS}


class Tuning(C.Structure):
    _fields_ = [("strategy", C.c_uint32), ("brick", C.c_uint32 * 3), ("block_threads", C.c_uint32),
                ("apply_blocks", C.c_uint32), ("chunk", C.c_uint32)]


class ServerConfig(C.Structure):
    _fields_ = [("n_streams", C.c_uint32), ("max_batch_scans", C.c_uint32), ("max_batch_points", C.c_uint64),
                ("memory_budget", C.c_uint64), ("queue_capacity", C.c_uint32), ("use_graph", C.c_uint32)]


class Completion(C.Structure):
    _fields_ = [("ticket", C.c_uint64), ("map_id", C.c_uint32), ("status", C.c_uint32),
                ("t_arrival_ns", C.c_uint64), ("t_launch_ns", C.c_uint64), ("t_done_ns", C.c_uint64),
                ("batch_scans", C.c_uint32), ("stats", ScanStats)]


class Metrics(C.Structure):
    _fields_ = [("accuracy", C.c_double), ("completeness", C.c_double), ("chamfer_l1", C.c_double),
                ("precision", C.c_double), ("recall", C.c_double), ("fscore", C.c_double),
                ("n_pred", C.c_uint64), ("n_gt", C.c_uint64), ("n_pred_within", C.c_uint64),
                ("n_gt_within", C.c_uint64)]


P = C.c_void_p
U32, U64, I32 = C.c_uint32, C.c_uint64, C.c_int32
PP = C.POINTER(C.c_void_p)

# name -> (restype, argtypes)
SIGNATURES = {
    "dbtsdf_status_string": (C.c_char_p, [C.c_int]),
    "dbtsdf_last_error": (C.c_char_p, []),
    "dbtsdf_kernel_set_create": (C.c_int, [C.POINTER(KernelParams), PP]),
    "dbtsdf_kernel_set_export": (C.c_int, [P, P, P, P, C.POINTER(U32)]),
    "dbtsdf_kernel_set_n_bins": (U32, [P]),
    "dbtsdf_kernel_set_bin": (I32, [P, C.c_float, C.c_float, C.c_float]),
    "dbtsdf_kernel_set_destroy": (None, [P]),
    "dbtsdf_grid_bytes": (U64, [C.POINTER(GridParams)]),
    "dbtsdf_create_grid": (C.c_int, [C.POINTER(GridParams), P, P, PP]),
    "dbtsdf_create_grid_on": (C.c_int, [C.POINTER(GridParams), P, P, P, P, PP]),
    "dbtsdf_grid_planes": (C.c_int, [P, PP, PP]),
    "dbtsdf_reset_grid": (C.c_int, [P]),
    "dbtsdf_get_tuning": (C.c_int, [P, C.POINTER(Tuning)]),
    "dbtsdf_set_tuning": (C.c_int, [P, C.POINTER(Tuning)]),
    "dbtsdf_integrate_scan": (C.c_int, [P, P, P, U64, C.c_int, C.POINTER(ScanStats)]),
    "dbtsdf_sync": (C.c_int, [P]),
    "dbtsdf_integrate_scan_noalloc": (C.c_int, [P, P, P, U64, C.POINTER(ScanStats)]),
    "dbtsdf_read_voxels": (C.c_int, [P, P, P, P, P]),
    "dbtsdf_read_distance": (C.c_int, [P, P, P, P]),
    "dbtsdf_write_voxels": (C.c_int, [P, P, P]),
    "dbtsdf_integrate_scan_every": (C.c_int, [P, P, P, U64, U32, C.c_int, P]),
    "dbtsdf_extract_mesh": (C.c_int, [P, P, P, P, U64, C.POINTER(U64)]),
    "dbtsdf_extract_points": (C.c_int, [P, P, P, P, U64, C.POINTER(U64)]),
    "dbtsdf_nearest_sq": (C.c_int, [C.c_int, P, U64, P, U64, P]),
    "dbtsdf_surface_metrics": (C.c_int, [C.c_int, P, U64, P, U64, C.c_double, C.POINTER(Metrics)]),
    "dbtsdf_deskew_constants": (C.c_int, [P, P, C.c_int, P]),
    "dbtsdf_integrate_scan_deskew": (C.c_int, [P, P, P, P, P, U64, U32, C.c_int, C.c_int, P]),
    "dbtsdf_batch_integrate_deskew": (C.c_int, [P, U32, P, P, P, C.c_int, P, P, P, C.c_int, P]),
    "dbtsdf_destroy_grid": (None, [P]),
    "dbtsdf_set_profiling": (C.c_int, [P, C.c_int]),
    "dbtsdf_read_profile": (C.c_int, [P, C.POINTER(C.c_double), C.POINTER(U64), C.POINTER(C.c_double),
                                      C.POINTER(U64)]),
    "dbtsdf_batch_set_profiling": (C.c_int, [P, C.c_int]),
    "dbtsdf_batch_read_profile": (C.c_int, [P, C.POINTER(C.c_double), C.POINTER(U64), C.POINTER(C.c_double),
                                            C.POINTER(U64)]),
    "dbtsdf_batch_create": (C.c_int, [P, C.c_int, PP]),
    "dbtsdf_batch_integrate": (C.c_int, [P, U32, P, P, P, P, C.c_int, P]),
    "dbtsdf_batch_sync": (C.c_int, [P]),
    "dbtsdf_batch_graph_stats": (C.c_int, [P, C.POINTER(U64), C.POINTER(U64)]),
    "dbtsdf_batch_destroy": (None, [P]),
    "dbtsdf_autotune": (C.c_int, [P, U32, P, P, P, C.POINTER(Tuning)]),
    "dbtsdf_server_create": (C.c_int, [C.POINTER(ServerConfig), PP]),
    "dbtsdf_server_add_map": (C.c_int, [P, C.POINTER(GridParams), P, C.POINTER(U32)]),
    "dbtsdf_server_remove_map": (C.c_int, [P, U32]),
    "dbtsdf_server_map_grid": (C.c_int, [P, U32, PP]),
    "dbtsdf_server_submit": (C.c_int, [P, U32, P, P, U64, U64, C.POINTER(U64)]),
    "dbtsdf_integrate_batch": (C.c_int, [U32, P, P, P, P, P]),
    "dbtsdf_server_submit_sweep": (C.c_int, [P, U32, P, P, C.c_int, P, P, U64, U64, C.POINTER(U64)]),
    "dbtsdf_server_poll": (C.c_int, [P, P, U32, C.POINTER(U32)]),
    "dbtsdf_server_drain": (C.c_int, [P]),
    "dbtsdf_server_memory": (C.c_int, [P, C.POINTER(U64), C.POINTER(U64)]),
    "dbtsdf_server_destroy": (None, [P]),
    "dbtsdf_now_ns": (U64, []),
}

_lib = None


class DbtsdfError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        name = STATUS_NAMES.get(status, str(status))
        super().__init__(f"{where}: {name}" + (f" ({detail})" if detail else ""))


def lib():
    """The loaded library. Raises if it has not been built: there is no fallback."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run paper_2509_20081_amd.build.build() "
                               "(hipcc --offload-arch=gfx950) first")
        h = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _lib = h
    return _lib


def check(status: int, where: str) -> None:
    if status != OK:
        detail = lib().dbtsdf_last_error()
        raise DbtsdfError(status, where, detail.decode() if detail else "")
