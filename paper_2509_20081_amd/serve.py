"""Serving front: binding of the C++ request loop plus a Poisson load generator.

The C++ server (``dbtsdf_server_*``) keeps every admitted map resident in HBM
and fuses scans as they arrive (continuous batching over several streams).
This module only marshals arguments and drives arrivals.
"""
from __future__ import annotations

import ctypes as C
import time

import numpy as np

from . import _lib as L


class Server:
    def __init__(self, n_streams=2, max_batch_scans=64, max_batch_points=4 << 20, memory_budget=0,
                 queue_capacity=4096, use_graph=True):
        cfg = L.ServerConfig(n_streams, max_batch_scans, max_batch_points, memory_budget, queue_capacity,
                             1 if use_graph else 0)
        h = C.c_void_p()
        self._lib = L.lib()
        L.check(self._lib.dbtsdf_server_create(C.byref(cfg), C.byref(h)), "server_create")
        self._h = h
        self._kernel_sets = []

    def add_map(self, dims, voxel_size, origin, kernel_set, hit_threshold=5, hit_max=65535, dedup=True) -> int:
        from . import grid_params
        p = grid_params(dims, voxel_size, origin, hit_threshold, hit_max, dedup, False)
        mid = C.c_uint32()
        L.check(L.lib().dbtsdf_server_add_map(self._h, C.byref(p), kernel_set._h, C.byref(mid)), "server_add_map")
        self._kernel_sets.append(kernel_set)
        return int(mid.value)

    def try_add_map(self, *a, **k):
        """add_map, or None when the memory budget refuses the map."""
        try:
            return self.add_map(*a, **k)
        except L.DbtsdfError as e:
            if e.status == 2:
                return None
            raise

    def remove_map(self, map_id: int) -> None:
        L.check(L.lib().dbtsdf_server_remove_map(self._h, map_id), "server_remove_map")

    def map_grid(self, map_id: int, dims, kernel_set):
        """A non-owning Grid view of a served map (for readout after drain())."""
        from . import Grid
        h = C.c_void_p()
        L.check(L.lib().dbtsdf_server_map_grid(self._h, map_id, C.byref(h)), "server_map_grid")
        return Grid(dims, 1.0, (0, 0, 0), kernel_set, _handle=h)

    def submit(self, map_id: int, pose, points, t_arrival_ns: int | None = None) -> int:
        pose = np.ascontiguousarray(np.asarray(pose, np.float32).reshape(16))
        pts = np.ascontiguousarray(np.asarray(points, np.float32).reshape(-1, 3))
        if t_arrival_ns is None:
            t_arrival_ns = int(L.lib().dbtsdf_now_ns())
        tk = C.c_uint64()
        L.check(L.lib().dbtsdf_server_submit(self._h, map_id, pose.ctypes.data_as(C.c_void_p),
                                             pts.ctypes.data_as(C.c_void_p), pts.shape[0], t_arrival_ns,
                                             C.byref(tk)), "server_submit")
        return int(tk.value)

    def submit_sweep(self, map_id: int, pose_start, pose_end, points, times, deskew="se3",
                     t_arrival_ns: int | None = None) -> int:
        """Queue a motion-compensated sweep: return i at time fraction times[i] between the two poses."""
        from . import DESKEW
        p0 = np.ascontiguousarray(np.asarray(pose_start, np.float32).reshape(16))
        p1 = np.ascontiguousarray(np.asarray(pose_end, np.float32).reshape(16))
        pts = np.ascontiguousarray(np.asarray(points, np.float32).reshape(-1, 3))
        tt = np.ascontiguousarray(np.asarray(times, np.float32).reshape(-1))
        if tt.shape[0] != pts.shape[0]:
            raise ValueError("times must hold one float32 per point")
        if t_arrival_ns is None:
            t_arrival_ns = int(L.lib().dbtsdf_now_ns())
        tk = C.c_uint64()
        L.check(L.lib().dbtsdf_server_submit_sweep(self._h, map_id, p0.ctypes.data_as(C.c_void_p),
                                                   p1.ctypes.data_as(C.c_void_p), DESKEW[deskew],
                                                   pts.ctypes.data_as(C.c_void_p), tt.ctypes.data_as(C.c_void_p),
                                                   pts.shape[0], t_arrival_ns, C.byref(tk)), "server_submit_sweep")
        return int(tk.value)

    def poll(self, max_n=1024) -> list[dict]:
        buf = (L.Completion * max_n)()
        n = C.c_uint32()
        L.check(L.lib().dbtsdf_server_poll(self._h, buf, max_n, C.byref(n)), "server_poll")
        out = []
        for i in range(n.value):
            c = buf[i]
            out.append(dict(ticket=int(c.ticket), map_id=int(c.map_id), status=int(c.status),
                            t_arrival_ns=int(c.t_arrival_ns), t_launch_ns=int(c.t_launch_ns),
                            t_done_ns=int(c.t_done_ns), batch_scans=int(c.batch_scans), stats=c.stats.as_dict()))
        return out

    def drain(self) -> None:
        L.check(L.lib().dbtsdf_server_drain(self._h), "server_drain")

    def memory(self):
        a, b = C.c_uint64(), C.c_uint64()
        L.check(L.lib().dbtsdf_server_memory(self._h, C.byref(a), C.byref(b)), "server_memory")
        return int(a.value), int(b.value)

    def close(self):
        h, lib = getattr(self, "_h", None), getattr(self, "_lib", None)
        if h and lib is not None:
            lib.dbtsdf_server_destroy(h)
        self._h = None

    def __del__(self):
        self.close()


def poisson_arrivals(rng: np.random.Generator, rate_hz: float, duration_s: float) -> np.ndarray:
    """Arrival offsets (s) of a Poisson process of the given rate over [0, duration)."""
    n_est = int(rate_hz * duration_s * 1.5) + 16
    gaps = rng.exponential(1.0 / rate_hz, size=n_est)
    t = np.cumsum(gaps)
    while t[-1] < duration_s:
        more = np.cumsum(rng.exponential(1.0 / rate_hz, size=n_est)) + t[-1]
        t = np.concatenate([t, more])
    return t[t < duration_s]


def run_open_loop(server: Server, schedule, warmup_s: float = 0.0, progress=None):
    """Submit ``schedule`` = [(t_offset_s, map_id, pose, points)] at their arrival times.

    Returns the completions of every scan (arrival stamps are the scheduled
    times, so queueing delay in front of the server counts as latency).
    Scans arriving before ``warmup_s`` are marked ``warmup``.
    """
    now = L.lib().dbtsdf_now_ns
    t0 = int(now()) + 5_000_000
    done = []
    warm_tickets = set()
    for k, (toff, mid, pose, pts) in enumerate(schedule):
        t_arr = t0 + int(toff * 1e9)
        while True:
            d = t_arr - int(now())
            if d <= 0:
                break
            if d > 200_000:
                time.sleep((d - 100_000) / 1e9)
            done.extend(server.poll())
        tk = server.submit(mid, pose, pts, t_arr)
        if toff < warmup_s:
            warm_tickets.add(tk)
        if progress and k % 2000 == 0:
            progress(k, len(schedule))
    server.drain()
    done.extend(server.poll(1 << 16))
    for c in done:
        c["warmup"] = c["ticket"] in warm_tickets
    return done
