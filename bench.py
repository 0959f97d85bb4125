#!/usr/bin/env python3
"""Benchmark of DB-TSDF scan integration on one MI355X.

Default workload: the 200-scan sequence at 10 Hz of 64x1024-point scans fused
into a 1024x1024x256 grid at 0.05 m (11^3 kernel, 26 direction bins). One step
is one scan through the whole path (transform, bounds, bins, first-return
dedup, brick bucketing, eq. 4 AND, eqs. 5-6 counter/sign), plain form: one
scan per launch sequence, points already resident in HBM.

Also reported on the same scans: the batched form (several scans per launch,
replayed from a captured HIP graph, bit-identical), the plain form's per-scan
latency, the served form on 32 robots with Poisson arrivals (continuous
batching, p50/p99 arrival-to-completion latency), the dominant kernel's HBM
roofline fraction, and the CPU oracle on the host.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import contextlib
import gc
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "voxel-updates/s & scans/s (batched vs plain, bit-exact); p50/p99 scan latency"
HBM_PEAK_GBS = 8000.0
LDS_ATOMIC_OPS = 256 * 32 * 2.4e9
RING_SLOTS = 16  # calls in flight per grid / batch context; each slot has its own graphs
# the plain form's timed region times every 4th call with HIP events (a timed
# call launches its apply kernel between events instead of inside the call's
# graph, which costs it some microseconds); 4 divides the ring, so each ring
# slot is always timed or never and the warm-up captures every graph used
PROF_EVERY = 4


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("kernels.hip", "internal.h"):
        with open(os.path.join(ROOT, "paper_2509_20081_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def pct(a, q):
    return float(np.percentile(np.asarray(a, dtype=np.float64), q)) if len(a) else None


def load_scans(cfg, n, torch):
    from synth import scene as synth
    t = time.time()
    scans = list(synth.config_scans(cfg, 0, range(n)))
    dev = [(pose, torch.from_numpy(pts).cuda()) for pose, pts in scans]
    torch.cuda.synchronize()
    log(f"generated {n} scans of config {cfg} in {time.time() - t:.1f}s "
        f"({np.mean([len(p) for _, p in scans]):.0f} points/scan)")
    return scans, dev


@contextlib.contextmanager
def no_gc():
    """Timed regions run without Python's cyclic collector (a full pass over
    this process's heap of scan arrays takes tens of milliseconds)."""
    gc.collect()
    gc.freeze()
    gc.disable()
    try:
        yield
    finally:
        gc.enable()
        gc.unfreeze()


def planes_equal(torch, a, b):
    """Both planes of two grids (torch-owned planes) equal word for word, compared on the device."""
    return bool(torch.equal(a.mask_tensor, b.mask_tensor)) and bool(torch.equal(a.packed_tensor, b.packed_tensor))


def far_pose():
    """A pose that puts every return of a scan outside any grid of these workloads: calls with it run the
    whole pass sequence (descriptors, front end, select, apply with no survivors) and change nothing. Used
    to visit every ring slot (and capture its graphs) before a timed region without integrating a scan
    twice."""
    p = np.eye(4, dtype=np.float32)
    p[:3, 3] = 1.0e6
    return p


def warm_ring(g, pts):
    for _ in range(RING_SLOTS):
        g.integrate(far_pose(), pts)
    g.sync()


def run_plain(db, torch, gdef, ks, dev, warmup, steps, tuning, profile=True):
    g = db.Grid(gdef["dims"], gdef["voxel_size"], gdef["origin"], ks, planes="torch")
    if tuning:
        g.set_tuning(**{k: v for k, v in tuning.items() if k != "apply_blocks"})
    # the warm-up runs as profiled as the timed region: every ring slot is
    # visited (and its graphs captured) by calls that integrate nothing, then
    # the warm-up scans 0 .. warmup-1 are integrated once each
    if profile:
        g.set_profiling(True, every=PROF_EVERY)
    warm_ring(g, dev[0][1])
    for k in range(warmup):
        pose, pts = dev[k]
        g.integrate(pose, pts)
    g.sync()
    if profile:
        g.set_profiling(True, every=PROF_EVERY)  # restart the totals (the call count runs on)
    torch.cuda.synchronize()
    with no_gc():
        t0 = time.perf_counter()
        stats = []
        for k in range(warmup, warmup + steps):
            pose, pts = dev[k]
            stats.append(g.integrate(pose, pts))
        g.sync()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    prof = g.read_profile() if profile else None
    return g, dt, stats, prof


def run_deskew(db, torch, gdef, ks, dev, warmup, steps, tuning, mode="se3"):
    """The plain form with every scan taken as a motion-compensated sweep from its pose to the next
    scan's pose, time fraction rising along the point array (as a spinning sensor's): the cost of the
    per-return pose against the plain calls."""
    g = db.Grid(gdef["dims"], gdef["voxel_size"], gdef["origin"], ks, planes="torch")
    if tuning:
        g.set_tuning(**{k: v for k, v in tuning.items() if k != "apply_blocks"})
    n_seq = len(dev)
    times = {}
    def sweep(k):
        pose, pts = dev[k]
        end = dev[k + 1][0] if k + 1 < n_seq else pose
        n = int(pts.shape[0])
        if n not in times:
            times[n] = torch.linspace(0.0, 1.0, n, dtype=torch.float32, device="cuda")
        return pose, pts, end, times[n]
    warm_ring(g, dev[0][1])
    for k in range(warmup):
        pose, pts, end, tt = sweep(k)
        g.integrate(pose, pts, pose_end=end, times=tt, deskew=mode)
    g.sync()
    torch.cuda.synchronize()
    args_k = [sweep(k) for k in range(warmup, warmup + steps)]
    with no_gc():
        t0 = time.perf_counter()
        stats = [g.integrate(pose, pts, pose_end=end, times=tt, deskew=mode) for pose, pts, end, tt in args_k]
        g.sync()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    upd = sum(s.as_dict()["voxel_updates"] for s in stats)
    g.close()
    return {"mode": mode, "value": upd / dt, "unit": "voxel-updates/s", "ms_per_scan": dt * 1e3 / steps,
            "scans": steps, "times": "linear in the point index from 0 to 1; end pose = the next scan's pose"}


def run_batched(db, torch, gdef, ks, dev, warmup, steps, tuning, per_launch):
    g = db.Grid(gdef["dims"], gdef["voxel_size"], gdef["origin"], ks, planes="torch")
    if tuning:
        g.set_tuning(**{k: v for k, v in tuning.items() if k != "apply_blocks"})
    b = db.Batch(use_graph=True)
    # capture the context's graphs for every ring slot on a scratch grid of the
    # same shape (the graphs do not depend on which grid a launch updates)
    b.set_profiling(True)
    scratch = db.Grid(gdef["dims"], gdef["voxel_size"], gdef["origin"], ks)
    if tuning:
        scratch.set_tuning(**{k: v for k, v in tuning.items() if k != "apply_blocks"})
    for _ in range(RING_SLOTS):
        b.integrate([(scratch, dev[k][0], dev[k][1]) for k in range(per_launch)])
    b.sync()
    scratch.close()
    b.set_profiling(False)

    def launch(ks_):
        return b.integrate([(g, dev[k][0], dev[k][1]) for k in ks_])

    for s in range(0, warmup, per_launch):
        launch(range(s, min(s + per_launch, warmup)))
    b.sync()
    b.set_profiling(True)
    torch.cuda.synchronize()
    with no_gc():
        t0 = time.perf_counter()
        stats = []
        for s in range(warmup, warmup + steps, per_launch):
            stats.extend(launch(range(s, min(s + per_launch, warmup + steps))))
        b.sync()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    prof = b.read_profile()
    caps, reps = b.graph_stats()
    return g, dt, stats, prof, (caps, reps)


def count_traffic(db, gdef, ks, dev, warmup, steps, tuning):
    """Untimed replay with the unique-word counters on: U_m, C_m, U_s of the timed scans."""
    g = db.Grid(gdef["dims"], gdef["voxel_size"], gdef["origin"], ks, count_traffic=True)
    if tuning:
        g.set_tuning(**{k: v for k, v in tuning.items() if k != "apply_blocks"})
    out = []
    for k in range(warmup + steps):
        pose, pts = dev[k]
        st = g.integrate(pose, pts)
        if k >= warmup:
            out.append(st)
        if k % 16 == 15:
            g.sync()
    g.sync()
    res = [s.as_dict() for s in out]
    g.close()
    return res


def plain_latency(db, torch, gdef, ks, dev, n, tuning):
    g = db.Grid(gdef["dims"], gdef["voxel_size"], gdef["origin"], ks)
    if tuning:
        g.set_tuning(**{k: v for k, v in tuning.items() if k != "apply_blocks"})
    lat = []
    warm_ring(g, dev[0][1])   # every ring slot visited before measuring, nothing integrated
    with no_gc():
        for k in range(min(n, len(dev))):
            pose, pts = dev[k]
            t0 = time.perf_counter()
            g.integrate(pose, pts)
            g.sync()
            lat.append((time.perf_counter() - t0) * 1e3)
    g.close()
    return lat


def run_serve(db, torch, seconds, warm_s, rate_hz, n_robots, seed=5, check_robot=0):
    """Served form: n_robots maps of 512^3 @ 0.05 m, Poisson arrivals totalling rate_hz for warm_s + seconds;
    every arrival brings the robot's next scan along its own trajectory (no scan repeats). At the end one
    map is compared word for word with the oracle (all-core leg) fed that robot's scans in order."""
    from paper_2509_20081_amd.serve import Server, poisson_arrivals, run_open_loop
    from synth import scene as synth
    ks = db.KernelSet(kernel_size=11, binning="cube26", shadow_r2=9)
    rng = np.random.default_rng([20081, 5, seed])
    arr = poisson_arrivals(rng, rate_hz, warm_s + seconds)
    robots = rng.integers(0, n_robots, size=len(arr))
    per_robot = np.bincount(robots, minlength=n_robots)
    t = time.time()
    streams = []
    for r in range(n_robots):
        sc = synth.served_scans(r, int(per_robot[r]), torch)
        streams.append([(pose, pts.cpu().numpy()) for pose, pts in sc])
        del sc
    torch.cuda.empty_cache()
    n_pts = sum(int(p.shape[0]) for st in streams for _, p in st)
    log(f"generated {len(arr)} distinct served scans ({n_pts} points) in {time.time() - t:.1f}s")
    srv = Server(n_streams=2, max_batch_scans=64, use_graph=True)
    ids = []
    for r in range(n_robots):
        gdef = synth.config_grid(5, r)
        ids.append(srv.add_map(gdef["dims"], gdef["voxel_size"], gdef["origin"], ks))
    counters = [0] * n_robots
    schedule = []
    for toff, r in zip(arr, robots):
        pose, pts = streams[r][counters[r]]
        counters[r] += 1
        schedule.append((float(toff), ids[r], pose, pts))
    log(f"serving {len(schedule)} scans over {warm_s + seconds:.1f}s")
    with no_gc():
        done = run_open_loop(srv, schedule, warmup_s=warm_s)
    meas = [c for c in done if not c["warmup"]]
    bad = [c for c in done if c["status"] != 0]
    lat = [(c["t_done_ns"] - c["t_arrival_ns"]) / 1e6 for c in meas]
    if meas:
        t_lo = min(c["t_arrival_ns"] for c in meas)
        t_hi = max(c["t_done_ns"] for c in meas)
        span = (t_hi - t_lo) / 1e9
    else:
        span = float("nan")
    upd = sum(c["stats"]["voxel_updates"] for c in meas)
    # one map against the oracle
    t = time.time()
    from oracle.oracle import Oracle
    gd = synth.config_grid(5, check_robot)
    kw = dict(synth.KERNEL_DEFAULTS)
    o = Oracle(dims=gd["dims"], voxel_size=gd["voxel_size"], origin=gd["origin"], **kw)
    m, p = o.new_grid()
    for pose, pts in streams[check_robot]:
        o.integrate_parallel(m, p, pose, pts)
    sm, sp = srv.map_grid(ids[check_robot], gd["dims"], ks).read_voxels()
    check = dict(robot=check_robot, scans=int(per_robot[check_robot]),
                 equal=bool(np.array_equal(sm, m) and np.array_equal(sp, p)), s=time.time() - t)
    del m, p, sm, sp
    out = dict(workload="c5_32robots_512cube_poisson", robots=n_robots, offered_scans_per_s=rate_hz,
               warmup_s=warm_s, measured_s=seconds, scans=len(meas), failed=len(bad),
               value=upd / span if span else None, unit="voxel-updates/s",
               scans_per_s=len(meas) / span if span else None,
               p50_ms=pct(lat, 50), p99_ms=pct(lat, 99), mean_batch_scans=float(np.mean([c["batch_scans"] for c in meas]))
               if meas else None, distinct_scans=True, points=n_pts, oracle_check=check)
    srv.close()
    return out


def cpu_baseline(gdef, scans, kparams, budget_s=15.0):
    """The CPU oracle on the first scans of the same sequence: single-threaded (as it stands) until the
    budget is spent, then the same scans on every host core (its OpenMP leg, the same planes bit for
    bit) on a fresh grid."""
    from oracle.oracle import Oracle
    from synth import scene as synth
    kw = dict(synth.KERNEL_DEFAULTS)
    kw.update(kparams)
    o = Oracle(dims=gdef["dims"], voxel_size=gdef["voxel_size"], origin=gdef["origin"], **kw)
    m, p = o.new_grid()
    upd, t_tot, n = 0, 0.0, 0
    for pose, pts in scans:
        t0 = time.perf_counter()
        st = o.integrate(m, p, pose, pts)
        t_tot += time.perf_counter() - t0
        upd += st["voxel_updates"]
        n += 1
        if t_tot > budget_s:
            break
    del m, p
    gc.collect()
    m, p = o.new_grid()
    upd_p, t_par, threads = 0, 0.0, 0
    for pose, pts in scans[:n]:
        t0 = time.perf_counter()
        st, threads = o.integrate_parallel(m, p, pose, pts)
        t_par += time.perf_counter() - t0
        upd_p += st["voxel_updates"]
    del m, p
    gc.collect()
    return dict(value=upd / t_tot, unit="voxel-updates/s", cores=1, kind="oracle",
                sample=f"first {n} scans of the same sequence, single-threaded C oracle, {t_tot:.1f}s",
                scans_per_s=n / t_tot, host=host_cpu(),
                all_cores=dict(value=upd_p / t_par, unit="voxel-updates/s", cores=threads,
                               kind="oracle, OpenMP leg (atomic AND and counter compare-and-swap)",
                               sample=f"the same {n} scans on a fresh grid, {t_par:.1f}s", scans_per_s=n / t_par,
                               speedup_vs_1core=(upd_p / t_par) / (upd / t_tot)))


def host_cpu():
    """The host the CPU legs ran on: logical CPUs visible to this process and the CPU model."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return dict(nproc=len(os.sched_getaffinity(0)), cpu_model=model)


def run_mesh(torch, g, dims, reps=3):
    """Mesh export (Marching Cubes at iso 0) of the whole grid after the timed scans: HIP events on the
    grid's stream around each extraction call (the call synchronises, so its host return is inside)."""
    n = g.count_mesh()
    out = torch.empty((max(n, 1), 3, 3), dtype=torch.float32, device="cuda")
    g.extract_mesh(out=out)
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        g.extract_mesh(out=out)
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    t = min(ms)
    vox = dims[0] * dims[1] * dims[2]
    nbytes = 8.0 * vox + 36.0 * n
    return dict(triangles=n, ms=t, cubes_per_s=(dims[0] - 1) * (dims[1] - 1) * (dims[2] - 1) / (t * 1e-3),
                roofline=dict(bound="hbm", achieved=nbytes / (t * 1e-3) / 1e9, peak=HBM_PEAK_GBS, unit="GB/s",
                              frac=nbytes / (t * 1e-3) / 1e9 / HBM_PEAK_GBS,
                              per_launch="8 B per voxel (both planes read once) + 36 B per triangle written"),
                timing="HIP events around one extraction call (best of %d), whole grid" % reps,
                points=run_points(torch, g, dims, reps))


def run_accuracy(db, torch, synth, g, gdef, cfg, n_scans, tolerance=0.1):
    """Accuracy metrics (Sec. IV-A) of the map after the plain leg's scans against the exact hits of the
    same rays (one per voxel-sized cube, inside the grid): for the mesh (one point per triangle, its
    centroid) and for the point export,
    each scored on the GPU (nearest squared distances in fp64, both directions)."""
    t0 = time.perf_counter()
    gt = synth.config_ground_truth(cfg, scan_ids=range(n_scans), cell=gdef["voxel_size"])
    lo = np.array(gdef["origin"], np.float64)
    hi = lo + np.array(gdef["dims"], np.float64) * gdef["voxel_size"]
    gt = gt[np.all((gt >= lo) & (gt < hi), axis=1)]
    t_gt = time.perf_counter() - t0
    gt_dev = torch.from_numpy(np.ascontiguousarray(gt)).cuda()
    out = dict(tolerance_m=tolerance, reference=f"exact hits of the rays of scans 0-{n_scans - 1}, first per "
               f"{gdef['voxel_size']:.3f} m cube", n_reference=int(gt.shape[0]), reference_s=t_gt)
    sets = {"mesh_centroids": lambda: db.mesh_centroids(g.extract_mesh()), "point_export": g.extract_points}
    for name, get in sets.items():
        pred = get()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        m = db.surface_metrics(pred, gt_dev, tolerance)
        m["gpu_s"] = time.perf_counter() - t1
        out[name] = m
        del pred
        torch.cuda.empty_cache()
    return out


MRES_SIZES = (0.3, 0.2, 0.1, 0.05)


def run_mres(db, torch, synth, ks, tuning, n_scans=10, reps=3):
    """Per-scan cost against voxel size (Sec. IV-B, eq. 7: constant per scan): scans 0 .. n_scans-1 of the
    second workload integrated into a fresh grid of the same room at each voxel size (the same K^3 kernel,
    so the same work per return), timed from the first call to the final sync; best of `reps` fresh grids."""
    scans = list(synth.config_scans(2, 0, range(n_scans)))
    dev = [(pose, torch.from_numpy(pts).cuda()) for pose, pts in scans]
    out = []
    for s in MRES_SIZES:
        gd = synth.resolution_grid(s)
        best = None
        for _ in range(reps):
            g = db.Grid(gd["dims"], gd["voxel_size"], gd["origin"], ks)
            if tuning:
                g.set_tuning(**{k: v for k, v in tuning.items() if k != "apply_blocks"})
            warm_ring(g, dev[0][1])
            g.sync()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = [g.integrate(pose, pts) for pose, pts in dev]
            g.sync()
            dt = time.perf_counter() - t0
            g.close()
            torch.cuda.empty_cache()
            if best is None or dt < best[0]:
                best = (dt, st)
        dt, st = best
        out.append(dict(voxel_size_m=s, grid=list(gd["dims"]), ms_per_scan=dt * 1e3 / n_scans,
                        integrated_per_scan=float(np.mean([x.as_dict()["n_integrated"] for x in st])),
                        revisit_frac=float(np.sum([x.as_dict()["n_revisit"] for x in st]) /
                                           max(1, np.sum([x.as_dict()["n_integrated"] for x in st])))))
    t = [r["ms_per_scan"] for r in out]
    return dict(scans=f"second workload, scans 0-{n_scans - 1} (64 x 1024 returns each)", by_voxel_size=out,
                max_over_min_ms=max(t) / min(t),
                timing="wall clock from the first integrate call to the final sync, best of %d fresh grids" % reps)


def run_points(torch, g, dims, reps=3):
    """Point export (centres of the occupied contact voxels) of the whole grid, one pass into a buffer
    sized by a counting call, timed like the mesh export."""
    n = int(g.extract_points().shape[0])
    out = torch.empty((max(n, 1), 3), dtype=torch.float32, device="cuda")
    g.extract_points(out=out)
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        g.extract_points(out=out)
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    t = min(ms)
    n_zero = int((g.mask_tensor == 0).sum().item())   # voxels whose packed word the export must read
    nbytes = 4.0 * dims[0] * dims[1] * dims[2] + 4.0 * n_zero + 12.0 * n
    return dict(points=n, ms=t, roofline=dict(bound="hbm", achieved=nbytes / (t * 1e-3) / 1e9, peak=HBM_PEAK_GBS,
                                              unit="GB/s", frac=nbytes / (t * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                              per_launch="4 B per voxel (mask) + 4 B per voxel of mask 0 (packed) "
                                                         "read + 12 B per point written"))


def copy_calibration(torch, nbytes=1 << 30):
    """A plain device copy of known size (for scaling HBM counters of a --pmc run)."""
    a = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"copy calibration: 3 copies of {nbytes} bytes")


def copy_bandwidth(torch, nbytes=2 << 30, reps=5):
    """Achieved device-copy bandwidth (read + write bytes per second), the practical HBM ceiling."""
    a = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def run_c4(db, torch, ks, n_maps, n_scans, tuning):
    """64 independent maps (sides 128..1024 @ 0.05 m) x 20 scans: plain (one scan per call) against
    batched (one launch per round holding every map's scan of that round, graph-replayed), on the
    same scans in the same order; grids of the smaller maps are compared bit for bit."""
    from synth import scene as synth
    t = time.time()
    maps = []
    for m in range(n_maps):
        gdef = synth.config_grid(4, m)
        sc = [(p, torch.from_numpy(x).cuda()) for p, x in synth.config_scans(4, m, range(n_scans))]
        maps.append((gdef, sc))
    n_pts = sum(int(x.shape[0]) for _, sc in maps for _, x in sc)
    log(f"c4: generated {n_maps} maps x {n_scans} scans ({n_pts} points) in {time.time() - t:.1f}s")
    # up to 16 maps every map is compared; beyond, those of side <= 384 (their plain grids stay resident)
    small = list(range(n_maps)) if n_maps <= 16 else [m for m, (gd, _) in enumerate(maps) if max(gd["dims"]) <= 384]

    def make_grids():
        gs = []
        for gd, _ in maps:
            g = db.Grid(gd["dims"], gd["voxel_size"], gd["origin"], ks, planes="torch")
            if tuning:
                g.set_tuning(**{k: v for k, v in tuning.items() if k != "apply_blocks"})
            gs.append(g)
        return gs

    # plain; scan 0 of every map is the untimed warm-up (workspaces, first launches) in both forms
    gs = make_grids()
    for m, (_, sc) in enumerate(maps):
        gs[m].integrate(sc[0][0], sc[0][1])
    for g in gs:
        g.sync()
    torch.cuda.synchronize()
    with no_gc():
        t0 = time.perf_counter()
        st_plain = []
        for r in range(1, n_scans):
            for m, (_, sc) in enumerate(maps):
                st_plain.append(gs[m].integrate(sc[r][0], sc[r][1]))
        for g in gs:
            g.sync()
        torch.cuda.synchronize()
        dt_plain = time.perf_counter() - t0
    upd = sum(s.as_dict()["voxel_updates"] for s in st_plain)
    kept = {m: gs[m] for m in small}   # the smaller maps' plain grids stay for the comparison
    for m, g in enumerate(gs):
        if m not in kept:
            g.close()
    del gs
    torch.cuda.empty_cache()
    # batched: one launch per round
    gs = make_grids()
    b = db.Batch(use_graph=True)
    b.integrate([(gs[m], sc[0][0], sc[0][1]) for m, (_, sc) in enumerate(maps)])
    b.sync()
    torch.cuda.synchronize()
    with no_gc():
        t0 = time.perf_counter()
        st_b = []
        for r in range(1, n_scans):
            st_b.extend(b.integrate([(gs[m], sc[r][0], sc[r][1]) for m, (_, sc) in enumerate(maps)]))
        b.sync()
        torch.cuda.synchronize()
        dt_b = time.perf_counter() - t0
    caps, reps = b.graph_stats()
    updb = sum(s.as_dict()["voxel_updates"] for s in st_b)
    same = all(planes_equal(torch, gs[m], kept[m]) for m in small)
    for g in kept.values():
        g.close()
    b.close()
    for g in gs:
        g.close()
    del gs
    torch.cuda.empty_cache()
    grid_gb = sum(2 * 4 * gd["dims"][0] * gd["dims"][1] * gd["dims"][2] for gd, _ in maps) / 1e9
    return dict(workload=f"c4_{n_maps}maps_x{n_scans}scans", maps=n_maps, scans_per_map=n_scans, points=n_pts,
                resident_grid_gb=grid_gb,
                timed_rounds=n_scans - 1,
                plain=dict(value=upd / dt_plain, unit="voxel-updates/s", scans_per_s=n_maps * (n_scans - 1) / dt_plain),
                batched=dict(value=updb / dt_b, unit="voxel-updates/s", scans_per_s=n_maps * (n_scans - 1) / dt_b,
                             scans_per_launch=n_maps, graph_captures=caps, graph_replays=reps),
                speedup=(updb / dt_b) / (upd / dt_plain), updates_equal=upd == updb,
                bit_exact_maps_checked=len(small), bit_exact=same,
                comparison="both planes of each checked map word for word on the device (torch.equal)")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed scans (plain form)")
    ap.add_argument("--warmup", type=int, default=5, help="scans integrated before the timed ones")
    ap.add_argument("--config", type=int, default=3, choices=(1, 2, 3),
                    help="3: 100 scans of 128x2048 into 2048x2048x512 @ 0.02 m (the large grid, default); "
                         "2: 200 scans of 64x1024 into 1024x1024x256 @ 0.05 m")
    ap.add_argument("--batch-scans", type=int, default=8, help="scans per batched launch")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-mesh", action="store_true", help="skip the mesh export leg")
    ap.add_argument("--no-deskew", action="store_true", help="skip the motion-compensated sweep leg")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the accuracy-metrics leg")
    ap.add_argument("--no-mres", action="store_true", help="skip the per-scan cost against voxel size leg")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--latency-scans", type=int, default=50)
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--serve-warmup", type=float, default=1.0)
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--serve-robots", type=int, default=32)
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--c4-maps", type=int, default=16,
                    help="maps of the batching workload (plain against batched, every map compared when <= 16; "
                         "64 is the full workload, about 160 GB of grids; 0 skips it)")
    ap.add_argument("--kernel", choices=("workload", "paper"), default="workload",
                    help="kernel set: the workload's (K = 11, 26 cube bins) or the paper's (K = 21, 40 x 40 bins)")
    ap.add_argument("--tuning", type=str, default="", help="JSON tuning to use instead of autotuning")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; multi-GPU sharding is not built",
                          "n_gpus": args.gpus}))
        return 2
    if int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "launched with WORLD_SIZE > 1; this benchmark is single-GPU"}))
        return 2

    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        return 2
    import paper_2509_20081_amd as db
    from synth import scene as synth

    if args.copy_calibration:
        copy_calibration(torch)

    cfg = args.config
    gdef = synth.config_grid(cfg)
    n_seq = synth.CONFIGS[cfg]["scans"]
    if args.warmup + args.steps > n_seq:
        # a timed region never integrates a scan twice (a repeated scan at the same pose finds every
        # window already applied and would time less work)
        print(json.dumps({"error": f"warmup + steps = {args.warmup + args.steps} exceeds the {n_seq} scans of "
                                   f"config {cfg}; no scan is integrated twice"}))
        return 2
    scans, dev = load_scans(cfg, args.warmup + args.steps, torch)
    kparams = dict(kernel_size=11, binning="cube26", shadow_r2=9) if args.kernel == "workload" else \
        dict(kernel_size=21, binning="azel", bins_az=40, bins_el=40, shadow_r2=9)
    ks = db.KernelSet(**kparams)

    tuning = json.loads(args.tuning) if args.tuning else None
    if tuning is None and not args.no_autotune:
        # tune on the state the timed scans meet: a grid that already holds the
        # warm-up scans (autotune works on scratch copies of it)
        g = db.Grid(gdef["dims"], gdef["voxel_size"], gdef["origin"], ks)
        for pose, pts in dev[: args.warmup]:
            g.integrate(pose, pts)
        g.sync()
        tuning = g.autotune(dev[args.warmup: args.warmup + 4], True)
        g.close()
        log(f"autotuned: {tuning}")
    if tuning is None:
        g = db.Grid(gdef["dims"], gdef["voxel_size"], gdef["origin"], ks)
        tuning = g.tuning
        g.close()

    # ---- plain form (the measured value)
    g, dt, stats, prof = run_plain(db, torch, gdef, ks, dev, args.warmup, args.steps, tuning)
    sd = [s.as_dict() for s in stats]
    upd = sum(s["voxel_updates"] for s in sd)
    value = upd / dt
    log(f"plain: {args.steps} scans in {dt * 1e3:.1f} ms -> {value / 1e9:.1f} G voxel-updates/s; profile {prof}")
    mesh = None if args.no_mesh else run_mesh(torch, g, gdef["dims"])
    if mesh:
        log(f"mesh: {mesh}")
    accuracy = None
    if not args.no_accuracy:
        accuracy = run_accuracy(db, torch, synth, g, gdef, cfg, args.warmup + args.steps)
        log(f"accuracy: {accuracy}")
    plain_grid = g          # kept for the batched form's word-for-word comparison
    if args.no_batched:
        g.close()
    torch.cuda.empty_cache()

    deskew = None
    if not args.no_deskew:
        deskew = run_deskew(db, torch, gdef, ks, dev, args.warmup, min(args.steps, 100), tuning)
        deskew["vs_plain_ms_per_scan"] = deskew["ms_per_scan"] / (dt * 1e3 / args.steps)
        log(f"deskew: {deskew}")
        torch.cuda.empty_cache()

    # ---- roofline of the dominant kernel (the brick merge / apply)
    tr = count_traffic(db, gdef, ks, dev, args.warmup, args.steps, tuning)
    u_m = np.array([t["u_mask"] for t in tr], dtype=np.float64)
    c_m = np.array([t["c_mask"] for t in tr], dtype=np.float64)
    u_s = np.array([t["u_shadow"] for t in tr], dtype=np.float64)
    n_in = np.array([t["n_in"] for t in tr], dtype=np.float64)
    apply_bytes = float(np.mean(4 * u_m + 4 * c_m + 8 * u_s))
    scan_bytes = float(np.mean(12 * n_in + 4 * u_m + 4 * c_m + 8 * u_s))
    apply_ms = prof["apply_ms"] / max(prof["applies"], 1)
    call_ms = prof["call_ms"] / max(prof["calls"], 1)
    achieved = apply_bytes / (apply_ms * 1e-3) / 1e9
    if tuning["strategy"] == "tile":
        kname = "k_apply_tile"
    elif tuning["strategy"] == "brick":
        kname = f"k_apply_brick<{tuning['brick'][0]},{tuning['brick'][1]},{tuning['brick'][2]},{tuning['block_threads']}>"
    elif kparams["kernel_size"] <= 11 and kparams["binning"] == "cube26" and gdef["dims"][0] % 4 == 0:
        kname = "k_apply_points<true>"   # the row kernel of the plain one-scan call
    else:
        kname = "k_apply_atomic"
    traffic = None
    tfile = os.path.join(ROOT, "profiles", f"traffic_c{cfg}.json")
    if os.path.exists(tfile):
        tj = json.load(open(tfile))
        if tj.get("kernel_source_hash") == kernel_source_hash() and tj.get("kernel") == kname:
            traffic = tj.get("bytes_per_launch")
    copy_gbs = copy_bandwidth(torch)
    visits = float(np.mean([t["voxel_updates"] for t in sd]))
    k3 = kparams["kernel_size"] ** 3
    n_int = float(np.sum([t["n_integrated"] for t in sd]))
    n_rev = float(np.sum([t["n_revisit"] for t in sd]))
    applied_frac = 1.0 - n_rev / n_int if n_int else None
    # operations the apply kernel executes: K^3 cells per applied window plus one counter step per shadow cell
    executed = float(np.mean([(t["n_integrated"] - t["n_revisit"]) * k3 + t["shadow_updates"] for t in sd]))
    roofline = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS,
                    traffic=traffic, kernel=kname, avg_launch_us=apply_ms * 1e3,
                    timed_launches=prof["applies"],
                    timing="HIP events around the apply kernel of every %dth call of the timed region" % PROF_EVERY,
                    measured_copy_gbs=copy_gbs, frac_vs_copy=achieved / copy_gbs,
                    secondary=dict(ceiling="LDS/atomic dword ops: 256 CUs x 32 per clock x 2.4 GHz",
                                   peak_ops_per_s=LDS_ATOMIC_OPS, achieved_ops_per_s=executed / (apply_ms * 1e-3),
                                   frac=executed / (apply_ms * 1e-3) / LDS_ATOMIC_OPS,
                                   per_launch="operations executed in one scan: K^3 per applied window (returns "
                                              "in voxels an earlier scan integrated skip theirs) + one per "
                                              "shadow cell"),
                    windows_applied_frac=applied_frac,
                    algorithmic_bytes_per_launch=apply_bytes,
                    per_launch="4*U_m + 4*C_m + 8*U_s of one scan (unique mask words read, changed words "
                               "written, unique shadow words read+written)",
                    whole_call=dict(avg_us=call_ms * 1e3, bytes=scan_bytes,
                                    frac=scan_bytes / (call_ms * 1e-3) / 1e9 / HBM_PEAK_GBS),
                    mean_U_m=float(u_m.mean()), mean_C_m=float(c_m.mean()), mean_U_s=float(u_s.mean()))
    log(f"roofline: {roofline}")

    # ---- batched form on the same scans
    batched = None
    if not args.no_batched:
        bg, bdt, bst, bprof, (caps, reps) = run_batched(db, torch, gdef, ks, dev, args.warmup, args.steps, tuning,
                                                          args.batch_scans)
        bupd = sum(s.as_dict()["voxel_updates"] for s in bst)
        batched = dict(value=bupd / bdt, unit="voxel-updates/s", scans_per_s=args.steps / bdt,
                       scans_per_launch=args.batch_scans, ms_per_scan=bdt * 1e3 / args.steps,
                       graph_captures=caps, graph_replays=reps, speedup_vs_plain=(bupd / bdt) / value,
                       bit_exact_vs_plain=planes_equal(torch, bg, plain_grid),
                       comparison="both planes word for word on the device (torch.equal)")
        bg.close()
        plain_grid.close()
        log(f"batched: {batched}")
        torch.cuda.empty_cache()

    mres = None
    if not args.no_mres:
        mres = run_mres(db, torch, synth, ks, tuning)
        log(f"mres: {mres}")
        torch.cuda.empty_cache()

    lat = plain_latency(db, torch, gdef, ks, dev, args.latency_scans, tuning) if args.latency_scans else []
    latency = dict(plain_p50_ms=pct(lat, 50), plain_p99_ms=pct(lat, 99), plain_scans=len(lat),
                   plain_definition="integrate_scan call to sync return, one scan at a time, scans 0.. of the "
                                    "sequence in order on a fresh grid (none repeated)")
    torch.cuda.empty_cache()

    served = None
    if not args.no_serve:
        served = run_serve(db, torch, args.serve_seconds, args.serve_warmup, args.serve_rate, args.serve_robots)
        latency.update(served_p50_ms=served["p50_ms"], served_p99_ms=served["p99_ms"],
                       served_definition="scheduled arrival to observed completion, Poisson arrivals")
        log(f"served: {served}")

    c4 = None
    if args.c4_maps:
        torch.cuda.empty_cache()
        c4 = run_c4(db, torch, ks, args.c4_maps, synth.CONFIGS[4]["scans"], tuning)
        log(f"c4: {c4}")

    cpu = None if args.no_cpu else cpu_baseline(gdef, scans[: min(len(scans), 80)], kparams)

    mean_pts = float(np.mean([int(p.shape[0]) for _, p in scans]))
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "voxel-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": synth.CONFIGS[cfg]["name"], "grid": list(gdef["dims"]),
                   "voxel_size_m": round(gdef["voxel_size"], 6), "mean_points_per_scan": mean_pts,
                   "kernel": ("K=11 (11^3), cube26 bins" if args.kernel == "workload" else
                              "K=21 (21^3), 40x40 azimuth/elevation bins (the paper's kernel set)")
                             + ", r_s^2=9, T=5, H_max=65535, first-return dedup",
                   "form": "plain: one scan per launch sequence, points resident in HBM",
                   "tuning": tuning},
        "scans_per_s": args.steps / dt,
        "mean_integrated_per_scan": float(np.mean([s["n_integrated"] for s in sd])),
        "windows_applied_frac": applied_frac,
        "timed_scans": [args.warmup, args.warmup + args.steps - 1],
        "batched": batched,
        "mesh_export": mesh,
        "accuracy": accuracy,
        "mres": mres,
        "deskew": deskew,
        "latency_ms": latency,
        "served": served,
        "c4_batching": c4,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernel_source_hash": kernel_source_hash(),
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
