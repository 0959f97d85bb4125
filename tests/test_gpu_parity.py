"""GPU parity: the HIP library against the CPU oracle, bit for bit (tolerance 0).

Every integer the method produces (masks, counters, signs, statistics) must be
identical; the result is unique because every update commutes (Sec. III-C).
All calls go through the C ABI via the Python binding.
"""
import json
import os

import numpy as np
import pytest

from oracle import brute
from synth import scene as synth
from tests import parity as P

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]


@pytest.fixture(scope="module")
def db():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2509_20081_amd as db
    return db


def tiny_scans(seed, K, dims, n_scans=3, n_max=200, nan_frac=0.03):
    rng = np.random.default_rng(seed)
    R = (K - 1) // 2
    c = np.array(dims, dtype=np.float64) / 2.0
    out = []
    for _ in range(n_scans):
        pose = synth.random_pose(rng, c - 2, c + 2)
        n = int(rng.integers(1, n_max))
        half = np.array(dims) / 2.0 - R + 1.5
        pts = synth.random_cloud(rng, n, -half, half)
        pts[rng.random(n) < nan_frac] = np.nan
        k = int(rng.integers(0, 5))
        if k:
            pts = np.concatenate([pts, pts[rng.integers(0, n, size=k)]])
        out.append((pose, pts))
    return out


TINY_CASES = [
    dict(seed=1, K=3, dims=(24, 24, 24), binning="cube26", shadow_r2=1, hit_threshold=1),
    dict(seed=2, K=5, dims=(40, 33, 29), binning="cube26", shadow_r2=4, hit_threshold=2, hit_max=3),
    dict(seed=3, K=11, dims=(70, 45, 37), binning="cube26", shadow_r2=9, hit_threshold=5),
    dict(seed=4, K=11, dims=(64, 64, 64), binning="azel", shadow_r2=9, hit_threshold=3, hit_max=255),
    dict(seed=5, K=7, dims=(50, 50, 50), binning="azel", bins_az=8, bins_el=5, shadow_r2=6, metric="l1"),
    dict(seed=6, K=11, dims=(48, 48, 48), binning="cube26", shadow_r2=16, hit_threshold=0, dedup=False),
    dict(seed=7, K=21, dims=(60, 60, 60), binning="cube26", shadow_r2=25, hit_threshold=2),
    dict(seed=8, K=37, dims=(80, 70, 75), binning="cube26", shadow_r2=36, hit_threshold=4),
    dict(seed=9, K=5, dims=(30, 30, 30), binning="cube26", shadow_r2=-1),
    dict(seed=10, K=11, dims=(48, 48, 40), binning="cube26", shadow_r2=9, hit_threshold=2, shadow_model="cone",
         cone_deg=35.0),
    dict(seed=11, K=7, dims=(44, 40, 36), binning="azel", bins_az=8, bins_el=5, shadow_r2=9, shadow_model="cone",
         cone_deg=50.0),
    # within the tile strategy's limits: the L1 metric (its mask table is even in dy and dz too), K = 9 with a
    # small counter ceiling, grid sides that are not multiples of the 32 x 16 x 8 tile
    dict(seed=12, K=7, dims=(45, 38, 27), binning="cube26", shadow_r2=4, hit_threshold=2, metric="l1"),
    dict(seed=13, K=9, dims=(53, 35, 41), binning="cube26", shadow_r2=9, hit_threshold=3, hit_max=7),
]

TUNINGS = [
    dict(strategy="brick", brick=(32, 8, 8), block_threads=256),
    dict(strategy="brick", brick=(16, 16, 8), block_threads=256),
    dict(strategy="brick", brick=(64, 16, 8), block_threads=512),
    dict(strategy="brick", brick=(16, 8, 8), block_threads=256, apply_blocks=7),
    dict(strategy="brick", brick=(32, 16, 8), block_threads=256, chunk=3),      # many split bricks
    dict(strategy="brick", brick=(32, 16, 16), block_threads=512, chunk=None),  # never split
    dict(strategy="atomic", block_threads=256),
    dict(strategy="sort"),
    dict(strategy="sort", chunk=7),                                              # rounds of 7 returns
    dict(strategy="tile"),
]


@pytest.mark.parametrize("case", TINY_CASES, ids=lambda c: f"seed{c['seed']}_K{c['K']}_{c['binning']}")
@pytest.mark.parametrize("tuning", TUNINGS,
                         ids=lambda t: f"{t['strategy']}{t.get('brick', '')}_c{t.get('chunk', 'd')}")
def test_tiny_grids_match_oracle(db, case, tuning):
    case = dict(case)
    seed, K, dims = case.pop("seed"), case.pop("K"), case.pop("dims")
    # unique-word counters are exact only when no brick is split over work units
    traffic = tuning["strategy"] == "brick" and "chunk" not in tuning
    o, g, _ = P.make_pair(dims, 1.0, (0.0, 0.0, 0.0), count_traffic=traffic, kernel_size=K, **case)
    try:
        g.set_tuning(**tuning)
    except db.DbtsdfError:
        # documented: the largest brick shapes cannot hold the tiles for K = 37,
        # and the tile strategy takes K <= 17
        if tuning["strategy"] == "tile":
            n_bins = 26 if case["binning"] == "cube26" else case.get("bins_az", 40) * case.get("bins_el", 40)
            assert K > 11 or n_bins > 31 or case.get("shadow_r2", 9) > 9
            pytest.skip("the tile strategy takes K <= 11, at most 31 bins, r_s^2 <= 9")
        assert K == 37 and tuning["brick"] == (32, 16, 16)
        pytest.skip("brick shape too small in LDS for this kernel radius")
    m, p = o.new_grid()
    for i, (pose, pts) in enumerate(tiny_scans(seed, K, dims)):
        ref = o.integrate(m, p, pose, pts, count_traffic=traffic)
        st = g.integrate(pose, P.to_device(pts))
        g.sync()
        P.assert_stats_equal(st.as_dict(), ref, traffic=traffic, what=f"scan {i}")
        gm, gp = P.gpu_planes(g)
        P.assert_grids_equal(gm, gp, m, p, what=f"scan {i}")


def test_hand_worked_scan_on_gpu(db):
    root = os.path.dirname(os.path.abspath(__file__))
    gold = json.load(open(os.path.join(root, "golden", "hand_worked_scan.json")))
    ks = db.KernelSet(**{k: v for k, v in gold["kernel"].items() if k in P.KW_KERNEL})
    gk = {k: v for k, v in gold["kernel"].items() if k in P.KW_GRID}
    g = db.Grid(gold["grid"]["dims"], gold["grid"]["voxel_size"], gold["grid"]["origin"], ks, **gk)
    pose = np.eye(4, dtype=np.float32)
    pose[:3, 3] = gold["pose_translation"]
    g.integrate(pose, np.array([gold["point"]], np.float32))
    g.sync()
    m, p = g.read_voxels()
    for (x, y, z), want in gold["expect"]["mask"]:
        assert m[z, y, x] == want
    sh = {tuple(v) for v in gold["expect"]["shadow_voxels"]}
    for z, y, x in np.ndindex(*p.shape):
        want = gold["expect"]["packed_in_shadow"] if (x, y, z) in sh else gold["expect"]["packed_elsewhere"]
        assert p[z, y, x] == want
    d = g.read_distance()
    for (x, y, z), want in gold["expect"]["distance"]:
        assert d[z, y, x] == want
    sub = g.read_distance((7, 7, 7), (10, 9, 8))
    assert sub.shape == (1, 2, 3) and np.array_equal(sub, d[7:8, 7:9, 7:10])


def test_edge_cases(db):
    dims, K = (32, 32, 32), 5
    o, g, _ = P.make_pair(dims, 1.0, (0, 0, 0), count_traffic=True, kernel_size=K, shadow_r2=4, hit_threshold=1)
    m, p = o.new_grid()
    eye = np.eye(4, dtype=np.float32)
    eye[:3, 3] = 16.0
    R = (K - 1) // 2
    cases = [
        np.zeros((0, 3), np.float32),                                           # empty scan
        np.full((7, 3), np.nan, np.float32),                                    # all invalid
        np.array([[100, 0, 0], [0, -100, 0], [0, 0, 1e30]], np.float32),        # all out of bounds
        np.zeros((5, 3), np.float32),                                           # zero range
        np.array([[0.25, 0.25, 0.25]], np.float32),                            # single point next to the sensor
        np.array([[R - 16.0, 0, 0], [R - 16.0 - 0.01, 0, 0],                   # exactly R from the face / just inside the halo
                  [dims[0] - 1 - R - 16.0 + 0.99, 0, 0], [dims[0] - R - 16.0, 0, 0]], np.float32),
        np.repeat(np.array([[3.3, -2.2, 1.1]], np.float32), 50, axis=0),       # 50 returns in one voxel
        np.array([[np.inf, 0, 0], [1, np.nan, 0], [2, 2, 2], [-2, -2, -2]], np.float32),
    ]
    for i, pts in enumerate(cases):
        ref = o.integrate(m, p, eye, pts, count_traffic=True)
        st = g.integrate(eye, P.to_device(pts) if len(pts) else pts)
        g.sync()
        P.assert_stats_equal(st.as_dict(), ref, traffic=True, what=f"case {i}")
        gm, gp = P.gpu_planes(g)
        P.assert_grids_equal(gm, gp, m, p, what=f"case {i}")


def test_host_points_and_permutation(db):
    """Host (numpy) points equal device points; any permutation of a scan gives the same grid."""
    dims, K = (64, 64, 48), 11
    pose, pts = next(synth.config_scans(1, 0, [0]))
    pts = pts[:4000]
    pose = pose.copy()
    pose[:3, 3] = [32 * 0.1 + 0.03, 32 * 0.1 - 0.07, 24 * 0.1]
    grids = []
    rng = np.random.default_rng(0)
    for order, host in ((None, False), (rng.permutation(len(pts)), False), (rng.permutation(len(pts)), True)):
        o, g, _ = P.make_pair(dims, 0.1, (0, 0, 0), kernel_size=K, dedup=False)
        q = pts if order is None else pts[order]
        g.integrate(pose, q if host else P.to_device(q))
        g.sync()
        grids.append(P.gpu_planes(g))
    m, p = o.new_grid()
    o.integrate(m, p, pose, pts)
    for gm, gp in grids:
        P.assert_grids_equal(gm, gp, m, p, what="permutation")


def _config_grid_pair(db, cfg, count_traffic=False):
    gdef = synth.config_grid(cfg)
    return P.make_pair(gdef["dims"], gdef["voxel_size"], gdef["origin"], count_traffic=count_traffic,
                       **synth.KERNEL_DEFAULTS), gdef


def test_config1_full_grid(db):
    """16x1024 scan into 256^3 @ 0.1 m: whole grid against the oracle."""
    (o, g, _), gdef = _config_grid_pair(db, 1, count_traffic=True)
    m, p = o.new_grid()
    for pose, pts in synth.config_scans(1, 0, [0]):
        ref = o.integrate(m, p, pose, pts, count_traffic=True)
        st = g.integrate(pose, P.to_device(pts))
        g.sync()
        P.assert_stats_equal(st.as_dict(), ref, traffic=True, what="c1")
    gm, gp = P.gpu_planes(g)
    P.assert_grids_equal(gm, gp, m, p, what="c1")
    assert ref["n_integrated"] > 5000


PAPER_KERNEL = dict(kernel_size=21, binning="azel", bins_az=40, bins_el=40, shadow_r2=9)


@pytest.mark.parametrize("tuning", [dict(strategy="atomic"), dict(strategy="brick", brick=(32, 8, 8), block_threads=256),
                                    dict(strategy="sort")],
                         ids=["atomic", "brick32x8x8", "sort"])
def test_paper_kernel_set_config1(db, tuning):
    """The paper's own kernel set (Sec. III-B: K = 21, 40 x 40 direction bins) on the 16x1024 scan
    into 256^3 @ 0.1 m: whole grid and statistics against the oracle."""
    gdef = synth.config_grid(1)
    kw = dict(synth.KERNEL_DEFAULTS)
    kw.update(PAPER_KERNEL)
    o, g, _ = P.make_pair(gdef["dims"], gdef["voxel_size"], gdef["origin"], **kw)
    g.set_tuning(**tuning)
    m, p = o.new_grid()
    for pose, pts in synth.config_scans(1, 0, [0]):
        ref = o.integrate(m, p, pose, pts)
        st = g.integrate(pose, P.to_device(pts))
        g.sync()
        P.assert_stats_equal(st.as_dict(), ref, traffic=False, what="c1 paper kernel")
    gm, gp = P.gpu_planes(g)
    P.assert_grids_equal(gm, gp, m, p, what="c1 paper kernel")
    assert ref["n_integrated"] > 3000


@pytest.mark.parametrize("strategy", ["atomic", "brick", "sort", "tile"])
def test_plain_calls_over_the_ring(db, strategy):
    """20 plain calls into one grid (more than the 16 ring slots, so every slot's descriptors, and with the
    brick strategy its captured graph, are used again), eager work between calls: statistics and grid
    checked after every call."""
    import torch
    dims = (64, 64, 48)
    o, g, _ = P.make_pair(dims, 0.1, (0.0, 0.0, 0.0), **synth.KERNEL_DEFAULTS)
    g.set_tuning(strategy=strategy)
    m, p = o.new_grid()
    rng = np.random.default_rng(7)
    for k in range(20):
        pose = synth.random_pose(rng, np.array(dims) * 0.05 - 0.5, np.array(dims) * 0.05 + 0.5)
        pts = synth.random_cloud(rng, int(rng.integers(200, 3000)), -np.array(dims) * 0.04, np.array(dims) * 0.04)
        ref = o.integrate(m, p, pose, pts)
        st = g.integrate(pose, P.to_device(pts))
        _ = torch.ones(4096, device="cuda").cumsum(0)[-1].item()   # unrelated eager work
        g.sync()
        P.assert_stats_equal(st.as_dict(), ref, traffic=False, what=f"call {k}")
        gm, gp = P.gpu_planes(g)
        P.assert_grids_equal(gm, gp, m, p, what=f"call {k}")


@pytest.mark.parametrize("hit", [(2, 3), (1, 1), (5, 65535)])
@pytest.mark.parametrize("dedup", [True, False])
@pytest.mark.parametrize("strategy", ["atomic", "sort", "tile"])
def test_dense_neighbouring_returns_saturate_exactly(db, hit, dedup, strategy):
    """Returns one voxel apart in input order (neighbours share most of their shadows, so the per-point
    kernel adds shared shadow cells once with their count) on a small hit cap: counters, signs and masks
    match the oracle scan after scan, through saturation."""
    T, H = hit
    dims = (32, 32, 32)
    o, g, _ = P.make_pair(dims, 1.0, (0.0, 0.0, 0.0), kernel_size=7, binning="cube26", shadow_r2=9,
                          hit_threshold=T, hit_max=H, dedup=dedup)
    g.set_tuning(strategy=strategy)
    m, p = o.new_grid()
    rng = np.random.default_rng(23)
    sensor = np.array([16.5, 16.5, 16.5])
    for i in range(6):
        pose = np.eye(4, dtype=np.float32)
        pose[:3, 3] = sensor + rng.uniform(-0.4, 0.4, 3)
        # a patch of a wall and a patch of a floor, walked row by row, plus repeats
        u, v = np.meshgrid(np.arange(-6, 7), np.arange(-6, 7), indexing="ij")
        wall = np.stack([np.full(u.size, 9.3), u.ravel() + 0.2, v.ravel() - 0.1], 1)
        floor = np.stack([u.ravel() - 0.3, v.ravel() + 0.4, np.full(u.size, -8.6)], 1)
        pts = np.concatenate([wall, floor, wall[::7]]) + rng.normal(0, 0.05, (2 * u.size + len(wall[::7]), 3))
        pts = pts.astype(np.float32)
        ref = o.integrate(m, p, pose, pts)
        st = g.integrate(pose, P.to_device(pts))
        g.sync()
        P.assert_stats_equal(st.as_dict(), ref, traffic=False, what=f"scan {i}")
        gm, gp = P.gpu_planes(g)
        P.assert_grids_equal(gm, gp, m, p, what=f"scan {i}")
    assert ref["n_integrated"] > 200


@pytest.mark.parametrize("strategy", ["atomic", "brick", "sort", "tile"])
def test_profiling_period_mixes_call_forms(db, strategy):
    """Profiling every 3rd call: timed calls (split launch) and untimed calls (one graph) interleave
    over the ring; the totals count the timed calls only and every call matches the oracle."""
    dims = (64, 64, 48)
    o, g, _ = P.make_pair(dims, 0.1, (0.0, 0.0, 0.0), **synth.KERNEL_DEFAULTS)
    g.set_tuning(strategy=strategy)
    with pytest.raises(ValueError):
        g.set_profiling(True, every=0)
    g.set_profiling(True, every=3)
    m, p = o.new_grid()
    rng = np.random.default_rng(11)
    n_calls = 19
    for k in range(n_calls):
        pose = synth.random_pose(rng, np.array(dims) * 0.05 - 0.5, np.array(dims) * 0.05 + 0.5)
        pts = synth.random_cloud(rng, int(rng.integers(200, 3000)), -np.array(dims) * 0.04, np.array(dims) * 0.04)
        ref = o.integrate(m, p, pose, pts)
        st = g.integrate(pose, P.to_device(pts))
        g.sync()
        P.assert_stats_equal(st.as_dict(), ref, traffic=False, what=f"call {k}")
    gm, gp = P.gpu_planes(g)
    P.assert_grids_equal(gm, gp, m, p, what="after the profiled run")
    pr = g.read_profile()
    assert pr["calls"] == pr["applies"] == (n_calls + 2) // 3   # call indices 0, 3, ..., 18
    assert 0.0 < pr["apply_ms"] <= pr["call_ms"]
    g.set_profiling(False)
    assert g.read_profile()["calls"] == 0


@pytest.mark.parametrize("every", [2, 3, 7])
@pytest.mark.parametrize("host", [False, True])
def test_sequential_downsampling(db, every, host):
    """DS = every (Sec. IV-B): the grid and statistics equal the oracle's on every `every`-th return."""
    dims = (96, 96, 64)
    origin = (-4.8, -4.8, -1.2)
    o, g, _ = P.make_pair(dims, 0.1, origin, **synth.KERNEL_DEFAULTS)
    m, p = o.new_grid()
    pose, full = next(synth.config_scans(1, 0, [0]))
    for k in range(2):
        pts = full[: 9000 + 3037 * k]
        ref = o.integrate(m, p, pose, np.ascontiguousarray(pts[::every]))
        st = g.integrate(pose, pts if host else P.to_device(pts), every=every)
        g.sync()
        P.assert_stats_equal(st.as_dict(), ref, traffic=False, what=f"DS={every} scan {k}")
    gm, gp = P.gpu_planes(g)
    P.assert_grids_equal(gm, gp, m, p, what=f"DS={every}")
    with pytest.raises(db.DbtsdfError):
        g.integrate(pose, P.to_device(pts), every=0)


def test_config2_full_grid_three_scans(db):
    """1024x1024x256 @ 0.05 m, 64x1024 scans along the trajectory: whole grid after 3 scans."""
    (o, g, _), gdef = _config_grid_pair(db, 2, count_traffic=True)
    m, p = o.new_grid()
    for k, (pose, pts) in enumerate(synth.config_scans(2, 0, [0, 1, 2])):
        ref = o.integrate(m, p, pose, pts, count_traffic=True)
        st = g.integrate(pose, P.to_device(pts))
        g.sync()
        P.assert_stats_equal(st.as_dict(), ref, traffic=True, what=f"c2 scan {k}")
    gm, gp = P.gpu_planes(g)
    P.assert_grids_equal(gm, gp, m, p, what="c2")


def _invariants_torch(g, T, H):
    import torch
    m, pk = g.mask_tensor, g.packed_tensor
    assert int(((m & (m + 1)) != 0).sum()) == 0
    assert int((pk & 0x7FFF0000).sum()) == 0
    h = pk & 0xFFFF
    assert int((h > H).sum()) == 0
    occ = pk >= 0                                  # bit 31 clear
    want = (h >= T) if (1 <= T <= H) else torch.zeros_like(occ)
    assert bool(torch.equal(occ, want))


def test_config2_bench_launch_sampled(db):
    """The plain form as the benchmark runs it (default tuning, device points), 24 scans;
    sampled voxels computed one by one from the closed form, plus whole-grid invariants."""
    (o, g, _), gdef = _config_grid_pair(db, 2)
    dims, K = gdef["dims"], 11
    integrated = []
    for pose, pts in synth.config_scans(2, 0, range(24)):
        g.integrate(pose, P.to_device(pts))
        integrated.append(P.integrated_of(o, pose, pts, dims, K))
    g.sync()
    rng = np.random.default_rng(2)
    smp = P.sample_voxels(rng, dims, K, integrated)
    sm, sp = brute.sampled_voxels(smp, dims, K, integrated, 9, 5, 65535)
    gm, gp = P.gpu_planes(g)
    P.assert_grids_equal(gm[smp[:, 2], smp[:, 1], smp[:, 0]], gp[smp[:, 2], smp[:, 1], smp[:, 0]], sm, sp,
                         what="c2 sampled")
    _invariants_torch(g, 5, 65535)


def test_config3_sampled(db):
    """2048x2048x512 @ 0.02 m (2^31 voxels, 17 GB): two 128x2048 scans, sampled voxels."""
    import torch
    gdef = synth.config_grid(3)
    ks = db.KernelSet(kernel_size=11, binning="cube26", shadow_r2=9)
    g = db.Grid(gdef["dims"], gdef["voxel_size"], gdef["origin"], ks, planes="torch")
    dims, K = gdef["dims"], 11
    integrated = []
    for pose, pts in synth.config_scans(3, 0, [0, 1]):
        g.integrate(pose, P.to_device(pts))
        integrated.append(_front_end_big(pose, pts, gdef, K))
    g.sync()
    rng = np.random.default_rng(3)
    smp = P.sample_voxels(rng, dims, K, integrated, n_near=2000, n_any=500)
    sm, sp = brute.sampled_voxels(smp, dims, K, integrated, 9, 5, 65535)
    idx = torch.from_numpy(smp[:, 2] * dims[1] * dims[0] + smp[:, 1] * dims[0] + smp[:, 0]).cuda()
    gm = g.mask_tensor.view(-1)[idx].cpu().numpy().view(np.uint32)
    gp = g.packed_tensor.view(-1)[idx].cpu().numpy().view(np.uint32)
    P.assert_grids_equal(gm, gp, sm, sp, what="c3 sampled")
    _invariants_torch(g, 5, 65535)
    g.close()
    del g
    torch.cuda.empty_cache()


def centred(cfg, map_id, side):
    """A side^3 grid with the same centre and voxel size as the configuration's map."""
    gdef = synth.config_grid(cfg, map_id)
    vs = gdef["voxel_size"]
    org = tuple(float(np.float32(o + (d - side) * vs / 2.0)) for o, d in zip(gdef["origin"], gdef["dims"]))
    return (side, side, side), vs, org


def _front_end_big(pose, pts, gdef, K):
    vox, bins, status = brute.front_end(pose, pts, gdef["dims"], gdef["voxel_size"], gdef["origin"], K)
    keep = brute.survivors(vox, status, gdef["dims"])
    return vox[keep], bins[keep]


def test_batch_and_graph_replays_equal_plain(db):
    """Batched launches (with and without graphs, same grid several times, host and device
    points) equal the plain per-scan form and the oracle; every graph replay is checked."""
    import torch
    maps = []
    for mid in range(3):
        side = min(synth.config_grid(4, mid)["dims"][0], 256)
        dims, vs, org = centred(4, mid, side)
        maps.append((dims, vs, org, list(synth.config_scans(4, mid, range(4)))))
    plain, batched_g, batched_n = [], [], []
    for dims, vs, org, scans in maps:
        _, g, _ = P.make_pair(dims, vs, org, **synth.KERNEL_DEFAULTS)
        for pose, pts in scans:
            g.integrate(pose, P.to_device(pts))
        g.sync()
        plain.append(P.gpu_planes(g))
    # graph-replayed and directly launched batches in lockstep: every replay is
    # compared with the direct launches, with eager work in between
    bg_, bn_ = db.Batch(use_graph=True), db.Batch(use_graph=False)
    grids_g = [P.make_pair(d, vs, org, **synth.KERNEL_DEFAULTS)[1] for d, vs, org, _ in maps]
    grids_n = [P.make_pair(d, vs, org, **synth.KERNEL_DEFAULTS)[1] for d, vs, org, _ in maps]
    for rnd in range(4):              # 4 batches: one scan of every map each, plus a repeat
        for b, grids in ((bg_, grids_g), (bn_, grids_n)):
            items = [(grids[i], maps[i][3][rnd][0], P.to_device(maps[i][3][rnd][1])) for i in range(3)]
            if rnd == 3:              # host points path
                items = [(g_, pose, pts.cpu().numpy()) for g_, pose, pts in items]
            b.integrate(items)
            b.sync()
            torch.cuda.synchronize()
            _ = torch.ones(1024, device="cuda").sum().item()   # unrelated eager work between replays
        for i in range(3):
            P.assert_grids_equal(*P.gpu_planes(grids_g[i]), *P.gpu_planes(grids_n[i]), what=f"replay {rnd} map {i}")
    batched_g.extend(P.gpu_planes(g_) for g_ in grids_g)
    batched_n.extend(P.gpu_planes(g_) for g_ in grids_n)
    caps, reps = bg_.graph_stats()
    assert reps == 4 and caps <= 4   # at most one graph per ring slot used
    caps_n, reps_n = bn_.graph_stats()
    assert reps_n == 0 and caps_n == 0
    for i in range(3):
        P.assert_grids_equal(*batched_g[i], *plain[i], what=f"graph batch map {i}")
        P.assert_grids_equal(*batched_n[i], *plain[i], what=f"batch map {i}")
    # one more: all scans of all maps in a single launch, against the oracle
    b = db.Batch(use_graph=True)
    pairs = [P.make_pair(d, vs, org, **synth.KERNEL_DEFAULTS) for d, vs, org, _ in maps]
    items = [(pairs[i][1], pose, P.to_device(pts)) for i in range(3) for pose, pts in maps[i][3]]
    stats = b.integrate(items)
    b.sync()
    k = 0
    for i, (o, g, _) in enumerate(pairs):
        m, p = o.new_grid()
        for pose, pts in maps[i][3]:
            ref = o.integrate(m, p, pose, pts)
            P.assert_stats_equal(stats[k].as_dict(), ref, what=f"batch stats {k}")
            k += 1
        P.assert_grids_equal(*P.gpu_planes(g), m, p, what=f"single-launch batch map {i}")


def test_autotune_keeps_result_identical(db):
    (o, g, _), gdef = _config_grid_pair(db, 1)
    scans = [(pose, P.to_device(pts)) for pose, pts in synth.config_scans(1, 0, [0])]
    tun = g.autotune(scans, True)
    assert tun["strategy"] in ("brick", "atomic", "sort", "tile")
    m, p = o.new_grid()
    for pose, pts in synth.config_scans(1, 0, [0]):
        o.integrate(m, p, pose, pts)
        g.integrate(pose, P.to_device(pts))
    g.sync()
    P.assert_grids_equal(*P.gpu_planes(g), m, p, what="tuned grid")


def test_server_mix_equals_alone(db):
    """Scans of several robots served concurrently equal each robot's scans integrated alone."""
    from paper_2509_20081_amd.serve import Server
    ks = db.KernelSet(kernel_size=11, binning="cube26", shadow_r2=9)
    robots = []
    for rid in range(4):
        dims, vs, org = centred(5, rid, 192)
        robots.append((dict(voxel_size=vs, origin=org), list(synth.config_scans(5, rid, range(5)))))
    srv = Server(n_streams=2, max_batch_scans=8)
    ids = [srv.add_map(dims, r[0]["voxel_size"], r[0]["origin"], ks) for r in robots]
    for k in range(5):
        for rid, (gdef, scans) in enumerate(robots):
            srv.submit(ids[rid], scans[k][0], scans[k][1])
    srv.drain()
    done = srv.poll(100)
    assert len(done) == 20 and all(c["status"] == 0 for c in done)
    assert all(c["t_done_ns"] >= c["t_launch_ns"] >= c["t_arrival_ns"] for c in done)
    for rid, (gdef, scans) in enumerate(robots):
        alone = db.Grid(dims, gdef["voxel_size"], gdef["origin"], ks)
        for pose, pts in scans:
            alone.integrate(pose, pts)
        alone.sync()
        a = alone.read_voxels()
        view = srv.map_grid(ids[rid], dims, ks)
        s = view.read_voxels()
        P.assert_grids_equal(s[0], s[1], a[0], a[1], what=f"robot {rid}")
    srv.close()


def test_server_admission_by_memory(db):
    from paper_2509_20081_amd.serve import Server
    ks = db.KernelSet(kernel_size=11)
    per_map = 128 ** 3 * 8
    srv = Server(memory_budget=int(2.5 * per_map))
    a = srv.try_add_map((128,) * 3, 0.05, (0, 0, 0), ks)
    b = srv.try_add_map((128,) * 3, 0.05, (0, 0, 0), ks)
    c = srv.try_add_map((128,) * 3, 0.05, (0, 0, 0), ks)
    assert a is not None and b is not None and c is None
    srv.remove_map(a)
    assert srv.try_add_map((128,) * 3, 0.05, (0, 0, 0), ks) is not None
    adm, bud = srv.memory()
    assert adm == 2 * per_map and bud == int(2.5 * per_map)
    srv.close()


def test_readout_and_restore(db):
    dims = (40, 40, 40)
    o, g, ks = P.make_pair(dims, 1.0, (0, 0, 0), kernel_size=5, shadow_r2=4, hit_threshold=2)
    for pose, pts in tiny_scans(11, 5, dims):
        g.integrate(pose, P.to_device(pts))
    g.sync()
    m, p = g.read_voxels()
    gm, gp = P.gpu_planes(g)
    assert np.array_equal(m, gm) and np.array_equal(p, gp)
    d = g.read_distance()
    pc = np.vectorize(lambda v: bin(int(v)).count("1"))(m)
    assert np.array_equal(d, np.where(p >> 31, pc, -pc))
    g2 = db.Grid(dims, 1.0, (0, 0, 0), ks, hit_threshold=2)
    g2.write_voxels(m, p)
    m2, p2 = g2.read_voxels()
    assert np.array_equal(m, m2) and np.array_equal(p, p2)
    bad = p.copy()
    bad.flat[0] = 0x00010000
    with pytest.raises(db.DbtsdfError):
        g2.write_voxels(m, bad)
    bad = m.copy()
    bad.flat[0] = 0x5
    with pytest.raises(db.DbtsdfError):
        g2.write_voxels(bad, p)
    with pytest.raises(db.DbtsdfError):
        g.read_voxels((0, 0, 0), (41, 1, 1))


@pytest.mark.parametrize("kernel", ["row", "generic"])
@pytest.mark.parametrize("strategy", ["atomic", "sort", "tile"])
def test_written_planes_integrate_every_window(db, strategy, kernel):
    """Planes written with zero masks at voxels whose windows were never stamped (not a state integration
    makes): returns landing there still get their whole eq. 4 window, as in the oracle; after a reset the
    grid integrates normally again."""
    dims = (48, 48, 40)
    kw = dict(synth.KERNEL_DEFAULTS)
    if kernel == "generic":
        kw.update(kernel_size=13)   # past the row kernel's tables: the generic per-point kernel
    if strategy == "tile" and kernel == "generic":
        pytest.skip("the tile strategy takes K <= 11")
    o, g, _ = P.make_pair(dims, 1.0, (0.0, 0.0, 0.0), **kw)
    g.set_tuning(strategy=strategy)
    rng = np.random.default_rng(17)
    pose = synth.random_pose(rng, np.array([20.0, 20.0, 16.0]), np.array([28.0, 28.0, 24.0]))
    pts = synth.random_cloud(rng, 600, -np.full(3, 12.0), np.full(3, 12.0))
    vox, _, st = o.front_end(pose, pts)
    m, p = o.new_grid()
    ok = vox[st == 0]
    m[ok[:, 2], ok[:, 1], ok[:, 0]] = 0          # "integrated" centres without their windows
    g.write_voxels(m, p)
    ref = o.integrate(m, p, pose, pts)
    assert ref["n_integrated"] > 100
    g.integrate(pose, P.to_device(pts))
    g.sync()
    gm, gp = P.gpu_planes(g)
    P.assert_grids_equal(gm, gp, m, p, what="after writing planes")
    g.reset()
    m, p = o.new_grid()
    for k in range(2):
        o.integrate(m, p, pose, pts)
        g.integrate(pose, P.to_device(pts))
    g.sync()
    gm, gp = P.gpu_planes(g)
    P.assert_grids_equal(gm, gp, m, p, what="after reset, twice")


def test_argument_errors_leave_grid_unchanged(db):
    dims = (24, 24, 24)
    o, g, ks = P.make_pair(dims, 1.0, (0, 0, 0), kernel_size=5)
    pose = np.eye(4, dtype=np.float32)
    pose[0, 3] = np.nan
    with pytest.raises(db.DbtsdfError):
        g.integrate(pose, np.ones((3, 3), np.float32))
    with pytest.raises(db.DbtsdfError):
        db.Grid((4, 24, 24), 1.0, (0, 0, 0), ks)
    with pytest.raises(db.DbtsdfError):
        db.Grid(dims, 0.0, (0, 0, 0), ks)
    with pytest.raises(db.DbtsdfError):
        db.Grid(dims, 1.0, (0, 0, 0), ks, hit_max=0)
    with pytest.raises(db.DbtsdfError):
        g.set_tuning(strategy="brick", brick=(48, 16, 8))
    with pytest.raises(db.DbtsdfError):
        g.set_tuning(strategy="brick", brick=(32, 8, 8), block_threads=512)
    gm, gp = P.gpu_planes(g)
    assert np.all(gm == 0xFFFFFFFF) and np.all(gp == 0x80000000)


def test_sort_strategy_batches_of_many_grids(db):
    """The sort strategy over one launch holding every scan of three maps of different sizes (the keys
    carry the grid index above the voxel bits), in rounds of 50 returns and in one round, against the
    oracle; statistics too."""
    maps = []
    for mid in range(3):
        side = min(synth.config_grid(4, mid)["dims"][0], 192)
        dims, vs, org = centred(4, mid, side)
        maps.append((dims, vs, org, list(synth.config_scans(4, mid, range(3)))))
    for chunk in (50, 0):
        pairs = [P.make_pair(d, vs, org, **synth.KERNEL_DEFAULTS) for d, vs, org, _ in maps]
        for _, g, _ in pairs:
            g.set_tuning(strategy="sort", chunk=chunk)
        b = db.Batch(use_graph=True)
        items = [(pairs[i][1], pose, P.to_device(pts)) for i in range(3) for pose, pts in maps[i][3]]
        stats = b.integrate(items)
        b.sync()
        assert b.graph_stats() == (0, 0)      # the sort strategy launches directly
        k = 0
        for i, (o, g, _) in enumerate(pairs):
            m, p = o.new_grid()
            for pose, pts in maps[i][3]:
                ref = o.integrate(m, p, pose, pts)
                P.assert_stats_equal(stats[k].as_dict(), ref, what=f"sort batch stats {k}")
                k += 1
            P.assert_grids_equal(*P.gpu_planes(g), m, p, what=f"sort batch map {i} chunk {chunk}")


def test_sort_strategy_config2_three_scans(db):
    """1024x1024x256 @ 0.05 m with the sort strategy (about 86 M pairs per scan on the empty grid): whole
    grid after three scans equals the oracle, and the per-point atomic strategy's grid."""
    (o, g, _), gdef = _config_grid_pair(db, 2)
    g.set_tuning(strategy="sort")
    m, p = o.new_grid()
    for k, (pose, pts) in enumerate(synth.config_scans(2, 0, [0, 1, 2])):
        ref = o.integrate(m, p, pose, pts)
        st = g.integrate(pose, P.to_device(pts))
        g.sync()
        P.assert_stats_equal(st.as_dict(), ref, traffic=False, what=f"c2 sort scan {k}")
    gm, gp = P.gpu_planes(g)
    P.assert_grids_equal(gm, gp, m, p, what="c2 sort")


def _turn(axis, ang):
    a = np.asarray(axis, float)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + np.sin(ang) * K + (1 - np.cos(ang)) * (K @ K)


def _sweep_times(rng, n):
    """Time fractions of n returns: increasing like a spinning sensor's, with exact ends and a few values
    outside the sweep (invalid returns)."""
    t = np.sort(rng.uniform(0, 1, n)).astype(np.float32)
    t[0], t[-1] = 0.0, 1.0
    t[7::97] = np.nan
    t[5::101] = 1.5
    t[3::103] = -0.25
    t[11::89] = np.float32(1.0) - np.float32(2 ** -24)
    return t


@pytest.mark.parametrize("mode", ["se3", "yaw"])
@pytest.mark.parametrize("strategy", ["atomic", "brick", "sort", "tile"])
def test_deskewed_sweeps_match_oracle(db, mode, strategy):
    """Motion-compensated sweeps (start and end poses, a time fraction per return) on a small grid: device
    and host points, DS = 1 and 2, invalid time fractions; statistics and whole grid equal the oracle's
    after every sweep."""
    import torch
    dims, vs = (48, 44, 40), 0.1
    o, g, _ = P.make_pair(dims, vs, (0.0, 0.0, 0.0), kernel_size=7, binning="cube26", shadow_r2=9, hit_threshold=2)
    g.set_tuning(**(dict(strategy="brick", brick=(32, 8, 8), block_threads=256) if strategy == "brick"
                    else dict(strategy=strategy)))
    m, p = o.new_grid()
    rng = np.random.default_rng(31 if mode == "se3" else 32)
    centre = np.array(dims) * vs / 2
    for k in range(4):
        P0 = synth.random_pose(rng, centre - 0.3, centre + 0.3)
        axis = (0.05, -0.03, 1.0) if mode == "yaw" else rng.normal(size=3)
        P1 = P0.copy()
        P1[:3, :3] = (_turn(axis, rng.uniform(-0.4, 0.4)) @ P0[:3, :3].astype(float)).astype(np.float32)
        P1[:3, 3] += rng.uniform(-0.2, 0.2, 3).astype(np.float32)
        pts = synth.random_cloud(rng, 1500, -centre * 0.9, centre * 0.9)
        times = _sweep_times(rng, len(pts))
        every = 1 if k % 2 == 0 else 2
        ref = o.integrate_deskew(m, p, P0, P1, pts[::every], times[::every], mode)
        if k == 3:
            st = g.integrate(P0, pts, every=every, pose_end=P1, times=times, deskew=mode)
        else:
            st = g.integrate(P0, P.to_device(pts), every=every, pose_end=P1,
                             times=torch.from_numpy(times).cuda(), deskew=mode)
        g.sync()
        P.assert_stats_equal(st.as_dict(), ref, traffic=False, what=f"sweep {k}")
        P.assert_grids_equal(*P.gpu_planes(g), m, p, what=f"sweep {k}")
        assert ref["n_invalid"] > 0 and ref["n_integrated"] > 100


def test_deskewed_config1_sweep(db):
    """The 16x1024 scan into 256^3 @ 0.1 m taken as a sweep that turns 4 degrees and moves 0.4 m, time
    fraction by column, integrated once per mode: whole grid and statistics against the oracle."""
    gdef = synth.config_grid(1)
    o, g, _ = P.make_pair(gdef["dims"], gdef["voxel_size"], gdef["origin"], **synth.KERNEL_DEFAULTS)
    m, p = o.new_grid()
    (pose, pts), = synth.config_scans(1, 0, [0])
    for k in range(2):
        P1 = pose.copy()
        P1[:3, :3] = (_turn((0.0, 0.0, 1.0), np.radians(4.0)) @ pose[:3, :3].astype(float)).astype(np.float32)
        P1[:3, 3] += np.array([0.4, 0.1, 0.0], np.float32)
        times = ((np.arange(len(pts)) % 1024) / 1023.0).astype(np.float32)
        mode = "se3" if k == 0 else "yaw"
        ref = o.integrate_deskew(m, p, pose, P1, pts, times, mode)
        st = g.integrate(pose, P.to_device(pts), pose_end=P1, times=P.to_device(times),
                         deskew=mode)
        g.sync()
        P.assert_stats_equal(st.as_dict(), ref, traffic=False, what=f"c1 sweep {k}")
        assert ref["n_integrated"] > 3000
    P.assert_grids_equal(*P.gpu_planes(g), m, p, what="c1 sweeps")


def test_sort_strategy_wide_keys(db):
    """The sort strategy with keys wider than 31 bits (64-bit sort): one launch holding two scans into the
    2048x2048x512 grid (2^31 voxels, 31 voxel bits) and a scan into a small grid (one grid bit above them),
    the c3 scans in two rounds (their pairs pass 2^28). Sampled c3 voxels against the brute-force closed
    form, the small grid whole against the oracle, and both grids' invariants."""
    import torch
    gdef = synth.config_grid(3)
    ks = db.KernelSet(kernel_size=11, binning="cube26", shadow_r2=9)
    big = db.Grid(gdef["dims"], gdef["voxel_size"], gdef["origin"], ks, planes="torch")
    big.set_tuning(strategy="sort")
    dims, K = gdef["dims"], 11
    sdims = (40, 36, 32)
    o, small, _ = P.make_pair(sdims, 0.1, (0.0, 0.0, 0.0), kernel_size=11, binning="cube26", shadow_r2=9)
    small.set_tuning(strategy="sort")
    rng = np.random.default_rng(41)
    centre = np.array(sdims) * 0.1 / 2
    spose = synth.random_pose(rng, centre - 0.2, centre + 0.2)
    spts = synth.random_cloud(rng, 3000, -centre * 0.9, centre * 0.9)
    items, integrated = [], []
    for pose, pts in synth.config_scans(3, 0, [0, 1]):
        items.append((big, pose, P.to_device(pts)))
        integrated.append(_front_end_big(pose, pts, gdef, K))
    items.append((small, spose, P.to_device(spts)))
    b = db.Batch(use_graph=False)
    stats = b.integrate(items)
    b.sync()
    m, p = o.new_grid()
    ref = o.integrate(m, p, spose, spts)
    P.assert_stats_equal(stats[2].as_dict(), ref, what="small grid in the wide-key batch")
    P.assert_grids_equal(*P.gpu_planes(small), m, p, what="small grid in the wide-key batch")
    smp = P.sample_voxels(np.random.default_rng(3), dims, K, integrated, n_near=2000, n_any=500)
    sm, sp = brute.sampled_voxels(smp, dims, K, integrated, 9, 5, 65535)
    idx = torch.from_numpy(smp[:, 2] * dims[1] * dims[0] + smp[:, 1] * dims[0] + smp[:, 0]).cuda()
    gm = big.mask_tensor.view(-1)[idx].cpu().numpy().view(np.uint32)
    gp = big.packed_tensor.view(-1)[idx].cpu().numpy().view(np.uint32)
    P.assert_grids_equal(gm, gp, sm, sp, what="c3 sampled, wide-key sort")
    _invariants_torch(big, 5, 65535)
    big.close()
    del big
    torch.cuda.empty_cache()


@pytest.mark.parametrize("strategy", ["atomic", "sort"])
@pytest.mark.parametrize("use_graph", [True, False])
def test_batched_sweeps_match_oracle(db, use_graph, strategy):
    """Motion-compensated sweeps of three grids of different sizes in one launch (the same grid twice),
    device and then host points, graph-replayed or direct: statistics and grids equal the oracle's."""
    import torch
    sizes = [(40, 36, 32), (56, 40, 48), (32, 32, 32)]
    pairs = [P.make_pair(d, 0.1, (0.0, 0.0, 0.0), kernel_size=7, binning="cube26", shadow_r2=9, hit_threshold=2)
             for d in sizes]
    refs = [o.new_grid() for o, _, _ in pairs]
    for _, g, _ in pairs:
        g.set_tuning(strategy=strategy)
    rng = np.random.default_rng(51)
    b = db.Batch(use_graph=use_graph)
    for rnd in range(3):
        items, plan = [], []
        for gi in (0, 1, 2, 0):
            dims = np.array(sizes[gi])
            centre = dims * 0.1 / 2
            P0 = synth.random_pose(rng, centre - 0.2, centre + 0.2)
            P1 = P0.copy()
            P1[:3, :3] = (_turn(rng.normal(size=3), rng.uniform(-0.3, 0.3)) @ P0[:3, :3].astype(float)).astype(np.float32)
            P1[:3, 3] += rng.uniform(-0.15, 0.15, 3).astype(np.float32)
            pts = synth.random_cloud(rng, int(rng.integers(300, 1500)), -centre * 0.9, centre * 0.9)
            times = _sweep_times(rng, len(pts))
            plan.append((gi, P0, P1, pts, times))
            if rnd < 2:
                items.append((pairs[gi][1], P0, P1, P.to_device(pts), torch.from_numpy(times).cuda()))
            else:
                items.append((pairs[gi][1], P0, P1, pts, times))
        stats = b.integrate_sweeps(items, deskew="se3" if rnd != 1 else "yaw")
        b.sync()
        for k, (gi, P0, P1, pts, times) in enumerate(plan):
            o = pairs[gi][0]
            ref = o.integrate_deskew(*refs[gi], P0, P1, pts, times, "se3" if rnd != 1 else "yaw")
            P.assert_stats_equal(stats[k].as_dict(), ref, what=f"round {rnd} scan {k}")
        for gi in range(3):
            P.assert_grids_equal(*P.gpu_planes(pairs[gi][1]), *refs[gi], what=f"round {rnd} grid {gi}")



@pytest.mark.parametrize("strategy", ["atomic", "sort"])
@pytest.mark.parametrize("kernel", [dict(kernel_size=13, binning="cube26", shadow_r2=9),
                                    dict(kernel_size=11, binning="azel", bins_az=40, bins_el=40, shadow_r2=9),
                                    dict(kernel_size=5, binning="azel", bins_az=256, bins_el=130, shadow_r2=4)],
                         ids=["K13", "azel1600", "azel33280"])
def test_revisits_with_generic_kernels(db, strategy, kernel):
    """Scans that land again in voxels earlier calls integrated (the same cloud from nearby poses, then a
    denser one), with kernel sets the row kernel does not cover: K = 13, 1600 bins (revisits skip their
    window, the flag beside the bin) and 33280 bins (the bin takes all 16 bits, no skip). Statistics and
    grid equal the oracle's after every call."""
    dims = (56, 52, 48)
    o, g, _ = P.make_pair(dims, 0.1, (0.0, 0.0, 0.0), hit_threshold=2, **kernel)
    g.set_tuning(strategy=strategy)
    m, p = o.new_grid()
    rng = np.random.default_rng(61)
    centre = np.array(dims) * 0.1 / 2
    cloud = synth.random_cloud(rng, 1200, -centre * 0.8, centre * 0.8)
    base = synth.random_pose(rng, centre - 0.1, centre + 0.1, max_angle=0.2)
    for k in range(4):
        pose = base.copy()
        pose[:3, 3] += rng.uniform(-0.02, 0.02, 3).astype(np.float32)
        pts = cloud if k < 3 else np.concatenate([cloud, synth.random_cloud(rng, 2000, -centre * 0.8, centre * 0.8)])
        ref = o.integrate(m, p, pose, pts)
        st = g.integrate(pose, P.to_device(pts))
        g.sync()
        P.assert_stats_equal(st.as_dict(), ref, traffic=False, what=f"call {k}")
        P.assert_grids_equal(*P.gpu_planes(g), m, p, what=f"call {k}")


def test_sweep_argument_errors_leave_grid_unchanged(db):
    """Bad sweeps are rejected before anything is enqueued: NULL times, an unknown mode, a non-finite end
    pose, time fractions on the other side of the points or of the wrong length; the grid is unchanged."""
    import ctypes as C
    import torch
    from paper_2509_20081_amd import _lib as L
    o, g, _ = P.make_pair((32, 32, 32), 0.1, (0.0, 0.0, 0.0), kernel_size=5, binning="cube26", shadow_r2=4)
    before = [x.copy() for x in P.gpu_planes(g)]
    pose = np.eye(4, dtype=np.float32)
    pose[:3, 3] = 1.6
    pts = P.to_device(synth.random_cloud(np.random.default_rng(3), 100, np.full(3, -1.0), np.full(3, 1.0)))
    times = torch.linspace(0, 1, 100, device="cuda")
    p0 = pose.ctypes.data_as(C.c_void_p)
    bad_end = pose.copy()
    bad_end[0, 3] = np.inf
    st = L.ScanStats()
    for end, tp, mode in ((pose, None, 0), (pose, times, 7), (bad_end, times, 0)):
        rc = L.lib().dbtsdf_integrate_scan_deskew(g._h, p0, end.ctypes.data_as(C.c_void_p), C.c_void_p(pts.data_ptr()),
                                                  None if tp is None else C.c_void_p(tp.data_ptr()), 100, 1, mode, 1,
                                                  C.byref(st))
        assert rc == 1   # DBTSDF_ERR_INVALID_ARG
    with pytest.raises(ValueError):
        g.integrate(pose, pts, pose_end=pose, times=times.cpu())          # host times, device points
    with pytest.raises(ValueError):
        g.integrate(pose, pts, pose_end=pose, times=times[:50])           # wrong length
    with pytest.raises(ValueError):
        g.integrate(pose, pts, pose_end=pose)                             # no times
    g.sync()
    after = P.gpu_planes(g)
    assert np.array_equal(after[0], before[0]) and np.array_equal(after[1], before[1])


def test_server_malformed_and_refused_scans(db):
    """Serving with bad input: a non-finite pose, an unknown or removed map and a full queue are refused at
    submit (nothing enqueued); scans with non-finite, zero-range and out-of-map returns, and an empty scan,
    complete with the oracle's statistics; the map equals the oracle's grid after them."""
    from paper_2509_20081_amd import _lib as L
    from paper_2509_20081_amd.serve import Server
    dims, vs, org = (64, 64, 48), 0.1, (0.0, 0.0, 0.0)
    ks = db.KernelSet(kernel_size=7, binning="cube26", shadow_r2=9)
    from oracle.oracle import Oracle
    o = Oracle(dims, vs, org, kernel_size=7, binning="cube26", shadow_r2=9)
    m, p = o.new_grid()
    srv = Server(n_streams=2, max_batch_scans=4, queue_capacity=64)
    mid = srv.add_map(dims, vs, org, ks)
    gone = srv.add_map((32, 32, 32), vs, org, ks)
    srv.remove_map(gone)
    rng = np.random.default_rng(71)
    pose = synth.random_pose(rng, np.array([3.0, 3.0, 2.2]), np.array([3.4, 3.4, 2.6]))
    bad_pose = pose.copy()
    bad_pose[1, 3] = np.nan
    scans = []
    for k in range(6):
        pts = synth.random_cloud(rng, 800, np.full(3, -3.5), np.full(3, 3.5))
        pts[::23] = np.nan                   # non-finite returns
        pts[5::31] = 0.0                     # zero range
        pts[7::29] *= 40.0                   # far outside the map
        scans.append(pts if k != 3 else pts[:0])   # one empty scan
    for bad in ((mid, bad_pose), (gone, pose), (mid + 7, pose)):
        with pytest.raises(L.DbtsdfError):
            srv.submit(bad[0], bad[1], scans[0])
    tickets = [srv.submit(mid, pose, pts) for pts in scans]
    srv.drain()
    done = {c["ticket"]: c for c in srv.poll(100)}
    assert sorted(done) == sorted(tickets)
    for t, pts in zip(tickets, scans):
        ref = o.integrate(m, p, pose, pts)
        assert done[t]["status"] == 0
        P.assert_stats_equal(done[t]["stats"], ref, traffic=False, what=f"ticket {t}")
    view = srv.map_grid(mid, dims, ks)
    got = view.read_voxels()
    P.assert_grids_equal(got[0], got[1], m, p, what="served map after malformed scans")
    # a full queue refuses with BUSY: 500 submits of tiny scans (microseconds each on the host) into a
    # queue of 2 that one stream drains a scan per launch sequence (tens of microseconds each)
    tiny = synth.random_cloud(rng, 8, np.full(3, -1.0), np.full(3, 1.0))
    srv2 = Server(n_streams=1, max_batch_scans=1, queue_capacity=2)
    mid2 = srv2.add_map(dims, vs, org, ks)
    busy = accepted = 0
    for _ in range(500):
        try:
            srv2.submit(mid2, pose, tiny)
            accepted += 1
        except L.DbtsdfError as e:
            assert e.status == 6   # DBTSDF_ERR_BUSY
            busy += 1
    srv2.drain()
    assert busy > 0 and accepted >= 2
    assert len(srv2.poll(1000)) == accepted
    srv2.close()
    srv.close()


def test_checkpoint_and_resume(db, tmp_path):
    """A grid saved after some scans and loaded into a new grid holds the same planes; integrating the
    remaining scans into the restored grid gives the oracle's grid for the whole sequence. A kernel set
    with other parameters is refused; the file loads without pickle."""
    from paper_2509_20081_amd.checkpoint import load_checkpoint, save_checkpoint
    dims = (48, 44, 40)
    o, g, ks = P.make_pair(dims, 0.1, (0.2, -0.1, 0.0), kernel_size=7, binning="cube26", shadow_r2=9,
                           hit_threshold=3, dedup=False)
    m, p = o.new_grid()
    rng = np.random.default_rng(81)
    centre = np.array((0.2, -0.1, 0.0)) + np.array(dims) * 0.1 / 2
    scans = [(synth.random_pose(rng, centre - 0.2, centre + 0.2),
              synth.random_cloud(rng, 900, -np.array(dims) * 0.04, np.array(dims) * 0.04)) for _ in range(5)]
    for pose, pts in scans[:3]:
        o.integrate(m, p, pose, pts)
        g.integrate(pose, P.to_device(pts))
    path = str(tmp_path / "grid.npz")
    save_checkpoint(path, g)
    with np.load(path, allow_pickle=False) as z:
        assert z["mask"].dtype == np.uint32 and z["mask"].shape == dims[::-1]
    g2 = load_checkpoint(path, planes="torch")
    assert g2.kernel_set.params == ks.params and g2.dims == dims
    P.assert_grids_equal(*P.gpu_planes(g2), m, p, what="restored")
    for pose, pts in scans[3:]:
        ref = o.integrate(m, p, pose, pts)
        st = g2.integrate(pose, P.to_device(pts))
        g2.sync()
        P.assert_stats_equal(st.as_dict(), ref, traffic=False, what="resumed scan")
    P.assert_grids_equal(*P.gpu_planes(g2), m, p, what="after resuming")
    with pytest.raises(ValueError):
        load_checkpoint(path, kernel_set=db.KernelSet(kernel_size=5, binning="cube26", shadow_r2=9))


def test_server_mixes_sweeps_and_plain_scans(db):
    """Three maps served with plain scans and motion-compensated sweeps of both modes interleaved: every
    completion carries the oracle's statistics and every map equals the oracle's grid."""
    from oracle.oracle import Oracle
    from paper_2509_20081_amd.serve import Server
    dims, vs = (48, 44, 40), 0.1
    kk = dict(kernel_size=7, binning="cube26", shadow_r2=9)
    ks = db.KernelSet(**kk)
    srv = Server(n_streams=2, max_batch_scans=4)
    origins = [(0.0, 0.0, 0.0), (0.5, -0.3, 0.1), (-0.2, 0.4, 0.0)]
    ids = [srv.add_map(dims, vs, org, ks, hit_threshold=2) for org in origins]
    oracles = [Oracle(dims, vs, org, hit_threshold=2, **kk) for org in origins]
    refs = [o.new_grid() for o in oracles]
    rng = np.random.default_rng(91)
    plan = {}
    for k in range(6):
        for i, org in enumerate(origins):
            centre = np.array(org) + np.array(dims) * vs / 2
            P0 = synth.random_pose(rng, centre - 0.2, centre + 0.2)
            pts = synth.random_cloud(rng, int(rng.integers(200, 900)), -np.array(dims) * 0.04, np.array(dims) * 0.04)
            kind = (k + i) % 3          # 0 plain, 1 se3 sweep, 2 yaw sweep
            if kind == 0:
                t = srv.submit(ids[i], P0, pts)
                plan[t] = (i, P0, None, pts, None, None)
            else:
                P1 = P0.copy()
                P1[:3, :3] = (_turn(rng.normal(size=3) if kind == 1 else (0.0, 0.0, 1.0), rng.uniform(-0.3, 0.3))
                              @ P0[:3, :3].astype(float)).astype(np.float32)
                P1[:3, 3] += rng.uniform(-0.1, 0.1, 3).astype(np.float32)
                times = _sweep_times(rng, len(pts))
                mode = "se3" if kind == 1 else "yaw"
                t = srv.submit_sweep(ids[i], P0, P1, pts, times, deskew=mode)
                plan[t] = (i, P0, P1, pts, times, mode)
    srv.drain()
    done = {c["ticket"]: c for c in srv.poll(100)}
    assert sorted(done) == sorted(plan)
    for t in sorted(plan):           # tickets rise with arrival, so this is each map's arrival order
        i, P0, P1, pts, times, mode = plan[t]
        if P1 is None:
            ref = oracles[i].integrate(*refs[i], P0, pts)
        else:
            ref = oracles[i].integrate_deskew(*refs[i], P0, P1, pts, times, mode)
        assert done[t]["status"] == 0
        P.assert_stats_equal(done[t]["stats"], ref, traffic=False, what=f"ticket {t}")
    for i in range(3):
        got = srv.map_grid(ids[i], dims, ks).read_voxels()
        P.assert_grids_equal(got[0], got[1], *refs[i], what=f"served map {i}")
    srv.close()


def test_context_free_batch_matches_oracle(db):
    """dbtsdf_integrate_batch (the library's own batch context): several grids, one of them twice, in one
    launch; statistics are filled when the call returns and the grids equal the oracle's."""
    sizes = [(40, 36, 32), (56, 40, 48)]
    pairs = [P.make_pair(d, 0.1, (0.0, 0.0, 0.0), kernel_size=5, binning="cube26", shadow_r2=4, hit_threshold=2)
             for d in sizes]
    refs = [o.new_grid() for o, _, _ in pairs]
    rng = np.random.default_rng(101)
    for rnd in range(2):
        items, plan = [], []
        for gi in (0, 1, 0):
            centre = np.array(sizes[gi]) * 0.1 / 2
            pose = synth.random_pose(rng, centre - 0.2, centre + 0.2)
            pts = synth.random_cloud(rng, int(rng.integers(100, 1200)), -centre * 0.9, centre * 0.9)
            items.append((pairs[gi][1], pose, P.to_device(pts)))
            plan.append((gi, pose, pts))
        stats = db.integrate_batch(items)
        for k, (gi, pose, pts) in enumerate(plan):
            ref = pairs[gi][0].integrate(*refs[gi], pose, pts)
            P.assert_stats_equal(stats[k].as_dict(), ref, what=f"round {rnd} scan {k}")
        for gi in range(2):
            P.assert_grids_equal(*P.gpu_planes(pairs[gi][1]), *refs[gi], what=f"round {rnd} grid {gi}")


# ---------------------------------------------------------------------------
# whole grids at full size, on the paths the benchmark times
# ---------------------------------------------------------------------------
_C2_ORACLE = {}


def _c2_oracle(n_scans):
    """Oracle planes after scans 0 .. n_scans-1 of the 1024x1024x256 @ 0.05 m sequence (computed once)."""
    if n_scans not in _C2_ORACLE:
        gdef = synth.config_grid(2)
        from oracle.oracle import Oracle
        kk, gk = P.split_kw(synth.KERNEL_DEFAULTS)
        o = Oracle(dims=gdef["dims"], voxel_size=gdef["voxel_size"], origin=gdef["origin"], **kk, **gk)
        m, p = o.new_grid()
        stats = [o.integrate(m, p, pose, pts) for pose, pts in synth.config_scans(2, 0, range(n_scans))]
        _C2_ORACLE.clear()
        _C2_ORACLE[n_scans] = (m, p, stats)
    return _C2_ORACLE[n_scans]


@pytest.mark.parametrize("strategy", ["tile", "atomic"])
def test_config2_default_paths_whole_grid(db, strategy):
    """The plain one-scan calls the benchmark times (device points, no traffic counting, so the per-point
    strategies run with their revisit skips) over 24 scans of 1024x1024x256 @ 0.05 m: every word of
    both planes and every scan's statistics against the oracle."""
    m, p, stats = _c2_oracle(24)
    gdef = synth.config_grid(2)
    ks = db.KernelSet(kernel_size=11, binning="cube26", shadow_r2=9)
    g = db.Grid(gdef["dims"], gdef["voxel_size"], gdef["origin"], ks, planes="torch")
    g.set_tuning(strategy=strategy)
    revisits = 0
    for k, (pose, pts) in enumerate(synth.config_scans(2, 0, range(24))):
        st = g.integrate(pose, P.to_device(pts))
        g.sync()   # a plain call's statistics arrive with the sync
        st = st.as_dict()
        P.assert_stats_equal(st, stats[k], what=f"c2 scan {k}")
        revisits += st["n_revisit"]
    assert revisits > 0, "the sequence must exercise the revisit skip"
    gm, gp = P.gpu_planes(g)
    P.assert_grids_equal(gm, gp, m, p, what=f"c2 24 scans, {strategy}")
    g.close()


@pytest.mark.parametrize("strategy", ["atomic", "sort"])
def test_paper_kernel_set_config2_whole_grid(db, strategy):
    """The paper's kernel set (K = 21, 40 x 40 direction bins) on three scans of 1024x1024x256 @ 0.05 m:
    whole grid and statistics against the oracle."""
    gdef = synth.config_grid(2)
    kw = dict(synth.KERNEL_DEFAULTS)
    kw.update(PAPER_KERNEL)
    o, g, _ = P.make_pair(gdef["dims"], gdef["voxel_size"], gdef["origin"], **kw)
    g.set_tuning(strategy=strategy)
    m, p = o.new_grid()
    for k, (pose, pts) in enumerate(synth.config_scans(2, 0, range(3))):
        ref = o.integrate(m, p, pose, pts)
        st = g.integrate(pose, P.to_device(pts))
        g.sync()
        P.assert_stats_equal(st.as_dict(), ref, what=f"paper kernel c2 scan {k}")
    gm, gp = P.gpu_planes(g)
    P.assert_grids_equal(gm, gp, m, p, what=f"paper kernel c2, {strategy}")
    g.close()


def test_config3_whole_grid(db):
    """2048x2048x512 @ 0.02 m (2^31 voxels): three scans on the default tuning, every word of both planes
    against the oracle (17 GB per side), compared a slab of 64 z layers at a time."""
    import torch
    gdef = synth.config_grid(3)
    kk, gk = P.split_kw(synth.KERNEL_DEFAULTS)
    from oracle.oracle import Oracle
    o = Oracle(dims=gdef["dims"], voxel_size=gdef["voxel_size"], origin=gdef["origin"], **kk, **gk)
    m, p = o.new_grid()
    ks = db.KernelSet(**kk)
    g = db.Grid(gdef["dims"], gdef["voxel_size"], gdef["origin"], ks, planes="torch", **gk)
    for k, (pose, pts) in enumerate(synth.config_scans(3, 0, range(3))):
        ref = o.integrate(m, p, pose, pts)
        st = g.integrate(pose, P.to_device(pts))
        g.sync()
        P.assert_stats_equal(st.as_dict(), ref, what=f"c3 scan {k}")
    torch.cuda.synchronize()
    nz = gdef["dims"][2]
    for z0 in range(0, nz, 64):
        gm = g.mask_tensor[z0:z0 + 64].cpu().numpy().view(np.uint32)
        gp = g.packed_tensor[z0:z0 + 64].cpu().numpy().view(np.uint32)
        P.assert_grids_equal(gm, gp, m[z0:z0 + 64], p[z0:z0 + 64], what=f"c3 z {z0}-{z0 + 63}")
    g.close()
    del g
    torch.cuda.empty_cache()


def test_served_mix_512_cubes_match_oracle(db):
    """Eight robots' maps of 512^3 @ 0.05 m served concurrently (continuous batching over two streams),
    four scans each: every map word for word against the oracle run of that robot's scans alone."""
    from paper_2509_20081_amd.serve import Server
    from oracle.oracle import Oracle
    kk, gk = P.split_kw(synth.KERNEL_DEFAULTS)
    ks = db.KernelSet(**kk)
    dims = synth.CONFIGS[5]["dims"]
    robots = []
    for rid in range(8):
        gd = synth.config_grid(5, rid)
        robots.append((gd, list(synth.config_scans(5, rid, range(4)))))
    srv = Server(n_streams=2, max_batch_scans=8)
    ids = [srv.add_map(dims, gd["voxel_size"], gd["origin"], ks) for gd, _ in robots]
    for k in range(4):
        for rid, (_, scans) in enumerate(robots):
            srv.submit(ids[rid], scans[k][0], scans[k][1])
    srv.drain()
    done = srv.poll(100)
    assert len(done) == 32 and all(c["status"] == 0 for c in done)
    for rid, (gd, scans) in enumerate(robots):
        o = Oracle(dims=dims, voxel_size=gd["voxel_size"], origin=gd["origin"], **kk, **gk)
        m, p = o.new_grid()
        for pose, pts in scans:
            o.integrate(m, p, pose, pts)
        s = srv.map_grid(ids[rid], dims, ks).read_voxels()
        P.assert_grids_equal(s[0], s[1], m, p, what=f"served robot {rid}")
    srv.close()


@pytest.mark.parametrize("s", [0.3, 0.2, 0.1, 0.05])
def test_resolution_sweep_scan0_whole_grid(db, s):
    """Scan 0 of the 64x1024 sequence into the same 51.2 x 51.2 x 12.8 m room at voxel size s (the
    per-scan cost against resolution leg): whole grid and statistics against the oracle."""
    gd = synth.resolution_grid(s)
    o, g, _ = P.make_pair(gd["dims"], gd["voxel_size"], gd["origin"], **synth.KERNEL_DEFAULTS)
    m, p = o.new_grid()
    for pose, pts in synth.config_scans(2, 0, [0]):
        ref = o.integrate(m, p, pose, pts)
        st = g.integrate(pose, P.to_device(pts))
        g.sync()
        P.assert_stats_equal(st.as_dict(), ref, what=f"scan 0 at {s} m")
    gm, gp = P.gpu_planes(g)
    P.assert_grids_equal(gm, gp, m, p, what=f"scan 0 at {s} m")
    assert ref["n_integrated"] > 1000
    g.close()
