"""Seeded synthetic scenes, LiDAR scans and trajectories.

Stand-in for the paper's datasets (Newer College, Mai City; Section IV), which
are not available: an indoor room with box and cylinder obstacles is ray-cast
analytically in fp64 from a spinning multi-beam sensor, and the returns are
written as fp32 points in the sensor frame together with an fp32 row-major
4x4 sensor->map pose per scan.

Nothing here belongs to the mapping method: no map-frame transform, no
voxelisation, no direction binning, no kernels.

Seeding: every random draw comes from ``numpy.random.default_rng`` seeded with
the integer list ``[20081, config, map_or_robot, stream, ...]`` so that any
scan of any configuration can be regenerated on its own.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_ROOT = 20081

# stream identifiers inside one (config, map) seed family
_S_SCENE = 0
_S_TRAJ = 1
_S_SCAN = 2
_S_MAPS = 3


@dataclass
class SensorModel:
    rows: int                 # beams, evenly spaced in elevation
    cols: int                 # azimuth columns at 2*pi*j/cols
    fov_deg: float            # beams span [-fov, +fov]
    max_range: float = 30.0   # a hit beyond this gives no return
    sigma: float = 0.02       # Gaussian range noise (m)


@dataclass
class Scene:
    room_lo: np.ndarray                              # (3,) fp64
    room_hi: np.ndarray                              # (3,) fp64
    boxes: np.ndarray = field(default_factory=lambda: np.zeros((0, 6)))      # x0 x1 y0 y1 z0 z1
    cylinders: np.ndarray = field(default_factory=lambda: np.zeros((0, 4)))  # cx cy r h (base z=0)


def _rng(*ids: int) -> np.random.Generator:
    return np.random.default_rng([SEED_ROOT, *[int(i) for i in ids]])


# ----------------------------------------------------------------------------
# scene
# ----------------------------------------------------------------------------
def make_scene(rng: np.random.Generator, room_w: float = 40.0, room_h: float = 10.0,
               n_obstacles: int = 20, path_xy: np.ndarray | None = None,
               clearance: float = 1.5) -> Scene:
    """Room [-w/2, w/2]^2 x [0, h] with ``n_obstacles`` boxes/cylinders on the floor.

    Obstacle sizes follow the 40 m room (box footprint sides U[0.5, 4] m, height
    U[0.5, 4] m; cylinder radius U[0.2, 1.5] m, height U[1, 6] m) and shrink with
    the room width below 40 m. Centres are U[-0.45 w, 0.45 w]^2; an obstacle whose
    footprint, grown by ``clearance``, contains a point of ``path_xy`` is redrawn.
    """
    half = room_w / 2.0
    f = min(1.0, room_w / 40.0)
    boxes, cyls = [], []
    path = np.zeros((1, 2)) if path_xy is None else np.asarray(path_xy, dtype=np.float64).reshape(-1, 2)
    attempts = 0
    while len(boxes) + len(cyls) < n_obstacles and attempts < 100 * max(1, n_obstacles):
        attempts += 1
        is_box = rng.random() < 0.5
        cx, cy = rng.uniform(-0.9 * half, 0.9 * half, size=2)
        if is_box:
            sx, sy = rng.uniform(0.5, 4.0, size=2) * f
            hgt = min(rng.uniform(0.5, 4.0), 0.9 * room_h)
            lo = np.array([cx - sx / 2, cy - sy / 2])
            hi = np.array([cx + sx / 2, cy + sy / 2])
        else:
            r = rng.uniform(0.2, 1.5) * f
            hgt = min(rng.uniform(1.0, 6.0), 0.9 * room_h)
            lo = np.array([cx - r, cy - r])
            hi = np.array([cx + r, cy + r])
        inside = np.all((path >= lo - clearance) & (path <= hi + clearance), axis=1)
        if inside.any():
            continue
        if is_box:
            boxes.append([lo[0], hi[0], lo[1], hi[1], 0.0, hgt])
        else:
            cyls.append([cx, cy, r, hgt])
    return Scene(room_lo=np.array([-half, -half, 0.0]), room_hi=np.array([half, half, room_h]),
                 boxes=np.array(boxes, dtype=np.float64).reshape(-1, 6),
                 cylinders=np.array(cyls, dtype=np.float64).reshape(-1, 4))


def cast_rays(scene: Scene, origin: np.ndarray, dirs: np.ndarray) -> np.ndarray:
    """Distance along each unit ray (fp64) to the first surface; inf if none."""
    o = np.asarray(origin, dtype=np.float64).reshape(3)
    d = np.asarray(dirs, dtype=np.float64)
    tiny = 1e-12
    ds = np.where(np.abs(d) < tiny, np.where(d < 0, -tiny, tiny), d)
    inv = 1.0 / ds
    # room interior: leave through the nearest wall / floor / ceiling
    bound = np.where(ds > 0, scene.room_hi[None, :], scene.room_lo[None, :])
    t = np.min((bound - o[None, :]) * inv, axis=1)
    # boxes: slab test
    for b in scene.boxes:
        lo = np.array([b[0], b[2], b[4]])
        hi = np.array([b[1], b[3], b[5]])
        t1 = (lo[None, :] - o[None, :]) * inv
        t2 = (hi[None, :] - o[None, :]) * inv
        tn = np.max(np.minimum(t1, t2), axis=1)
        tf = np.min(np.maximum(t1, t2), axis=1)
        hit = (tn <= tf) & (tn > 0)
        t = np.where(hit & (tn < t), tn, t)
    # vertical cylinders standing on the floor
    for cx, cy, r, h in scene.cylinders:
        ox, oy, oz = o[0] - cx, o[1] - cy, o[2]
        a = d[:, 0] ** 2 + d[:, 1] ** 2
        bq = 2.0 * (ox * d[:, 0] + oy * d[:, 1])
        c = ox * ox + oy * oy - r * r
        disc = bq * bq - 4.0 * a * c
        ok = (a > 1e-18) & (disc >= 0)
        sq = np.sqrt(np.where(ok, disc, 0.0))
        t0 = np.where(ok, (-bq - sq) / np.where(ok, 2.0 * a, 1.0), np.inf)
        z0 = oz + t0 * d[:, 2]
        side = ok & (t0 > 0) & (z0 >= 0) & (z0 <= h)
        t = np.where(side & (t0 < t), t0, t)
        # top cap
        tc = (h - oz) * inv[:, 2]
        xc = ox + tc * d[:, 0]
        yc = oy + tc * d[:, 1]
        cap = (tc > 0) & (xc * xc + yc * yc <= r * r)
        t = np.where(cap & (tc < t), tc, t)
    return t


# ----------------------------------------------------------------------------
# sensor and trajectory
# ----------------------------------------------------------------------------
def sensor_directions(sensor: SensorModel) -> np.ndarray:
    """Unit beam directions in the sensor frame, azimuth outer, beams inner (bottom to top)."""
    el = np.deg2rad(np.linspace(-sensor.fov_deg, sensor.fov_deg, sensor.rows))
    az = 2.0 * np.pi * np.arange(sensor.cols) / sensor.cols
    a, e = np.meshgrid(az, el, indexing="ij")          # (cols, rows)
    dirs = np.stack([np.cos(e) * np.cos(a), np.cos(e) * np.sin(a), np.sin(e)], axis=-1)
    return dirs.reshape(-1, 3)


def pose_from_xyz_rpy(x: float, y: float, z: float, roll: float, pitch: float, yaw: float) -> np.ndarray:
    """fp64 4x4 sensor->map pose from ZYX Euler angles (R = Rz(yaw) Ry(pitch) Rx(roll))."""
    cr, sr = math.cos(roll), math.sin(roll)
    cp, sp = math.cos(pitch), math.sin(pitch)
    cyw, syw = math.cos(yaw), math.sin(yaw)
    rz = np.array([[cyw, -syw, 0], [syw, cyw, 0], [0, 0, 1.0]])
    ry = np.array([[cp, 0, sp], [0, 1.0, 0], [-sp, 0, cp]])
    rx = np.array([[1.0, 0, 0], [0, cr, -sr], [0, sr, cr]])
    pose = np.eye(4)
    pose[:3, :3] = rz @ ry @ rx
    pose[:3, 3] = [x, y, z]
    return pose


def make_trajectory(rng: np.random.Generator, n_scans: int, rate_hz: float = 10.0,
                    amp=(8.0, 14.0), freq=(0.01, 0.03), height: float = 1.5) -> np.ndarray:
    """(n_scans, 4, 4) fp64 poses along x = A_x sin(2 pi f_x t + phi_x), y likewise.

    z = height + 0.05 sin(.), yaw follows the heading, roll and pitch are 2 degree
    sinusoids (0.1-0.5 Hz) so that the full rotation is exercised.
    """
    ax, ay = rng.uniform(*amp, size=2)
    fx, fy = rng.uniform(*freq, size=2)
    px, py, pz, pr, pp = rng.uniform(0, 2 * np.pi, size=5)
    fz, fr, fp = rng.uniform(0.1, 0.5, size=3)
    poses = np.zeros((n_scans, 4, 4))
    for k in range(n_scans):
        t = k / rate_hz
        x = ax * math.sin(2 * math.pi * fx * t + px)
        y = ay * math.sin(2 * math.pi * fy * t + py)
        z = height + 0.05 * math.sin(2 * math.pi * fz * t + pz)
        vx = ax * 2 * math.pi * fx * math.cos(2 * math.pi * fx * t + px)
        vy = ay * 2 * math.pi * fy * math.cos(2 * math.pi * fy * t + py)
        yaw = math.atan2(vy, vx)
        roll = math.radians(2.0) * math.sin(2 * math.pi * fr * t + pr)
        pitch = math.radians(2.0) * math.sin(2 * math.pi * fp * t + pp)
        poses[k] = pose_from_xyz_rpy(x, y, z, roll, pitch, yaw)
    return poses


def synth_scan(scene: Scene, pose64: np.ndarray, sensor: SensorModel,
               rng: np.random.Generator) -> np.ndarray:
    """One scan: fp32 (N, 3) points in the sensor frame, misses and far hits dropped."""
    dirs_s = sensor_directions(sensor)
    rot = pose64[:3, :3]
    dirs_w = dirs_s @ rot.T
    t = cast_rays(scene, pose64[:3, 3], dirs_w)
    noise = rng.normal(0.0, sensor.sigma, size=t.shape)
    keep = np.isfinite(t) & (t <= sensor.max_range)
    rng_m = t + noise
    pts = dirs_s[keep] * rng_m[keep, None]
    return np.ascontiguousarray(pts.astype(np.float32))


# ----------------------------------------------------------------------------
# the five workload configurations
# ----------------------------------------------------------------------------
# c1: one 16x1024 scan into 256^3 @ 0.1 m (small parity case)
# c2: 200 scans of 64x1024 into 1024x1024x256 @ 0.05 m (plain form, one scan per launch)
# c3: 100 scans of 128x2048 into 2048x2048x512 @ 0.02 m (2^31 voxels)
# c4: 64 independent maps x 20 scans, cubic sides U{128..1024} @ 0.05 m,
#     points per scan log-uniform in [4096, 131072] (batched form)
# c5: 32 robots, 512^3 @ 0.05 m each, 23x23x10 m rooms, 16-64 beams x 1024,
#     Poisson arrivals totalling 2000 scans/s (served form)
CONFIGS = {
    1: dict(name="c1_256cube_16x1024", dims=(256, 256, 256), voxel=0.1, scans=1,
            sensor=SensorModel(16, 1024, 15.0), room=(40.0, 10.0), static=True),
    2: dict(name="c2_1024x1024x256_64x1024", dims=(1024, 1024, 256), voxel=0.05, scans=200,
            sensor=SensorModel(64, 1024, 22.5), room=(40.0, 10.0), static=False),
    3: dict(name="c3_2048x2048x512_128x2048", dims=(2048, 2048, 512), voxel=0.02, scans=100,
            sensor=SensorModel(128, 2048, 22.5), room=(40.0, 10.0), static=False),
    4: dict(name="c4_64maps_x20scans", maps=64, scans=20, voxel=0.05, side=(128, 1024),
            npts=(4096, 131072), fov=22.5, cols=1024),
    5: dict(name="c5_32robots_512cube", robots=32, dims=(512, 512, 512), voxel=0.05,
            room=(23.0, 10.0), rows=(16, 64), cols=1024, fov=22.5, rate_hz=2000.0),
}

KERNEL_DEFAULTS = dict(kernel_size=11, binning="cube26", shadow_r2=9, hit_threshold=5, hit_max=65535)


def _c4_map_spec(map_id: int) -> dict:
    r = _rng(4, map_id, _S_MAPS)
    side = int(r.integers(CONFIGS[4]["side"][0], CONFIGS[4]["side"][1] + 1))
    lo, hi = CONFIGS[4]["npts"]
    npts = [math.exp(r.uniform(math.log(lo), math.log(hi))) for _ in range(CONFIGS[4]["scans"])]
    rows = [max(4, int(round(n / 1024.0))) for n in npts]
    return dict(side=side, rows=rows)


def config_grid(cfg: int, map_id: int = 0) -> dict:
    """Grid of a configuration: dims, voxel size, fp32 origin (min corner of voxel 0)."""
    if cfg in (1, 2, 3):
        c = CONFIGS[cfg]
        dims, vs, room_h = c["dims"], c["voxel"], c["room"][1]
    elif cfg == 4:
        spec = _c4_map_spec(map_id)
        dims, vs = (spec["side"],) * 3, CONFIGS[4]["voxel"]
        room_h = min(10.0, 0.8 * spec["side"] * vs)
    elif cfg == 5:
        c = CONFIGS[5]
        dims, vs, room_h = c["dims"], c["voxel"], c["room"][1]
    else:
        raise ValueError(f"unknown config {cfg}")
    centre = np.array([0.0, 0.0, room_h / 2.0])
    origin = (centre - np.array(dims, dtype=np.float64) * vs / 2.0).astype(np.float32)
    return dict(dims=tuple(int(d) for d in dims), voxel_size=float(np.float32(vs)),
                origin=tuple(float(v) for v in origin))


def _room_and_sensor(cfg: int, map_id: int, scan: int):
    if cfg in (1, 2, 3):
        c = CONFIGS[cfg]
        return c["room"][0], c["room"][1], c["sensor"]
    if cfg == 4:
        spec = _c4_map_spec(map_id)
        ext = spec["side"] * CONFIGS[4]["voxel"]
        return (min(40.0, 0.9 * ext), min(10.0, 0.8 * ext),
                SensorModel(spec["rows"][scan], CONFIGS[4]["cols"], CONFIGS[4]["fov"]))
    c = CONFIGS[5]
    rows = int(_rng(5, map_id, _S_SCAN, scan).integers(c["rows"][0], c["rows"][1] + 1))
    return c["room"][0], c["room"][1], SensorModel(rows, c["cols"], c["fov"])


def config_poses(cfg: int, map_id: int = 0, n_scans: int | None = None) -> np.ndarray:
    """fp64 poses of a configuration's sequence (identity rotation at (0,0,1.5) for c1)."""
    room_w, _, _ = _room_and_sensor(cfg, map_id, 0)
    if cfg == 1:
        pose = np.eye(4)
        pose[:3, 3] = [0.0, 0.0, 1.5]
        return pose[None]
    if n_scans is None:
        n_scans = {2: 200, 3: 100, 4: 20, 5: 200}[cfg]
    scale = room_w / 40.0
    return make_trajectory(_rng(cfg, map_id, _S_TRAJ), n_scans,
                           amp=(8.0 * scale, 14.0 * scale))


def config_scans(cfg: int, map_id: int = 0, scan_ids=None, n_scans: int | None = None):
    """Yield ``(pose_f32[4,4], points_f32[N,3])`` for the chosen scans of a configuration."""
    poses = config_poses(cfg, map_id, n_scans)
    room_w, room_h, _ = _room_and_sensor(cfg, map_id, 0)
    scene = make_scene(_rng(cfg, map_id, _S_SCENE), room_w=room_w, room_h=room_h,
                       path_xy=poses[:, :2, 3])
    if scan_ids is None:
        scan_ids = range(len(poses))
    for k in scan_ids:
        _, _, sensor = _room_and_sensor(cfg, map_id, k)
        pts = synth_scan(scene, poses[k], sensor, _rng(cfg, map_id, _S_SCAN, k))
        yield poses[k].astype(np.float32), pts


def random_cloud(rng: np.random.Generator, n: int, lo, hi) -> np.ndarray:
    """Uniform fp32 points in a box (small structured-free test clouds)."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    return (lo + (hi - lo) * rng.random((n, 3))).astype(np.float32)


def random_pose(rng: np.random.Generator, t_lo, t_hi, max_angle: float = math.pi) -> np.ndarray:
    """fp32 pose with a random rotation (ZYX angles) and translation in [t_lo, t_hi]."""
    ang = rng.uniform(-max_angle, max_angle, size=3)
    t = rng.uniform(t_lo, t_hi)
    return pose_from_xyz_rpy(t[0], t[1], t[2], ang[0], ang[1] * 0.5, ang[2]).astype(np.float32)


def config_ground_truth(cfg: int, map_id: int = 0, scan_ids=None, n_scans: int | None = None,
                        cell: float = 0.02) -> np.ndarray:
    """Reference surface points for the accuracy metrics: the exact (noise-free)
    first hits of the same rays as ``config_scans`` on the analytic scene, in
    the map frame (fp64 ray casting, then fp32), within the sensor's range,
    thinned to the first point (in scan, then ray order) of each cube of side
    ``cell`` so that the density does not follow the sensor's range falloff."""
    poses = config_poses(cfg, map_id, n_scans)
    room_w, room_h, _ = _room_and_sensor(cfg, map_id, 0)
    scene = make_scene(_rng(cfg, map_id, _S_SCENE), room_w=room_w, room_h=room_h,
                       path_xy=poses[:, :2, 3])
    if scan_ids is None:
        scan_ids = range(len(poses))
    chunks = []
    for k in scan_ids:
        _, _, sensor = _room_and_sensor(cfg, map_id, k)
        pose = poses[k]
        dirs_w = sensor_directions(sensor) @ pose[:3, :3].T
        t = cast_rays(scene, pose[:3, 3], dirs_w)
        keep = np.isfinite(t) & (t <= sensor.max_range)
        chunks.append(pose[:3, 3][None, :] + dirs_w[keep] * t[keep, None])
    pts = np.concatenate(chunks) if chunks else np.zeros((0, 3))
    k = np.floor(pts / cell).astype(np.int64) + (1 << 20)   # cells within +-2^20 of the origin
    key = k[:, 0] | (k[:, 1] << 21) | (k[:, 2] << 42)
    _, first = np.unique(key, return_index=True)
    return np.ascontiguousarray(pts[np.sort(first)].astype(np.float32))


def resolution_grid(s: float) -> dict:
    """The second configuration's room (1024 x 1024 x 256 voxels at 0.05 m: 51.2 x 51.2 x 12.8 m, same
    centre) at voxel size ``s``, for the per-scan cost against resolution sweep."""
    base = config_grid(2)
    ext = np.array(base["dims"], np.float64) * base["voxel_size"]
    dims = tuple(int(round(e / s)) for e in ext)
    centre = np.array(base["origin"], np.float64) + ext / 2.0
    origin = (centre - np.array(dims, np.float64) * np.float32(s) / 2.0).astype(np.float32)
    return dict(dims=dims, voxel_size=float(np.float32(s)), origin=tuple(float(v) for v in origin))


# ----------------------------------------------------------------------------
# the served form's scan streams, generated on the GPU (torch)
# ----------------------------------------------------------------------------
def _cast_rays_torch(torch, scene: Scene, origins, dirs):
    """``cast_rays`` for a batch on the GPU: origins (S, 3), unit dirs (S, R, 3), fp64; distance (S, R)."""
    o = origins[:, None, :]
    tiny = 1e-12
    ds = torch.where(dirs.abs() < tiny, torch.where(dirs < 0, torch.full_like(dirs, -tiny),
                                                     torch.full_like(dirs, tiny)), dirs)
    inv = 1.0 / ds
    lo = torch.tensor(scene.room_lo, dtype=dirs.dtype, device=dirs.device)
    hi = torch.tensor(scene.room_hi, dtype=dirs.dtype, device=dirs.device)
    bound = torch.where(ds > 0, hi, lo)
    t = ((bound - o) * inv).amin(dim=-1)
    for b in scene.boxes:
        blo = torch.tensor([b[0], b[2], b[4]], dtype=dirs.dtype, device=dirs.device)
        bhi = torch.tensor([b[1], b[3], b[5]], dtype=dirs.dtype, device=dirs.device)
        t1 = (blo - o) * inv
        t2 = (bhi - o) * inv
        tn = torch.minimum(t1, t2).amax(dim=-1)
        tf = torch.maximum(t1, t2).amin(dim=-1)
        hit = (tn <= tf) & (tn > 0) & (tn < t)
        t = torch.where(hit, tn, t)
    for cx, cy, r, h in scene.cylinders:
        ox, oy, oz = o[..., 0] - cx, o[..., 1] - cy, o[..., 2]
        dx, dy, dz = dirs[..., 0], dirs[..., 1], dirs[..., 2]
        a = dx * dx + dy * dy
        bq = 2.0 * (ox * dx + oy * dy)
        c = ox * ox + oy * oy - r * r
        disc = bq * bq - 4.0 * a * c
        ok = (a > 1e-18) & (disc >= 0)
        sq = torch.sqrt(torch.where(ok, disc, torch.zeros_like(disc)))
        t0 = torch.where(ok, (-bq - sq) / torch.where(ok, 2.0 * a, torch.ones_like(a)),
                         torch.full_like(a, float("inf")))
        z0 = oz + t0 * dz
        side = ok & (t0 > 0) & (z0 >= 0) & (z0 <= h) & (t0 < t)
        t = torch.where(side, t0, t)
        tc = (h - oz) * inv[..., 2]
        xc = ox + tc * dx
        yc = oy + tc * dy
        cap = (tc > 0) & (xc * xc + yc * yc <= r * r) & (tc < t)
        t = torch.where(cap, tc, t)
    return t


def served_scans(map_id: int, n_scans: int, torch, device="cuda", seed_stream: int = 7):
    """Robot ``map_id``'s stream for the served form: ``n_scans`` distinct scans along its own trajectory
    in its own room (the fifth configuration's rooms, sensors and 10 Hz trajectory sampling), ray cast on
    the GPU in fp64 with Gaussian range noise from a seeded device generator. Returns
    ``[(pose_f32[4,4] numpy, points_f32[N,3] CUDA tensor in the sensor frame)]`` in scan order."""
    poses = config_poses(5, map_id, n_scans)
    room_w, room_h, _ = _room_and_sensor(5, map_id, 0)
    scene = make_scene(_rng(5, map_id, _S_SCENE), room_w=room_w, room_h=room_h, path_xy=poses[:, :2, 3])
    sensors = [_room_and_sensor(5, map_id, k)[2] for k in range(n_scans)]
    gen = torch.Generator(device=device)
    gen.manual_seed(int(_rng(5, map_id, seed_stream).integers(0, 2 ** 62)))
    out = [None] * n_scans
    by_rows = {}
    for k, s in enumerate(sensors):
        by_rows.setdefault(s.rows, []).append(k)
    for rows in sorted(by_rows):
        ks = by_rows[rows]
        sensor = sensors[ks[0]]
        dirs_s = torch.from_numpy(sensor_directions(sensor)).to(device)                 # (R, 3)
        for c0 in range(0, len(ks), 64):
            idx = ks[c0:c0 + 64]
            P = torch.from_numpy(poses[idx]).to(device)                                  # (S, 4, 4)
            rot_t = P[:, :3, :3].transpose(1, 2).contiguous()
            dirs_w = torch.matmul(dirs_s[None, :, :].expand(len(idx), -1, -1).contiguous(), rot_t)
            t = _cast_rays_torch(torch, scene, P[:, :3, 3].contiguous(), dirs_w)
            noise = torch.randn(t.shape, generator=gen, device=device, dtype=torch.float64) * sensor.sigma
            keep = torch.isfinite(t) & (t <= sensor.max_range)
            rng_m = t + noise
            for j, k in enumerate(idx):
                kk = keep[j]
                pts = (dirs_s[kk] * rng_m[j][kk][:, None]).to(torch.float32).contiguous()
                out[k] = (poses[k].astype(np.float32), pts)
    return out
