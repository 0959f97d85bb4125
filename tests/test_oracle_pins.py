"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the passage it follows. The oracle is the C implementation in
``oracle/``; the closed-form voxel-by-voxel definition in ``oracle/brute.py``
is a second, independent formulation used for brute-force checks on tiny grids.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

from oracle import brute
from oracle.oracle import Oracle
from synth import scene as synth

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def popcount(a):
    a = np.asarray(a, dtype=np.uint64)
    return np.array([bin(int(v)).count("1") for v in a.ravel()]).reshape(a.shape)


def tiny(K=3, dims=(16, 16, 16), **kw):
    kw.setdefault("shadow_r2", 1)
    return Oracle(dims=dims, voxel_size=1.0, origin=(0.0, 0.0, 0.0), kernel_size=K, **kw)


# ----------------------------------------------------------- eq. 3 kernels ---
def test_mask_histograms_eq3(golden_dir):
    """Eq. (3): cells per bit count for K = 3, 5, 11 and the paper's K = 21."""
    g = json.load(open(os.path.join(golden_dir, "mask_histograms.json")))
    for K, hist in g["histograms"].items():
        m, _, _ = Oracle(dims=(int(K),) * 3, voxel_size=1.0, kernel_size=int(K)).tables()
        vals, cnt = np.unique(popcount(m), return_counts=True)
        assert {str(v): int(c) for v, c in zip(vals, cnt)} == hist
    m, _, _ = Oracle(dims=(21,) * 3, voxel_size=1.0, kernel_size=21).tables()
    pc = popcount(m)
    p = g["k21_partial"]
    assert pc.size == p["total"] and pc.max() == p["max_bits"]
    assert (pc == 17).sum() == p["count_17"] and (pc == 18).sum() == p["count_18"]


def test_mask_values_are_low_bit_runs_eq3():
    """Eq. (3): m = 0 at the centre, else (2^32-1) >> (32 - ceil r) (a run of low ones)."""
    for K in (3, 7, 11, 37):
        m, _, _ = Oracle(dims=(K,) * 3, voxel_size=1.0, kernel_size=K).tables()
        R = (K - 1) // 2
        o = np.arange(-R, R + 1)
        DZ, DY, DX = np.meshgrid(o, o, o, indexing="ij")
        n = brute.bits_of_offset(DX, DY, DZ)
        assert m[R, R, R] == 0
        assert np.array_equal(m.astype(np.uint64) + 1, np.left_shift(np.uint64(1), n.astype(np.uint64)))
    # K = 37 reaches the 32-bit limit at its corners: ceil(18 sqrt 3) = 32
    m, _, _ = Oracle(dims=(37,) * 3, voxel_size=1.0, kernel_size=37).tables()
    assert m[0, 0, 0] == 0xFFFFFFFF


def test_k3_kernel_by_hand_eq3():
    """Eq. (3) for K = 3: centre 0x0, 6 faces 0x1, 12 edges and 8 corners 0x3."""
    m, _, _ = tiny(K=3).tables()
    for dz, dy, dx in itertools.product((-1, 0, 1), repeat=3):
        nz = abs(dx) + abs(dy) + abs(dz)
        want = 0x0 if nz == 0 else (0x1 if nz == 1 else 0x3)
        assert m[dz + 1, dy + 1, dx + 1] == want


def test_l1_option_mask():
    """The L1 option named in Sec. III-A: n = |x| + |y| + |z|."""
    m, _, _ = Oracle(dims=(5,) * 3, voxel_size=1.0, kernel_size=5, metric="l1").tables()
    assert m[2, 2, 2] == 0 and m[2, 2, 3] == 0x1 and m[2, 3, 3] == 0x3 and m[4, 4, 4] == 0x3F
    with pytest.raises(ValueError):
        Oracle(dims=(23,) * 3, voxel_size=1.0, kernel_size=23, metric="l1")


# ------------------------------------------------------ shadow (Sec. III-B) ---
def test_cube26_shadow_sizes(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "cube26_shadow_sizes.json")))
    for i, r in enumerate(g["r_s"]):
        _, sh, _ = Oracle(dims=(11,) * 3, voxel_size=1.0, kernel_size=11, shadow_r2=r * r).tables()
        sizes = sh.reshape(26, -1).sum(axis=1)
        for b in range(26):
            s = brute.cube26_sign_vector(b)
            kind = {1: "face", 2: "edge", 3: "corner"}[int(np.abs(s).sum())]
            assert sizes[b] == g[kind][i], (r, b, kind)


def test_cube26_shadow_symmetry_and_halfspace():
    """All 26 shadows are signed axis permutations of the face/edge/corner ones and lie behind the contact voxel."""
    _, sh, dirs = Oracle(dims=(11,) * 3, voxel_size=1.0, kernel_size=11, shadow_r2=9).tables()
    R = 5

    def cells(b):
        z, y, x = np.nonzero(sh[b])
        return np.stack([x, y, z], 1) - R

    refs = {}
    for b in range(26):
        s = brute.cube26_sign_vector(b)
        assert np.allclose(dirs[b], s / np.linalg.norm(s))
        off = cells(b)
        assert np.all(off @ s >= 0) and np.all((off ** 2).sum(1) <= 9)
        assert sh[b][R, R, R] == 1                      # contact voxel included
        kind = int(np.abs(s).sum())
        if kind not in refs:
            refs[kind] = (s, {tuple(o) for o in off})
            continue
        s0, set0 = refs[kind]
        found = False
        for perm in itertools.permutations(range(3)):
            for sg in itertools.product((-1, 1), repeat=3):
                sg = np.array(sg)
                if np.array_equal(sg * s0[list(perm)], s):
                    img = {tuple(sg * np.array(o)[list(perm)]) for o in set0}
                    assert img == {tuple(o) for o in off}
                    found = True
        assert found


def test_shadow_off_is_unsigned_tdf():
    """shadow_r2 < 0: the D-LIO unsigned TDF special case (Sec. III): packed words never change."""
    o = Oracle(dims=(24,) * 3, voxel_size=1.0, kernel_size=5, shadow_r2=-1)
    m, p = o.new_grid()
    rng = np.random.default_rng(5)
    pose = synth.random_pose(rng, (9, 9, 9), (15, 15, 15))
    st = o.integrate(m, p, pose, synth.random_cloud(rng, 40, -6, 6))
    assert st["n_integrated"] > 0 and st["shadow_updates"] == 0
    assert np.all(p == 0x80000000)
    assert np.any(m != 0xFFFFFFFF)


def test_azel_shadow_matches_definition():
    """AZEL shadows: o.o <= r_s^2 and o.u_b >= 0 (u_b = bin centre, eq. 2 grid of bins)."""
    o = Oracle(dims=(11,) * 3, voxel_size=1.0, kernel_size=11, binning="azel", shadow_r2=9)
    _, sh, dirs = o.tables()
    assert sh.shape[0] == 1600
    for b in (0, 17, 800, 820, 1599, 1234):
        want = brute.shadow_set(b, 11, 9, "azel", 40, 40)
        assert np.array_equal(sh[b].astype(bool), want)
        ia, ie = b % 40, b // 40
        a = 2 * math.pi * (ia + 0.5) / 40
        e = -math.pi / 2 + math.pi * (ie + 0.5) / 40
        assert np.allclose(dirs[b], [math.cos(e) * math.cos(a), math.cos(e) * math.sin(a), math.sin(e)])


@pytest.mark.parametrize("baz,bel", [(40, 40), (8, 5), (256, 130)])
def test_azel_bin_centres_fall_in_their_own_bin(baz, bel):
    """Every AZEL bin centre (eq. 2 grid: azimuth from +x counter-clockwise, elevation from the
    nadir) lies in the middle of its own bin, half a bin from each boundary, so binning the
    centre returns the bin. A centre table shifted by half a bin would sit on a boundary, one
    counted from the zenith would land in the mirrored elevation row."""
    o = Oracle(dims=(3,) * 3, voxel_size=1.0, kernel_size=3, binning="azel", bins_az=baz, bins_el=bel,
               shadow_r2=1)
    _, _, dirs = o.tables()
    assert dirs.shape == (baz * bel, 3)
    got = np.array([o.bin(d) for d in dirs])
    assert np.array_equal(got, np.arange(baz * bel))


def test_azel_two_by_one_reduces_to_cube26_y_faces(golden_dir):
    """With 2 azimuth bins and 1 elevation bin, bin 0 spans azimuths [0, pi) around +y and bin 1
    [pi, 2 pi) around -y (elevation centre 0). Their r_s = 3 hemispheres are the closed half-balls
    dy >= 0 and dy <= 0: the same cell sets as the 26-direction shadows of +y and -y, which are
    built from an exact integer dot product, 76 cells each (face entry of the golden table)."""
    sizes = json.load(open(os.path.join(golden_dir, "cube26_shadow_sizes.json")))
    face = sizes["face"][sizes["r_s"].index(3)]
    az = Oracle(dims=(7,) * 3, voxel_size=1.0, kernel_size=7, binning="azel", bins_az=2, bins_el=1, shadow_r2=9)
    cu = Oracle(dims=(7,) * 3, voxel_size=1.0, kernel_size=7, binning="cube26", shadow_r2=9)
    _, sh_az, dirs = az.tables()
    _, sh_cu, _ = cu.tables()
    assert np.allclose(dirs[0], [0.0, 1.0, 0.0], atol=1e-15)
    assert np.allclose(dirs[1], [0.0, -1.0, 0.0], atol=1e-15)
    for b, y in ((0, 1), (1, -1)):
        cb = cu.bin((0.0, float(y), 0.0))
        assert np.array_equal(sh_az[b], sh_cu[cb])
        assert int(sh_az[b].sum()) == face
        # and the directions themselves: +y falls in bin 0, -y in bin 1
        assert az.bin((0.0, float(y), 0.0)) == b


def _ball_offsets(r2):
    rng = range(-3, 4)
    return [(x, y, z) for z in rng for y in rng for x in rng if x * x + y * y + z * z <= r2]


def test_azel_tilted_bin_shadow_sizes_by_symmetry():
    """Shadow sizes fixed by the ball's central symmetry (r_s^2 = 9: 123 lattice cells).

    A direction u with no nonzero cell of the ball on its plane o.u = 0: of each pair o, -o exactly
    one has o.u > 0, so the hemisphere holds the contact cell and half of the other 122: 62 cells.
    The 40 x 40 bin (az 3, el 25), centre azimuth 31.5 deg, elevation 24.75 deg, is such a direction.

    The 8 x 5 bin (az 0, el 2) has centre azimuth 22.5 deg and elevation 0: its plane holds the six
    z-axis cells (dx cos 22.5 + dy sin 22.5 = 0 forces dx = dy = 0, tan 22.5 deg = sqrt 2 - 1 being
    irrational), which the closed hemisphere keeps, and half of the other 116: 1 + 6 + 58 = 65."""
    ball = _ball_offsets(9)
    assert len(ball) == 123
    for baz, bel, ia, ie, on_plane, want in ((40, 40, 3, 25, 0, 62), (8, 5, 0, 2, 6, 65)):
        # the precondition of the count: which nonzero cells lie on the plane (angles as stated above)
        a = math.radians((ia + 0.5) * 360.0 / baz)
        e = math.radians(-90.0 + (ie + 0.5) * 180.0 / bel)
        u = (math.cos(e) * math.cos(a), math.cos(e) * math.sin(a), math.sin(e))
        flat = [c for c in ball if c != (0, 0, 0) and abs(c[0] * u[0] + c[1] * u[1] + c[2] * u[2]) < 1e-6]
        assert len(flat) == on_plane
        o = Oracle(dims=(7,) * 3, voxel_size=1.0, kernel_size=7, binning="azel", bins_az=baz, bins_el=bel,
                   shadow_r2=9)
        _, sh, _ = o.tables()
        assert int(sh[ie * baz + ia].sum()) == want


# --------------------------------------------------------- eq. 2 binning ---
def test_azel_named_directions_eq2():
    o = Oracle(dims=(11,) * 3, voxel_size=1.0, kernel_size=11, binning="azel")
    assert o.bin((1, 0, 0)) == 20 * 40 + 0
    assert o.bin((0, 0, 1)) == 39 * 40 + 0
    assert o.bin((-1, 0, 0)) == 20 * 40 + 20
    assert o.bin((0, -1, 0)) == 20 * 40 + 30
    assert o.bin((0, 1, 0)) == 20 * 40 + 10
    assert o.bin((0, 0, -1)) == 0


def test_azel_agrees_with_atan2_asin_eq2():
    """Eq. (2) with atan2 wrapped to [0, 2 pi): equal away from bin boundaries."""
    o = Oracle(dims=(11,) * 3, voxel_size=1.0, kernel_size=11, binning="azel")
    rng = np.random.default_rng(11)
    d = rng.normal(size=(4000, 3)).astype(np.float32)
    dd = d.astype(np.float64)
    az = np.mod(np.arctan2(dd[:, 1], dd[:, 0]), 2 * np.pi)
    el = np.arcsin(dd[:, 2] / np.linalg.norm(dd, axis=1))
    b_az = np.floor(az / (2 * np.pi) * 40).astype(int)
    b_el = np.minimum(np.floor((el + np.pi / 2) / np.pi * 40).astype(int), 39)
    near = (np.abs(az * 40 / (2 * np.pi) - np.round(az * 40 / (2 * np.pi))) < 1e-4) | \
           (np.abs((el + np.pi / 2) * 40 / np.pi - np.round((el + np.pi / 2) * 40 / np.pi)) < 1e-4)
    got = np.array([o.bin(v) for v in d])
    want = b_el * 40 + b_az
    assert np.all(got[~near] == want[~near])
    # vectorised brute front end agrees exactly everywhere
    vb = brute._bins_azel(d, 40, 40)
    assert np.array_equal(got, vb)


def test_cube26_lattice_directions_and_sector_edges():
    o = tiny()
    seen = set()
    for s in itertools.product((-1, 0, 1), repeat=3):
        if s == (0, 0, 0):
            continue
        b = o.bin(s)
        assert np.array_equal(brute.cube26_sign_vector(b), s)
        seen.add(b)
    assert seen == set(range(26))
    # boundary at tan(pi/8) = 0.41421356...: below it the axis stays 0
    assert np.array_equal(brute.cube26_sign_vector(o.bin((1.0, 0.4142, 0.0))), (1, 0, 0))
    assert np.array_equal(brute.cube26_sign_vector(o.bin((1.0, 0.4143, 0.0))), (1, 1, 0))
    assert np.array_equal(brute.cube26_sign_vector(o.bin((-2.0, 0.0, -0.83))), (-1, 0, -1))


# ---------------------------------------------------- front end (III-C) ---
def test_hand_worked_scan(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "hand_worked_scan.json")))
    o = Oracle(dims=g["grid"]["dims"], voxel_size=g["grid"]["voxel_size"],
               origin=g["grid"]["origin"], **g["kernel"])
    pose = np.eye(4, dtype=np.float32)
    pose[:3, 3] = g["pose_translation"]
    pts = np.array([g["point"]], dtype=np.float32)
    vox, _, status = o.front_end(pose, pts)
    assert status[0] == 0 and list(vox[0]) == g["expect"]["voxel"]
    m, p = o.new_grid()
    st = o.integrate(m, p, pose, pts)
    assert st["n_integrated"] == 1 and st["voxel_updates"] == 27 and st["shadow_updates"] == 6
    for (x, y, z), want in g["expect"]["mask"]:
        assert m[z, y, x] == want
    sh = {tuple(v) for v in g["expect"]["shadow_voxels"]}
    for z, y, x in itertools.product(range(16), repeat=3):
        want = g["expect"]["packed_in_shadow"] if (x, y, z) in sh else g["expect"]["packed_elsewhere"]
        assert p[z, y, x] == want
    # untouched voxels outside the 3^3 cube
    cube = np.zeros((16, 16, 16), bool)
    cube[7:10, 7:10, 7:10] = True
    assert np.all(m[~cube] == 0xFFFFFFFF)
    d = o.read_distance(m, p)
    for (x, y, z), want in g["expect"]["distance"]:
        assert d[z, y, x] == want


def test_rotated_pose_row_major():
    """Sec. III-C transform w = R p + t with the pose row-major: a 90 degree yaw maps +x to +y.

    A transposed pose would send the point to -y and the voxel below the centre.
    """
    o = tiny(K=3)
    pose = np.array([[0, -1, 0, 8.5], [1, 0, 0, 8.5], [0, 0, 1, 8.5], [0, 0, 0, 1]], np.float32)
    vox, bins, status = o.front_end(pose, np.array([[3.0, 0.0, 0.0], [0.0, 0.0, 2.0]], np.float32))
    assert list(vox[0]) == [8, 11, 8] and list(vox[1]) == [8, 8, 10]
    assert np.array_equal(brute.cube26_sign_vector(bins[0]), (0, 1, 0))
    assert np.array_equal(brute.cube26_sign_vector(bins[1]), (0, 0, 1))


def test_origin_and_voxel_size():
    o = Oracle(dims=(20, 20, 20), voxel_size=0.25, origin=(-1.0, 2.0, 0.5), kernel_size=3)
    pose = np.eye(4, dtype=np.float32)
    vox, _, st = o.front_end(pose, np.array([[0.13, 3.0, 2.3]], np.float32))
    # (0.13+1)/0.25 = 4.52 ; (3-2)/0.25 = 4 ; (2.3-0.5)/0.25 = 7.2
    assert st[0] == 0 and list(vox[0]) == [4, 4, 7]


def test_bounds_rule():
    """Sec. III-C: a return whose K^3 neighbourhood would leave the map is discarded."""
    o = tiny(K=5, dims=(16, 16, 16))   # R = 2: valid voxel range [2, 13]
    pose = np.eye(4, dtype=np.float32)
    pts = np.array([[1.5, 8, 8], [2.0, 8, 8], [13.9, 8, 8], [14.0, 8, 8],
                    [8, 8, 1.99], [8, 8, 2.0], [-0.5, 8, 8]], np.float32)
    _, _, st = o.front_end(pose, pts)
    assert list(st) == [2, 0, 0, 2, 2, 0, 2]
    m, p = o.new_grid()
    o.integrate(m, p, pose, pts[1:2])
    assert m[8, 8, 0] == 0x3 and m[8, 8, 4] == 0x3   # touches x = 0 face voxel row


def test_invalid_returns():
    o = tiny(K=3)
    pose = np.eye(4, dtype=np.float32)
    pose[:3, 3] = 8.5
    pts = np.array([[np.nan, 0, 0], [np.inf, 1, 1], [0, 0, 0], [1, 0, 0], [0, -np.inf, 0]], np.float32)
    m, p = o.new_grid()
    st = o.integrate(m, p, pose, pts)
    assert st["n_invalid"] == 4 and st["n_integrated"] == 1
    with pytest.raises(ValueError):
        bad = pose.copy()
        bad[0, 0] = np.nan
        o.integrate(m, p, bad, pts)


# ---------------------------------------------- dedup and counter (III-C, IV-B) ---
def test_dedup_first_return_wins():
    """Sec. IV-B: only the first return per voxel within a frame is integrated."""
    o = tiny(K=3, shadow_r2=1, hit_threshold=1)
    pose = np.eye(4, dtype=np.float32)
    pose[:3, 3] = 8.5
    a = [1.0, 0.2, 0.2]      # voxel (9,8,8), direction +x
    b = [0.6, 0.45, 0.45]    # same voxel, direction (+,+,+)
    for first, second, sh in ((a, b, (1, 0, 0)), (b, a, (1, 1, 1))):
        m, p = o.new_grid()
        st = o.integrate(m, p, pose, np.array([first, second], np.float32))
        assert st["n_duplicate"] == 1 and st["n_integrated"] == 1
        # offset (0,-1,0) from voxel (9,8,8) is on the planar face of the +x
        # shadow, but in front of the (+,+,+) one
        assert (p[8, 7, 9] == 1) == (sh == (1, 0, 0))
        assert p[8, 8, 10] == 1
    oo = tiny(K=3, shadow_r2=1, hit_threshold=1, dedup=False)
    m, p = oo.new_grid()
    st = oo.integrate(m, p, pose, np.array([a, b], np.float32))
    assert st["n_duplicate"] == 0 and st["n_integrated"] == 2 and (p[8, 8, 9] & 0xFFFF) == 2


def test_counter_saturates_and_sign_crossing():
    """Eq. (5) saturation at H_max and eq. (6) sign on the crossing h_old < T <= h_new."""
    pose = np.eye(4, dtype=np.float32)
    pose[:3, 3] = 8.5
    pt = np.array([[2.0, 0, 0]], np.float32)
    o = tiny(K=3, shadow_r2=1, hit_threshold=5, hit_max=3)  # T > H_max: never occupied
    m, p = o.new_grid()
    for _ in range(10):
        o.integrate(m, p, pose, pt)
    assert p[8, 8, 10] == (0x80000000 | 3)
    o = tiny(K=3, shadow_r2=1, hit_threshold=3, hit_max=3)
    m, p = o.new_grid()
    for i in range(10):
        o.integrate(m, p, pose, pt)
        assert p[8, 8, 10] == (min(i + 1, 3) | (0 if i + 1 >= 3 else 0x80000000))
    o = tiny(K=3, shadow_r2=1, hit_threshold=0)  # T = 0: eq. 6 never fires
    m, p = o.new_grid()
    o.integrate(m, p, pose, pt)
    assert p[8, 8, 10] == (0x80000000 | 1)


def test_idempotent_masks_and_doubling_hits():
    o = Oracle(dims=(24,) * 3, voxel_size=1.0, kernel_size=5, shadow_r2=4)
    rng = np.random.default_rng(3)
    pose = synth.random_pose(rng, (10, 10, 10), (14, 14, 14))
    pts = synth.random_cloud(rng, 50, -7, 7)
    m1, p1 = o.new_grid()
    o.integrate(m1, p1, pose, pts)
    m2, p2 = m1.copy(), p1.copy()
    o.integrate(m2, p2, pose, pts)
    assert np.array_equal(m1, m2)
    assert np.array_equal(p2 & 0xFFFF, np.minimum(2 * (p1 & 0xFFFF), 65535))


# ----------------------------------------- brute force, order independence ---
def _random_case(seed, K, binning="cube26", dims=(24, 24, 24)):
    rng = np.random.default_rng(seed)
    R = (K - 1) // 2
    c = np.array(dims) / 2.0
    scans = []
    for _ in range(int(rng.integers(1, 4))):
        pose = synth.random_pose(rng, c - 3, c + 3)
        n = int(rng.integers(1, 61))
        pts = synth.random_cloud(rng, n, -dims[0] / 2 + R - 2, dims[0] / 2 - R + 2)
        pts[rng.random(n) < 0.05] = np.nan
        # a few exact duplicates of earlier returns
        k = int(rng.integers(0, 4))
        if k:
            pts = np.concatenate([pts, pts[rng.integers(0, n, size=k)]])
        scans.append((pose, pts))
    return scans


@pytest.mark.parametrize("seed,K,binning,metric,T,hmax,r2", [
    (1, 3, "cube26", "l2", 1, 65535, 1),
    (2, 5, "cube26", "l2", 2, 3, 4),
    (3, 11, "cube26", "l2", 5, 65535, 9),
    (4, 5, "azel", "l2", 2, 255, 4),
    (5, 7, "azel", "l1", 1, 2, 9),
    (6, 11, "cube26", "l1", 3, 65535, 16),
    (7, 3, "azel", "l2", 0, 65535, 2),
])
def test_brute_force_closed_form(seed, K, binning, metric, T, hmax, r2):
    """Closed-form definition (order-independent) equals the sequential oracle on tiny grids."""
    dims = (24, 24, 24)
    kw = dict(dims=dims, voxel_size=1.0, kernel_size=K, binning=binning, bins_az=40, bins_el=40,
              metric=metric, hit_threshold=T, hit_max=hmax, shadow_r2=r2)
    o = Oracle(**kw)
    m, p = o.new_grid()
    integrated = []
    for pose, pts in _random_case(seed, K, binning, dims):
        st = o.integrate(m, p, pose, pts)
        vox, bins, status = brute.front_end(pose, pts, dims, 1.0, (0, 0, 0), K, binning, 40, 40)
        vo, bo, so = o.front_end(pose, pts)
        assert np.array_equal(vox[status == 0], vo[so == 0]) and np.array_equal(status, so)
        assert np.array_equal(bins, bo)
        keep = brute.survivors(vox, status, dims)
        assert st["n_integrated"] == len(keep)
        integrated.append((vox[keep], bins[keep]))
    bm, bp = brute.closed_form_grid(dims, K, integrated, r2, T, hmax, metric, binning, 40, 40)
    assert np.array_equal(m, bm)
    assert np.array_equal(p, bp)
    # sampled path of the closed form agrees too
    rng = np.random.default_rng(seed)
    smp = rng.integers(0, 24, size=(60, 3))
    sm, sp = brute.sampled_voxels(smp, dims, K, integrated, r2, T, hmax, metric, binning, 40, 40)
    assert np.array_equal(sm, m[smp[:, 2], smp[:, 1], smp[:, 0]])
    assert np.array_equal(sp, p[smp[:, 2], smp[:, 1], smp[:, 0]])


def test_permutation_and_scan_order_independence():
    """Within a scan points commute; whole scans commute (AND, unit saturating steps)."""
    dims = (24, 24, 24)
    o = Oracle(dims=dims, voxel_size=1.0, kernel_size=5, shadow_r2=4, hit_threshold=2, dedup=False)
    scans = _random_case(21, 5, dims=dims) + _random_case(22, 5, dims=dims)
    m1, p1 = o.new_grid()
    for pose, pts in scans:
        o.integrate(m1, p1, pose, pts)
    m2, p2 = o.new_grid()
    rng = np.random.default_rng(0)
    for pose, pts in reversed(scans):
        o.integrate(m2, p2, pose, pts[rng.permutation(len(pts))])
    assert np.array_equal(m1, m2) and np.array_equal(p1, p2)


def test_invariants_after_integration():
    """Sec. III-A: masks only lose bits and stay low-bit runs; bits 16-30 stay zero; sign iff h >= T."""
    dims = (32, 32, 32)
    T, H = 3, 200
    o = Oracle(dims=dims, voxel_size=0.5, kernel_size=11, shadow_r2=9, hit_threshold=T, hit_max=H)
    m, p = o.new_grid()
    rng = np.random.default_rng(8)
    prev = m.copy()
    for _ in range(4):
        pose = synth.random_pose(rng, (7, 7, 7), (9, 9, 9))
        o.integrate(m, p, pose, synth.random_cloud(rng, 300, -5, 5))
        assert np.all((m & prev) == m)      # monotone non-increasing
        prev = m.copy()
        mm = m.astype(np.uint64)
        assert np.all(((mm + 1) & mm) == 0)  # 2^n - 1 patterns
        assert popcount(m[m != 0xFFFFFFFF]).max() <= 9
        assert np.all((p & 0x7FFF0000) == 0)
        h = p & 0xFFFF
        assert h.max() <= H
        assert np.array_equal((p >> 31) == 0, h >= T)


def test_traffic_counts():
    """Unique touched / changed mask words and unique shadow words per scan."""
    o = tiny(K=3, shadow_r2=1)
    pose = np.eye(4, dtype=np.float32)
    pose[:3, 3] = 8.5
    m, p = o.new_grid()
    st = o.integrate(m, p, pose, np.array([[2, 0, 0], [3, 0, 0]], np.float32), count_traffic=True)
    # voxels (10,8,8) and (11,8,8): union of two 3^3 cubes = 36 words
    assert st["u_mask"] == 36 and st["c_mask"] == 36
    assert st["u_shadow"] == 6 + 5
    st = o.integrate(m, p, pose, np.array([[2, 0, 0], [3, 0, 0]], np.float32), count_traffic=True)
    assert st["u_mask"] == 36 and st["c_mask"] == 0 and st["u_shadow"] == 11


def test_synthetic_config_scan_front_end_matches_numpy():
    """The two front ends (C oracle, numpy) agree on a real synthetic scan (c1)."""
    g = synth.config_grid(1)
    pose, pts = next(synth.config_scans(1, 0, [0]))
    o = Oracle(dims=g["dims"], voxel_size=g["voxel_size"], origin=g["origin"], kernel_size=11)
    vo, bo, so = o.front_end(pose, pts)
    vb, bb, sb = brute.front_end(pose, pts, g["dims"], g["voxel_size"], g["origin"], 11)
    assert np.array_equal(so, sb) and np.array_equal(bo, bb)
    assert np.array_equal(vo[so == 0], vb[sb == 0])
    assert (so == 0).sum() > 5000


# ------------------------------------------------------ conical shadow ---
def _shadows(**kw):
    o = Oracle(dims=(16, 16, 16), voxel_size=1.0, kernel_size=11, shadow_r2=9, **kw)
    _, sh, dirs = o.tables()
    return sh.astype(bool), dirs


def _cube_kind(d):
    return int(np.count_nonzero(np.abs(d) > 1e-9))   # 1 face, 2 edge, 3 corner


def test_cone_of_90_degrees_is_the_hemisphere():
    """Sec. IV-A contrasts the hemispherical shadow with a conical one; a cone of half-angle 90 degrees
    is the hemisphere itself, planar face included, for both binnings."""
    for kw in (dict(binning="cube26"), dict(binning="azel", bins_az=8, bins_el=5)):
        hemi, _ = _shadows(**kw)
        cone, _ = _shadows(shadow_model="cone", cone_deg=90.0, **kw)
        assert np.array_equal(hemi, cone)


def test_narrow_cone_keeps_the_lattice_points_on_the_ray():
    """Half-angle 1 degree, r_s = 3: only the voxels on the beam's own line behind the contact voxel:
    0..3 steps along a face direction, 0..2 along an edge (|(2,2,0)|^2 = 8), 0..1 along a corner."""
    sh, dirs = _shadows(shadow_model="cone", cone_deg=1.0)
    R = 5
    for b in range(26):
        s = np.rint(dirs[b] / np.abs(dirs[b]).max()).astype(int)
        want = np.zeros_like(sh[b])
        for k in range(4):
            o = k * s
            if o @ o <= 9:
                want[o[2] + R, o[1] + R, o[0] + R] = True
        assert np.array_equal(sh[b], want), b
        assert sh[b].sum() == {1: 4, 2: 3, 3: 2}[_cube_kind(dirs[b])]


def test_cone_sizes_by_hand():
    """Face direction, r_s = 3: cells with o_x >= 0 and o_y^2 + o_z^2 <= tan^2(alpha) o_x^2 in the ball.
    40 deg (tan^2 = 0.704): 1 + 1 + 9 + 1 = 12; 50 deg (tan^2 = 1.420): 1 + 5 + 21 + 1 = 28."""
    for deg, want in ((40.0, 12), (50.0, 28)):
        sh, dirs = _shadows(shadow_model="cone", cone_deg=deg)
        faces = [int(sh[b].sum()) for b in range(26) if _cube_kind(dirs[b]) == 1]
        assert faces == [want] * 6


def test_cones_nest_and_bad_angles_are_rejected():
    for kw in (dict(binning="cube26"), dict(binning="azel", bins_az=8, bins_el=5)):
        prev = None
        for deg in (5.0, 20.0, 35.0, 60.0, 90.0):
            sh, _ = _shadows(shadow_model="cone", cone_deg=deg, **kw)
            assert sh[:, 5, 5, 5].all()          # the contact voxel is always in
            if prev is not None:
                assert not (prev & ~sh).any()
            prev = sh
    for deg in (0.0, -3.0, 90.5):
        with pytest.raises(ValueError):
            Oracle(dims=(16, 16, 16), voxel_size=1.0, kernel_size=5, shadow_model="cone", cone_deg=deg)


def test_parallel_oracle_equals_serial():
    """The all-core timing leg of the oracle (OpenMP, atomic AND and counter CAS) leaves the planes of the
    single-threaded oracle bit for bit, with the same statistics, over scans that collide, repeat voxels
    and saturate counters."""
    import numpy as np
    from oracle.oracle import Oracle
    from synth import scene as synth
    rng = np.random.default_rng(31)
    for kw in (dict(kernel_size=11, binning="cube26", shadow_r2=9, hit_threshold=2, hit_max=3),
               dict(kernel_size=7, binning="azel", bins_az=8, bins_el=5, shadow_r2=6, dedup=False)):
        dims = (48, 40, 36)
        a = Oracle(dims=dims, voxel_size=0.1, origin=(0.0, 0.0, 0.0), **kw)
        ma, pa = a.new_grid()
        mb, pb = a.new_grid()
        c = np.array(dims) * 0.05
        for _ in range(4):
            pose = synth.random_pose(rng, c - 0.5, c + 0.5)
            pts = synth.random_cloud(rng, 3000, -c * 0.9, c * 0.9)
            pts = np.concatenate([pts, pts[:500]])          # repeated voxels
            pts[rng.random(len(pts)) < 0.02] = np.nan
            s1 = a.integrate(ma, pa, pose, pts)
            s2, thr = a.integrate_parallel(mb, pb, pose, pts)
            assert thr >= 1
            for k in ("n_in", "n_invalid", "n_out_of_bounds", "n_duplicate", "n_integrated", "voxel_updates",
                      "shadow_updates"):
                assert s1[k] == s2[k], (k, s1[k], s2[k])
        assert np.array_equal(ma, mb) and np.array_equal(pa, pb)
