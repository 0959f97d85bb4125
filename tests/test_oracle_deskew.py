"""Pins of the oracle's motion compensation (deskew of a sweep, Sec. III-C).

The reading: the rotation over the sweep Q = R1 R0^T becomes a unit quaternion q
(w >= 0; for yaw-only, the rotation about z of Q's projected x axis), and a
return at time fraction tau gets R(tau) = M(nlerp(1, q, tau)) R0 and
t(tau) = t0 + tau (t1 - t0). The pins tie this to closed forms reached another
way: quaternions of rotations built from axis and angle, the angle of the
normalised interpolation from trigonometry, exact special cases (tau = 0, no
motion, axis-aligned turns) and single returns whose contact voxel is computed
in fp64.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O


def rot_axis_angle(axis, ang):
    """Rotation matrix from axis and angle (fp64, Rodrigues)."""
    a = np.asarray(axis, float)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * (K @ K)


def pose_of(R, t):
    P = np.eye(4, dtype=np.float32)
    P[:3, :3] = np.asarray(R, np.float32)
    P[:3, 3] = np.asarray(t, np.float32)
    return P


def test_constants_of_known_rotations():
    eye = np.eye(4, dtype=np.float32)
    assert O.deskew_constants(eye, eye).tolist() == [1, 0, 0, 0, 0, 0, 0]
    # a quarter turn about z, written exactly
    Rz = np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1]], np.float32)
    k = O.deskew_constants(eye, pose_of(Rz, (0.5, -2.0, 0.25)))
    c = np.float32(math.sqrt(0.5))
    assert np.allclose(k[:4], [c, 0, 0, c], rtol=0, atol=1e-7) and k[1] == 0 and k[2] == 0
    assert k[4:].tolist() == [0.5, -2.0, 0.25]
    # a half turn about x: Shepperd's second branch, exactly (0, 1, 0, 0)
    Rx = np.diag([1, -1, -1]).astype(np.float32)
    assert O.deskew_constants(eye, pose_of(Rx, (0, 0, 0)))[:4].tolist() == [0, 1, 0, 0]
    # three quarters of a turn about z is a quarter turn the other way (w >= 0)
    k = O.deskew_constants(eye, pose_of(Rz.T, (0, 0, 0)))
    assert np.allclose(k[:4], [c, 0, 0, -c], atol=1e-7)


@pytest.mark.parametrize("seed", range(6))
def test_constants_match_axis_angle(seed):
    """General rotations: the quaternion of R1 R0^T is (cos(a/2), sin(a/2) u) for the relative axis u and
    angle a used to build R1 from R0; the yaw constants of Rz(psi) Ry(b) Rx(g) R0 are those of the
    z rotation by psi alone."""
    rng = np.random.default_rng(seed)
    R0 = rot_axis_angle(rng.normal(size=3), rng.uniform(0, math.pi))
    u = rng.normal(size=3)
    u /= np.linalg.norm(u)
    ang = rng.uniform(0.01, 3.0)
    R1 = rot_axis_angle(u, ang) @ R0
    P0, P1 = pose_of(R0, rng.normal(size=3)), pose_of(R1, rng.normal(size=3))
    k = O.deskew_constants(P0, P1, "se3")
    want = np.concatenate([[math.cos(ang / 2)], math.sin(ang / 2) * u])
    assert np.allclose(k[:4], want, atol=3e-6)
    assert np.array_equal(k[4:], P1[:3, 3] - P0[:3, 3])
    psi, b, g = rng.uniform(-3.0, 3.0), rng.uniform(-0.3, 0.3), rng.uniform(-0.3, 0.3)
    R1 = rot_axis_angle((0, 0, 1), psi) @ rot_axis_angle((0, 1, 0), b) @ rot_axis_angle((1, 0, 0), g) @ R0
    k = O.deskew_constants(P0, pose_of(R1, (0, 0, 0)), "yaw")
    assert k[1] == 0 and k[2] == 0
    assert np.allclose(k[:4], [math.cos(psi / 2), 0, 0, math.sin(psi / 2)], atol=3e-6)


def test_pose_along_the_sweep():
    """tau = 0 gives the start pose exactly; tau = 1 the end pose to fp32 rounding; in between the
    rotation angle is the normalised interpolation's, 2 atan2(tau sin(a/2), 1 - tau + tau cos(a/2))."""
    rng = np.random.default_rng(4)
    R0 = rot_axis_angle(rng.normal(size=3), 1.1)
    u = np.array([0.3, -0.2, 0.9])
    u /= np.linalg.norm(u)
    a = 0.7
    R1 = rot_axis_angle(u, a) @ R0
    P0, P1 = pose_of(R0, (1.0, 2.0, 3.0)), pose_of(R1, (1.5, 1.0, 3.25))
    k = O.deskew_constants(P0, P1)
    assert np.array_equal(O.deskew_pose(P0, k, 0.0), P0)
    assert np.allclose(O.deskew_pose(P0, k, 1.0), P1, atol=2e-6)
    for tau in (0.1, 0.25, 0.5, 0.9):
        phi = 2 * math.atan2(tau * math.sin(a / 2), 1 - tau + tau * math.cos(a / 2))
        want = rot_axis_angle(u, phi) @ R0
        P = O.deskew_pose(P0, k, tau)
        assert np.allclose(P[:3, :3], want, atol=3e-6), tau
        assert np.allclose(P[:3, 3], np.array([1.0, 2.0, 3.0]) + tau * np.array([0.5, -1.0, 0.25]), atol=1e-6)
        assert np.allclose(P[:3, :3] @ P[:3, :3].T, np.eye(3), atol=3e-6)   # a rotation for every tau


def _oracle():
    return O.Oracle((40, 40, 40), 0.25, (-5.0, -5.0, -5.0), kernel_size=5, binning="cube26", shadow_r2=4,
                    hit_threshold=2)


def _scan(rng, n=400):
    return rng.uniform(-3.0, 3.0, size=(n, 3)).astype(np.float32)


def test_tau_zero_and_no_motion_equal_the_plain_scan():
    rng = np.random.default_rng(7)
    o = _oracle()
    pts = _scan(rng)
    P0 = pose_of(rot_axis_angle((0.2, 0.1, 1.0), 0.4), (0.3, -0.2, 0.1))
    P1 = pose_of(rot_axis_angle((0.0, 1.0, 0.3), 0.9), (0.8, 0.2, -0.4))
    m, p = o.new_grid()
    ref = o.integrate(m, p, P0, pts)
    for mode in ("se3", "yaw"):
        m2, p2 = o.new_grid()
        st = o.integrate_deskew(m2, p2, P0, P1, pts, np.zeros(len(pts), np.float32), mode)
        assert st == ref and np.array_equal(m, m2) and np.array_equal(p, p2)
    # no motion with an axis-aligned rotation (exactly orthonormal): any tau is the start pose
    Pa = pose_of(np.array([[0, 0, 1], [1, 0, 0], [0, 1, 0]]), (0.3, -0.2, 0.1))
    m, p = o.new_grid()
    ref = o.integrate(m, p, Pa, pts)
    m2, p2 = o.new_grid()
    st = o.integrate_deskew(m2, p2, Pa, Pa, pts, rng.uniform(0, 1, len(pts)).astype(np.float32))
    assert st == ref and np.array_equal(m, m2) and np.array_equal(p, p2)


def test_times_outside_the_sweep_are_invalid():
    o = _oracle()
    pts = np.array([[1.0, 0.5, 0.2]] * 6, np.float32) + np.arange(6, dtype=np.float32)[:, None] * 0.3
    times = np.array([0.0, 1.0, np.nan, -0.01, 1.01, np.inf], np.float32)
    m, p = o.new_grid()
    st = o.integrate_deskew(m, p, np.eye(4), pose_of(np.eye(3), (0.1, 0, 0)), pts, times)
    assert st["n_invalid"] == 4 and st["n_integrated"] == 2


@pytest.mark.parametrize("mode", ["se3", "yaw"])
def test_single_returns_land_in_the_closed_form_voxel(mode):
    """A sweep turning 90 degrees about z while moving: one return at a time, its contact voxel (mask 0)
    is floor((R(tau) p + t(tau) - o) / s) with R(tau) from the interpolation angle, computed in fp64
    (returns within 1e-3 voxel of a face are skipped)."""
    rng = np.random.default_rng(11 if mode == "se3" else 12)
    o = _oracle()
    R0 = rot_axis_angle((0, 0, 1), 0.3)
    psi = math.pi / 2
    P0 = pose_of(R0, (0.2, -0.1, 0.05))
    P1 = pose_of(rot_axis_angle((0, 0, 1), psi) @ R0, (0.7, 0.4, -0.2))
    t0, dt = P0[:3, 3].astype(float), (P1[:3, 3] - P0[:3, 3]).astype(float)
    checked = 0
    for _ in range(40):
        p = rng.uniform(-2.0, 2.0, 3).astype(np.float32)
        tau = np.float32(rng.uniform(0, 1))
        phi = 2 * math.atan2(tau * math.sin(psi / 2), 1 - tau + tau * math.cos(psi / 2))
        w = rot_axis_angle((0, 0, 1), phi) @ R0 @ p.astype(float) + t0 + float(tau) * dt
        f = (w + 5.0) / 0.25
        if np.min(np.abs(f - np.round(f))) < 1e-3:
            continue
        v = np.floor(f).astype(int)
        m, pk = o.new_grid()
        st = o.integrate_deskew(m, pk, P0, P1, p[None], np.array([tau], np.float32), mode)
        if st["n_integrated"] == 0:
            continue
        assert m[v[2], v[1], v[0]] == 0
        assert int((m == 0).sum()) == 1
        checked += 1
    assert checked > 20
