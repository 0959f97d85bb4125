"""Closed-form definition of the integrated DB-TSDF grid, voxel by voxel (numpy).

Test infrastructure only. Shares no code with the C oracle or the GPU library.

Because the eq. 4 AND only clears bits of masks of the form 2^n - 1, it is a
minimum over n; because eq. 5 adds unit steps that saturate, and eq. 6 flips
the sign exactly once when the count passes T, the grid after any sequence of
scans has a plain definition that does not depend on the order in which points
or scans were applied. With P_j the returns integrated from scan j (valid, in
bounds, first per voxel within the scan):

    n(u)  = min(32, min over i in P_1..P_m with |u - v_i|_inf <= R of ceil(|u - v_i|))
    mask  = 2^n(u) - 1                  (all ones when n = 32; 0 when n = 0)
    h(u)  = min(H_max, #{i : u - v_i in S(b_i)})
    sign  = 0  iff  1 <= T <= H_max and h(u) >= T,  else 1 (free)

``ceil(|o|)`` is eq. 3's bit count (or |ox|+|oy|+|oz| in the L1 option), and
S(b) = {o : o.o <= r_s^2, o.u_b >= 0} is the hemispherical shadow of
Section III-B. The front end (fp32 transform, voxelisation, bounds test, bins)
is written again here in vectorised numpy float32, one IEEE operation per
step, in the paper's order.
"""
from __future__ import annotations

import math

import numpy as np

TAN_PI_8 = np.float32(0.414213562373095)


# ---------------------------------------------------------------- kernels ---
def bits_of_offset(dx, dy, dz, metric: str = "l2"):
    """eq. 3 bit count n(o) for integer offsets (arrays ok)."""
    dx, dy, dz = (np.asarray(a, dtype=np.int64) for a in (dx, dy, dz))
    if metric == "l1":
        return np.abs(dx) + np.abs(dy) + np.abs(dz)
    q = dx * dx + dy * dy + dz * dz
    n = np.floor(np.sqrt(q.astype(np.float64))).astype(np.int64)
    n = np.where(n * n < q, n + 1, n)       # exact integer ceil of sqrt
    n = np.where((n > 0) & ((n - 1) * (n - 1) >= q), n - 1, n)
    return n


def mask_of_bits(n):
    n = np.asarray(n, dtype=np.int64)
    full = np.uint64(0xFFFFFFFF)
    m = (np.left_shift(np.uint64(1), n.astype(np.uint64)) - np.uint64(1)) & full
    return np.where(n >= 32, full, m).astype(np.uint32)


def cube26_sign_vector(b: int):
    idx = b + 1 if b >= 13 else b
    return np.array([idx // 9 - 1, (idx // 3) % 3 - 1, idx % 3 - 1], dtype=np.int64)


def azel_centre(b: int, bins_az: int, bins_el: int):
    ia, ie = b % bins_az, b // bins_az
    a = 2.0 * math.pi * (ia + 0.5) / bins_az
    e = -math.pi / 2.0 + math.pi * (ie + 0.5) / bins_el
    return np.array([math.cos(e) * math.cos(a), math.cos(e) * math.sin(a), math.sin(e)])


def shadow_set(b: int, K: int, shadow_r2: int, binning: str = "cube26", bins_az: int = 40,
               bins_el: int = 40):
    """bool[K,K,K] indexed [dz+R, dy+R, dx+R]: o.o <= r_s^2 and o.u_b >= 0."""
    R = (K - 1) // 2
    o = np.arange(-R, R + 1)
    dz, dy, dx = np.meshgrid(o, o, o, indexing="ij")
    ball = (dx * dx + dy * dy + dz * dz) <= shadow_r2
    if binning == "cube26":
        s = cube26_sign_vector(b)
        behind = (dx * s[0] + dy * s[1] + dz * s[2]) >= 0
    else:
        u = azel_centre(b, bins_az, bins_el)
        behind = (dx * u[0] + dy * u[1] + dz * u[2]) >= -1e-9
    if shadow_r2 < 0:
        return np.zeros((K, K, K), dtype=bool)
    return ball & behind


# -------------------------------------------------------------- front end ---
def _bins_cube26(d):
    a = np.abs(d)
    m = np.max(a, axis=1)
    t = (TAN_PI_8 * m).astype(np.float32)
    s = np.where(a >= t[:, None], np.where(d > 0, 1, -1), 0)
    idx = 9 * (s[:, 0] + 1) + 3 * (s[:, 1] + 1) + (s[:, 2] + 1)
    return np.where(idx > 13, idx - 1, idx)


def _snap(v):
    return 0.0 if abs(v) < 1e-12 else v


def _bins_azel(d, bins_az, bins_el):
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    half = (y < 0) | ((y == 0) & (x < 0))
    xp = np.where(half, -x, x).astype(np.float32)
    yp = np.where(half, -y, y).astype(np.float32)
    cnt = np.zeros(len(d), dtype=np.int64)
    for k in range(1, bins_az // 2):
        th = 2.0 * math.pi * k / bins_az
        ck = np.float32(_snap(math.cos(th)))
        sk = np.float32(_snap(math.sin(th)))
        cnt += ((ck * yp) - (sk * xp) >= np.float32(0)).astype(np.int64)
    b_az = np.where((x == 0) & (y == 0), 0, half.astype(np.int64) * (bins_az // 2) + cnt)
    q = ((x * x) + (y * y)) + (z * z)
    zz = z * z
    b_el = np.zeros(len(d), dtype=np.int64)
    for k in range(1, bins_el):
        sg = np.float32(_snap(math.sin((2.0 * k - bins_el) * math.pi / (2.0 * bins_el))))
        s2 = np.float32(sg * sg)
        rhs = s2 * q
        if sg >= 0:
            ok = (z >= 0) & (zz >= rhs)
        else:
            ok = (z >= 0) | (zz <= rhs)
        b_el += ok.astype(np.int64)
    return b_el * bins_az + b_az


def front_end(pose, pts, dims, voxel_size, origin, K, binning="cube26", bins_az=40, bins_el=40):
    """(vox int64[N,3], bins int64[N], status int64[N]: 0 ok, 1 invalid, 2 out of bounds)."""
    P = np.asarray(pose, dtype=np.float32).reshape(16)
    p = np.asarray(pts, dtype=np.float32).reshape(-1, 3)
    n = p.shape[0]
    R = (K - 1) // 2
    inv_s = np.float32(np.float32(1.0) / np.float32(voxel_size))
    org = np.asarray(origin, dtype=np.float32)
    with np.errstate(all="ignore"):
        d = np.zeros((n, 3), dtype=np.float32)
        w = np.zeros((n, 3), dtype=np.float32)
        for k in range(3):
            d[:, k] = ((P[4 * k] * p[:, 0]) + (P[4 * k + 1] * p[:, 1])) + (P[4 * k + 2] * p[:, 2])
            w[:, k] = d[:, k] + P[4 * k + 3]
        invalid = ~np.all(np.isfinite(p), axis=1) | np.all(d == 0, axis=1)
        f = np.floor((w - org[None, :]) * inv_s)
        lo = np.float32(R)
        hi = np.array([dims[0] - 1 - R, dims[1] - 1 - R, dims[2] - 1 - R], dtype=np.float32)
        inb = np.all((f >= lo) & (f <= hi[None, :]), axis=1)
        vox = np.where(inb[:, None], f, 0).astype(np.int64)
        if binning == "cube26":
            bins = _bins_cube26(d)
        else:
            bins = _bins_azel(d, bins_az, bins_el)
    status = np.where(invalid, 1, np.where(inb, 0, 2))
    bins = np.where(status == 0, bins, -1)
    return vox, bins, status


def survivors(vox, status, dims, dedup=True):
    """Indices of integrated returns: valid, in bounds, and (with dedup) first per voxel."""
    ok = np.nonzero(status == 0)[0]
    if not dedup:
        return ok
    key = vox[ok, 0] + dims[0] * (vox[ok, 1] + dims[1] * vox[ok, 2])
    _, first = np.unique(key, return_index=True)   # first occurrence = lowest index
    return np.sort(ok[first])


# ------------------------------------------------------------ closed form ---
def closed_form_grid(dims, K, scans, shadow_r2, hit_threshold, hit_max, metric="l2",
                     binning="cube26", bins_az=40, bins_el=40, state=None):
    """Whole grid (mask, packed as uint32[Nz,Ny,Nx]) from integrated voxels/bins per scan.

    ``scans`` is a list of (vox int[M,3], bins int[M]) of the integrated returns of
    each scan; ``state`` an optional starting (n_bits, hits) pair.
    """
    nx, ny, nz = dims
    R = (K - 1) // 2
    nb = np.full((nz, ny, nx), 32, dtype=np.int64) if state is None else state[0].copy()
    hits = np.zeros((nz, ny, nx), dtype=np.int64) if state is None else state[1].copy()
    o = np.arange(-R, R + 1)
    DZ, DY, DX = np.meshgrid(o, o, o, indexing="ij")
    bits = bits_of_offset(DX, DY, DZ, metric)
    cache = {}
    for vox, bins in scans:
        for (x, y, z), b in zip(np.asarray(vox), np.asarray(bins)):
            sl = (slice(z - R, z + R + 1), slice(y - R, y + R + 1), slice(x - R, x + R + 1))
            nb[sl] = np.minimum(nb[sl], bits)
            if b not in cache:
                cache[b] = shadow_set(int(b), K, shadow_r2, binning, bins_az, bins_el)
            hits[sl] += cache[b]
    return _encode(nb, hits, hit_threshold, hit_max)


def _encode(nb, hits, T, hmax):
    h = np.minimum(hits, hmax)
    mask = mask_of_bits(nb)
    occupied = (T >= 1) & (T <= hmax) & (h >= T)
    packed = (np.where(occupied, 0, 0x80000000) | h).astype(np.uint32)
    return mask, packed


def sampled_voxels(samples, dims, K, scans, shadow_r2, hit_threshold, hit_max, metric="l2",
                   binning="cube26", bins_az=40, bins_el=40):
    """(mask, packed) of selected voxels (int[S,3], x y z) computed one by one.

    Every integrated return whose K^3 window holds the voxel is found by a sorted
    lookup of the K^3 candidate positions; used for grids too big for the whole
    closed form.
    """
    nx, ny, nz = dims
    R = (K - 1) // 2
    s = np.asarray(samples, dtype=np.int64).reshape(-1, 3)
    o = np.arange(-R, R + 1)
    DZ, DY, DX = np.meshgrid(o, o, o, indexing="ij")
    offs = np.stack([DX.ravel(), DY.ravel(), DZ.ravel()], axis=1)          # K^3 x 3
    bits = bits_of_offset(offs[:, 0], offs[:, 1], offs[:, 2], metric)
    nb = np.full(len(s), 32, dtype=np.int64)
    hits = np.zeros(len(s), dtype=np.int64)
    sh_cache = {}
    for vox, bins in scans:
        vox = np.asarray(vox, dtype=np.int64).reshape(-1, 3)
        bins = np.asarray(bins, dtype=np.int64)
        key = vox[:, 0] + nx * (vox[:, 1] + ny * vox[:, 2])
        order = np.argsort(key, kind="stable")
        skey, sbin = key[order], bins[order]
        # candidate source voxel v = u - o for each sample u and offset o
        src = s[:, None, :] - offs[None, :, :]                              # S x K^3 x 3
        inside = np.all((src >= 0) & (src < np.array([nx, ny, nz])), axis=2)
        ck = src[..., 0] + nx * (src[..., 1] + ny * src[..., 2])
        lo = np.searchsorted(skey, ck, side="left")
        hi = np.searchsorted(skey, ck, side="right")
        cnt = np.where(inside, hi - lo, 0)
        have = cnt > 0
        nb = np.minimum(nb, np.where(have, bits[None, :], 32).min(axis=1))
        si, oi = np.nonzero(have)
        for a, b_off in zip(si, oi):
            for j in range(lo[a, b_off], hi[a, b_off]):
                b = int(sbin[j])
                if b not in sh_cache:
                    sh_cache[b] = shadow_set(b, K, shadow_r2, binning, bins_az, bins_el).ravel()
                hits[a] += int(sh_cache[b][b_off])
    return _encode(nb, hits, hit_threshold, hit_max)
