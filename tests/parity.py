"""Helpers shared by the GPU parity tests: run the HIP library and the CPU oracle
on the same seeded inputs and compare grids element by element."""
from __future__ import annotations

import numpy as np

from oracle import brute
from oracle.oracle import Oracle

KW_KERNEL = ("kernel_size", "binning", "bins_az", "bins_el", "shadow_r2", "metric", "shadow_model", "cone_deg")
KW_GRID = ("hit_threshold", "hit_max", "dedup")


def split_kw(kw):
    k = {n: kw[n] for n in KW_KERNEL if n in kw}
    g = {n: kw[n] for n in KW_GRID if n in kw}
    return k, g


def make_pair(dims, voxel_size, origin, count_traffic=False, **kw):
    """(oracle, gpu Grid with torch-owned planes, KernelSet) for the same parameters."""
    import paper_2509_20081_amd as db
    kk, gk = split_kw(kw)
    ks = db.KernelSet(**kk)
    g = db.Grid(dims, voxel_size, origin, ks, planes="torch", count_traffic=count_traffic, **gk)
    o = Oracle(dims=dims, voxel_size=voxel_size, origin=origin, **kk, **gk)
    return o, g, ks


def gpu_planes(g):
    """(mask, packed) of a torch-planed grid as uint32 numpy arrays (z, y, x)."""
    import torch
    torch.cuda.synchronize()
    return (g.mask_tensor.cpu().numpy().view(np.uint32), g.packed_tensor.cpu().numpy().view(np.uint32))


def to_device(pts):
    import torch
    return torch.from_numpy(np.ascontiguousarray(pts, np.float32)).cuda()


def assert_grids_equal(m_gpu, p_gpu, m_ref, p_ref, what=""):
    dm = np.count_nonzero(m_gpu != m_ref)
    dp = np.count_nonzero(p_gpu != p_ref)
    if dm or dp:
        idx = np.argwhere((m_gpu != m_ref) | (p_gpu != p_ref))[:5]
        detail = [(tuple(int(v) for v in i[::-1]), hex(int(m_gpu[tuple(i)])), hex(int(m_ref[tuple(i)])),
                   hex(int(p_gpu[tuple(i)])), hex(int(p_ref[tuple(i)]))) for i in idx]
        raise AssertionError(f"{what}: {dm} mask and {dp} packed words differ; first (x,y,z, gpu/ref): {detail}")


STAT_KEYS = ("n_in", "n_invalid", "n_out_of_bounds", "n_duplicate", "n_integrated", "voxel_updates",
             "shadow_updates")


def assert_stats_equal(gpu: dict, ref: dict, traffic=False, what=""):
    keys = STAT_KEYS + (("u_mask", "c_mask", "u_shadow") if traffic else ())
    bad = {k: (gpu[k], ref[k]) for k in keys if gpu[k] != ref[k]}
    assert not bad, f"{what}: statistics differ (gpu, oracle): {bad}"


def sample_voxels(rng, dims, K, integrated, n_near=1500, n_any=300):
    """Voxels worth checking: around integrated returns, plus uniform ones."""
    R = (K - 1) // 2
    vox = np.concatenate([v for v, _ in integrated]) if integrated else np.zeros((0, 3), np.int64)
    out = []
    if len(vox):
        pick = vox[rng.integers(0, len(vox), size=n_near)]
        out.append(pick + rng.integers(-R, R + 1, size=pick.shape))
    out.append(np.stack([rng.integers(0, d, size=n_any) for d in dims], axis=1))
    s = np.concatenate(out)
    s = np.clip(s, 0, np.array(dims) - 1)
    return np.unique(s, axis=0)


def integrated_of(o: Oracle, pose, pts, dims, K, binning="cube26", dedup=True, bins_az=40, bins_el=40):
    """(vox, bins) of the returns the oracle integrates from one scan (its own front end)."""
    vox, bins, status = o.front_end(pose, pts)
    keep = brute.survivors(vox.astype(np.int64), status, dims, dedup)
    return vox[keep].astype(np.int64), bins[keep].astype(np.int64)
