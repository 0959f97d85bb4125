"""Serving on the GPU: maps added and removed while others are served, and a served mix of many
robots' scans at full map size, every map compared with the CPU oracle word for word."""
import threading

import numpy as np
import pytest

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


def test_server_adds_maps_while_a_busy_map_is_removed(db):
    """remove_map waits (lock released) for its map's queued and running scans; maps added by another
    thread meanwhile must not disturb it, and the removed map is gone afterwards."""
    from paper_2509_20081_amd.serve import Server
    ks = db.KernelSet(kernel_size=11, binning="cube26", shadow_r2=9)
    gdef = synth.config_grid(5, 0)
    srv = Server(n_streams=2, max_batch_scans=4)
    m0 = srv.add_map(gdef["dims"], gdef["voxel_size"], gdef["origin"], ks)
    scans = list(synth.config_scans(5, 0, range(6)))
    for pose, pts in scans:
        srv.submit(m0, pose, pts)
    errors = []

    def remover():
        try:
            srv.remove_map(m0)
        except Exception as e:  # reported by the main thread
            errors.append(e)

    th = threading.Thread(target=remover)
    th.start()
    small = []
    for k in range(48):     # enough push_backs to move a growing array of slots several times
        small.append(srv.add_map((64, 64, 64), 0.05, (-1.6, -1.6, -0.1), ks))
    th.join(timeout=120)
    assert not th.is_alive(), "remove_map did not return"
    assert not errors, errors
    srv.drain()
    done = srv.poll(100)
    assert len(done) == len(scans) and all(c["status"] == 0 for c in done)
    with pytest.raises(db.DbtsdfError):
        srv.map_grid(m0, gdef["dims"], ks)
    with pytest.raises(db.DbtsdfError):
        srv.remove_map(m0)
    # a map added during the removal works: one scan against the oracle
    rng = np.random.default_rng(3)
    pose = synth.random_pose(rng, (1.4, 1.4, 1.4), (1.8, 1.8, 1.8))
    pts = synth.random_cloud(rng, 3000, -1.2, 1.2)
    srv.submit(small[-1], pose, pts)
    srv.drain()
    assert all(c["status"] == 0 for c in srv.poll(10))
    o, _, _ = P.make_pair((64, 64, 64), 0.05, (-1.6, -1.6, -0.1), kernel_size=11, binning="cube26", shadow_r2=9)
    m, p = o.new_grid()
    o.integrate(m, p, pose, pts)
    view = srv.map_grid(small[-1], (64, 64, 64), ks).read_voxels()
    P.assert_grids_equal(view[0], view[1], m, p, what="map added during a removal")
    srv.close()


def test_server_eight_robots_full_maps_match_oracle(db):
    """Eight robots, each with its own 512^3 map at 0.05 m and its own scene, three distinct scans each,
    submitted interleaved so that batches mix robots: every served map equals the oracle's."""
    from oracle.oracle import Oracle
    from paper_2509_20081_amd.serve import Server
    kw = dict(kernel_size=11, binning="cube26", shadow_r2=9)
    ks = db.KernelSet(**kw)
    srv = Server(n_streams=2, max_batch_scans=16)
    robots = []
    for r in range(8):
        gdef = synth.config_grid(5, r)
        robots.append((gdef, srv.add_map(gdef["dims"], gdef["voxel_size"], gdef["origin"], ks),
                       list(synth.config_scans(5, r, range(3)))))
    for k in range(3):
        for gdef, mid, scans in robots:
            srv.submit(mid, *scans[k])
    srv.drain()
    done = srv.poll(100)
    assert len(done) == 24 and all(c["status"] == 0 for c in done)
    assert max(c["batch_scans"] for c in done) > 1, "no batch mixed robots"
    by_ticket = {}
    for c in done:
        by_ticket.setdefault(c["map_id"], []).append(c)
    for r, (gdef, mid, scans) in enumerate(robots):
        o = Oracle(dims=gdef["dims"], voxel_size=gdef["voxel_size"], origin=gdef["origin"], **kw)
        m, p = o.new_grid()
        want = [o.integrate(m, p, pose, pts) for pose, pts in scans]
        got = sorted(by_ticket[mid], key=lambda c: c["ticket"])
        for k, (g_st, w_st) in enumerate(zip(got, want)):
            P.assert_stats_equal(g_st["stats"], w_st, what=f"robot {r} scan {k}")
        view = srv.map_grid(mid, gdef["dims"], ks).read_voxels()
        P.assert_grids_equal(view[0], view[1], m, p, what=f"robot {r}")
        del m, p, view
    srv.close()


def test_write_voxels_refuses_planes_of_the_wrong_shape(db):
    g = db.Grid((16, 12, 8), 0.1, (0.0, 0.0, 0.0), db.KernelSet(kernel_size=3, binning="cube26", shadow_r2=1))
    good = np.full((8, 12, 16), 0xFFFFFFFF, np.uint32)
    pk = np.full((8, 12, 16), 0x80000000, np.uint32)
    with pytest.raises(ValueError):
        g.write_voxels(good[:, :, :15], pk)
    with pytest.raises(ValueError):
        g.write_voxels(good, pk.reshape(16, 12, 8))
    g.write_voxels(good, pk)
    m, p = g.read_voxels()
    assert np.array_equal(m, good) and np.array_equal(p, pk)
    g.close()
