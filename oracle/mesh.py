"""Marching-cubes mesh of the DB-TSDF zero level -- test infrastructure only.

The paper exports the fused map as a mesh by Marching Cubes at iso = 0.0 (the
export block of its pipeline figure, Sec. III). It names the method and the
iso value only; this module fixes the rest as follows, and the GPU path must
give the same triangles (as a set: the order of output is not part of the
result).

Field. ``d(u) = (s ? +1 : -1) * popcount(mask)`` at every voxel centre, the
signed distance the grid reads out (untouched voxels read +32).

Cells. The cubes of the dual grid: the cube with lower corner voxel (i, j, k)
has the eight voxels (i + cx, j + cy, k + cz), c = cx + 2 cy + 4 cz.

Readings (M1-M6):

M1  A corner is inside when d < 0 (d = 0 is outside: the zero level is the
    boundary of the negative region).
M2  Edges are numbered 4 a + r: axis a (x, y, z) and r the rank of the edge's
    lower corner among the four corners whose bit a is clear. An edge is
    crossed when exactly one of its corners is inside. Its vertex, with d_lo
    and d_hi at the lower and upper voxel u and u + e_a, is at
    ``t = d_lo / (d_lo - d_hi)`` and coordinates ``c_q(u)`` for q != a and
    ``c_a(u) + t * s`` along a, with ``c_q(u) = o_q + (u_q + 0.5) * s``: every
    operation one IEEE fp32 operation in this order, no fused multiply-add.
M3  Faces with two crossed edges take one segment. Faces with four (a saddle:
    inside corners on a diagonal) take two, each cutting off one inside
    corner (inside corners are kept apart), so two cubes sharing the face
    agree and the mesh has no holes.
M4  Each segment runs from the crossed edge where the face's cycle of corners,
    taken counter-clockwise as seen from outside the cube, enters an inside
    run of corners to the edge where it leaves it. Segments chain into closed
    loops (each crossed edge is the end of one segment and the start of
    another); a loop starts at its smallest edge number w0. Triangles so
    oriented have their normal (right hand rule) pointing to the outside
    (d >= 0).
M5  A loop is fanned from w0: (w0, w_i, w_(i+1)). A loop that holds all four
    crossed edges of a saddle face would then have a chord lying in that face,
    which the neighbouring cube can draw too (an edge of four triangles); such
    a loop is fanned instead from its centre c, the mean of its vertices
    (each coordinate summed in loop order from w0, then divided by the count,
    fp32): (c, w_i, w_(i+1)) for every i, wrapping round.
M6  The cubes taken are those with all eight corners in the box [lo, hi).
"""
from __future__ import annotations

import numpy as np

N_EDGES = 12


def corner_offset(c: int):
    return (c & 1, (c >> 1) & 1, (c >> 2) & 1)


def edge_list():
    """[(axis, lower corner)] in edge-number order (M2)."""
    out = []
    for a in range(3):
        lows = [c for c in range(8) if not (c >> a) & 1]
        out += [(a, c) for c in lows]
    return out


EDGES = edge_list()
EDGE_OF = {(min(c, c | (1 << a)), max(c, c | (1 << a))): n for n, (a, c) in enumerate(EDGES)}


def face_cycles():
    """The six faces, each as its four corners counter-clockwise seen from outside (M4)."""
    out = []
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3           # e_b x e_c = e_a
        for v in (0, 1):
            # (b, c) coordinates counter-clockwise about +e_a; reversed about -e_a
            ring = [(0, 0), (1, 0), (1, 1), (0, 1)] if v == 1 else [(0, 0), (0, 1), (1, 1), (1, 0)]
            corners = []
            for pb, pc in ring:
                bits = [0, 0, 0]
                bits[a], bits[b], bits[c] = v, pb, pc
                corners.append(bits[0] + 2 * bits[1] + 4 * bits[2])
            out.append(corners)
    return out


FACES = face_cycles()


def edge_between(c0: int, c1: int) -> int:
    return EDGE_OF[(min(c0, c1), max(c0, c1))]


def case_loops(case: int):
    """Closed loops of crossed edges (lists of edge numbers) for a corner case (bit c = corner c inside)."""
    inside = [(case >> c) & 1 for c in range(8)]
    nxt = {}
    for ring in FACES:
        flags = [inside[q] for q in ring]
        if all(flags) or not any(flags):
            continue
        # runs of inside corners in the counter-clockwise cycle; on a saddle
        # face each inside corner is its own run, which is what M3 asks for
        for i in range(4):
            if flags[i] and not flags[i - 1]:
                j = i
                while flags[(j + 1) % 4]:
                    j = (j + 1) % 4
                enter = edge_between(ring[i - 1], ring[i])
                leave = edge_between(ring[j], ring[(j + 1) % 4])
                assert enter not in nxt
                nxt[enter] = leave
    loops = []
    left = set(nxt)
    while left:
        start = min(left)
        loop = [start]
        left.discard(start)
        e = nxt[start]
        while e != start:
            loop.append(e)
            left.discard(e)
            e = nxt[e]
        loops.append(loop)
    return loops


CENTRE = 12   # stands for the centre vertex of a loop in a triangle


def saddle_faces(case: int):
    """Faces (as sets of their four edge numbers) with four crossed edges."""
    inside = [(case >> c) & 1 for c in range(8)]
    out = []
    for ring in FACES:
        flags = [inside[q] for q in ring]
        if flags == [1, 0, 1, 0] or flags == [0, 1, 0, 1]:
            out.append({edge_between(ring[i], ring[(i + 1) % 4]) for i in range(4)})
    return out


def case_polygons(case: int):
    """[(loop from its smallest edge, fanned from the centre?)] of a case (M4, M5)."""
    out = []
    saddles = saddle_faces(case)
    for loop in case_loops(case):
        k = loop.index(min(loop))
        w = loop[k:] + loop[:k]
        out.append((w, any(f <= set(w) for f in saddles)))
    return out


def case_triangles(case: int):
    """Triangles of a case as edge-number triples (CENTRE for a loop's centre)."""
    tris = []
    for w, centred in case_polygons(case):
        if centred:
            tris += [(CENTRE, w[i], w[(i + 1) % len(w)]) for i in range(len(w))]
        else:
            tris += [(w[0], w[i], w[i + 1]) for i in range(1, len(w) - 1)]
    return tris


TABLE = [case_triangles(c) for c in range(256)]


def signed_distance(mask: np.ndarray, packed: np.ndarray) -> np.ndarray:
    """d = (s ? +1 : -1) * popcount(mask), as int32, same shape (z, y, x)."""
    m = np.ascontiguousarray(mask, dtype=np.uint32)
    pc = np.zeros(m.shape, dtype=np.int32)
    for b in range(32):
        pc += ((m >> np.uint32(b)) & np.uint32(1)).astype(np.int32)
    sign = np.where((np.asarray(packed, dtype=np.uint32) >> np.uint32(31)) != 0, 1, -1).astype(np.int32)
    return sign * pc


def _coord(o: float, u: int, s: float) -> np.float32:
    return np.float32(np.float32(o) + np.float32(np.float32(np.float32(u) + np.float32(0.5)) * np.float32(s)))


def edge_vertex(d, ijk, edge: int, origin, s):
    """The vertex of a crossed edge of the cube with lower corner ijk (M2), as three fp32 values."""
    a, c = EDGES[edge]
    off = corner_offset(c)
    u = [ijk[q] + off[q] for q in range(3)]
    hi = list(u)
    hi[a] += 1
    d_lo = np.float32(d[u[2], u[1], u[0]])
    d_hi = np.float32(d[hi[2], hi[1], hi[0]])
    t = np.float32(d_lo / np.float32(d_lo - d_hi))
    out = []
    for q in range(3):
        cq = _coord(origin[q], u[q], s)
        if q == a:
            cq = np.float32(cq + np.float32(t * np.float32(s)))
        out.append(cq)
    return out


def extract_mesh(mask, packed, origin, voxel_size, lo=None, hi=None) -> np.ndarray:
    """Triangles (n, 3, 3) float32 of the zero level over the cubes inside box [lo, hi) (x, y, z)."""
    d = signed_distance(mask, packed)
    nz, ny, nx = d.shape
    lo = (0, 0, 0) if lo is None else tuple(int(v) for v in lo)
    hi = (nx, ny, nz) if hi is None else tuple(int(v) for v in hi)
    tris = []
    if any(hi[q] - lo[q] < 2 for q in range(3)):
        return np.zeros((0, 3, 3), np.float32)
    sub = d[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] < 0
    case = np.zeros((sub.shape[0] - 1, sub.shape[1] - 1, sub.shape[2] - 1), np.int32)
    for c in range(8):
        cx, cy, cz = corner_offset(c)
        case |= sub[cz:cz + case.shape[0], cy:cy + case.shape[1], cx:cx + case.shape[2]].astype(np.int32) << c
    for kz, ky, kx in zip(*np.nonzero((case != 0) & (case != 255))):
        ijk = (lo[0] + int(kx), lo[1] + int(ky), lo[2] + int(kz))
        for w, centred in case_polygons(int(case[kz, ky, kx])):
            v = [edge_vertex(d, ijk, e, origin, voxel_size) for e in w]
            if centred:
                c = []
                for q in range(3):
                    acc = v[0][q]
                    for i in range(1, len(v)):
                        acc = np.float32(acc + v[i][q])
                    c.append(np.float32(acc / np.float32(len(v))))
                tris += [[c, v[i], v[(i + 1) % len(v)]] for i in range(len(v))]
            else:
                tris += [[v[0], v[i], v[i + 1]] for i in range(1, len(v) - 1)]
    return np.asarray(tris, np.float32).reshape(-1, 3, 3)


def canonical(tris: np.ndarray) -> np.ndarray:
    """Triangles as a sorted array of rows, each rotated (orientation kept) to start at its least vertex."""
    t = np.asarray(tris, np.float32).reshape(-1, 3, 3)
    if len(t) == 0:
        return t.reshape(0, 9)
    keys = t.view(np.uint32).reshape(-1, 3, 3).astype(np.uint64)
    # least vertex by (x, y, z) bit patterns, compared lexicographically
    code = (keys[:, :, 0] << np.uint64(32)) | keys[:, :, 1]
    best = np.zeros(len(t), np.int64)
    for i in (1, 2):
        b = best
        cb, ci = code[np.arange(len(t)), b], code[:, i]
        zb, zi = keys[np.arange(len(t)), b, 2], keys[:, i, 2]
        better = (ci < cb) | ((ci == cb) & (zi < zb))
        best = np.where(better, i, b)
    idx = (np.arange(3)[None, :] + best[:, None]) % 3
    rows = np.take_along_axis(t, idx[:, :, None], axis=1).reshape(-1, 9)
    order = np.lexsort(rows.view(np.uint32).T[::-1])
    return rows[order]


def occupied_points(mask, packed, origin, voxel_size, lo=None, hi=None) -> np.ndarray:
    """The map exported as a point cloud (the CSV/PCL export beside the mesh in
    the paper's pipeline figure): the centres of the occupied contact voxels,
    those a return landed in (mask 0) whose hit counter confirmed them (sign
    0), in the box [lo, hi), x fastest, as (n, 3) fp32 with the coordinate
    rule of M2. (The paper does not say which voxels the point export holds;
    this is the reading.)"""
    m = np.asarray(mask, np.uint32)
    p = np.asarray(packed, np.uint32)
    nz, ny, nx = m.shape
    lo = (0, 0, 0) if lo is None else tuple(int(v) for v in lo)
    hi = (nx, ny, nz) if hi is None else tuple(int(v) for v in hi)
    sub = (m[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] == 0) & ((p[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] >> np.uint32(31)) == 0)
    kz, ky, kx = np.nonzero(sub)
    out = np.empty((len(kx), 3), np.float32)
    for col, (k, base) in enumerate(((kx, lo[0]), (ky, lo[1]), (kz, lo[2]))):
        u = (k + base).astype(np.float32)
        out[:, col] = np.float32(origin[col]) + (u + np.float32(0.5)) * np.float32(voxel_size)
    return out

