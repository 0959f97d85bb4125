"""Checkpoint and resume of a grid (its state after any scans, Sec. III-A).

One ``.npz`` file holds the two planes (uint32, shape (Nz, Ny, Nx)) and a JSON
header with the grid's and the kernel set's parameters, which give the planes
their meaning. Nothing in the file is a pickled object: it loads with
``numpy.load(allow_pickle=False)``. Restoring goes through
``dbtsdf_write_voxels``, which checks the planes' invariants.
"""
from __future__ import annotations

import json

import numpy as np

from . import _lib as L

FORMAT = "dbtsdf-grid-v1"


def save_checkpoint(path: str, grid) -> None:
    """Write ``grid`` (synchronised first) to ``path``."""
    grid.sync()
    mask, packed = grid.read_voxels()
    p = grid.params
    header = dict(format=FORMAT, dims=list(grid.dims), voxel_size=float(p.voxel_size),
                  origin=[float(x) for x in p.origin], hit_threshold=int(p.hit_threshold), hit_max=int(p.hit_max),
                  dedup=bool(p.flags & L.DEDUP_FIRST), kernel=grid.kernel_set.params)
    with open(path, "wb") as f:
        np.savez(f, header=np.array(json.dumps(header)), mask=mask, packed=packed)


def load_checkpoint(path: str, kernel_set=None, **grid_kw):
    """A new grid holding the checkpoint at ``path``. ``kernel_set`` (else one built from the header) must
    have the saved parameters; ``grid_kw`` go to ``Grid`` (e.g. ``planes="torch"``)."""
    from . import Grid, KernelSet
    with np.load(path, allow_pickle=False) as z:
        header = json.loads(str(z["header"]))
        if header.get("format") != FORMAT:
            raise ValueError(f"{path}: not a {FORMAT} checkpoint")
        dims = header.get("dims")
        if not (isinstance(dims, list) and len(dims) == 3 and all(isinstance(d, int) and d > 0 for d in dims)):
            raise ValueError(f"{path}: bad grid dims {dims!r} in the header")
        shape = (dims[2], dims[1], dims[0])
        for name in ("mask", "packed"):
            if z[name].shape != shape or z[name].dtype != np.uint32:
                raise ValueError(f"{path}: {name} plane is {z[name].dtype} {z[name].shape}, "
                                 f"the header's grid needs uint32 {shape}")
        ks = KernelSet(**header["kernel"]) if kernel_set is None else kernel_set
        if ks.params != header["kernel"]:
            raise ValueError(f"kernel set {ks.params} differs from the checkpoint's {header['kernel']}")
        g = Grid(header["dims"], header["voxel_size"], header["origin"], ks, hit_threshold=header["hit_threshold"],
                 hit_max=header["hit_max"], dedup=header["dedup"], **grid_kw)
        g.write_voxels(z["mask"], z["packed"])
    return g
