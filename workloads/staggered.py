"""Synthetic inputs of the ensemble projection step: the staggered channel
geometry (the same faces and spacings as ``grids.channel7``) and seeded
preliminary velocity fields u* for m realizations.

This module holds no arithmetic of the method: velocities are i.i.d. U[-1, 1)
draws of ``rng`` (one stream per component), geometry is the grid generator's.
"""
from __future__ import annotations

import numpy as np

from . import grids, rng


def channel_geometry(nx: int, ny: int, nz: int, beta: float = 2.0, lx: float = 2.0 * np.pi,
                     ly: float = 2.0, lz: float = np.pi) -> dict:
    """dx, dz and the wall-normal face coordinates of ``grids.channel7`` with
    the same arguments."""
    return {"nx": nx, "ny": ny, "nz": nz, "dx": lx / nx, "dz": lz / nz,
            "y_faces": grids.tanh_faces(ny, ly, beta)}


def velocity_blocks(nx: int, ny: int, nz: int, m: int, seed: int):
    """(U, V, W) face blocks of m preliminary fields: U and W with
    nx*ny*nz rows, V with nx*(ny+1)*nz rows, all values U[-1, 1).  Values on
    closed faces (walls, solids) are drawn too; the projection ignores them."""
    cells = nx * ny * nz
    return (rng.rhs_block(cells, m, seed),
            rng.rhs_block(nx * (ny + 1) * nz, m, seed + 1),
            rng.rhs_block(cells, m, seed + 2))
