"""Oracle of the ensemble projection step (CPU, binary64, numpy).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``: the GPU library never
imports it and it imports nothing from the library.

Section 2.2, eqs. (3)-(4): a substep predicts m velocity fields u*, solves
the pressure Poisson equation lap p = (1/tau) div u* for all m at once, and
corrects u = u* - tau grad p.  Discretised with the finite-volume reading of
the channel pressure operator (pressure at cell centres, face-normal
velocities on the staggered faces):

* divergence(g, U, V, W): for every fluid cell, the sum over its faces of
  face area times outward normal velocity, areas dy_j*dz (x-faces), dx*dz
  (y-faces), dx*dy_j (z-faces); a face on a wall or next to a solid cell
  passes nothing.
* gradient(g, P): on every face between two fluid cells, the pressure
  difference (upper cell minus lower cell) over the distance between the two
  centres: dx, yc_j - yc_{j-1}, dz.  Closed faces get 0.
* correct(g, U, V, W, P, tau) = (U, V, W) - tau * gradient(g, P).
* rhs(g, U, V, W, tau) = -(1/tau) * divergence(g, U, V, W).  The channel
  matrix A (A p = sum over a cell's open faces of area/distance times
  (p_cell - p_neighbour)) satisfies D G = -A, so solving A p = rhs and
  correcting gives D u = D u* - tau D G p = D u* + tau A p = 0.

Face arrays are (rows, m) in the library's layout: U and W have one row per
cell (the x-face west of it, the z-face behind it), V has (ny + 1) rows per
(x, z) column (the y-face below cell j, j = 0..ny).  Every function works on
whole numpy arrays in the order written above; nothing is fused or reordered.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Grid:
    nx: int
    ny: int
    nz: int
    dx: float
    dz: float
    y_faces: np.ndarray
    solid: np.ndarray | None = None  # (nz, ny, nx) bool

    @property
    def fluid(self) -> np.ndarray:
        shape = (self.nz, self.ny, self.nx)
        return np.ones(shape, bool) if self.solid is None else ~np.asarray(self.solid, bool).reshape(shape)

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def v_faces(self) -> int:
        return self.nx * (self.ny + 1) * self.nz

    @property
    def n(self) -> int:
        return int(self.fluid.sum())


def _open_faces(g: Grid):
    """Masks of the open faces: x-face west of each cell, y-face below each
    cell (j = 0..ny), z-face behind each cell."""
    f = g.fluid
    ox = f & np.roll(f, 1, axis=2)                      # cell and its west neighbour (periodic)
    oz = f & np.roll(f, 1, axis=0)                      # cell and its back neighbour (periodic)
    oy = np.zeros((g.nz, g.ny + 1, g.nx), bool)         # face j between cells j-1 and j
    oy[:, 1:g.ny, :] = f[:, 1:, :] & f[:, :-1, :]       # walls (j = 0, ny) stay closed
    return ox, oy, oz


def _geometry(g: Grid):
    yf = np.asarray(g.y_faces, dtype=np.float64)
    dy = np.diff(yf)                                     # cell heights, j = 0..ny-1
    yc = 0.5 * (yf[:-1] + yf[1:])                        # cell centres
    dyc = np.zeros(g.ny + 1)
    dyc[1:g.ny] = np.diff(yc)                            # centre distance across face j
    return dy, dyc


def divergence(g: Grid, U, V, W) -> np.ndarray:
    """(n_fluid, m): sum over each fluid cell's faces of area x outward velocity."""
    m = U.shape[1]
    ox, oy, oz = _open_faces(g)
    dy, _ = _geometry(g)
    U3 = np.where(ox[..., None], U.reshape(g.nz, g.ny, g.nx, m), 0.0)
    V3 = np.where(oy[..., None], V.reshape(g.nz, g.ny + 1, g.nx, m), 0.0)
    W3 = np.where(oz[..., None], W.reshape(g.nz, g.ny, g.nx, m), 0.0)
    ax = (dy * g.dz)[None, :, None, None]                # x-face area of row j
    ay = g.dx * g.dz
    az = (g.dx * dy)[None, :, None, None]
    # outward flux: east face minus west face, north minus south, front minus back
    D = (ax * (np.roll(U3, -1, axis=2) - U3)
         + ay * (V3[:, 1:, :, :] - V3[:, :-1, :, :])
         + az * (np.roll(W3, -1, axis=0) - W3))
    return D[g.fluid]


def gradient(g: Grid, P) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Face-normal pressure gradient on the open faces (U, V, W layout)."""
    m = P.shape[1]
    ox, oy, oz = _open_faces(g)
    _, dyc = _geometry(g)
    P3 = np.zeros((g.nz, g.ny, g.nx, m))
    P3[g.fluid] = P
    GU = np.where(ox[..., None], (P3 - np.roll(P3, 1, axis=2)) / g.dx, 0.0)
    GW = np.where(oz[..., None], (P3 - np.roll(P3, 1, axis=0)) / g.dz, 0.0)
    GV = np.zeros((g.nz, g.ny + 1, g.nx, m))
    inner = (P3[:, 1:, :, :] - P3[:, :-1, :, :]) / np.where(dyc[1:g.ny] > 0, dyc[1:g.ny], 1.0)[None, :, None, None]
    GV[:, 1:g.ny, :, :] = np.where(oy[:, 1:g.ny, :, None], inner, 0.0)
    return (GU.reshape(g.cells, m), GV.reshape(g.v_faces, m), GW.reshape(g.cells, m))


def rhs(g: Grid, U, V, W, tau: float) -> np.ndarray:
    """Pressure right-hand side -(1/tau) D u* of eq. (4) in the sign of the
    positive semidefinite channel matrix A = -lap."""
    return -divergence(g, U, V, W) / tau


def correct(g: Grid, U, V, W, P, tau: float):
    """Eq. (3): the corrected fields U - tau G P (new arrays)."""
    GU, GV, GW = gradient(g, P)
    return U - tau * GU, V - tau * GV, W - tau * GW
