"""Seeded synthetic pressure-Poisson matrices in CSR form.

The paper's matrices come from its in-house DNS code (second-order finite
differences on a staggered, orthogonal, wall-stretched grid, Section 3) and are
not available; these generators produce stand-ins with the same structure:
a 7-point, cell-centred pressure operator on a structured grid, stored as
general CSR with 32-bit row offsets and column indices and binary64 values
(the storage assumed by the paper's CRS traffic model, Section 2.3).

* ``dirichlet7``: the unit 7-point stencil (diagonal 6, neighbours -1) on a
  uniform grid whose outside neighbours are zero (homogeneous Dirichlet).
* ``channel7``: the finite-volume (flux) form of -div(grad p) on a channel of
  size Lx x Ly x Lz, periodic in x and z, impermeable walls in y (zero normal
  flux, i.e. Neumann), with tanh wall-normal stretching.  Optional solid cells
  (wall-mounted cubes) are removed from the unknowns and their faces carry no
  flux.  The operator is symmetric with zero row sums, so its null space is
  the constant vector.
* ``permute_symmetric``: the relabelling P A P^T (rows and columns together),
  which keeps the diagonal on the diagonal.

Columns within each row are sorted ascending.  This module holds no
arithmetic of the solver.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class CSRMatrix:
    """General CSR: ``row_ptr`` int32[n+1], ``col`` int32[nnz], ``val`` f64[nnz]."""

    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    name: str = ""
    nullspace_const: bool = False
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1]) if self.n > 0 else 0

    def to_dense(self) -> np.ndarray:
        """Dense copy (tiny matrices only); duplicate entries add."""
        d = np.zeros((self.n, self.n))
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        np.add.at(d, (rows, self.col.astype(np.int64)), self.val)
        return d


def _from_padded(cols: np.ndarray, vals: np.ndarray, n: int) -> tuple:
    """CSR arrays from ``(n, K)`` candidate entries; ``cols >= n`` marks a
    missing entry.  Entries are sorted by column within each row."""
    order = np.argsort(cols, axis=1, kind="stable")
    cols = np.take_along_axis(cols, order, axis=1)
    vals = np.take_along_axis(vals, order, axis=1)
    mask = cols < n
    counts = mask.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("nnz does not fit 32-bit row offsets")
    col = cols[mask].astype(np.int32)
    val = vals[mask].astype(np.float64)
    return row_ptr.astype(np.int32), col, val


def dirichlet7(nx: int, ny: int | None = None, nz: int | None = None) -> CSRMatrix:
    """Unit 7-point stencil on an ``nx*ny*nz`` grid, x fastest."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    n = nx * ny * nz
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    idx = np.arange(n, dtype=np.int64)
    sentinel = np.int64(n)
    cols = np.full((n, 7), sentinel, dtype=np.int64)
    vals = np.zeros((n, 7))
    cols[:, 0] = idx
    vals[:, 0] = 6.0
    nbrs = [
        (i > 0, -1), (i < nx - 1, 1),
        (j > 0, -nx), (j < ny - 1, nx),
        (k > 0, -nx * ny), (k < nz - 1, nx * ny),
    ]
    for s, (ok, off) in enumerate(nbrs, start=1):
        cols[ok, s] = idx[ok] + off
        vals[ok, s] = -1.0
    rp, c, v = _from_padded(cols, vals, n)
    return CSRMatrix(n, rp, c, v, name=f"dirichlet7_{nx}x{ny}x{nz}",
                     nullspace_const=False, meta={"shape": (nx, ny, nz)})


def tanh_faces(ny: int, ly: float, beta: float) -> np.ndarray:
    """Wall-normal face coordinates y_0..y_ny, clustered at both walls:
    y_j = (ly/2) * (1 - tanh(beta*(1 - 2j/ny)) / tanh(beta))."""
    jj = np.arange(ny + 1, dtype=np.float64)
    y = 0.5 * ly * (1.0 - np.tanh(beta * (1.0 - 2.0 * jj / ny)) / np.tanh(beta))
    y[0], y[-1] = 0.0, ly
    return y


def channel7(nx: int, ny: int, nz: int, beta: float = 2.0,
             lx: float = 2.0 * np.pi, ly: float = 2.0, lz: float = np.pi,
             solid: np.ndarray | None = None, name: str | None = None) -> CSRMatrix:
    """Flux-form pressure operator on a stretched channel.

    ``solid`` is an optional boolean array of shape ``(nz, ny, nx)`` marking
    cells removed from the unknowns.  Fluid cells are numbered in natural
    order (x fastest, then y, then z).  Off-diagonal coefficients:
    x-faces -dy_j*dz/dx, z-faces -dx*dy_j/dz, y-faces -dx*dz/(yc_{j+1}-yc_j);
    the diagonal is minus the sum of the off-diagonals of its row.
    """
    if nx < 3 or nz < 3:
        raise ValueError("periodic directions need at least 3 cells")
    yf = tanh_faces(ny, ly, beta)
    dy = np.diff(yf)
    yc = 0.5 * (yf[:-1] + yf[1:])
    dx, dz = lx / nx, lz / nz
    cx = dy * dz / dx                      # per j
    cz = dx * dy / dz                      # per j
    cy = dx * dz / np.diff(yc)             # face between j and j+1, j < ny-1

    shape = (nz, ny, nx)
    fluid = np.ones(shape, dtype=bool) if solid is None else ~np.asarray(solid, dtype=bool)
    ncell = nx * ny * nz
    number = np.full(ncell, -1, dtype=np.int64)
    fl = fluid.ravel()
    n = int(fl.sum())
    number[fl] = np.arange(n, dtype=np.int64)
    number = number.reshape(shape)
    sentinel = np.int64(n)

    jgrid = np.broadcast_to(np.arange(ny)[None, :, None], shape)
    cols = np.full(shape + (7,), sentinel, dtype=np.int64)
    vals = np.zeros(shape + (7,))
    diag = np.zeros(shape)

    def put(slot, nbr_num, ok, coef):
        ok = ok & fluid & (nbr_num >= 0)
        cols[..., slot] = np.where(ok, nbr_num, sentinel)
        vals[..., slot] = np.where(ok, -coef, 0.0)
        diag[...] += np.where(ok, coef, 0.0)

    cxg = cx[jgrid]
    czg = cz[jgrid]
    true = np.ones(shape, dtype=bool)
    put(1, np.roll(number, 1, axis=2), true, cxg)    # west (i-1, periodic)
    put(2, np.roll(number, -1, axis=2), true, cxg)   # east (i+1, periodic)
    put(3, np.roll(number, 1, axis=0), true, czg)    # back (k-1, periodic)
    put(4, np.roll(number, -1, axis=0), true, czg)   # front (k+1, periodic)
    # south (j-1) and north (j+1): no face beyond the walls
    south = np.full(shape, -1, dtype=np.int64)
    south[:, 1:, :] = number[:, :-1, :]
    csouth = np.zeros(shape)
    csouth[:, 1:, :] = cy[None, :, None]
    put(5, south, jgrid > 0, csouth)
    north = np.full(shape, -1, dtype=np.int64)
    north[:, :-1, :] = number[:, 1:, :]
    cnorth = np.zeros(shape)
    cnorth[:, :-1, :] = cy[None, :, None]
    put(6, north, jgrid < ny - 1, cnorth)
    cols[..., 0] = np.where(fluid, number, sentinel)
    vals[..., 0] = diag

    cols = cols.reshape(ncell, 7)[fl]
    vals = vals.reshape(ncell, 7)[fl]
    rp, c, v = _from_padded(cols, vals, n)
    nm = name or f"channel7_{nx}x{ny}x{nz}_b{beta:g}"
    return CSRMatrix(n, rp, c, v, name=nm, nullspace_const=True,
                     meta={"shape": (nx, ny, nz), "beta": beta,
                           "lengths": (lx, ly, lz), "y_faces": yf})


def cube_array_solid(nx: int = 192, ny: int = 96, nz: int = 128, ncube: int = 4,
                     h: int = 16, pitch_x: int = 48, pitch_z: int = 32,
                     off_x: int = 16, off_z: int = 8) -> np.ndarray:
    """Solid mask of an ``ncube x ncube`` array of ``h^3``-cell cubes on the
    lower wall: cube (a, b) occupies x in [pitch_x*a+off_x, +h),
    z in [pitch_z*b+off_z, +h), y in [0, h)."""
    solid = np.zeros((nz, ny, nx), dtype=bool)
    for a in range(ncube):
        for b in range(ncube):
            x0 = pitch_x * a + off_x
            z0 = pitch_z * b + off_z
            solid[z0:z0 + h, 0:h, x0:x0 + h] = True
    return solid


def permute_symmetric(A: CSRMatrix, perm: np.ndarray) -> CSRMatrix:
    """``P A P^T``: new row ``r`` is old row ``perm[r]`` with every column
    relabelled the same way; columns re-sorted within rows."""
    n = A.n
    perm = np.asarray(perm, dtype=np.int64)
    inv = np.empty(n, dtype=np.int64)
    inv[perm] = np.arange(n, dtype=np.int64)
    rp_old = A.row_ptr.astype(np.int64)
    lens = np.diff(rp_old)[perm]
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=rp[1:])
    nnz = int(rp[-1])
    src = np.repeat(rp_old[perm] - rp[:-1], lens) + np.arange(nnz, dtype=np.int64)
    newcol = inv[A.col.astype(np.int64)[src]]
    newval = A.val[src]
    kmax = int(lens.max()) if n else 0
    if kmax <= 16:
        # pad every row to kmax slots and sort each row's slots
        slot = np.arange(nnz, dtype=np.int64) - np.repeat(rp[:-1], lens)
        row_of = np.repeat(np.arange(n, dtype=np.int64), lens)
        cols = np.full((n, max(kmax, 1)), n, dtype=np.int64)
        vals = np.zeros((n, max(kmax, 1)))
        cols[row_of, slot] = newcol
        vals[row_of, slot] = newval
        rp32, col, val = _from_padded(cols, vals, n)
    else:
        row_of = np.repeat(np.arange(n, dtype=np.int64), lens)
        order = np.lexsort((newcol, row_of))
        rp32, col, val = rp.astype(np.int32), newcol[order].astype(np.int32), newval[order]
    meta = dict(A.meta)
    meta["perm"] = perm
    return CSRMatrix(n, rp32, col, val, name=A.name + "_perm",
                     nullspace_const=A.nullspace_const, meta=meta)
