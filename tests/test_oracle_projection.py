"""Pins of the projection-step oracle (Section 2.2, eqs. (3)-(4)) against facts
that do not come from the oracle itself:

* D G = -A with A the channel pressure matrix built independently by
  ``grids.channel7`` (coefficients area/distance, diagonal = minus the row's
  off-diagonals), with solid cells;
* a discrete stream-function field is divergence-free to rounding, which
  fixes the face areas (a wrong area breaks the cancellation);
* the divergence sums to zero over the domain (fluxes telescope: periodic in
  x and z, closed walls and solids);
* a single open face's flux appears with opposite signs in its two cells, with
  the exact area;
* the full projection (rhs, oracle BiCGStab, correction) leaves D u at the
  solver's residual.
"""
import numpy as np
import pytest

import oracle
from oracle import projection as proj
from workloads import grids, rng, staggered


def make(nx, ny, nz, solid=None, beta=2.0):
    geo = staggered.channel_geometry(nx, ny, nz, beta=beta)
    g = proj.Grid(nx, ny, nz, geo["dx"], geo["dz"], geo["y_faces"], solid)
    A = grids.channel7(nx, ny, nz, beta=beta, solid=solid)
    return g, A


def small_solid(nx=10, ny=6, nz=8):
    s = np.zeros((nz, ny, nx), bool)
    s[2:5, 0:2, 3:6] = True   # a block on the lower wall
    s[6, 3, 0] = True         # an isolated solid cell at the periodic seam
    return s


@pytest.mark.parametrize("solid", [None, "block"])
def test_div_grad_is_minus_channel_matrix(solid):
    nx, ny, nz = 10, 6, 8
    s = small_solid(nx, ny, nz) if solid else None
    g, A = make(nx, ny, nz, s)
    assert g.n == A.n
    P = rng.rhs_block(A.n, 3, 77)
    GU, GV, GW = proj.gradient(g, P)
    DG = proj.divergence(g, GU, GV, GW)
    AP = oracle.gspmv(A, P)
    absA = grids.CSRMatrix(A.n, A.row_ptr, A.col, np.abs(A.val))
    scale = oracle.gspmv(absA, np.abs(P))
    assert np.all(np.abs(DG + AP) <= 1e-13 * scale)


def test_stream_function_field_is_divergence_free():
    """psi on the cell corners (x-face, y-face), periodic in x, constant on
    each wall: U = (psi(i, j+1) - psi(i, j)) / dy_j and
    V = -(psi(i+1, j) - psi(i, j)) / dx carry fluxes that cancel around
    every cell; W = 0."""
    nx, ny, nz = 12, 7, 5
    g, _ = make(nx, ny, nz)
    dy = np.diff(g.y_faces)
    r = np.random.default_rng(5)
    psi = r.uniform(-1, 1, size=(nz, ny + 1, nx))
    psi[:, 0, :] = 0.3
    psi[:, ny, :] = -0.7
    U = (psi[:, 1:, :] - psi[:, :-1, :]) / dy[None, :, None]
    V = -(np.roll(psi, -1, axis=2) - psi) / g.dx
    W = np.zeros((nz, ny, nx))
    D = proj.divergence(g, U.reshape(-1, 1), V.reshape(-1, 1), W.reshape(-1, 1))
    flux_scale = g.dz * (np.abs(psi).max())
    assert np.all(np.abs(D) <= 1e-14 * flux_scale * 8)
    # the same field with the x-face area taken as dx*dz instead of dy_j*dz
    wrong = (g.dx * g.dz) * (np.roll(U, -1, axis=2) - U) + g.dx * g.dz * (V[:, 1:, :] - V[:, :-1, :])
    assert np.abs(wrong).max() > 1e-3


def test_divergence_telescopes_to_zero():
    nx, ny, nz = 10, 6, 8
    g, _ = make(nx, ny, nz, small_solid(nx, ny, nz))
    U, V, W = staggered.velocity_blocks(nx, ny, nz, 4, 123)
    D = proj.divergence(g, U, V, W)
    total = np.abs(D).sum(axis=0)
    assert np.all(np.abs(D.sum(axis=0)) <= 1e-13 * total)


def test_single_face_flux():
    nx, ny, nz = 6, 4, 5
    g, _ = make(nx, ny, nz)
    dy = np.diff(g.y_faces)
    U = np.zeros((g.cells, 1)); V = np.zeros((g.v_faces, 1)); W = np.zeros((g.cells, 1))
    i, j, k = 0, 2, 3                       # x-face west of cell (0, 2, 3): the periodic seam
    U[(k * ny + j) * nx + i] = 1.0
    D = proj.divergence(g, U, V, W).reshape(nz, ny, nx)
    area = dy[j] * g.dz
    assert D[k, j, i] == -area and D[k, j, nx - 1] == area
    assert np.count_nonzero(D) == 2
    # a wall face (j = 0 row of V) carries nothing
    V[(k * (ny + 1) + 0) * nx + 2] = 5.0
    assert np.array_equal(proj.divergence(g, U, V, W).reshape(nz, ny, nx), D)


def test_projection_with_oracle_solve():
    nx, ny, nz = 10, 6, 8
    s = small_solid(nx, ny, nz)
    g, A = make(nx, ny, nz, s)
    U, V, W = staggered.velocity_blocks(nx, ny, nz, 2, 9)
    tau = 0.01
    b = proj.rhs(g, U, V, W, tau)
    P, info, _ = oracle.bicgstab(A, b, tol=1e-12)
    assert all(i["status"] == 0 for i in info)
    U2, V2, W2 = proj.correct(g, U, V, W, P, tau)
    D0 = proj.divergence(g, U, V, W)
    D1 = proj.divergence(g, U2, V2, W2)
    assert np.all(np.linalg.norm(D1, axis=0) <= 1e-10 * np.linalg.norm(D0, axis=0))
    # closed faces keep their values
    ox, oy, oz = proj._open_faces(g)
    assert np.array_equal(U2[~ox.ravel()], U[~ox.ravel()])
    assert np.array_equal(V2[~oy.ravel()], V[~oy.ravel()])
