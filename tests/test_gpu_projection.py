"""GPU parity of the ensemble projection step (Section 2.2, eqs. (3)-(4))
against the oracle.

projection_rhs and projection_correct are compared with the oracle element by
element on the same seeded fields (binary64; bound 1e-13 of the sum of the
absolute terms), on channels with solid cells whose cell counts are not
multiples of the kernels' rows per pass, for several m.  The full projection
(rhs, block_bicgstab, correction on the GPU) must leave the divergence of
every corrected field (computed by the oracle) at the solver's tolerance.
"""
import ctypes

import numpy as np
import pytest

from oracle import projection as proj
from workloads import grids, rng, staggered

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


@pytest.fixture(scope="module")
def mrhs():
    import paper_1711_10622_amd as p
    p.load(build_if_missing=False)
    return p


def solid_for(nx, ny, nz):
    s = np.zeros((nz, ny, nx), bool)
    s[1:max(2, nz // 2), 0:max(1, ny // 3), 2:max(3, nx // 2)] = True
    s[nz - 1, ny // 2, 0] = True
    return s


def setup(mrhs, nx, ny, nz, solid):
    geo = staggered.channel_geometry(nx, ny, nz)
    g = proj.Grid(nx, ny, nz, geo["dx"], geo["dz"], geo["y_faces"], solid)
    G = mrhs.ChannelGrid(nx, ny, nz, geo["dx"], geo["dz"], geo["y_faces"], solid)
    return g, G


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _abs_terms(g, U, V, W):
    m = U.shape[1]
    dy = np.diff(g.y_faces)
    U3 = np.abs(U.reshape(g.nz, g.ny, g.nx, m)); V3 = np.abs(V.reshape(g.nz, g.ny + 1, g.nx, m))
    W3 = np.abs(W.reshape(g.nz, g.ny, g.nx, m))
    t = ((dy * g.dz)[None, :, None, None] * (np.roll(U3, -1, axis=2) + U3)
         + g.dx * g.dz * (V3[:, 1:] + V3[:, :-1])
         + (g.dx * dy)[None, :, None, None] * (np.roll(W3, -1, axis=0) + W3))
    return t[g.fluid]


CASES = [(10, 6, 8, True), (37, 9, 5, True), (64, 32, 16, False)]


@pytest.mark.parametrize("nx,ny,nz,with_solid", CASES)
@pytest.mark.parametrize("m", [1, 3, 8, 16])
def test_rhs_parity(torch_cuda, mrhs, nx, ny, nz, with_solid, m):
    solid = solid_for(nx, ny, nz) if with_solid else None
    g, G = setup(mrhs, nx, ny, nz, solid)
    assert G.n == g.n and G.cells == g.cells and G.v_faces == g.v_faces
    U, V, W = staggered.velocity_blocks(nx, ny, nz, m, 40 + m)
    tau = 0.37
    B = G.rhs(dev(torch_cuda, U), dev(torch_cuda, V), dev(torch_cuda, W), tau)
    torch_cuda.cuda.synchronize()
    ref = proj.rhs(g, U, V, W, tau)
    bound = _abs_terms(g, U, V, W) / tau
    assert np.all(np.abs(B.cpu().numpy() - ref) <= 1e-13 * bound)
    D = G.rhs(dev(torch_cuda, U), dev(torch_cuda, V), dev(torch_cuda, W), -1.0).cpu().numpy()
    assert np.all(np.abs(D - proj.divergence(g, U, V, W)) <= 1e-13 * _abs_terms(g, U, V, W))
    G.close()


@pytest.mark.parametrize("nx,ny,nz,with_solid", CASES)
@pytest.mark.parametrize("m", [1, 5, 16])
def test_correct_parity(torch_cuda, mrhs, nx, ny, nz, with_solid, m):
    solid = solid_for(nx, ny, nz) if with_solid else None
    g, G = setup(mrhs, nx, ny, nz, solid)
    U, V, W = staggered.velocity_blocks(nx, ny, nz, m, 60 + m)
    P = rng.rhs_block(g.n, m, 80 + m)
    tau = 0.21
    Ud, Vd, Wd = dev(torch_cuda, U), dev(torch_cuda, V), dev(torch_cuda, W)
    G.correct(Ud, Vd, Wd, dev(torch_cuda, P), tau)
    torch_cuda.cuda.synchronize()
    rU, rV, rW = proj.correct(g, U, V, W, P, tau)
    # both sides form the same pressure difference; the scaling by tau over
    # the distance and the final subtraction round differently (a few ulp of
    # |u*| + |tau G P|)
    for got, ref, orig in ((Ud, rU, U), (Vd, rV, V), (Wd, rW, W)):
        got = got.cpu().numpy()
        assert np.all(np.abs(got - ref) <= 1e-13 * (np.abs(orig) + np.abs(ref - orig)))
    # closed faces untouched, bitwise
    ox, oy, oz = proj._open_faces(g)
    assert np.array_equal(Ud.cpu().numpy()[~ox.ravel()], U[~ox.ravel()])
    assert np.array_equal(Vd.cpu().numpy()[~oy.ravel()], V[~oy.ravel()])
    assert np.array_equal(Wd.cpu().numpy()[~oz.ravel()], W[~oz.ravel()])
    G.close()


def test_argument_errors(torch_cuda, mrhs):
    import paper_1711_10622_amd._lib as L
    geo = staggered.channel_geometry(6, 4, 5)
    lib = L.load()
    h = ctypes.c_void_p()
    yf = np.ascontiguousarray(geo["y_faces"])
    assert lib.grid_create(2, 4, 5, geo["dx"], geo["dz"], yf.ctypes.data, None, ctypes.byref(h)) == L.EINVAL
    bad = yf.copy(); bad[2] = bad[1]
    assert lib.grid_create(6, 4, 5, geo["dx"], geo["dz"], bad.ctypes.data, None, ctypes.byref(h)) == L.EINVAL
    assert lib.grid_create(6, 4, 5, -1.0, geo["dz"], yf.ctypes.data, None, ctypes.byref(h)) == L.EINVAL
    G = mrhs.ChannelGrid(6, 4, 5, geo["dx"], geo["dz"], geo["y_faces"])
    t = torch_cuda
    m = 2
    U = t.zeros((G.cells, m), dtype=t.float64, device="cuda")
    V = t.zeros((G.v_faces, m), dtype=t.float64, device="cuda")
    W = t.zeros((G.cells, m), dtype=t.float64, device="cuda")
    B = t.zeros((G.n, m), dtype=t.float64, device="cuda")
    vp = lambda x: ctypes.c_void_p(x.data_ptr())
    assert lib.projection_rhs(G.handle, vp(U), vp(V), vp(W), 0.0, vp(B), m, None) == L.EINVAL
    assert lib.projection_rhs(G.handle, vp(U), vp(V), vp(W), 1.0, vp(B), 17, None) == L.EINVAL
    assert lib.projection_rhs(G.handle, vp(U), vp(V), vp(U), 1.0, vp(B), m, None) == L.EINVAL
    assert lib.projection_correct(G.handle, vp(U), vp(V), vp(W), vp(V), 1.0, m, None) == L.EINVAL
    assert lib.projection_rhs(G.handle, vp(U), vp(V), vp(W), 1.0, vp(B), m, None) == L.OK
    t.cuda.synchronize()
    G.close()


@pytest.mark.parametrize("name,nx,ny,nz,with_solid,m", [
    ("cube-like", 48, 24, 32, True, 8),
    ("chan128", 128, 64, 64, False, 16),
])
def test_projection_end_to_end(torch_cuda, mrhs, name, nx, ny, nz, with_solid, m):
    """rhs -> block_bicgstab -> correct, all on the GPU: the corrected fields
    are divergence-free to the solve's tolerance (oracle divergence)."""
    solid = solid_for(nx, ny, nz) if with_solid else None
    g, G = setup(mrhs, nx, ny, nz, solid)
    A = grids.channel7(nx, ny, nz, beta=2.0, solid=solid)
    M = mrhs.CsrMatrix.from_csr(A)
    U, V, W = staggered.velocity_blocks(nx, ny, nz, m, 500)
    tau = 0.05
    Ud, Vd, Wd = dev(torch_cuda, U), dev(torch_cuda, V), dev(torch_cuda, W)
    B = G.rhs(Ud, Vd, Wd, tau)
    P, infos, st = M.solve(B, tol=1e-11)
    assert st == 0, infos
    G.correct(Ud, Vd, Wd, P, tau)
    torch_cuda.cuda.synchronize()
    D0 = proj.divergence(g, U, V, W)
    D1 = proj.divergence(g, Ud.cpu().numpy(), Vd.cpu().numpy(), Wd.cpu().numpy())
    assert np.all(np.linalg.norm(D1, axis=0) <= 1e-9 * np.linalg.norm(D0, axis=0))
    M.close()
    G.close()
