"""GPU parity of matrices created with MRHS_CSR_REORDER: the solvers work on
P A P^T (reverse Cuthill-McKee) while every call keeps the caller's numbering.

* gspmv on such a handle uses the caller's arrays: bitwise the plain handle's.
* A reordered solve is the solve of P A P^T with the right-hand sides
  renumbered, so after k iterations its iterate equals the oracle's on
  (P A P^T, P B), renumbered back, up to rounding; converged solves (binary64,
  mixed, odd m, AMG, the server) meet the tolerance and agree with the plain
  handle's solutions within it.
* The hierarchy of a reordered handle is bitwise the oracle's of P A P^T and
  its V-cycle bitwise the plain V-cycle of P A P^T on P B.
"""
import numpy as np
import pytest

import oracle
from oracle import amg as oamg
from helpers import mean_free, true_relres
from paper_1711_10622_amd._lib import SHADOW_SEED
from workloads import configs, grids, rng

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1711_10622_amd as p
    p.load(build_if_missing=False)
    return torch, p


def cube48():
    solid = grids.cube_array_solid(48, 24, 32, ncube=2, h=4, pitch_x=24, pitch_z=16, off_x=4, off_z=4)
    C = grids.channel7(48, 24, 32, beta=2.0, lx=3.0, ly=1.5, lz=2.0, solid=solid)
    return grids.permute_symmetric(C, rng.permutation(C.n, 10622))


@pytest.fixture(scope="module")
def cube(env):
    _, p = env
    A = cube48()
    perm = p.reorder_permutation(A)
    Ap = grids.permute_symmetric(A, perm)
    return A, perm, Ap


def cuda(torch, B):
    return torch.from_numpy(np.ascontiguousarray(B)).cuda()


@pytest.mark.parametrize("m", [1, 3, 8, 16])
def test_gspmv_bitwise_plain(env, cube, m):
    torch, p = env
    A, _, _ = cube
    X = rng.rhs_block(A.n, m, 40 + m)
    Mr = p.CsrMatrix.from_csr(A, reorder=True)
    M0 = p.CsrMatrix.from_csr(A)
    Yr = p.gspmv(Mr, cuda(torch, X)).cpu().numpy()
    Y0 = p.gspmv(M0, cuda(torch, X)).cpu().numpy()
    assert np.array_equal(Yr, Y0)
    assert np.allclose(Yr, oracle.gspmv(A, X), rtol=0, atol=1e-12 * np.abs(Y0).max())
    Mr.close()
    M0.close()


@pytest.mark.parametrize("k", [1, 3, 8])
def test_trajectory_is_that_of_the_renumbered_matrix(env, k):
    torch, p = env
    A = grids.permute_symmetric(grids.dirichlet7(16), rng.permutation(16 ** 3, 31))
    perm = p.reorder_permutation(A)
    Ap = grids.permute_symmetric(A, perm)
    B = configs.WORKLOADS["dir16"].rhs(A.n, 4)
    M = p.CsrMatrix.from_csr(A, reorder=True)
    X, infos, st = M.solve(cuda(torch, B), tol=1e-14, maxit=k)
    X = X.cpu().numpy()
    M.close()
    Xo, io, _ = oracle.bicgstab(Ap, B[perm], tol=1e-14, maxit=k, shadow_seed=SHADOW_SEED)
    assert st == -4 and all(i["iters"] == k for i in infos)
    for l in range(4):
        err = np.linalg.norm(X[perm, l] - Xo[:, l]) / np.linalg.norm(Xo[:, l])
        assert err <= 1e-11, (l, err)
        assert abs(infos[l]["relres"] - io[l]["relres"]) <= 1e-9 * io[l]["relres"]


@pytest.mark.parametrize("m,mixed", [(8, False), (8, True), (3, False), (7, True), (16, True)])
def test_converged_solves_agree_with_plain(env, cube, m, mixed):
    torch, p = env
    A, _, _ = cube
    B = rng.rhs_block(A.n, m, 900 + m, mean_zero=True)
    X0 = rng.rhs_block(A.n, m, 950 + m)
    out = []
    for reorder in (False, True):
        M = p.CsrMatrix.from_csr(A, reorder=reorder)
        X, infos, st = M.solve(cuda(torch, B), tol=1e-10, maxit=20000, mixed=mixed, X0=cuda(torch, X0))
        X = X.cpu().numpy()
        M.close()
        assert st == 0, infos
        assert np.all(true_relres(A, X, B) <= 1e-10)
        out.append(X)
    d = np.linalg.norm(mean_free(out[1]) - mean_free(out[0]), axis=0) / np.linalg.norm(mean_free(out[0]), axis=0)
    assert np.all(d <= 1e-5), d


def test_hierarchy_and_vcycle_of_renumbered_matrix(env, cube):
    torch, p = env
    A, perm, Ap = cube
    Mr = p.CsrMatrix.from_csr(A, reorder=True)
    Hr = p.AmgHierarchy(Mr)
    ref = oamg.setup(Ap.n, Ap.row_ptr, Ap.col, Ap.val, nullspace_const=True)
    assert Hr.levels == len(ref.levels)
    for l, lev in enumerate(ref.levels):
        rp, ci, va = Hr.level_arrays(l, "A")
        assert np.array_equal(rp, lev.A.rp) and np.array_equal(ci, lev.A.ci) and np.array_equal(va, lev.A.va)
    Mp = p.CsrMatrix.from_csr(Ap)
    Hp = p.AmgHierarchy(Mp)
    for m in (1, 5, 8):
        B = rng.rhs_block(A.n, m, 300 + m)
        Xr = Hr.vcycle(cuda(torch, B)).cpu().numpy()
        Xp = Hp.vcycle(cuda(torch, B[perm])).cpu().numpy()
        assert np.array_equal(Xr[perm], Xp), m
    B = rng.rhs_block(A.n, 8, 777, mean_zero=True)
    X, infos, st = Hr.solve(cuda(torch, B), tol=1e-10, maxit=200)
    X = X.cpu().numpy()
    assert st == 0, infos
    assert np.all(true_relres(A, X, B) <= 1e-10)
    Xp, _, stp = Hp.solve(cuda(torch, B[perm]), tol=1e-10, maxit=200)
    assert stp == 0
    assert np.array_equal(X[perm], Xp.cpu().numpy())
    for h in (Hr, Hp, Mr, Mp):
        h.close()


@pytest.mark.parametrize("mixed", [False, True])
def test_server_with_renumbered_matrix(env, cube, mixed):
    torch, p = env
    A, _, _ = cube
    M = p.CsrMatrix.from_csr(A, reorder=True)
    srv = p.SolveServer(4 << 30, mixed=mixed)
    mid = srv.register(M)
    sent = []
    for i, k in enumerate((3, 1, 6, 2)):
        B = rng.rhs_block(A.n, k, 500 + i, mean_zero=True)
        sent.append((B, srv.submit(mid, B, tol=1e-10)))
    for B, t in sent:
        X, infs, st = srv.wait(t, timeout=120)
        assert st == 0, infs
        assert np.all(true_relres(A, X, B) <= 1e-10)
    srv.close()
    M.close()


def test_degenerate_matrices(env):
    """Renumbering an empty matrix, a single row and a diagonal matrix (every
    row its own component): creation, products and solves behave as without
    renumbering."""
    torch, p = env
    from workloads.grids import CSRMatrix
    E = CSRMatrix(0, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0))
    Me = p.CsrMatrix.from_csr(E, reorder=True)
    Me.close()
    for n in (1, 37):
        D = CSRMatrix(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32),
                      np.linspace(1.0, 2.0, n))
        assert np.array_equal(np.sort(p.reorder_permutation(D)), np.arange(n))
        B = rng.rhs_block(n, 3, 88)
        M = p.CsrMatrix.from_csr(D, reorder=True)
        Y = p.gspmv(M, cuda(torch, B)).cpu().numpy()
        assert np.array_equal(Y, D.val[:, None] * B)
        X, infos, st = M.solve(cuda(torch, B), tol=1e-12, maxit=10)
        assert st == 0, infos
        assert np.allclose(X.cpu().numpy(), B / D.val[:, None], rtol=1e-12, atol=0)
        M.close()
