"""Pins for the oracle's per-column Jacobi BiCGStab (Section 2.2: one matrix,
m right-hand sides; BiCGStab as cited in Section 1).

Independent references: LAPACK dense solves (plain and bordered for the
singular Neumann/periodic operator), scipy's BiCGStab trajectory with the same
right preconditioner, closed-form condition numbers for manufactured
solutions, finite termination on an operator with two distinct eigenvalues,
one-step convergence on a diagonal operator, and an exactly-zero sigma.
The random shadow residual (a SplitMix64 vector) is pinned against the
workload generator's independent implementation of the same stream, and the
solve pins run in both shadow modes.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spl

import oracle
from workloads import grids, rng

SEED = 17110622          # the library's MRHS_SHADOW_SEED
SHADOWS = [None, SEED]   # r^ = r0, and the random shadow vector


def dense_to_csr(D):
    S = sp.csr_matrix(D)
    S.sort_indices()
    return grids.CSRMatrix(D.shape[0], S.indptr.astype(np.int32), S.indices.astype(np.int32),
                           S.data.astype(np.float64))


def scipy_of(A):
    return sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n, A.n))


def test_shadow_vector_is_the_splitmix64_stream():
    for n, seed in ((1, SEED), (1000, SEED), (4097, 12345)):
        ref = rng.uniform_pm1(seed, np.arange(n, dtype=np.uint64))
        assert np.array_equal(oracle.shadow(n, seed), ref)
    v = oracle.shadow(200000, SEED)
    assert -1.0 <= v.min() and v.max() < 1.0 and abs(v.mean()) < 0.01


@pytest.mark.parametrize("shadow", SHADOWS)
@pytest.mark.parametrize("N", [4, 5, 6])
def test_dense_lapack_dirichlet(N, shadow):
    A = grids.dirichlet7(N)
    B = rng.rhs_block(A.n, 3, 21)
    X, infos, _ = oracle.bicgstab(A, B, tol=1e-12, shadow_seed=shadow)
    ref = np.linalg.solve(A.to_dense(), B)
    lam = [3 * (2 - 2 * np.cos(q * np.pi / (N + 1))) for q in (1, N)]
    kappa = lam[1] / lam[0]
    for l in range(3):
        assert infos[l]["status"] == 0
        err = np.linalg.norm(X[:, l] - ref[:, l]) / np.linalg.norm(ref[:, l])
        assert err <= kappa * 1e-12 * 1.01


@pytest.mark.parametrize("shadow", SHADOWS)
def test_bordered_lapack_singular_channel(shadow):
    nx, ny, nz = 6, 4, 6
    solid = np.zeros((nz, ny, nx), dtype=bool)
    solid[2:4, 0:2, 2:4] = True
    A = grids.channel7(nx, ny, nz, beta=2.0, lx=6.0, ly=4.0, lz=6.0, solid=solid)
    assert A.n == nx * ny * nz - 8
    B = rng.rhs_block(A.n, 2, 22, mean_zero=True)
    X, infos, _ = oracle.bicgstab(A, B, tol=1e-11, nullspace_const=True, shadow_seed=shadow)
    D = A.to_dense()
    K = np.zeros((A.n + 1, A.n + 1))
    K[:A.n, :A.n] = D
    K[:A.n, A.n] = 1.0
    K[A.n, :A.n] = 1.0
    ev = np.linalg.eigvalsh(D)
    kappa = ev[-1] / ev[1]               # on the complement of the null space
    for l in range(2):
        rhs = np.concatenate([B[:, l], [0.0]])
        ref = np.linalg.solve(K, rhs)[:A.n]
        assert infos[l]["status"] == 0
        assert abs(X[:, l].mean()) <= 1e-14 * np.abs(X[:, l]).max()
        err = np.linalg.norm(X[:, l] - ref) / np.linalg.norm(ref)
        assert err <= kappa * 1e-11 * 1.01


def nonsymmetric_stencil(N):
    """Dirichlet 7-point operator with an upwind-like skew in x: (6, -1.3, -0.7)."""
    A = grids.dirichlet7(N)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    val = A.val.copy()
    val[A.col == rows - 1] = -1.3
    val[A.col == rows + 1] = -0.7
    return grids.CSRMatrix(A.n, A.row_ptr, A.col, val)


def test_trajectory_matches_scipy_bicgstab():
    A = nonsymmetric_stencil(10)
    S = scipy_of(A)
    b = rng.rhs_block(A.n, 1, 23)[:, 0]
    dinv = 1.0 / S.diagonal()
    M = spl.LinearOperator(S.shape, matvec=lambda v: dinv * v)
    xs = []
    x_sp, code = spl.bicgstab(S, b, rtol=1e-10, atol=0.0, M=M, maxiter=500,
                              callback=lambda xk: xs.append(xk.copy()))
    assert code == 0
    nb = np.linalg.norm(b)
    sp_hist = [1.0] + [np.linalg.norm(b - S @ xk) / nb for xk in xs]
    X, infos, hist = oracle.bicgstab(A, b[:, None], tol=1e-10, hist_len=200)
    assert infos[0]["status"] == 0 and infos[0]["restarts"] == 0
    assert abs(infos[0]["iters"] - len(xs)) <= 1
    # BiCGStab's irregular convergence (residual spikes) amplifies rounding
    # differences to ~1e-8 relative within 20 steps; 1e-7 still fails on any
    # changed term, sign or index.
    k = min(20, len(xs))
    h = hist[0, :k + 1]
    assert np.all(np.abs(h - np.array(sp_hist[:k + 1])) <= 1e-7 * np.array(sp_hist[:k + 1]))
    assert np.linalg.norm(X[:, 0] - x_sp) <= 1e-8 * np.linalg.norm(x_sp)


@pytest.mark.parametrize("shadow", SHADOWS)
def test_finite_termination_two_eigenvalues(shadow):
    n, c, a = 50, 3.0, 0.05
    D = c * np.eye(n) + a * np.ones((n, n))      # constant diagonal c + a
    A = dense_to_csr(D)
    B = rng.rhs_block(n, 2, 24)
    X, infos, _ = oracle.bicgstab(A, B, tol=1e-12, shadow_seed=shadow)
    for inf in infos:
        assert inf["status"] == 0
        assert inf["iters"] <= 2
        assert inf["relres"] <= 1e-12


@pytest.mark.parametrize("shadow", SHADOWS)
def test_diagonal_operator_one_step(shadow):
    n = 37
    d = 1.0 + np.arange(n) / 7.0
    A = dense_to_csr(np.diag(d))
    b = rng.rhs_block(n, 1, 25)
    X, infos, _ = oracle.bicgstab(A, b, tol=1e-14, shadow_seed=shadow)
    assert infos[0]["iters"] == 1 and infos[0]["status"] == 0
    assert np.allclose(X[:, 0], b[:, 0] / d, rtol=1e-15, atol=0)


def test_forced_breakdown():
    A = dense_to_csr(np.array([[1.0, -1.25], [-1.25, 1.0]]))
    b = np.array([[1.0], [2.0]])
    # sigma = b^T A b = 1 - 5 + 4 = 0 exactly
    assert float(b[:, 0] @ A.to_dense() @ b[:, 0]) == 0.0
    X, infos, _ = oracle.bicgstab(A, b, tol=1e-10, maxit=50)
    inf = infos[0]
    assert inf["status"] == oracle.EBREAKDOWN
    assert inf["breakdowns"] == 4 and inf["restarts"] == 3 and inf["iters"] == 4


@pytest.mark.parametrize("shadow", SHADOWS)
def test_forced_breakdown_any_shadow(shadow):
    # b spans the null space of a singular operator: v = A p = 0, so sigma = 0
    # whatever the shadow residual; every restart meets it again
    A = dense_to_csr(np.array([[1.0, -1.0], [-1.0, 1.0]]))
    X, infos, _ = oracle.bicgstab(A, np.array([[1.0], [1.0]]), tol=1e-10, maxit=50, shadow_seed=shadow)
    inf = infos[0]
    assert inf["status"] == oracle.EBREAKDOWN
    assert inf["breakdowns"] == 4 and inf["restarts"] == 3 and inf["iters"] == 4


def test_random_shadow_converges_like_r0():
    # both shadow choices reach the tolerance on the 16^3 Dirichlet operator
    # in a similar number of iterations
    A = grids.dirichlet7(16)
    B = rng.rhs_block(A.n, 2, 26)
    _, i0, _ = oracle.bicgstab(A, B, tol=1e-10)
    _, i1, _ = oracle.bicgstab(A, B, tol=1e-10, shadow_seed=SEED)
    for a, b in zip(i0, i1):
        assert a["status"] == b["status"] == 0 and b["relres"] <= 1e-10
        assert abs(a["iters"] - b["iters"]) <= 0.25 * a["iters"]


def test_manufactured_integer_solution():
    N = 16
    A = grids.dirichlet7(N)
    xstar = rng.int_block(A.n, 2, 26, -50, 50)
    B = oracle.gspmv(A, xstar)                   # exact: integers below 2**53
    X, infos, _ = oracle.bicgstab(A, B, tol=1e-10)
    lmin = 3 * (2 - 2 * np.cos(np.pi / (N + 1)))
    lmax = 3 * (2 - 2 * np.cos(N * np.pi / (N + 1)))
    assert abs(lmax / lmin - 116.46) < 0.01
    for l in range(2):
        err = np.linalg.norm(X[:, l] - xstar[:, l]) / np.linalg.norm(xstar[:, l])
        assert err <= (lmax / lmin) * infos[l]["relres"] * 1.0001


def test_iteration_count_small_dirichlet():
    A = grids.dirichlet7(16)
    B = rng.rhs_block(A.n, 4, 1711)
    X, infos, _ = oracle.bicgstab(A, B, tol=1e-10)
    for inf in infos:
        assert inf["status"] == 0 and inf["restarts"] == 0
        assert 40 <= inf["iters"] <= 70
        assert inf["relres"] <= 1e-10


def test_maxit_reports_noconv():
    A = grids.dirichlet7(8)
    B = rng.rhs_block(A.n, 1, 27)
    X, infos, _ = oracle.bicgstab(A, B, tol=1e-10, maxit=1)
    assert infos[0]["status"] == oracle.ENOCONV and infos[0]["iters"] == 1
    assert 0 < infos[0]["relres"] < 1


def test_nan_column_isolated_and_zero_rhs():
    A = grids.dirichlet7(6)
    B = rng.rhs_block(A.n, 3, 28)
    B[:, 2] = 0.0
    Bn = B.copy()
    Bn[5, 1] = np.nan
    X, infos, _ = oracle.bicgstab(A, B, tol=1e-10)
    Xn, infos_n, _ = oracle.bicgstab(A, Bn, tol=1e-10)
    assert infos_n[1]["status"] == oracle.EBREAKDOWN
    assert np.array_equal(X[:, 0], Xn[:, 0])
    assert infos[2]["status"] == 0 and infos[2]["iters"] == 0 and np.all(X[:, 2] == 0)


def test_zero_diagonal_rejected():
    A = dense_to_csr(np.array([[0.0, 1.0], [1.0, 2.0]]))
    X, infos, _ = oracle.bicgstab(A, np.ones((2, 1)))
    assert infos[0]["status"] == oracle.EINVAL


def test_initial_guess_exact():
    A = grids.dirichlet7(6)
    xstar = rng.int_block(A.n, 1, 29, -5, 5)
    B = oracle.gspmv(A, xstar)
    X, infos, _ = oracle.bicgstab(A, B, tol=1e-10, X0=xstar)
    assert infos[0]["iters"] == 0 and infos[0]["status"] == 0
    assert np.array_equal(X, xstar)


@pytest.mark.parametrize("shadow", SHADOWS)
def test_restart_continues_as_a_fresh_start(shadow):
    """A restart from the true residual is a fresh start from the current
    iterate: the shadow residual is re-taken as the new residual (r^ = r0
    mode) or stays the one fixed vector (random mode), and the recurrence
    scalars reset.  So the residual history after the first restart must
    equal, bit for bit, that of a new solve started at the restart iterate.
    A tolerance below the attainable accuracy forces the restarts: the
    recurrence residual keeps falling while the true one stalls."""
    A = grids.channel7(16, 12, 8, beta=2.0)
    B = rng.rhs_block(A.n, 1, 31, mean_zero=True)
    tol = 1e-15
    K = None
    for mx in range(60, 200):  # smallest maxit that ends right at the first restart
        Xk, inf, _ = oracle.bicgstab(A, B, tol=tol, maxit=mx, shadow_seed=shadow, nullspace_const=False)
        if inf[0]["restarts"] >= 1:
            K = mx
            break
    assert K is not None and inf[0]["status"] == oracle.ENOCONV
    J = 30
    _, inf_l, hist_l = oracle.bicgstab(A, B, tol=tol, maxit=K + J, shadow_seed=shadow, hist_len=K + J + 1,
                                       nullspace_const=False)
    _, inf_f, hist_f = oracle.bicgstab(A, B, tol=tol, maxit=J, shadow_seed=shadow, hist_len=J + 1, X0=Xk,
                                       nullspace_const=False)
    assert inf_l[0]["restarts"] >= 2          # the continuation restarts again
    a, b = hist_l[0, K:K + J + 1], hist_f[0, :J + 1]
    used = ~np.isnan(a)
    assert used.sum() >= 8 and np.array_equal(np.isnan(a), np.isnan(b))
    assert np.array_equal(a[used], b[used])
    assert inf_l[0]["restarts"] - 1 == inf_f[0]["restarts"]
    assert inf_l[0]["iters"] - K == inf_f[0]["iters"]
