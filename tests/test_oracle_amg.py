"""Pins for the oracle's classical AMG preconditioner (BiCGStab with classical
algebraic multigrid, Section 4.1; the construction is Ruge-Stueben's).

Independent references: the closed-form coarse operator of the 1-D Laplacian
(every other point coarse, weights 1/2, A_c = A/2 on the coarse grid), a
brute-force C/F splitting that rescans every row for the largest measure,
dense Galerkin products, the splitting's defining properties, constants
reproduced by interpolation, the exact inverse on a one-level hierarchy,
symmetry of the V-cycle for symmetric operators, LAPACK solves, and the
contraction of the stationary V-cycle iteration.
"""
import numpy as np
import pytest

from oracle import amg
from workloads import grids, rng


def tridiag(n):
    rp, ci, va = [0], [], []
    for i in range(n):
        for j, v in ((i - 1, -1.0), (i, 2.0), (i + 1, -1.0)):
            if 0 <= j < n:
                ci.append(j)
                va.append(v)
        rp.append(len(ci))
    return grids.CSRMatrix(n, np.array(rp, dtype=np.int32), np.array(ci, dtype=np.int32), np.array(va))


def small_cases():
    yield grids.dirichlet7(6, 5, 4), False
    solid = np.zeros((6, 4, 8), dtype=bool)
    solid[2:4, 0:2, 3:5] = True
    yield grids.channel7(8, 4, 6, beta=2.0, lx=4.0, ly=2.0, lz=3.0, solid=solid), True


def brute_force_split(S, n):
    """The Ruge-Stueben first pass by direct rescanning (O(n^2))."""
    ST = [[i for i in range(n) if j in S[i]] for j in range(n)]
    state = ["U"] * n
    for i in range(n):
        if not S[i] and not ST[i]:
            state[i] = "F"
    lam = [len(ST[i]) for i in range(n)]
    while "U" in state:
        best = max((lam[i], -i) for i in range(n) if state[i] == "U")
        i = -best[1]
        state[i] = "C"
        for j in ST[i]:
            if state[j] == "U":
                state[j] = "F"
                for k in S[j]:
                    if state[k] == "U":
                        lam[k] += 1
        for k in S[i]:
            if state[k] == "U":
                lam[k] -= 1
    return np.array([1 if s == "C" else 0 for s in state])


def test_1d_laplacian_closed_form():
    n = 15
    A1 = tridiag(n)
    A = amg.canonical(n, A1.row_ptr, A1.col, A1.val)
    S = amg.strength(A)
    cf = amg.rs_split(S, n)
    assert list(np.nonzero(cf)[0]) == list(range(1, n, 2))      # every other point
    P = amg.direct_interpolation(A, S, cf)
    D = P.to_dense()
    for i in range(0, n, 2):                                      # F rows: weight 1/2 to each neighbour
        for j in (i - 1, i + 1):
            if 0 <= j < n:
                assert D[i, j // 2] == 0.5
    Ac = amg.spgemm(amg.transpose(P), amg.spgemm(A, P)).to_dense()
    nc = n // 2
    want = 0.5 * (2 * np.eye(nc) - np.eye(nc, k=1) - np.eye(nc, k=-1))
    assert np.array_equal(Ac, want)


@pytest.mark.parametrize("case", range(2))
def test_split_matches_brute_force_and_its_properties(case):
    A0, _ = list(small_cases())[case]
    A = amg.canonical(A0.n, A0.row_ptr, A0.col, A0.val)
    S = amg.strength(A)
    cf = amg.rs_split(S, A.n_rows)
    assert np.array_equal(cf, brute_force_split(S, A.n_rows))
    Sset = [set(s) for s in S]
    for i in range(A.n_rows):
        if not cf[i] and Sset[i]:
            assert any(cf[j] for j in Sset[i])                   # F rows see a strong C row
        if cf[i]:
            assert not any(cf[j] and i in Sset[j] for j in Sset[i])  # no mutually strong C pair


def test_strength_threshold():
    # row 0: -a = (4, 1, 0.9, -2): threshold 0.25 * 4 = 1 keeps 4 and 1 only
    rp = np.array([0, 5, 6, 7, 8, 9])
    ci = np.array([0, 1, 2, 3, 4, 1, 2, 3, 4])
    va = np.array([10.0, -4.0, -1.0, -0.9, 2.0, 1.0, 1.0, 1.0, 1.0])
    A = amg.canonical(5, rp, ci, va)
    S = amg.strength(A)
    assert S[0] == [1, 2] and S[1] == []


@pytest.mark.parametrize("case", range(2))
def test_galerkin_against_dense(case):
    A0, ns = list(small_cases())[case]
    H = amg.setup(A0.n, A0.row_ptr, A0.col, A0.val, nullspace_const=ns, max_coarse=8)
    assert len(H.levels) >= 3
    for l in range(len(H.levels) - 1):
        lev, nxt = H.levels[l], H.levels[l + 1]
        Pd, Ad = lev.P.to_dense(), lev.A.to_dense()
        assert np.array_equal(lev.R.to_dense(), Pd.T)
        ref = Pd.T @ Ad @ Pd
        assert np.abs(nxt.A.to_dense() - ref).max() <= 1e-13 * np.abs(ref).max()
        # C rows inject; interpolation reproduces constants on zero-row-sum rows
        cidx = np.cumsum(lev.cf) - 1
        for i in np.nonzero(lev.cf)[0]:
            assert Pd[i].tolist() == [1.0 if c == cidx[i] else 0.0 for c in range(Pd.shape[1])]
        rs = Ad.sum(axis=1)
        zero_rows = np.abs(rs) <= 1e-12 * np.abs(Ad).sum(axis=1)
        assert np.all(np.abs(Pd[zero_rows].sum(axis=1) - 1.0) <= 1e-14)
        assert np.all(Pd >= 0.0)


def test_one_level_is_the_exact_inverse():
    A0 = grids.dirichlet7(5, 4, 3)
    H = amg.setup(A0.n, A0.row_ptr, A0.col, A0.val, max_coarse=1000)
    assert len(H.levels) == 1
    B = rng.rhs_block(A0.n, 3, 40)
    X = amg.vcycle(H, B)
    ref = np.linalg.solve(A0.to_dense(), B)
    assert np.abs(X - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("case", range(2))
def test_vcycle_is_symmetric(case):
    A0, ns = list(small_cases())[case]
    H = amg.setup(A0.n, A0.row_ptr, A0.col, A0.val, nullspace_const=ns, max_coarse=8)
    U = rng.rhs_block(A0.n, 2, 41)
    V = rng.rhs_block(A0.n, 2, 42)
    MU, MV = amg.vcycle(H, U), amg.vcycle(H, V)
    lhs, rhs = np.sum(U * MV, axis=0), np.sum(MU * V, axis=0)
    assert np.all(np.abs(lhs - rhs) <= 1e-13 * np.abs(lhs))


def test_vcycle_contracts_the_error():
    """Stationary iteration e <- (I - M^-1 A) e on the 16^3 Dirichlet
    operator: a working two-sided cycle contracts every error component
    (measured factor ~0.39); a wrong weight, a missing coarse correction or
    a transposed transfer pushes it towards or past 1."""
    A0 = grids.dirichlet7(16)
    H = amg.setup(A0.n, A0.row_ptr, A0.col, A0.val)
    A = H.levels[0].A
    e = rng.rhs_block(A0.n, 1, 43)
    rate = 1.0
    for _ in range(15):
        e_new = e - amg.vcycle(H, A.matvec(e))
        rate = np.linalg.norm(e_new) / np.linalg.norm(e)
        e = e_new
    assert rate < 0.5


@pytest.mark.parametrize("case", range(2))
def test_amg_bicgstab_against_lapack(case):
    A0, ns = list(small_cases())[case]
    H = amg.setup(A0.n, A0.row_ptr, A0.col, A0.val, nullspace_const=ns, max_coarse=8)
    A = H.levels[0].A
    B = rng.rhs_block(A0.n, 2, 44, mean_zero=ns)
    D = A0.to_dense()
    for l in range(2):
        x, info = amg.bicgstab(A, H, B[:, l], tol=1e-11, maxit=100, nullspace_const=ns)
        assert info["status"] == 0 and info["relres"] <= 1e-11 and info["iters"] <= 20
        if ns:
            K = np.zeros((A0.n + 1, A0.n + 1))
            K[:A0.n, :A0.n] = D
            K[:A0.n, A0.n] = K[A0.n, :A0.n] = 1.0
            ref = np.linalg.solve(K, np.concatenate([B[:, l], [0.0]]))[:A0.n]
            ev = np.linalg.eigvalsh(D)
            kappa = ev[-1] / ev[1]
        else:
            ref = np.linalg.solve(D, B[:, l])
            ev = np.linalg.eigvalsh(D)
            kappa = ev[-1] / ev[0]
        assert np.linalg.norm(x - ref) <= kappa * 1e-11 * np.linalg.norm(ref) * 1.01


def test_l1_jacobi_weights_closed_form():
    """The l1-Jacobi weights of the unit 7-point Dirichlet stencil: a row's
    absolute sum is 6 plus one per neighbour inside the box, so interior,
    face, edge and corner rows weigh 1/12, 1/11, 1/10 and 1/9."""
    N = 6
    A = grids.dirichlet7(N)
    H = amg.setup(A.n, A.row_ptr, A.col, A.val)
    w = H.levels[0].dl1_inv
    for z in range(N):
        for y in range(N):
            for x in range(N):
                inside = sum(1 for c in (x, y, z) for d in (-1, 1) if 0 <= c + d < N)
                assert w[(z * N + y) * N + x] == 1.0 / (6 + inside)


def test_singular_coarsest_level_solves_mean_free():
    """A channel operator (periodic x, z; Neumann walls) has the constants as
    null space.  With one level the V-cycle applies (A + s 1 1^T)^-1, which on
    a mean-free b returns the mean-free solution of A x = b exactly (to
    rounding): 1^T A = 0 forces 1^T x = 0 and then A x = b."""
    A = grids.channel7(6, 5, 4, beta=2.0)
    H = amg.setup(A.n, A.row_ptr, A.col, A.val, nullspace_const=True, max_coarse=10**6)
    assert len(H.levels) == 1 and H.shift > 0.0
    b = rng.rhs_block(A.n, 3, 55, mean_zero=True)
    x = amg.vcycle(H, b)
    Ad = H.levels[0].A.to_dense()
    assert np.abs(Ad @ x - b).max() <= 1e-11 * np.abs(b).max()
    assert np.abs(x.mean(axis=0)).max() <= 1e-12 * np.abs(x).max()
