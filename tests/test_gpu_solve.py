"""GPU parity of the block BiCGStab solve (Section 2.2: one matrix, m
right-hand sides) against the FP64 oracle.

Several solutions satisfy the stopping rule, so parity is: every column's
true relative residual (recomputed with compensated products) <= tol, the
solution within kappa * 2 tol of the oracle's (mean-free for the singular
channel operator), and iteration counts within 10% of the oracle's.
"""
import numpy as np
import pytest

import oracle
from helpers import mean_free, true_relres
from paper_1711_10622_amd._lib import SHADOW_SEED
from workloads import configs, grids, rng

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


def gpu_solve(mrhs, torch, A, B, **kw):
    M = mrhs.CsrMatrix.from_csr(A)
    Bt = torch.from_numpy(np.ascontiguousarray(B)).to("cuda")
    X0 = kw.pop("X0", None)
    if X0 is not None:
        kw["X0"] = torch.from_numpy(np.ascontiguousarray(X0)).to("cuda")
    X, infos, st = M.solve(Bt, **kw)
    torch.cuda.synchronize()
    out = X.cpu().numpy()
    M.close()
    return out, infos, st


def dir16_kappa():
    N = 16
    return (2 - 2 * np.cos(N * np.pi / (N + 1))) / (2 - 2 * np.cos(np.pi / (N + 1)))


@pytest.mark.parametrize("mixed", [False, True])
def test_dir16_m4(torch_cuda, mrhs, mixed):
    A = configs.MATRICES["dir16"]()
    B = configs.WORKLOADS["dir16"].rhs(A.n, 4)
    X, infos, st = gpu_solve(mrhs, torch_cuda, A, B, tol=1e-10, mixed=mixed)
    Xo, io, _ = oracle.bicgstab(A, B, tol=1e-10, shadow_seed=SHADOW_SEED)
    assert st == 0
    rr = true_relres(A, X, B)
    assert np.all(rr <= 1e-10), rr
    for l in range(4):
        assert infos[l]["status"] == 0
        assert abs(infos[l]["relres"] - rr[l]) <= 1e-3 * rr[l] + 1e-16
        err = np.linalg.norm(X[:, l] - Xo[:, l]) / np.linalg.norm(Xo[:, l])
        assert err <= dir16_kappa() * 2e-10
        if not mixed:
            assert abs(infos[l]["iters"] - io[l]["iters"]) <= max(2, 0.1 * io[l]["iters"])


@pytest.mark.parametrize("m", [1, 3, 8, 16])
def test_channel_small_all_shapes(torch_cuda, mrhs, m):
    A = grids.channel7(32, 16, 24, beta=2.0)
    B = rng.rhs_block(A.n, m, 700 + m, mean_zero=True)
    X, infos, st = gpu_solve(mrhs, torch_cuda, A, B, tol=1e-10)
    assert st == 0
    assert np.all(true_relres(A, X, B) <= 1e-10)
    assert np.abs(X.mean(axis=0)).max() <= 1e-12 * np.abs(X).max()
    Xo, io, _ = oracle.bicgstab(A, B[:, :2], tol=1e-10, shadow_seed=SHADOW_SEED)
    for l in range(min(m, 2)):
        assert abs(infos[l]["iters"] - io[l]["iters"]) <= max(3, 0.1 * io[l]["iters"])
        assert np.linalg.norm(mean_free(X[:, l:l + 1]) - Xo[:, l:l + 1]) <= 1e-6 * np.linalg.norm(Xo[:, l])


@pytest.mark.parametrize("m", [1, 2, 3, 5, 6, 7, 9, 10, 12, 13, 15])
def test_channel_small_mixed_all_widths(torch_cuda, mrhs, m):
    """Mixed precision at block widths whose binary32 lanes hold 1 (odd m),
    2 (m = 2 mod 4) or 4 columns, with the shadow residual's sign bytes laid
    out per lane: every column reaches the binary64 true residual 1e-10 and
    agrees with the binary64 block solve."""
    A = grids.channel7(32, 16, 24, beta=2.0)
    B = rng.rhs_block(A.n, m, 710 + m, mean_zero=True)
    X, infos, st = gpu_solve(mrhs, torch_cuda, A, B, tol=1e-10, mixed=True)
    assert st == 0, infos
    assert np.all(true_relres(A, X, B) <= 1e-10)
    X64, _, st64 = gpu_solve(mrhs, torch_cuda, A, B, tol=1e-10)
    assert st64 == 0
    err = np.linalg.norm(mean_free(X) - mean_free(X64), axis=0) / np.linalg.norm(mean_free(X64), axis=0)
    assert np.all(err <= 1e-5), err


def test_mixed_nan_and_zero_columns_isolated(torch_cuda, mrhs):
    """Mixed precision: a zero right-hand side returns x = 0 at once, a NaN
    column fails alone, and the other columns still converge."""
    A = grids.dirichlet7(10)
    B = rng.rhs_block(A.n, 6, 910)
    B[:, 4] = 0.0
    X1, i1, st1 = gpu_solve(mrhs, torch_cuda, A, B, tol=1e-10, mixed=True)
    assert st1 == 0 and i1[4]["iters"] == 0 and np.all(X1[:, 4] == 0)
    Bn = B.copy()
    Bn[11, 2] = np.nan
    Xn, inn, st = gpu_solve(mrhs, torch_cuda, A, Bn, tol=1e-10, mixed=True)
    assert st < 0 and inn[2]["status"] < 0
    for l in (0, 1, 3, 5):
        assert inn[l]["status"] == 0
        assert np.all(true_relres(A, Xn[:, l:l + 1], B[:, l:l + 1]) <= 1e-10)


def test_block_equals_singles(torch_cuda, mrhs):
    A = grids.dirichlet7(12, 10, 14)
    B = rng.rhs_block(A.n, 5, 800)
    X, infos, st = gpu_solve(mrhs, torch_cuda, A, B, tol=1e-11)
    # Block and single solves sum their dot products in different orders; at
    # tol 1e-11 plain BiCGStab's iteration count moves by up to ~10% under a
    # change of summation order alone (51-58 on this problem in binary64 on
    # the CPU), so counts are compared to that bound.
    for l in range(5):
        x1, i1, _ = gpu_solve(mrhs, torch_cuda, A, np.ascontiguousarray(B[:, l:l + 1]), tol=1e-11)
        assert abs(i1[0]["iters"] - infos[l]["iters"]) <= max(3, 0.1 * infos[l]["iters"])
        assert np.linalg.norm(x1[:, 0] - X[:, l]) <= 1e-8 * np.linalg.norm(X[:, l])


def test_nan_column_isolated_zero_rhs_and_determinism(torch_cuda, mrhs):
    A = grids.dirichlet7(10)
    B = rng.rhs_block(A.n, 4, 900)
    B[:, 2] = 0.0
    X1, i1, _ = gpu_solve(mrhs, torch_cuda, A, B, tol=1e-10)
    X2, _, _ = gpu_solve(mrhs, torch_cuda, A, B, tol=1e-10)
    assert np.array_equal(X1, X2)                 # bitwise reproducible
    assert i1[2]["status"] == 0 and i1[2]["iters"] == 0 and np.all(X1[:, 2] == 0)
    Bn = B.copy()
    Bn[7, 1] = np.nan
    Xn, inn, st = gpu_solve(mrhs, torch_cuda, A, Bn, tol=1e-10)
    assert st == -5 and inn[1]["status"] == -5
    for l in (0, 3):
        assert np.array_equal(Xn[:, l], X1[:, l])  # other columns untouched


def test_maxit_forced_breakdown_zero_diag(torch_cuda, mrhs):
    A = grids.dirichlet7(8)
    B = rng.rhs_block(A.n, 2, 901)
    X, infos, st = gpu_solve(mrhs, torch_cuda, A, B, tol=1e-10, maxit=1)
    assert st == -4 and all(i["status"] == -4 and i["iters"] == 1 for i in infos)
    assert all(0 < i["relres"] < 1 for i in infos)
    import scipy.sparse as sp
    # A singular operator with b in its null space: v = A p = 0, so sigma = 0
    # for any shadow residual; four breakdowns in a row end the column.
    D = sp.csr_matrix(np.array([[1.0, -1.0], [-1.0, 1.0]]))
    A2 = grids.CSRMatrix(2, D.indptr.astype(np.int32), D.indices.astype(np.int32), D.data)
    X, infos, st = gpu_solve(mrhs, torch_cuda, A2, np.array([[1.0], [1.0]]), tol=1e-10, maxit=50)
    _, io, _ = oracle.bicgstab(A2, np.array([[1.0], [1.0]]), tol=1e-10, maxit=50, shadow_seed=SHADOW_SEED)
    assert st == -5 and infos[0]["status"] == -5 and io[0]["status"] == -5
    assert infos[0]["iters"] == io[0]["iters"] == 4 and infos[0]["restarts"] == io[0]["restarts"] == 3
    Z = sp.csr_matrix(np.array([[0.0, 1.0], [1.0, 2.0]]))
    A3 = grids.CSRMatrix(2, Z.indptr.astype(np.int32), Z.indices.astype(np.int32), Z.data)
    import paper_1711_10622_amd as p
    with pytest.raises(p.MrhsError):
        gpu_solve(mrhs, torch_cuda, A3, np.ones((2, 1)))


def test_overlapping_blocks_rejected(torch_cuda, mrhs):
    """B and X, or the workspace and either of them, may not share a byte."""
    import ctypes
    import paper_1711_10622_amd._lib as L
    torch = torch_cuda
    A = grids.dirichlet7(6)
    M = mrhs.CsrMatrix.from_csr(A)
    lib = L.load()
    m = 2
    blk = A.n * m * 8
    ws_n = M.workspace_size(m)
    P = torch.zeros(3 * blk + ws_n, dtype=torch.uint8, device="cuda")
    p0 = P.data_ptr()

    def call(b, x, ws, ws_bytes):
        return lib.block_bicgstab_ex(M.handle, ctypes.c_void_p(b), ctypes.c_void_p(x), m, ctypes.c_double(1e-10),
                                     100, 0, ctypes.c_void_p(ws), ctypes.c_size_t(ws_bytes), None, None)

    assert call(p0, p0 + 16, p0 + 2 * blk, ws_n) == L.EINVAL          # X starts inside B
    assert call(p0 + 16, p0, p0 + 2 * blk, ws_n) == L.EINVAL          # B starts inside X
    assert call(p0, p0 + blk, p0 + blk + 16, ws_n) == L.EINVAL        # workspace inside X
    assert call(p0 + ws_n, p0 + ws_n + blk, p0, ws_n + 16) == L.EINVAL  # workspace runs into B
    # disjoint ranges are accepted (B = 0 converges at once)
    assert call(p0, p0 + blk, p0 + 2 * blk, ws_n) == L.OK
    torch.cuda.synchronize()
    M.close()


@pytest.mark.parametrize("k", [1, 2, 5, 12])
def test_trajectory_after_k_iterations(torch_cuda, mrhs, k):
    """The iterate after exactly k iterations equals the oracle's (same shadow
    residual, same recurrences) up to rounding."""
    A = configs.MATRICES["dir16"]()
    B = configs.WORKLOADS["dir16"].rhs(A.n, 4)
    X, infos, st = gpu_solve(mrhs, torch_cuda, A, B, tol=1e-14, maxit=k)
    Xo, io, _ = oracle.bicgstab(A, B, tol=1e-14, maxit=k, shadow_seed=SHADOW_SEED)
    assert st == -4 and all(i["iters"] == k for i in infos)
    for l in range(4):
        assert io[l]["iters"] == k
        err = np.linalg.norm(X[:, l] - Xo[:, l]) / np.linalg.norm(Xo[:, l])
        assert err <= 1e-11, (l, err)
        assert abs(infos[l]["relres"] - io[l]["relres"]) <= 1e-9 * io[l]["relres"]


def test_initial_guess(torch_cuda, mrhs):
    A = grids.dirichlet7(9)
    xs = rng.int_block(A.n, 3, 902, -5, 5)
    B = oracle.gspmv(A, xs)
    X, infos, st = gpu_solve(mrhs, torch_cuda, A, B, tol=1e-10, X0=xs)
    assert st == 0 and all(i["iters"] == 0 for i in infos)
    assert np.array_equal(X, xs)
    for mixed in (False, True):
        X, infos, st = gpu_solve(mrhs, torch_cuda, A, B, tol=1e-10, X0=xs + 0.01, mixed=mixed)
        assert st == 0 and np.all(true_relres(A, X, B) <= 1e-10)


@pytest.mark.parametrize("mixed", [False, True])
def test_channel_full_m16(torch_cuda, mrhs, mixed):
    """The 128x64x64 stretched channel at full size with m = 16."""
    A = configs.MATRICES["chan128"]()
    B = configs.WORKLOADS["chan128"].rhs(A.n, 16)
    X, infos, st = gpu_solve(mrhs, torch_cuda, A, B, tol=1e-10, maxit=20000, mixed=mixed)
    assert st == 0, infos
    rr = true_relres(A, X, B)
    assert np.all(rr <= 1e-10), rr
    Xo, io, _ = oracle.bicgstab(A, B[:, :2], tol=1e-10, threads=2, shadow_seed=SHADOW_SEED)
    for l in range(2):
        err = np.linalg.norm(X[:, l] - Xo[:, l]) / np.linalg.norm(Xo[:, l])
        assert err <= 1e-5, err
        if not mixed:
            # at 1e-10 on this operator the count moves with summation order
            # alone: 456-512 iterations for one column under three dot-product
            # orders in binary64 on the CPU, 473-551 for one column under two
            # workgroup counts on the GPU
            assert abs(infos[l]["iters"] - io[l]["iters"]) <= 0.3 * io[l]["iters"]


@pytest.fixture(scope="module")
def chunked_channel():
    """A channel with planes of 192 tiles of 256 rows and a short last plane,
    a mean-free block of 16 right-hand sides, and the oracle's solution of
    the first column."""
    solid = np.zeros((5, 192, 256), dtype=bool)
    solid[4, 100:, :] = True
    A = grids.channel7(256, 192, 5, beta=2.0, solid=solid)
    B = mean_free(rng.rhs_block(A.n, 16, 1717))
    Xo, _, _ = oracle.bicgstab(A, B[:, :1], tol=1e-10, threads=1, shadow_seed=SHADOW_SEED)
    return A, B, Xo


@pytest.mark.parametrize("mixed", [False, True])
def test_chunked_channel_solve(torch_cuda, mrhs, chunked_channel, mixed):
    """m = 16 on a matrix whose products sweep its planes in chunks (binary64
    spmv_omega in 4, the other products in 2 or 3)."""
    A, B, Xo = chunked_channel
    X, infos, st = gpu_solve(mrhs, torch_cuda, A, B, tol=1e-10, maxit=20000, mixed=mixed)
    assert st == 0, infos
    rr = true_relres(A, X, B)
    assert np.all(rr <= 1e-10), rr
    err = np.linalg.norm(X[:, 0] - Xo[:, 0]) / np.linalg.norm(Xo[:, 0])
    assert err <= 1e-5, err


@pytest.mark.parametrize("name,m", [("cube192", 8), ("chan256", 16)])
def test_full_size_fp64_and_mixed(torch_cuda, mrhs, name, m):
    """The two workloads the mixed solve is measured on, at full size: the
    relabelled cube channel (2.29M rows, m = 8) and the 256x192x256 channel
    (12.6M rows, m = 16).  Every column of both solves reaches a true
    residual of 1e-10 (compensated products on the CPU), and the binary64
    and mixed solutions agree mean-free to 1e-5 (both within kappa * tol of
    the exact solution)."""
    A = configs.MATRICES[name]()
    B = configs.WORKLOADS[name].rhs(A.n, m)
    X64, i64, st64 = gpu_solve(mrhs, torch_cuda, A, B, tol=1e-10, maxit=20000)
    assert st64 == 0, i64
    Xmx, imx, stmx = gpu_solve(mrhs, torch_cuda, A, B, tol=1e-10, maxit=20000, mixed=True)
    assert stmx == 0, imx
    for X in (X64, Xmx):
        rr = true_relres(A, X, B)
        assert np.all(rr <= 1e-10), rr
    d = mean_free(Xmx) - mean_free(X64)
    err = np.linalg.norm(d, axis=0) / np.linalg.norm(mean_free(X64), axis=0)
    assert np.all(err <= 1e-5), err


def _merge_env(flag):
    import os
    old = os.environ.get("MRHS_MERGE")
    os.environ["MRHS_MERGE"] = flag
    return old


def _merge_restore(old):
    import os
    if old is None:
        os.environ.pop("MRHS_MERGE", None)
    else:
        os.environ["MRHS_MERGE"] = old


@pytest.mark.parametrize("m", [1, 3, 4, 8, 16])
def test_merged_iteration(torch_cuda, mrhs, m):
    """Two kernels per iteration (the x/r/p update fused with the next
    iteration's v = A p, MRHS_MERGE=2) against three (MRHS_MERGE=0): the
    iterate after k iterations matches the oracle's, converged solves meet
    the tolerance and agree, iteration counts within 15 %."""
    A = grids.channel7(24, 16, 20, beta=2.0)
    B = mean_free(rng.rhs_block(A.n, m, 3300 + m))
    out = {}
    for flag in ("2", "0"):
        old = _merge_env(flag)
        try:
            Xk, ik, sk = gpu_solve(mrhs, torch_cuda, A, B, tol=1e-14, maxit=3)
            X, infos, st = gpu_solve(mrhs, torch_cuda, A, B, tol=1e-10, maxit=20000)
        finally:
            _merge_restore(old)
        assert st == 0, infos
        assert np.all(true_relres(A, X, B) <= 1e-10)
        out[flag] = (Xk, X, infos)
    Xo, io, _ = oracle.bicgstab(A, B, tol=1e-14, maxit=3, shadow_seed=SHADOW_SEED)
    for flag in ("2", "0"):
        Xk = out[flag][0]
        for l in range(m):
            err = np.linalg.norm(Xk[:, l] - Xo[:, l]) / np.linalg.norm(Xo[:, l])
            assert err <= 1e-11, (flag, l, err)
    d = np.linalg.norm(mean_free(out["2"][1]) - mean_free(out["0"][1]), axis=0)
    assert np.all(d <= 1e-6 * np.linalg.norm(mean_free(out["0"][1]), axis=0)), d
    for a, b in zip(out["2"][2], out["0"][2]):
        assert abs(a["iters"] - b["iters"]) <= max(3, 0.15 * b["iters"]), (a, b)
