"""Pins for the oracle's generalized SpMV (Section 2.3, Figure 1).

Each check rests on something other than the oracle itself: closed-form
eigenpairs of the generated operators, exact integer arithmetic done in
int64, a dense matrix product, the compensated Dot2 reference with the
textbook error bound, and algebraic identities (symmetry, relabelling).
"""
import numpy as np
import pytest

import oracle
from workloads import grids, rng

U64 = 2.0 ** -53


def sine_mode(nx, ny, nz, a, b, c):
    i = np.arange(nx)
    j = np.arange(ny)
    k = np.arange(nz)
    vx = np.sin(a * np.pi * (i + 1) / (nx + 1))
    vy = np.sin(b * np.pi * (j + 1) / (ny + 1))
    vz = np.sin(c * np.pi * (k + 1) / (nz + 1))
    v = vz[:, None, None] * vy[None, :, None] * vx[None, None, :]
    lam = sum(2 - 2 * np.cos(q * np.pi / (N + 1)) for q, N in ((a, nx), (b, ny), (c, nz)))
    return v.ravel(), lam


def test_dirichlet_sine_eigenmodes():
    nx, ny, nz = 16, 12, 10
    A = grids.dirichlet7(nx, ny, nz)
    modes = [(1, 1, 1), (2, 3, 1), (16, 12, 10), (5, 1, 7), (8, 6, 5)]
    X = np.stack([sine_mode(nx, ny, nz, *q)[0] for q in modes], axis=1)
    lams = np.array([sine_mode(nx, ny, nz, *q)[1] for q in modes])
    Y = oracle.gspmv(A, X)
    err = np.abs(Y - X * lams[None, :]).max(axis=0)
    assert np.all(err <= 1e-14 * 12 * np.abs(X).max(axis=0))


def test_channel_fourier_modes():
    nx, ny, nz = 16, 8, 12
    A = grids.channel7(nx, ny, nz, beta=2.0)
    yf = A.meta["y_faces"]
    dy = np.diff(yf)
    lx, ly, lz = A.meta["lengths"]
    dx, dz = lx / nx, lz / nz
    i = np.arange(nx)[None, None, :]
    k = np.arange(nz)[:, None, None]
    jj = np.broadcast_to(np.arange(ny)[None, :, None], (nz, ny, nx)).ravel()
    cols, want = [], []
    for kx in (1, 3, 8):
        v = np.broadcast_to(np.cos(2 * np.pi * kx * i / nx), (nz, ny, nx)).ravel()
        cols.append(v)
        want.append((dy[jj] * dz / dx) * (2 - 2 * np.cos(2 * np.pi * kx / nx)) * v)
    for kz in (1, 5):
        v = np.broadcast_to(np.sin(2 * np.pi * kz * k / nz), (nz, ny, nx)).ravel()
        cols.append(v)
        want.append((dx * dy[jj] / dz) * (2 - 2 * np.cos(2 * np.pi * kz / nz)) * v)
    X = np.stack(cols, axis=1)
    W = np.stack(want, axis=1)
    Y = oracle.gspmv(A, X)
    scale = np.abs(A.val).max() * 7
    assert np.abs(Y - W).max() <= 1e-13 * scale


def test_channel_constant_nullspace_and_symmetry():
    A = grids.channel7(12, 10, 8, beta=2.0)
    y = oracle.gspmv(A, np.ones(A.n))
    assert np.abs(y).max() <= 1e-14 * np.abs(A.val).max()
    X = rng.rhs_block(A.n, 3, 5)
    Z = rng.rhs_block(A.n, 3, 6)
    AX = oracle.gspmv(A, X)
    AZ = oracle.gspmv(A, Z)
    lhs = np.einsum("il,il->l", X, AZ)
    rhs = np.einsum("il,il->l", AX, Z)
    assert np.allclose(lhs, rhs, rtol=1e-12, atol=1e-12 * np.abs(lhs).max())


def _int_reference(A, Xi):
    """Exact int64 product: every nonzero of the unit stencil is an integer."""
    vals = A.val.astype(np.int64)
    assert np.all(vals == A.val)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    Y = np.zeros((A.n, Xi.shape[1]), dtype=np.int64)
    np.add.at(Y, rows, vals[:, None] * Xi[A.col.astype(np.int64)])
    return Y


def test_integer_exactness_bitwise():
    A = grids.dirichlet7(16)
    X = rng.int_block(A.n, 7, 99, -1000, 1000)
    Y = oracle.gspmv(A, X)
    ref = _int_reference(A, X.astype(np.int64))
    assert np.array_equal(Y, ref.astype(np.float64))


def test_dot2_bound_random():
    A = grids.channel7(16, 12, 8, beta=2.0)
    X = rng.rhs_block(A.n, 5, 7)
    Y = oracle.gspmv(A, X)
    Y2 = oracle.gspmv_dot2(A, X)
    absA = grids.CSRMatrix(A.n, A.row_ptr, A.col, np.abs(A.val))
    bound = oracle.gspmv(absA, np.abs(X))
    k = np.diff(A.row_ptr).max()
    gamma = k * U64 / (1 - k * U64)
    assert np.all(np.abs(Y - Y2) <= gamma * bound * (1 + 1e-12) + 1e-300)


def test_dense_product_duplicates_empty_rows():
    # row 1 is empty, row 2 holds a duplicate column (entries add), row 3 unsorted
    rp = np.array([0, 2, 2, 5, 7], dtype=np.int32)
    col = np.array([0, 3, 1, 1, 2, 3, 0], dtype=np.int32)
    val = np.array([2.0, -1.0, 0.5, 0.25, 3.0, 4.0, -2.0])
    A = grids.CSRMatrix(4, rp, col, val)
    X = rng.rhs_block(4, 3, 11)
    Y = oracle.gspmv(A, X)
    D = A.to_dense()
    assert D[2, 1] == 0.75
    assert np.allclose(Y, D @ X, rtol=0, atol=1e-15)
    assert np.all(Y[1] == 0.0)


def test_relabelling_commutes():
    A = grids.channel7(10, 6, 8, beta=2.0)
    perm = rng.permutation(A.n, 3)
    PA = grids.permute_symmetric(A, perm)
    X = rng.rhs_block(A.n, 4, 12)
    left = oracle.gspmv(PA, X[perm])
    right = oracle.gspmv(A, X)[perm]
    absA = grids.CSRMatrix(A.n, A.row_ptr, A.col, np.abs(A.val))
    scale = oracle.gspmv(absA, np.abs(X))[perm]
    assert np.all(np.abs(left - right) <= 16 * U64 * scale)


def test_block_equals_columns():
    A = grids.dirichlet7(8, 9, 7)
    X = rng.rhs_block(A.n, 6, 13)
    Y = oracle.gspmv(A, X)
    for l in range(6):
        assert np.array_equal(Y[:, l], oracle.gspmv(A, np.ascontiguousarray(X[:, l])))


@pytest.mark.parametrize("shape", [(4, 4, 4), (7, 3, 5)])
def test_generator_counts(shape):
    nx, ny, nz = shape
    A = grids.dirichlet7(nx, ny, nz)
    n = nx * ny * nz
    assert A.n == n
    assert A.nnz == 7 * n - 2 * (ny * nz + nx * nz + nx * ny)
    C = grids.channel7(max(nx, 3), ny, max(nz, 3))
    assert C.nnz == 7 * C.n - 2 * max(nx, 3) * max(nz, 3)


def _exact_rows(rp, col, val, X):
    """Exact row sums (rationals) and sum |a||x| of a CSR product, column 0."""
    from fractions import Fraction
    out, mag = [], []
    for i in range(len(rp) - 1):
        s = Fraction(0)
        a = Fraction(0)
        for j in range(rp[i], rp[i + 1]):
            t = Fraction(val[j]) * Fraction(X[col[j], 0])
            s += t
            a += abs(t)
        out.append(s)
        mag.append(a)
    return out, mag


def _cancelling_rows():
    """Rows whose plain left-to-right sum loses everything: huge terms that
    cancel around small ones, and products whose low-order half decides the
    result.  Column j of row i multiplies X[j]; X holds the chosen factors."""
    r = np.random.default_rng(1711)
    rows = []
    # (2^53, 1, -2^53) . (1, 1, 1) = 1; plain summation gives 0
    rows.append([(2.0 ** 53, 1.0), (1.0, 1.0), (-(2.0 ** 53), 1.0)])
    # (1 + 2^-30)(1 - 2^-30) - 1 = -2^-60; the rounded product is exactly 1
    rows.append([(1.0 + 2.0 ** -30, 1.0 - 2.0 ** -30), (-1.0, 1.0)])
    # a stencil-length row: two cancelling giants around three random terms,
    # then minus the rounded sum of those terms, so the exact result is the
    # rounding error of that sum
    for _ in range(6):
        small = r.uniform(-1, 1, 3) * 2.0 ** r.integers(-20, 20, 3)
        big = float(2.0 ** int(r.integers(60, 90)))
        s = float(sum(small))
        rows.append([(big, 1.0), (small[0], 1.0), (small[1], 1.0), (-big, 1.0), (small[2], 1.0),
                     (-s, 1.0), (r.uniform(-1, 1) * 2.0 ** -70, 1.0)])
    # products with many significant bits: x_j y_j summed against the
    # negated double-rounded sum of the products
    for _ in range(6):
        a = r.uniform(1, 2, 6) * np.where(r.random(6) < 0.5, -1, 1)
        b = r.uniform(1, 2, 6)
        s = float(np.sum(a * b))
        rows.append([(a[k], b[k]) for k in range(6)] + [(-s, 1.0)])
    return rows


def test_dot2_compensation_on_cancelling_rows():
    """Dot2 against the exact (rational) row sums on rows where plain
    summation fails: within u|s| + gamma_k^2 sum|a||x| (Ogita, Rump & Oishi
    2005, the Dot2 error bound), while the plain oracle product is wrong."""
    rows = _cancelling_rows()
    rp = [0]
    col, val, xs = [], [], []
    for row in rows:
        for a, x in row:
            col.append(len(xs))
            val.append(a)
            xs.append(x)
        rp.append(len(col))
    n = len(xs)
    # square CSR: pad with empty rows so every factor has a row index
    rp = rp + [rp[-1]] * (n - len(rows))
    A = grids.CSRMatrix(n, np.array(rp, dtype=np.int32), np.array(col, dtype=np.int32),
                        np.array(val, dtype=np.float64))
    X = np.array(xs, dtype=np.float64)[:, None]
    exact, mag = _exact_rows(rp, col, val, X)
    Y2 = oracle.gspmv_dot2(A, X)[:, 0]
    Y1 = oracle.gspmv(A, X)[:, 0]
    wrong_plain = 0
    for i in range(len(rows)):
        k = rp[i + 1] - rp[i]
        g = k * U64 / (1 - k * U64)
        bound = U64 * abs(float(exact[i])) + g * g * float(mag[i])
        from fractions import Fraction
        assert abs(Fraction(Y2[i]) - exact[i]) <= Fraction(bound) * (1 + 1e-9), (i, Y2[i], float(exact[i]))
        wrong_plain += Fraction(Y1[i]) != exact[i]
    # the rows are hard: plain summation misses most of them
    assert wrong_plain >= len(rows) - 2
    assert Y2[0] == 1.0 and Y1[0] == 0.0
    assert Y2[1] == -(2.0 ** -60)
