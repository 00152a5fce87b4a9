"""Shared helpers for the GPU parity tests (no solver arithmetic here)."""
import numpy as np

import oracle
from workloads import grids

U64 = 2.0 ** -53
U32 = 2.0 ** -24


def gamma(k, u):
    return k * u / (1 - k * u)


def abs_matrix(A):
    return grids.CSRMatrix(A.n, A.row_ptr, A.col, np.abs(A.val))


def abs_bound(A, X, rows=None):
    """(|A| |X|), the scale of the rounding error of a row sum."""
    if rows is None:
        return oracle.gspmv(abs_matrix(A), np.abs(X))
    return oracle.gspmv_rows(abs_matrix(A), np.abs(X), rows)


def round32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def f32_matrix(A):
    return grids.CSRMatrix(A.n, A.row_ptr, A.col, round32(A.val))


def max_row_len(A):
    return int(np.diff(A.row_ptr).max()) if A.n else 0


def true_relres(A, X, B):
    """||b - A x|| / ||b|| per column with compensated products (oracle Dot2)."""
    R = B - oracle.gspmv_dot2(A, X)
    nb = np.linalg.norm(B, axis=0)
    return np.linalg.norm(R, axis=0) / np.where(nb > 0, nb, 1.0)


def mean_free(X):
    return X - X.mean(axis=0, keepdims=True)
