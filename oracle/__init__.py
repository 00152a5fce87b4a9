"""Oracle for the block-RHS pressure-Poisson solve (CPU, binary64).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the GPU library never does, and
this package imports nothing from it.  The arithmetic lives in ``oracle.c``
(plain loops, no FMA contraction); this module only marshals numpy arrays.

Functions
---------
gspmv(A, X)         Y = A X as m separate SpMVs (Section 2.3, Figure 1).
gspmv_dot2(A, X)    the same with compensated Dot2 row sums (reference for
                    error bounds).
bicgstab(A, B, ...) m independent right-Jacobi-preconditioned BiCGStab solves
                    of A x_l = b_l (Section 2.2: one matrix, m right-hand
                    sides; BiCGStab cited in Section 1), columns optionally
                    spread over host threads.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, EINVAL, ENOMEM, ENOCONV, EBREAKDOWN = 0, -1, -2, -4, -5
X0_GIVEN, NULLSPACE_CONST, SHADOW_RANDOM = 1, 2, 4

_lock = threading.Lock()
_lib = None


class OracleInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("status", ctypes.c_int32), ("breakdowns", ctypes.c_int32),
                ("relres", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


def build(force: bool = False) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` with gcc."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                        "-fno-fast-math", "-Wall", "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            i32, f64p, i32p = ctypes.c_int32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)
            for nm in ("oracle_gspmv", "oracle_gspmv_dot2"):
                f = getattr(lib, nm)
                f.argtypes = [i32, i32p, i32p, f64p, i32, f64p, f64p]
                f.restype = None
            lib.oracle_bicgstab.argtypes = [i32, i32p, i32p, f64p, f64p, f64p, ctypes.c_double,
                                            i32, ctypes.c_uint32, ctypes.c_uint64,
                                            ctypes.POINTER(OracleInfo), f64p, i32]
            lib.oracle_bicgstab.restype = ctypes.c_int
            lib.oracle_shadow.argtypes = [i32, ctypes.c_uint64, f64p]
            lib.oracle_shadow.restype = None
            _lib = lib
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _csr(A):
    rp = np.ascontiguousarray(A.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(A.col, dtype=np.int32)
    va = np.ascontiguousarray(A.val, dtype=np.float64)
    return rp, ci, va


def _gspmv_impl(name, A, X):
    lib = _load()
    X = np.ascontiguousarray(X, dtype=np.float64)
    squeeze = X.ndim == 1
    if squeeze:
        X = X[:, None]
    n, m = X.shape
    assert n == A.n
    Y = np.empty((n, m), dtype=np.float64)
    rp, ci, va = _csr(A)
    getattr(lib, name)(n, _p(rp, ctypes.c_int32), _p(ci, ctypes.c_int32), _p(va, ctypes.c_double),
                       m, _p(X, ctypes.c_double), _p(Y, ctypes.c_double))
    return Y[:, 0] if squeeze else Y


def gspmv(A, X):
    """Y = A X, X an (n, m) row-interleaved block (or an n-vector)."""
    return _gspmv_impl("oracle_gspmv", A, X)


def gspmv_dot2(A, X):
    """Y = A X with compensated (Dot2) row sums."""
    return _gspmv_impl("oracle_gspmv_dot2", A, X)


class _Rows:
    def __init__(self, n, row_ptr, col, val):
        self.n, self.row_ptr, self.col, self.val = n, row_ptr, col, val


def row_subset(A, rows):
    """The rows ``rows`` of A as a CSR with len(rows) rows and A's columns."""
    rows = np.asarray(rows, dtype=np.int64)
    rp = A.row_ptr.astype(np.int64)
    lens = rp[rows + 1] - rp[rows]
    srp = np.zeros(len(rows) + 1, dtype=np.int64)
    np.cumsum(lens, out=srp[1:])
    src = np.repeat(rp[rows] - srp[:-1], lens) + np.arange(int(srp[-1]), dtype=np.int64)
    return _Rows(len(rows), srp.astype(np.int32), A.col[src], A.val[src])


def gspmv_part(S, X):
    """S X for a row subset S of a matrix (from ``row_subset``) and the full
    block X: the rows of A X that S holds."""
    lib = _load()
    X = np.ascontiguousarray(X, dtype=np.float64)
    if X.ndim == 1:
        X = X[:, None]
    m = X.shape[1]
    Y = np.empty((S.n, m), dtype=np.float64)
    rp, ci, va = _csr(S)
    lib.oracle_gspmv(S.n, _p(rp, ctypes.c_int32), _p(ci, ctypes.c_int32), _p(va, ctypes.c_double), m,
                     _p(X, ctypes.c_double), _p(Y, ctypes.c_double))
    return Y


def gspmv_rect(n_rows, row_ptr, col, val, X):
    """Y = A X for an n_rows-row CSR whose columns index the rows of X (a
    rectangular operator: restriction or prolongation), each row summed in
    storage order; X is an (n_cols, m) block."""
    lib = _load()
    X = np.ascontiguousarray(X, dtype=np.float64)
    if X.ndim == 1:
        X = X[:, None]
    m = X.shape[1]
    Y = np.empty((n_rows, m), dtype=np.float64)
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col, dtype=np.int32)
    va = np.ascontiguousarray(val, dtype=np.float64)
    if n_rows:
        lib.oracle_gspmv(n_rows, _p(rp, ctypes.c_int32), _p(ci, ctypes.c_int32), _p(va, ctypes.c_double), m,
                         _p(X, ctypes.c_double), _p(Y, ctypes.c_double))
    return Y


def gspmv_rows(A, X, rows, dot2=False):
    """Rows ``rows`` of A X, for sampled checks of products too large to
    recompute whole."""
    lib = _load()
    X = np.ascontiguousarray(X, dtype=np.float64)
    if X.ndim == 1:
        X = X[:, None]
    n, m = X.shape
    assert n == A.n
    S = row_subset(A, rows)
    Y = np.empty((S.n, m), dtype=np.float64)
    rp, ci, va = _csr(S)
    fn = lib.oracle_gspmv_dot2 if dot2 else lib.oracle_gspmv
    fn(S.n, _p(rp, ctypes.c_int32), _p(ci, ctypes.c_int32), _p(va, ctypes.c_double), m,
       _p(X, ctypes.c_double), _p(Y, ctypes.c_double))
    return Y


def bicgstab(A, B, tol=1e-10, maxit=10000, nullspace_const=None, X0=None,
             hist_len=0, threads=1, shadow_seed=None):
    """Solve A x_l = b_l for every column l of B independently.

    ``shadow_seed`` None takes the shadow residual r^ = r0 (renewed at every
    restart); an integer takes the fixed vector of SplitMix64 values of that
    seed mapped to [-1, 1), the same for every column.

    Returns ``(X, infos, hists)``: the (n, m) solution block, a list of
    per-column info dicts and, if ``hist_len`` > 0, an (m, hist_len) array of
    residual histories (NaN where unused).
    """
    lib = _load()
    B = np.ascontiguousarray(B, dtype=np.float64)
    if B.ndim == 1:
        B = B[:, None]
    n, m = B.shape
    assert n == A.n
    if nullspace_const is None:
        nullspace_const = bool(getattr(A, "nullspace_const", False))
    flags = (NULLSPACE_CONST if nullspace_const else 0) | (X0_GIVEN if X0 is not None else 0)
    if shadow_seed is not None:
        flags |= SHADOW_RANDOM
    rp, ci, va = _csr(A)
    X = np.zeros((n, m)) if X0 is None else np.array(X0, dtype=np.float64).reshape(n, m)
    hists = np.full((m, max(hist_len, 1)), np.nan)
    infos = [OracleInfo() for _ in range(m)]
    cols_out = [None] * m

    def run(l):
        b = np.ascontiguousarray(B[:, l])
        x = np.ascontiguousarray(X[:, l])
        h = np.full(max(hist_len, 1), np.nan)
        lib.oracle_bicgstab(n, _p(rp, ctypes.c_int32), _p(ci, ctypes.c_int32),
                            _p(va, ctypes.c_double), _p(b, ctypes.c_double),
                            _p(x, ctypes.c_double), float(tol), int(maxit), flags,
                            int(shadow_seed or 0), ctypes.byref(infos[l]),
                            _p(h, ctypes.c_double) if hist_len > 0 else None, int(hist_len))
        cols_out[l] = x
        hists[l] = h

    if threads > 1 and m > 1:
        with ThreadPoolExecutor(max_workers=min(threads, m)) as ex:
            list(ex.map(run, range(m)))
    else:
        for l in range(m):
            run(l)
    Xo = np.stack(cols_out, axis=1) if m else np.zeros((n, 0))
    return Xo, [i.as_dict() for i in infos], (hists if hist_len > 0 else None)


def shadow(n, seed):
    """The shadow residual vector of the random-shadow mode."""
    out = np.empty(n, dtype=np.float64)
    _load().oracle_shadow(int(n), int(seed), _p(out, ctypes.c_double))
    return out
