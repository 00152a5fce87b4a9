"""GPU parity of the generalized SpMV (Section 2.3, Figure 1) against the oracle.

Tolerances: binary64 products must lie within 1e-13 * (|A||X|)_il of the
oracle element by element (the rounding bound of a <= 8-term row sum is
~1e-15 of that scale); binary32 products are compared with the oracle applied
to the binary32-rounded inputs within gamma_k(2^-24) * (|A32||X32|)_il,
k = longest row.  Integer-valued inputs must agree bitwise.
"""
import numpy as np
import pytest

import oracle
from helpers import U32, abs_bound, f32_matrix, gamma, max_row_len, round32
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


def gpu_gspmv(mrhs, torch, A, X, dtype=np.float64):
    M = mrhs.CsrMatrix.from_csr(A)
    tdt = torch.float64 if dtype == np.float64 else torch.float32
    Xt = torch.from_numpy(np.ascontiguousarray(X.astype(dtype))).to("cuda", tdt)
    Y = M.gspmv(Xt)
    torch.cuda.synchronize()
    out = Y.cpu().numpy().astype(np.float64)
    M.close()
    return out


def small_cases():
    # (matrix, label): several tiles and a ragged tail (n not a multiple of 256)
    yield grids.dirichlet7(16), "dir16"
    yield grids.dirichlet7(13, 11, 7), "dir13x11x7"
    yield grids.channel7(24, 10, 9, beta=2.0), "chan24x10x9"
    solid = grids.cube_array_solid(48, 24, 32, ncube=2, h=4, pitch_x=24, pitch_z=16, off_x=4, off_z=4)
    C = grids.channel7(48, 24, 32, beta=2.0, lx=3.0, ly=1.5, lz=2.0, solid=solid)
    yield grids.permute_symmetric(C, rng.permutation(C.n, 10622)), "cube48_perm"


@pytest.mark.parametrize("m", list(range(1, 17)))
def test_f64_all_m(torch_cuda, mrhs, m):
    for A, label in small_cases():
        X = rng.rhs_block(A.n, m, 100 + m)
        Y = gpu_gspmv(mrhs, torch_cuda, A, X)
        ref = oracle.gspmv(A, X)
        bound = abs_bound(A, X)
        err = np.abs(Y - ref)
        assert np.all(err <= 1e-13 * bound), (label, m, float((err / np.maximum(bound, 1e-300)).max()))


@pytest.mark.parametrize("m", list(range(1, 17)))
def test_f32_all_m(torch_cuda, mrhs, m):
    for A, label in small_cases():
        X = round32(rng.rhs_block(A.n, m, 200 + m))
        A32 = f32_matrix(A)
        Y = gpu_gspmv(mrhs, torch_cuda, A, X, dtype=np.float32)
        ref = oracle.gspmv(A32, X)
        bound = abs_bound(A32, X)
        tol = gamma(max_row_len(A), U32) * bound
        assert np.all(np.abs(Y - ref) <= tol), (label, m)


@pytest.mark.parametrize("m", [1, 4, 7, 16])
def test_integer_exact_bitwise(torch_cuda, mrhs, m):
    A = grids.dirichlet7(16)
    X = rng.int_block(A.n, m, 300 + m, -1000, 1000)
    ref = oracle.gspmv(A, X)
    assert np.array_equal(gpu_gspmv(mrhs, torch_cuda, A, X), ref)
    assert np.array_equal(gpu_gspmv(mrhs, torch_cuda, A, X, dtype=np.float32), ref)


def test_block_equals_single_columns_bitwise(torch_cuda, mrhs):
    A = grids.channel7(24, 10, 9, beta=2.0)
    X = rng.rhs_block(A.n, 6, 400)
    Y = gpu_gspmv(mrhs, torch_cuda, A, X)
    for l in range(6):
        y = gpu_gspmv(mrhs, torch_cuda, A, np.ascontiguousarray(X[:, l:l + 1]))
        assert np.array_equal(Y[:, l], y[:, 0])


def test_eigenmode_and_symmetry(torch_cuda, mrhs):
    N = 20
    A = grids.dirichlet7(N)
    i = np.arange(N)
    cols, lams = [], []
    for a, b, c in [(1, 1, 1), (3, 7, 2), (20, 20, 20)]:
        v = (np.sin(c * np.pi * (i + 1) / (N + 1))[:, None, None] * np.sin(b * np.pi * (i + 1) / (N + 1))[None, :, None]
             * np.sin(a * np.pi * (i + 1) / (N + 1))[None, None, :]).ravel()
        cols.append(v)
        lams.append(sum(2 - 2 * np.cos(q * np.pi / (N + 1)) for q in (a, b, c)))
    X = np.stack(cols, axis=1)
    Y = gpu_gspmv(mrhs, torch_cuda, A, X)
    assert np.abs(Y - X * np.array(lams)).max() <= 1e-13 * 12
    C = grids.channel7(16, 12, 10, beta=2.0)
    X1 = rng.rhs_block(C.n, 2, 401)
    X2 = rng.rhs_block(C.n, 2, 402)
    AX1 = gpu_gspmv(mrhs, torch_cuda, C, X1)
    AX2 = gpu_gspmv(mrhs, torch_cuda, C, X2)
    assert np.allclose(np.sum(X1 * AX2, 0), np.sum(AX1 * X2, 0), rtol=1e-12)


def test_irregular_rows(torch_cuda, mrhs):
    # empty rows, duplicates, unsorted columns and one very long row that
    # overflows the LDS staging of its tile
    n = 700
    r = np.random.default_rng(5)
    rows = []
    for i in range(n):
        if i % 17 == 3:
            rows.append(([], []))
            continue
        k = 3000 if i == 300 else r.integers(1, 12)
        c = r.integers(0, n, size=k)
        c[0] = i
        rows.append((c, r.standard_normal(k)))
    rp = np.zeros(n + 1, dtype=np.int32)
    rp[1:] = np.cumsum([len(c) for c, _ in rows])
    col = np.concatenate([np.asarray(c, dtype=np.int32) for c, _ in rows])
    val = np.concatenate([np.asarray(v, dtype=np.float64) for _, v in rows])
    A = grids.CSRMatrix(n, rp, col, val)
    for m in (1, 3, 8, 16):
        X = rng.rhs_block(n, m, 500 + m)
        Y = gpu_gspmv(mrhs, torch_cuda, A, X)
        ref = oracle.gspmv(A, X)
        assert np.all(np.abs(Y - ref) <= 1e-13 * abs_bound(A, X) + 1e-300)
        assert np.all(Y[3::17] == 0.0)


def test_argument_errors(torch_cuda, mrhs):
    import paper_1711_10622_amd._lib as L
    A = grids.dirichlet7(4)
    M = mrhs.CsrMatrix.from_csr(A)
    X = torch_cuda.zeros((A.n, 2), dtype=torch_cuda.float64, device="cuda")
    lib = L.load()
    import ctypes
    assert lib.gspmv(M.handle, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(X.data_ptr()), 2) == L.EINVAL
    assert lib.gspmv(M.handle, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(X.data_ptr()), 17) == L.EINVAL
    assert lib.gspmv(M.handle, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(X.data_ptr()), 0) == L.EINVAL
    # partial overlap: Y starts one row (16 bytes) into X
    P = torch_cuda.zeros((A.n + 1) * 2, dtype=torch_cuda.float64, device="cuda")
    p0 = P.data_ptr()
    assert lib.gspmv(M.handle, ctypes.c_void_p(p0), ctypes.c_void_p(p0 + 16), 2) == L.EINVAL
    assert lib.gspmv(M.handle, ctypes.c_void_p(p0 + 16), ctypes.c_void_p(p0), 2) == L.EINVAL
    E = mrhs.CsrMatrix(0, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0))
    assert lib.gspmv(E.handle, None, None, 4) == L.OK
    M.close()
    E.close()


def test_sampled_trace(torch_cuda, mrhs):
    """mrhs_trace_enable(k) times launches 0, k, 2k, ... of each kernel class."""
    A = grids.dirichlet7(6)
    M = mrhs.CsrMatrix.from_csr(A)
    X = torch_cuda.ones((A.n, 4), dtype=torch_cuda.float64, device="cuda")
    Y = torch_cuda.empty_like(X)
    mrhs.trace_enable(True, every=3)
    for _ in range(7):
        M.gspmv(X, out=Y)
    M.gspmv(X[:, :2].contiguous())
    tr = mrhs.trace_read()
    mrhs.trace_enable(False)
    M.close()
    keys = sorted(tr)
    assert len(keys) == 2 and keys[0].startswith("gspmv/f64/m2/") and keys[1].startswith("gspmv/f64/m4/")
    assert tr[keys[1]]["seen"] == 7 and tr[keys[1]]["launches"] == 3
    assert tr[keys[0]]["seen"] == 1 and tr[keys[0]]["launches"] == 1
    assert 0 < tr[keys[1]]["min_ms"] <= tr[keys[1]]["max_ms"] < 1e3


@pytest.mark.parametrize("m", [1, 8, 16])
def test_full_size_channel_f64(torch_cuda, mrhs, m):
    """The 128x64x64 stretched channel at full size, every row checked."""
    A = configs.MATRICES["chan128"]()
    X = configs.WORKLOADS["chan128"].rhs(A.n, m)
    Y = gpu_gspmv(mrhs, torch_cuda, A, X)
    ref = oracle.gspmv(A, X)
    assert np.all(np.abs(Y - ref) <= 1e-13 * abs_bound(A, X))


@pytest.mark.parametrize("dtype,m", [(np.float64, 8), (np.float64, 16), (np.float32, 16)])
def test_plane_chunked_schedule(torch_cuda, mrhs, dtype, m):
    """A channel with planes of 192 tiles of 256 rows: wide blocks make the
    products sweep every plane in 2 (binary64 m = 8, binary32 m = 16) or 3
    (binary64 m = 16) chunks.  The last plane is short of cells, so the final
    plane of tiles is partial; every row is checked."""
    solid = np.zeros((5, 192, 256), dtype=bool)
    solid[4, 100:, :] = True
    A = grids.channel7(256, 192, 5, beta=2.0, solid=solid)
    assert A.n == 4 * 192 * 256 + 100 * 256
    X = rng.rhs_block(A.n, m, 500 + m)
    if dtype == np.float64:
        Y = gpu_gspmv(mrhs, torch_cuda, A, X)
        ref = oracle.gspmv(A, X)
        assert np.all(np.abs(Y - ref) <= 1e-13 * abs_bound(A, X))
    else:
        X = round32(X)
        A32 = f32_matrix(A)
        Y = gpu_gspmv(mrhs, torch_cuda, A, X, dtype=np.float32)
        ref = oracle.gspmv(A32, X)
        assert np.all(np.abs(Y - ref) <= gamma(max_row_len(A), U32) * abs_bound(A32, X))


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_large_channel_sampled(torch_cuda, mrhs, dtype):
    """The 256x192x256 channel (12.6M rows, m = 16, the chunked plane
    schedule), on 20k sampled rows including the first and last tiles."""
    A = configs.MATRICES["chan256"]()
    X = configs.WORKLOADS["chan256"].rhs(A.n, 16)
    r = np.random.default_rng(0)
    rows = np.unique(np.concatenate([np.arange(512), np.arange(A.n - 512, A.n),
                                     r.integers(0, A.n, size=20000)]))
    if dtype == np.float64:
        Y = gpu_gspmv(mrhs, torch_cuda, A, X)
        ref = oracle.gspmv_rows(A, X, rows)
        assert np.all(np.abs(Y[rows] - ref) <= 1e-13 * abs_bound(A, X, rows))
    else:
        X = round32(X)
        A32 = f32_matrix(A)
        Y = gpu_gspmv(mrhs, torch_cuda, A, X, dtype=np.float32)
        ref = oracle.gspmv_rows(A32, X, rows)
        assert np.all(np.abs(Y[rows] - ref) <= gamma(max_row_len(A), U32) * abs_bound(A32, X, rows))


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_cube_full_sampled(torch_cuda, mrhs, dtype):
    """The relabelled wall-mounted-cube channel (2.29M rows, random row order)
    at m = 8, the case the mixed solve is measured on: 20k sampled rows plus
    the first and last tiles."""
    A = configs.MATRICES["cube192"]()
    X = configs.WORKLOADS["cube192"].rhs(A.n, 8)
    r = np.random.default_rng(1)
    rows = np.unique(np.concatenate([np.arange(512), np.arange(A.n - 512, A.n),
                                     r.integers(0, A.n, size=20000)]))
    if dtype == np.float64:
        Y = gpu_gspmv(mrhs, torch_cuda, A, X)
        ref = oracle.gspmv_rows(A, X, rows)
        assert np.all(np.abs(Y[rows] - ref) <= 1e-13 * abs_bound(A, X, rows))
    else:
        X = round32(X)
        A32 = f32_matrix(A)
        Y = gpu_gspmv(mrhs, torch_cuda, A, X, dtype=np.float32)
        ref = oracle.gspmv_rows(A32, X, rows)
        tol = gamma(max_row_len(A), U32) * abs_bound(A32, X, rows)
        assert np.all(np.abs(Y[rows] - ref) <= tol)


def march_cases():
    # planes of 64 x 63 = 4032 rows (63 march tiles of 64 rows, 48 of 84, 84 of
    # 48, 112 of 36 rows): every lane layout's march tile divides the plane;
    # one with a solid block in three of its planes (rows renumbered past it,
    # a ragged last plane)
    yield grids.channel7(64, 63, 10, beta=2.0), "chan64x63x10"
    solid = np.zeros((10, 63, 64), dtype=bool)
    solid[2:5, 0:7, 10:30] = True
    yield grids.channel7(64, 63, 10, beta=2.0, solid=solid), "chan64x63x10_solid"


def march_tile(elem, m):
    """Rows of a march tile: whole passes of the lane layout's rows, at least 64."""
    if elem == 8:
        vw = 2 if m % 2 == 0 else 1
    else:
        vw = 4 if m % 4 == 0 else (2 if m % 2 == 0 else 1)
    g = -(-m // vw)
    p2 = 1
    while p2 < g:
        p2 *= 2
    exact = (vw == 1 or g == 5) and 64 // g > 64 // p2
    rpp = 4 * (64 // (g if exact else p2))
    return rpp * (1 if rpp >= 64 else 64 // rpp)


def _with_march(mrhs, torch, flag, fn):
    import os
    old = os.environ.get("MRHS_MARCH")
    os.environ["MRHS_MARCH"] = flag
    try:
        mrhs.trace_enable(True)
        out = fn()
        torch.cuda.synchronize()
        tr = mrhs.trace_read()
        mrhs.trace_enable(False)
    finally:
        if old is None:
            del os.environ["MRHS_MARCH"]
        else:
            os.environ["MRHS_MARCH"] = old
    return out, set(tr)


@pytest.mark.parametrize("m", list(range(1, 17)))
def test_plane_march_bitwise_tiled(torch_cuda, mrhs, m):
    """Products on grid operators may walk planes with the gathered block rows
    of three planes in LDS (MRHS_MARCH=1); each row's sum must be bitwise that
    of the tiled product (same order, same values), binary64 and binary32,
    and within the oracle's bound."""
    for A, label in march_cases():
        for dt in (np.float64, np.float32):
            X = rng.rhs_block(A.n, m, 300 + m)
            if dt == np.float32:
                X = round32(X)
            Ym, km = _with_march(mrhs, torch_cuda, "1", lambda: gpu_gspmv(mrhs, torch_cuda, A, X, dtype=dt))
            Yt, kt = _with_march(mrhs, torch_cuda, "0", lambda: gpu_gspmv(mrhs, torch_cuda, A, X, dtype=dt))
            assert np.array_equal(Ym, Yt), (label, m, dt)
            if dt == np.float64:
                assert np.all(np.abs(Ym - oracle.gspmv(A, X)) <= 1e-13 * abs_bound(A, X)), (label, m)
            # where the march tile divides the plane into at least 16 tiles
            # the march ran: its launches carry another grid size
            tr = march_tile(np.dtype(dt).itemsize, m)
            assert (km != kt) == (4032 % tr == 0 and 4032 // tr >= 16), (label, m, dt, tr, km, kt)


@pytest.mark.parametrize("mixed", [False, True])
def test_plane_march_solve(torch_cuda, mrhs, mixed):
    """A solve whose products march (MRHS_MARCH=1, the 128x64x64 channel,
    m = 16) and the same solve on tiled products (the default) both reach
    1e-10 and agree within it."""
    from helpers import mean_free, true_relres
    A = configs.MATRICES["chan128"]()
    B = configs.WORKLOADS["chan128"].rhs(A.n, 16)

    def solve():
        M = mrhs.CsrMatrix.from_csr(A)
        X, infos, st = M.solve(torch_cuda.from_numpy(B).cuda(), tol=1e-10, maxit=20000, mixed=mixed)
        out = X.cpu().numpy(), infos, st
        M.close()
        return out

    (Xm, im, sm), km = _with_march(mrhs, torch_cuda, "1", solve)
    (Xt, it, stt), kt = _with_march(mrhs, torch_cuda, "0", solve)
    assert sm == 0 and stt == 0, (im, it)
    assert km != kt
    for X in (Xm, Xt):
        assert np.all(true_relres(A, X, B) <= 1e-10)
    d = np.linalg.norm(mean_free(Xm) - mean_free(Xt), axis=0) / np.linalg.norm(mean_free(Xt), axis=0)
    assert np.all(d <= 1e-5), d
    # the order of the partial dot products differs, and at 1e-10 on this
    # operator the iteration count moves with that order alone (one column:
    # 473 against 551 between two grid sizes of the update pass; the
    # restarted binary32 inner solves' by up to ~20 %)
    for a, b in zip(im, it):
        assert abs(a["iters"] - b["iters"]) <= 0.3 * b["iters"], (a, b)
