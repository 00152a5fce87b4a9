"""block_bicgstab_noalloc (workspace in the library's fixed scratch array)
against block_bicgstab_ex (caller workspace), through the C ABI: the two run
the same kernels on the same inputs with deterministic reductions, so the
solutions and per-column outcomes must agree bit for bit.  Two calls in a
row, the second smaller than the first, in binary64 and in mixed precision,
and a solve whose workspace exceeds the scratch array is rejected."""
import ctypes

import numpy as np
import pytest

from workloads import grids, rng

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1711_10622_amd as p
    from paper_1711_10622_amd import _lib
    lib = p.load(build_if_missing=False)
    return torch, p, _lib, lib


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _solve_both(env, A, m, flags, seed):
    torch, p, _lib, lib = env
    M = p.CsrMatrix.from_csr(A)
    B = torch.from_numpy(rng.rhs_block(A.n, m, seed, mean_zero=A.nullspace_const)).cuda()
    X1 = torch.full_like(B, np.nan)
    X2 = torch.full_like(B, np.nan)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    need = ctypes.c_size_t()
    assert lib.block_bicgstab_workspace_size(M.handle, m, flags, ctypes.byref(need)) == 0
    ws = torch.empty(need.value, dtype=torch.uint8, device="cuda")
    i1 = (_lib.ColInfo * m)()
    i2 = (_lib.ColInfo * m)()
    s1 = lib.block_bicgstab_ex(M.handle, _ptr(B), _ptr(X1), m, 1e-10, 5000, flags, _ptr(ws), need.value,
                               stream, i1)
    s2 = lib.block_bicgstab_noalloc(M.handle, _ptr(B), _ptr(X2), m, 1e-10, 5000, flags, stream, i2)
    torch.cuda.synchronize()
    assert s1 == 0 and s2 == 0, (s1, s2, lib.mrhs_last_error())
    assert torch.equal(X1, X2)
    assert [c.as_dict() for c in i1] == [c.as_dict() for c in i2]
    M.close()
    return need.value


@pytest.mark.parametrize("flags", [0, 2])
def test_noalloc_matches_workspace_solve_twice(env, flags):
    big = _solve_both(env, grids.channel7(24, 16, 20, beta=2.0), 8, flags, 901)
    small = _solve_both(env, grids.dirichlet7(10, 9, 7), 3, flags, 902)
    assert small < big


def test_noalloc_rejects_oversized_workspace(env):
    torch, p, _lib, lib = env
    A = grids.dirichlet7(64)
    M = p.CsrMatrix.from_csr(A)
    need = ctypes.c_size_t()
    assert lib.block_bicgstab_workspace_size(M.handle, 8, 0, ctypes.byref(need)) == 0
    assert need.value > _lib.NOALLOC_SCRATCH_BYTES
    B = torch.zeros((A.n, 8), dtype=torch.float64, device="cuda")
    X = torch.zeros_like(B)
    st = lib.block_bicgstab_noalloc(M.handle, _ptr(B), _ptr(X), 8, 1e-10, 10, 0, None, None)
    assert st == _lib.EINVAL and b"scratch" in lib.mrhs_last_error()
    M.close()
