"""The benchmark's offline rule for the bytes a product streams from a matrix
(bench.matrix_stream_bytes, used when the rocprofv3 summaries are written
without a device), on matrices whose form follows from their construction:
a 7-point stencil has 7 offsets and 2 values (16-bit codes), the same rows
relabelled have thousands of offsets (32-bit column codes), and per-entry
perturbed values exceed the 2048-entry table (plain arrays).  The GPU tests
check the same rule against csr_stream_bytes of the library."""
import numpy as np
import pytest

import bench
from workloads import grids, rng
from workloads.grids import CSRMatrix


def plain(A, S):
    return 4 * (A.n + 1) + (4 + S) * A.nnz


@pytest.mark.parametrize("S", [8, 4])
@pytest.mark.parametrize("scaled", [False, True])
def test_forms(S, scaled):
    D = grids.dirichlet7(10)
    assert bench.matrix_stream_bytes(D, S, scaled) == 4 * (D.n + 1) + 2 * D.nnz
    R = grids.permute_symmetric(D, rng.permutation(D.n, 3))
    assert bench.matrix_stream_bytes(R, S, scaled) == 4 * (R.n + 1) + 4 * R.nnz
    g = np.random.default_rng(5)
    P = CSRMatrix(D.n, D.row_ptr, D.col, D.val * (1.0 + 1e-3 * g.random(D.nnz)))
    assert bench.matrix_stream_bytes(P, S, scaled) == plain(P, S)


def test_value_table_limit():
    """At most 2048 distinct values per table: a diagonal matrix with 2048
    values takes 16-bit codes (one offset); a relabelled tridiagonal matrix
    (many offsets) takes 32-bit column codes with 2048 distinct values and
    the plain arrays with 2049."""
    n = 3000
    rows = np.arange(n)
    vals = 4.0 + (rows % 2048) * 2.0 ** -10
    rp = np.arange(n + 1, dtype=np.int32)
    D = CSRMatrix(n, rp, rows.astype(np.int32), vals)
    assert bench.matrix_stream_bytes(D, 8, False) == 4 * (n + 1) + 2 * n
    # the same values on a tridiagonal pattern, relabelled: many offsets,
    # 2049 distinct values -> plain; 2048 -> column codes
    for k, per in ((2047, 4), (2048, 12)):
        ci, va, rps = [], [], [0]
        for i in range(n):
            for o in (-1, 0, 1):
                if 0 <= i + o < n:
                    ci.append(i + o)
                    va.append(4.0 + (i % k) * 2.0 ** -10 if o == 0 else -1.0)
            rps.append(len(ci))
        T = CSRMatrix(n, np.array(rps, np.int32), np.array(ci, np.int32), np.array(va))
        R = grids.permute_symmetric(T, rng.permutation(n, 11))
        assert bench.matrix_stream_bytes(R, 8, False) == 4 * (n + 1) + per * R.nnz, k
