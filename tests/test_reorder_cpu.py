"""The row renumbering of MRHS_CSR_REORDER (csr_reorder_permutation, host
code, no device): reverse Cuthill-McKee on the pattern of A + A^T.

Pinned by properties of a Cuthill-McKee order that do not depend on how it is
computed (every row after the first of its component has an earlier-numbered
neighbour; the first-numbered neighbours of successive rows never decrease;
rows sharing that neighbour come in order of degree), by the exact bandwidth 1
on a relabelled path, and by SciPy's reverse Cuthill-McKee (another choice of
starting rows), whose bandwidth it must match within 10% on relabelled grids.
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components, reverse_cuthill_mckee

from paper_1711_10622_amd import _lib, api
from workloads import grids, rng
from workloads.grids import CSRMatrix


def bandwidth(A):
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    return int(np.abs(rows - A.col).max()) if A.col.size else 0


def sym_adjacency(A):
    S = sp.csr_matrix((np.ones(A.col.size), A.col, A.row_ptr), shape=(A.n, A.n))
    S = ((S + S.T) > 0).tolil()
    S.setdiag(0)
    S = S.tocsr()
    S.eliminate_zeros()
    return [set(S.indices[S.indptr[i]:S.indptr[i + 1]].tolist()) for i in range(A.n)]


def check_cuthill_mckee(A, perm):
    """perm[new] = old must be the reverse of a Cuthill-McKee order of A + A^T."""
    n = A.n
    assert np.array_equal(np.sort(perm), np.arange(n))
    adj = sym_adjacency(A)
    deg = np.array([len(a) for a in adj])
    cm = perm[::-1]                       # the Cuthill-McKee order itself
    pos = np.empty(n, dtype=np.int64)
    pos[cm] = np.arange(n)
    S = sp.csr_matrix((np.ones(A.col.size), A.col, A.row_ptr), shape=(n, n))
    _, comp = connected_components(S, directed=True, connection="weak")
    seen = set()
    prev_parent = -1
    prev_deg = -1
    for k, v in enumerate(cm):
        earlier = [pos[u] for u in adj[v] if pos[u] < k]
        if comp[v] not in seen:
            # a component starts: nothing of it numbered before, and every
            # row of the previous component is already numbered
            seen.add(comp[v])
            assert not earlier
            prev_parent, prev_deg = -1, -1
            continue
        assert earlier, (k, v)
        parent = min(earlier)
        assert parent >= prev_parent, (k, parent, prev_parent)
        if parent == prev_parent:
            assert deg[v] >= prev_deg, (k, v)
        prev_parent, prev_deg = parent, deg[v]
    # components are contiguous in the order
    runs = comp[cm]
    assert len(set(runs.tolist())) == np.count_nonzero(np.diff(runs) != 0) + 1
    # the reversal never enlarges the envelope (Liu and Sherman 1976)
    assert envelope(adj, perm) <= envelope(adj, cm)


def envelope(adj, order):
    """Sum over rows of the distance to the row's first nonzero left of the
    diagonal, in the numbering order[new] = old."""
    pos = np.empty(len(order), dtype=np.int64)
    pos[order] = np.arange(len(order))
    return int(sum(max(0, pos[v] - min((pos[u] for u in adj[v]), default=pos[v])) for v in range(len(order))))


def relabelled(A, seed):
    return grids.permute_symmetric(A, rng.permutation(A.n, seed))


def test_star_is_reversed():
    """A star of k leaves: a Cuthill-McKee order from a leaf puts the centre
    second and leaves its k - 1 later leaves an envelope of order k^2; the
    reversed order has envelope k."""
    k = 12
    rows = [0] * (k + 1) + list(range(1, k + 1)) * 2
    cols = list(range(k + 1)) + [0] * k + list(range(1, k + 1))
    order = np.lexsort((cols, rows))
    rows, cols = np.array(rows)[order], np.array(cols)[order]
    rp = np.zeros(k + 2, dtype=np.int32)
    np.add.at(rp, rows + 1, 1)
    A = relabelled(CSRMatrix(k + 1, np.cumsum(rp).astype(np.int32), cols.astype(np.int32), np.ones(cols.size)), 9)
    perm = api.reorder_permutation(A)
    check_cuthill_mckee(A, perm)
    adj = sym_adjacency(A)
    assert envelope(adj, perm) == k and envelope(adj, perm[::-1]) > k * (k - 1) // 2


def test_relabelled_path_gets_bandwidth_one():
    A = relabelled(grids.dirichlet7(97, 1, 1), 3)
    assert bandwidth(A) > 1
    perm = api.reorder_permutation(A)
    check_cuthill_mckee(A, perm)
    assert bandwidth(grids.permute_symmetric(A, perm)) == 1


@pytest.mark.parametrize("name", ["dir12", "dir13x11x7", "chan24x16x20", "cube48"])
def test_relabelled_grids(name):
    if name == "dir12":
        A = grids.dirichlet7(12)
    elif name == "dir13x11x7":
        A = grids.dirichlet7(13, 11, 7)
    elif name == "chan24x16x20":
        A = grids.channel7(24, 16, 20, beta=2.0)
    else:
        solid = grids.cube_array_solid(48, 24, 32, ncube=2, h=4, pitch_x=24, pitch_z=16, off_x=4, off_z=4)
        A = grids.channel7(48, 24, 32, beta=2.0, lx=3.0, ly=1.5, lz=2.0, solid=solid)
    natural = bandwidth(A)
    R = relabelled(A, 10622)
    perm = api.reorder_permutation(R)
    check_cuthill_mckee(R, perm)
    ours = bandwidth(grids.permute_symmetric(R, perm))
    S = sp.csr_matrix((R.val, R.col, R.row_ptr), shape=(R.n, R.n))
    ref = bandwidth(grids.permute_symmetric(R, reverse_cuthill_mckee(S, symmetric_mode=True)))
    assert ours <= 1.1 * ref, (ours, ref)
    assert ours <= 1.25 * natural and ours * 8 < bandwidth(R), (ours, natural, bandwidth(R))
    # deterministic
    assert np.array_equal(perm, api.reorder_permutation(R))


def test_components_isolated_rows_and_one_sided_pattern():
    # two grids, three rows with only a diagonal, one empty row, and a chain
    # stored upper-triangular only (the pattern is symmetrized)
    a = grids.dirichlet7(5, 4, 3)
    b = grids.dirichlet7(3, 3, 3)
    rows, cols = [], []
    for blk, off in ((a, 0), (b, a.n)):
        r = np.repeat(np.arange(blk.n), np.diff(blk.row_ptr))
        rows += (r + off).tolist()
        cols += (blk.col + off).tolist()
    base = a.n + b.n
    rows += [base, base + 1, base + 2]
    cols += [base, base + 1, base + 2]
    chain = base + 4
    for i in range(6):
        rows += [chain + i]
        cols += [chain + i + 1]
    n = chain + 7
    rows, cols = np.array(rows), np.array(cols)
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    rp = np.zeros(n + 1, dtype=np.int32)
    np.add.at(rp, rows + 1, 1)
    rp = np.cumsum(rp).astype(np.int32)
    A = CSRMatrix(n, rp, cols.astype(np.int32), np.ones(cols.size), name="mix")
    R = relabelled(A, 77)
    perm = api.reorder_permutation(R)
    check_cuthill_mckee(R, perm)


def test_empty_and_invalid():
    lib = _lib.load()
    assert lib.csr_reorder_permutation(0, None, None, None) == _lib.OK
    perm = np.empty(2, dtype=np.int32)
    for rp, ci in (([1, 1, 2], [0, 1]), ([0, 2, 1], [0, 1]), ([0, 1, 2], [0, 2]), ([0, 1, 2], [0, -1])):
        rp = np.array(rp, dtype=np.int32)
        ci = np.array(ci, dtype=np.int32)
        assert lib.csr_reorder_permutation(2, rp.ctypes.data, ci.ctypes.data, perm.ctypes.data) == _lib.EINVAL
    assert lib.csr_reorder_permutation(-1, None, None, None) == _lib.EINVAL
    rp = np.array([0, 1, 2], dtype=np.int32)
    assert lib.csr_reorder_permutation(2, rp.ctypes.data, None, perm.ctypes.data) == _lib.EINVAL
    assert "NULL" in lib.mrhs_last_error().decode()
