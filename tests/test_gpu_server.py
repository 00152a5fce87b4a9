"""GPU tests of the continuous-batching solve server.

Each request's result must satisfy the solve's tolerance, agree with the
oracle, and be the same whether the request is served alone or in a mix of
other requests arriving while it runs (bitwise: every column's arithmetic is
independent of the other columns in its block).
"""
import time

import numpy as np
import pytest

import oracle
from helpers import true_relres
from workloads import grids, rng

pytestmark = pytest.mark.gpu

GiB = 1 << 30


@pytest.fixture(scope="module")
def mrhs():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1711_10622_amd as p
    p.load(build_if_missing=False)
    return p


@pytest.fixture(scope="module")
def mats(mrhs):
    As = {
        "dir12": grids.dirichlet7(12),
        "dir20": grids.dirichlet7(20, 18, 16),
        "chan": grids.channel7(24, 16, 20, beta=2.0),
    }
    Ms = {k: mrhs.CsrMatrix.from_csr(A) for k, A in As.items()}
    yield As, Ms
    for M in Ms.values():
        M.close()


def rhs_for(A, k, seed):
    return rng.rhs_block(A.n, k, seed, mean_zero=A.nullspace_const)


@pytest.mark.parametrize("mixed", [False, True])
def test_alone_vs_mix_bitwise(mrhs, mats, mixed):
    As, Ms = mats
    A = As["chan"]
    R = rhs_for(A, 3, 4242)
    # alone
    srv = mrhs.SolveServer(4 * GiB, mixed=mixed)
    mid = srv.register(Ms["chan"])
    X_alone, inf_alone, st = srv.wait(srv.submit(mid, R, tol=1e-10))
    assert st == 0, inf_alone
    srv.close()
    assert np.all(true_relres(A, X_alone, R) <= 1e-10)
    Xo, _, _ = oracle.bicgstab(A, R, tol=1e-10, shadow_seed=mrhs.SHADOW_SEED)
    assert np.linalg.norm(X_alone - Xo) <= 1e-6 * np.linalg.norm(Xo)
    # in a mix: other requests on all three matrices before, during and after
    srv = mrhs.SolveServer(4 * GiB, mixed=mixed)
    ids = {k: srv.register(M) for k, M in Ms.items()}
    r = np.random.default_rng(7)
    tickets = []
    for i in range(6):
        name = ["dir12", "dir20", "chan"][i % 3]
        tickets.append(srv.submit(ids[name], rhs_for(As[name], int(r.integers(1, 9)), 100 + i), tol=1e-10))
    time.sleep(0.02)
    tR = srv.submit(ids["chan"], R, tol=1e-10)
    for i in range(6, 12):
        name = ["dir12", "dir20", "chan"][i % 3]
        tickets.append(srv.submit(ids[name], rhs_for(As[name], int(r.integers(1, 9)), 100 + i), tol=1e-10))
    X_mix, inf_mix, st = srv.wait(tR)
    assert st == 0
    for t in tickets:
        _, infs, st = srv.wait(t)
        assert st == 0, infs
    stats = srv.stats()
    srv.close()
    assert np.array_equal(X_mix, X_alone)
    assert [i["iters"] for i in inf_mix] == [i["iters"] for i in inf_alone]
    assert stats["completed"] == 13 and stats["submitted"] == 13
    assert stats["p50_ms"] > 0 and stats["p99_ms"] >= stats["p50_ms"] and stats["rhs_per_s"] > 0


def test_stream_of_requests_all_correct(mrhs, mats):
    As, Ms = mats
    srv = mrhs.SolveServer(4 * GiB, mixed=True)
    ids = {k: srv.register(M) for k, M in Ms.items()}
    r = np.random.default_rng(11)
    sent = []
    for i in range(30):
        name = ["dir12", "dir20", "chan"][int(r.integers(0, 3))]
        B = rhs_for(As[name], int(r.integers(1, 17)), 500 + i)
        sent.append((name, B, srv.submit(ids[name], B, tol=1e-10)))
        time.sleep(float(r.exponential(0.002)))
    total = 0
    for name, B, t in sent:
        X, infs, st = srv.wait(t)
        assert st == 0, infs
        assert np.all(true_relres(As[name], X, B) <= 1e-10)
        total += B.shape[1]
    s = srv.stats()
    srv.close()
    assert s["completed"] == 30 and s["rhs_completed"] == total and s["queued"] == 0


def test_budget_and_errors(mrhs, mats):
    As, Ms = mats
    import paper_1711_10622_amd._lib as L
    srv = mrhs.SolveServer(1 << 20)  # 1 MiB: nothing fits
    with pytest.raises(mrhs.MrhsError) as e:
        srv.register(Ms["dir20"])
    assert e.value.status == L.EBUDGET
    srv.close()
    srv = mrhs.SolveServer(4 * GiB)
    mid = srv.register(Ms["dir12"])
    with pytest.raises(mrhs.MrhsError):
        srv.submit(mid + 5, np.ones((As["dir12"].n, 1)))
    B = rhs_for(As["dir12"], 2, 9)
    B[:, 1] = 0.0
    X, infs, st = srv.wait(srv.submit(mid, B, tol=1e-10, maxit=2))
    assert st == L.ENOCONV and infs[0]["status"] == L.ENOCONV and infs[1]["status"] == 0
    assert np.all(X[:, 1] == 0)
    srv.close()


def test_budget_shared_between_matrices(mrhs, mats):
    """A budget that holds only one engine at a time still serves both matrices."""
    As, Ms = mats
    from paper_1711_10622_amd import _lib
    eb = [Ms[k].device_bytes() for k in ("dir12", "chan")]
    ws = [Ms[k].workspace_size(16) + 3 * 8 * 16 * As[k].n for k in ("dir12", "chan")]
    budget = sum(eb) + max(ws) + (1 << 20)
    srv = mrhs.SolveServer(budget)
    a = srv.register(Ms["dir12"])
    b = srv.register(Ms["chan"])
    ta = srv.submit(a, rhs_for(As["dir12"], 4, 1), tol=1e-10)
    tb = srv.submit(b, rhs_for(As["chan"], 4, 2), tol=1e-10)
    for t in (ta, tb):
        _, infs, st = srv.wait(t, timeout=120)
        assert st == 0, infs
    assert srv.stats()["admitted_bytes"] <= budget
    srv.close()


def test_budget_registration_keeps_every_engine_feasible(mrhs, mats):
    """A matrix is refused when the registered matrices plus the largest engine
    of any of them would exceed the budget, even if its own engine would fit:
    otherwise the larger engine could never be allocated again."""
    As, Ms = mats
    import paper_1711_10622_amd._lib as L
    dev = {k: Ms[k].device_bytes() for k in ("dir12", "chan")}
    eng = {k: Ms[k].workspace_size(16) + 3 * 8 * 16 * As[k].n for k in ("dir12", "chan")}
    assert eng["chan"] > eng["dir12"]
    budget = dev["chan"] + dev["dir12"] + eng["chan"] - 1
    assert dev["chan"] + eng["chan"] <= budget and dev["chan"] + dev["dir12"] + eng["dir12"] <= budget
    srv = mrhs.SolveServer(budget)
    b = srv.register(Ms["chan"])
    with pytest.raises(mrhs.MrhsError) as e:
        srv.register(Ms["dir12"])
    assert e.value.status == L.EBUDGET
    _, infs, st = srv.wait(srv.submit(b, rhs_for(As["chan"], 2, 3), tol=1e-10), timeout=120)
    assert st == 0, infs
    srv.close()


def test_budget_turns_no_starvation(mrhs, mats):
    """With room for one engine, a matrix kept busy by a long stream of
    requests yields its engine to a waiting matrix between batches: the
    waiting request finishes while most of the stream is still queued."""
    As, Ms = mats
    dev = sum(Ms[k].device_bytes() for k in ("dir12", "chan"))
    eng = max(Ms[k].workspace_size(16) + 3 * 8 * 16 * As[k].n for k in ("dir12", "chan"))
    srv = mrhs.SolveServer(dev + eng + (1 << 20))
    a = srv.register(Ms["dir12"])
    b = srv.register(Ms["chan"])
    stream = [srv.submit(a, rhs_for(As["dir12"], 16, 100 + i), tol=1e-10) for i in range(60)]
    tb = srv.submit(b, rhs_for(As["chan"], 4, 7), tol=1e-10)
    _, infs, st = srv.wait(tb, timeout=120)
    assert st == 0, infs
    pending = 0
    done = []
    for t in stream:
        r = srv.poll(t)
        if r is None:
            pending += 1
        else:
            done.append(r)
    assert pending >= 30, pending
    for t in stream:
        if srv._k.get(t) is not None:
            done.append(srv.wait(t, timeout=120))
    assert len(done) == 60 and all(st == 0 for _, _, st in done)
    srv.close()


@pytest.mark.parametrize("vc32", [False, True])
def test_amg_server(mrhs, mats, vc32):
    """MRHS_SERVER_AMG: every request is solved by AMG-preconditioned block
    BiCGStab (a hierarchy per registered matrix; with MRHS_SERVER_MIXED the
    V-cycle in binary32); each result meets the tolerance in few iterations,
    equals bitwise the same request served alone, and agrees with
    block_bicgstab_amg on the matrix."""
    import torch
    As, Ms = mats
    A = As["chan"]
    R = rhs_for(A, 3, 4343)
    srv = mrhs.SolveServer(4 * GiB, amg=True, mixed=vc32)
    mid = srv.register(Ms["chan"])
    X_alone, inf_alone, st = srv.wait(srv.submit(mid, R, tol=1e-10))
    srv.close()
    assert st == 0, inf_alone
    assert np.all(true_relres(A, X_alone, R) <= 1e-10)
    assert max(i["iters"] for i in inf_alone) <= 40, inf_alone
    H = mrhs.AmgHierarchy(Ms["chan"])
    Xh, ih, sh = H.solve(torch.from_numpy(R).cuda(), tol=1e-10, maxit=20000, mixed=vc32)
    H.close()
    assert sh == 0
    Xh = Xh.cpu().numpy()
    assert np.linalg.norm(X_alone - Xh) <= 1e-6 * np.linalg.norm(Xh)
    srv = mrhs.SolveServer(4 * GiB, amg=True, mixed=vc32)
    ids = {k: srv.register(M) for k, M in Ms.items()}
    r = np.random.default_rng(8)
    sent = []
    for i in range(9):
        name = ["dir12", "dir20", "chan"][i % 3]
        B = rhs_for(As[name], int(r.integers(1, 9)), 700 + i)
        sent.append((name, B, srv.submit(ids[name], B, tol=1e-10)))
    tR = srv.submit(ids["chan"], R, tol=1e-10)
    X_mix, inf_mix, st = srv.wait(tR)
    assert st == 0
    for name, B, t in sent:
        X, infs, st = srv.wait(t)
        assert st == 0, infs
        assert np.all(true_relres(As[name], X, B) <= 1e-10)
        assert max(i["iters"] for i in infs) <= 40, infs
    srv.close()
    assert np.array_equal(X_mix, X_alone)
