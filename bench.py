#!/usr/bin/env python3
"""Benchmark of the block multi-RHS pressure-Poisson solve on one MI355X.

Workload (the large channel case of the metric): the finite-volume pressure
operator of a 256 x 192 x 256 channel (periodic x/z, Neumann walls, tanh
beta = 2 wall stretching; n = 12,582,912, nnz = 87,949,312) with m = 16
mean-zero U[-1,1) right-hand sides (seed 1715), solved by block
Jacobi-BiCGStab in binary64 to a true relative residual of 1e-10 from x0 = 0.
One step = one such block solve (every kernel of the path: products, fused
vector updates, per-column dots, device-side scalar control, true residual
checks, the null-space projection and the final residual).  ``value`` =
seconds per right-hand side = step time / m, with the matrix, B and the
workspace already resident in HBM.

``roofline`` prices the kernel with the largest share of the timed steps:
its algorithmic bytes per launch over its mean launch time, both taken from
HIP events recorded around every 8th launch of each kernel class on the
library's stream during the timed steps.  ``traffic`` is the HBM bytes per
launch that rocprofv3's FETCH_SIZE and WRITE_SIZE counters saw for that
kernel (scaled by what they read for a plain 1 GiB copy), taken from the
committed profile summary and reported only while the kernel sources are the
ones that were profiled.

``cpu_baseline``: the oracle's per-column BiCGStab on the same 16 columns,
one host thread per column, run for 2 and for 12 iterations; the difference
gives the time per iteration, and s/RHS is setup plus the GPU solve's
iteration count times that, over m.

Also reported (not part of ``value``): the library's streaming kernels'
read/write/copy rates (the attainable memory ceilings), the mixed binary32 /
binary64 solve of the same block, the time per iteration at a fixed count for
m = 1, 2, 4, 8, 16 with the speedup per right-hand side beside the paper's
traffic models (Section 2.3), the generalized SpMV sweep m = 1..16 (binary64
and binary32), the 524k-row channel (solves per m, mixed, error against the
oracle), the relabelled cube channel (m = 8) in both precisions, the ensemble
projection step, and open-loop serving (p50/p99 latency, RHS/s).
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "block-BiCGStab s/RHS to 1e-10 and GSpMV GB/s, m=1..16, FP64 vs FP32+refine"
HBM_PEAK_GBS = 8000.0
# every 8th launch of each kernel class is timed with a pair of HIP events:
# a pair leaves the stream idle for a few microseconds, which timing every
# launch would add to every step
TRACE_EVERY = 8
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_solve_chan256_m16.md")
HEADLINE = "chan256"


def log(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


def kernel_bytes(name, n, nnz, m, S, mat=None):
    """Algorithmic HBM bytes of one launch of a library kernel with all m
    columns active: each block (n x m, S bytes/element) read or written once,
    the matrix read once: ``mat`` bytes (csr_stream_bytes: row offsets plus
    2-byte codes in the dictionary form), by default the plain arrays (int32
    row offsets and columns, S-byte values)."""
    if mat is None:
        mat = 4 * (n + 1) + (4 + S) * nnz
    blk = S * m * n
    # the binary64 shadow residual is generated in the kernels; binary32
    # inner solves read its sign bits, one byte per lane of a row
    VW = 4 if m % 4 == 0 else 2 if m % 2 == 0 else 1
    G = m // VW
    L = G if (VW == 1 or G == 5) and 64 // G > 64 // next_pow2(G) else next_pow2(G)
    sgn = 0 if S == 8 else n * L
    table = {
        "gspmv": mat + 2 * blk,             # read X, write Y
        "spmv_sigma": mat + 2 * blk + sgn,  # read p (gathered); write v
        "spmv_omega": mat + 3 * blk + sgn,  # read r, v (gathered); write t
        "xr_update": 8 * blk + sgn,         # read y, r, p, v, t; write y, r, p
    }
    return table.get(name)


_MAT_CACHE = {}


def matrix_stream_bytes(A, S, scaled):
    """Bytes a product streams from A's arrays, by the rule csr_create uses
    for the dictionary form (at most 2048 distinct values in the value array:
    A or A D^-1, binary64 or its binary32 rounding; 2-byte codes with at most
    32 distinct column offsets, else 4-byte codes when n fits 32 minus the
    value index's bits), for offline summaries; runs on a device use
    CsrMatrix.stream_bytes."""
    import numpy as np
    key = (id(A), S, bool(scaled))
    if key not in _MAT_CACHE or _MAT_CACHE[key][0] is not A:
        plain = 4 * (A.n + 1) + (4 + S) * A.nnz
        rows = np.repeat(np.arange(A.n, dtype=np.int64), np.diff(A.row_ptr))
        off = A.col.astype(np.int64) - rows
        by_offset = np.unique(off).size <= 32
        v = A.val
        if scaled:
            d = np.zeros(A.n)
            np.add.at(d, rows[off == 0], A.val[off == 0])
            dc = d[A.col]
            v = np.where(dc != 0.0, A.val / np.where(dc != 0.0, dc, 1.0), 0.0)
        if S == 4:
            v = v.astype(np.float32)
        nv = np.unique(v.view(np.uint64 if S == 8 else np.uint32)).size
        per = 4 + S
        if nv <= 2048:
            vb = max(1, int(np.ceil(np.log2(nv))) if nv > 1 else 1)
            per = 2 if by_offset else 4 if A.n <= 2 ** (32 - vb) else per
        # (the entry keeps A alive, so its id is not reused while cached)
        _MAT_CACHE[key] = (A, 4 * (A.n + 1) + per * A.nnz)
    return _MAT_CACHE[key][1]


def next_pow2(x):
    return 1 if x <= 1 else 2 * next_pow2((x + 1) // 2)


def summary_mat(A, name, S):
    """Matrix bytes of a product kernel in an offline summary (gspmv reads A,
    the solvers' products A D^-1)."""
    if name not in ("gspmv", "spmv_sigma", "spmv_omega"):
        return None
    return matrix_stream_bytes(A, S, scaled=name != "gspmv")


def kernel_sources_digest():
    """sha256 over the HIP sources and the C header, so a stored counter
    reading is used only for the kernels it was taken on."""
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(ROOT, "paper_1711_10622_amd", "csrc", "*")))
    files.append(os.path.join(ROOT, "include", "mrhs.h"))
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def stored_traffic(kernel):
    """HBM bytes per launch of ``kernel`` from the profile summary, or None
    when there is none for it or the sources changed since it was taken."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    digest = kernel_sources_digest()
    for mo in re.finditer(r"^traffic: kernel=(\S+) bytes_per_launch=(\d+) sources_sha256=([0-9a-f]{64})\s*$",
                          text, re.M):
        if mo.group(1) == kernel and mo.group(3) == digest:
            return int(mo.group(2))
    return None


def dominant_kernel(trace, n, nnz, mats=None):
    """The kernel class with the largest estimated total time; ``mats``:
    matrix bytes per product by element size (the solvers' scaled matrix)."""
    best = None
    for key, st in trace.items():
        name, dt, mtag, _ = key.split("/")
        share = st["total_ms"] / max(st["launches"], 1) * st["seen"]   # estimated total time
        if st["launches"] and (best is None or share > best[5]):
            best = (key, st, name, 8 if dt == "f64" else 4, int(mtag[1:]), share)
    key, st, name, S, m, _ = best
    avg_ms = st["total_ms"] / st["launches"]
    byt = kernel_bytes(name, n, nnz, m, S, (mats or {}).get(S))
    achieved = byt / (avg_ms * 1e-3) / 1e9 if byt else None
    return {"kernel": key, "class": "/".join(key.split("/")[:3]), "launches": st["seen"], "timed": st["launches"],
            "avg_us": avg_ms * 1e3, "bytes_per_launch": byt, "achieved": achieved}


def timed_solves(torch, M, B, X, ws, steps, mixed=False, trace=False, tol=1e-10, maxit=20000,
                 expect_ok=True, label=None):
    """``steps`` block solves; each returns once its columns are decided (the
    library reads their states back), so a ``label`` line after every solve
    reports progress without adding a synchronization."""
    import paper_1711_10622_amd as mrhs
    infos = None
    torch.cuda.synchronize()
    if trace:
        mrhs.trace_enable(True, every=TRACE_EVERY)
    t0 = time.perf_counter()
    for k in range(steps):
        _, infos, st = M.solve(B, tol=tol, maxit=maxit, mixed=mixed, out=X, workspace=ws)
        if expect_ok and st != 0:
            raise RuntimeError(f"solve did not converge: {infos}")
        if label:
            log(f"{label} solve {k + 1}/{steps} done")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tr = None
    if trace:
        tr = mrhs.trace_read()
        mrhs.trace_enable(False)
    return (t1 - t0) / steps, infos, tr


def event_times_us(torch, fn, reps, warm, between=None):
    """Per-repetition durations of fn() from HIP events on the current
    stream, after ``warm`` untimed calls; ``between`` runs untimed before
    every repetition (cache flushing)."""
    for _ in range(warm):
        fn()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        if between is not None:
            between()
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    import numpy as np
    return np.array([a.elapsed_time(b) * 1e3 for a, b in ev])


def projection_step(torch, ms=(1, 16), tau=0.05, reps=20):
    """The ensemble projection step on the 128x64x64 channel (Section 2.2,
    eqs. (3)-(4)): pressure right-hand sides, block solve to 1e-10,
    correction, for m fields at once.  Kernel times from HIP events (median of
    ``reps``) with their algorithmic bytes, the solve's share theta of the
    step, and the whole-step gain m t_1 / t_m."""
    import numpy as np
    import paper_1711_10622_amd as mrhs
    from paper_1711_10622_amd import estimates as est
    from workloads import configs, staggered
    nx, ny, nz = 128, 64, 64
    geo = staggered.channel_geometry(nx, ny, nz)
    G = mrhs.ChannelGrid(nx, ny, nz, geo["dx"], geo["dz"], geo["y_faces"])
    M = mrhs.CsrMatrix.from_csr(configs.MATRICES["chan128"]())
    out = {}
    for m in ms:
        U, V, W = (torch.from_numpy(a).cuda() for a in staggered.velocity_blocks(nx, ny, nz, m, 1716))
        B = torch.empty((G.n, m), dtype=torch.float64, device="cuda")
        P = torch.empty_like(B)
        ws = torch.empty(M.workspace_size(m), dtype=torch.uint8, device="cuda")
        U0, V0, W0 = U.clone(), V.clone(), W.clone()
        t_rhs = float(np.median(event_times_us(torch, lambda: G.rhs(U, V, W, tau, out=B), reps, 3)))
        t_cor = float(np.median(event_times_us(
            torch, lambda: G.correct(U, V, W, P, tau), reps, 3,
            between=lambda: (U.copy_(U0), V.copy_(V0), W.copy_(W0)))))
        U.copy_(U0); V.copy_(V0); W.copy_(W0)
        G.rhs(U, V, W, tau, out=B)
        timed_solves(torch, M, B, P, ws, 1)  # warm-up
        t_solve, infos, _ = timed_solves(torch, M, B, P, ws, 2)
        t0 = time.perf_counter()
        G.rhs(U, V, W, tau, out=B)
        M.solve(B, tol=1e-10, out=P, workspace=ws)
        G.correct(U, V, W, P, tau)
        torch.cuda.synchronize()
        t_step = time.perf_counter() - t0
        S = 8 * m
        rhs_bytes = S * (2 * G.cells + G.v_faces + G.n) + 4 * G.cells
        cor_bytes = S * (G.n + 2 * (2 * G.cells + G.v_faces)) + 4 * G.cells
        out[str(m)] = {
            "rhs_us": round(t_rhs, 2), "rhs_GBps": round(rhs_bytes / t_rhs / 1e3, 1),
            "correct_us": round(t_cor, 2), "correct_GBps": round(cor_bytes / t_cor / 1e3, 1),
            "solve_ms": round(t_solve * 1e3, 3), "step_ms": round(t_step * 1e3, 3),
            "theta_solve": round(t_solve / (t_solve + (t_rhs + t_cor) * 1e-6), 5),
            "iters_max": max(i["iters"] for i in infos),
        }
        del U, V, W, U0, V0, W0, B, P, ws
    if "1" in out:
        # eq. est2_1 with measured inputs: the step gain predicted from the
        # m = 1 solve share theta and the measured solve gain, beside the
        # measured step gain
        th = out["1"]["theta_solve"]
        for k, v in out.items():
            v["solve_gain_vs_m1"] = round(int(k) * out["1"]["solve_ms"] / v["solve_ms"], 3)
            v["step_gain_vs_m1"] = round(int(k) * out["1"]["step_ms"] / v["step_ms"], 3)
            v["est2_1_step_gain"] = round(est.step_gain(th, v["solve_gain_vs_m1"]), 3)
    M.close()
    G.close()
    return out


def gspmv_sweep(torch, A, ms, dtypes, flush=False, reps=50, plain=False):
    """GSpMV times over block widths ``ms``; ``plain``: the handle is made
    with MRHS_CSR_DICT=0, so the products read the index and value arrays."""
    import numpy as np
    import paper_1711_10622_amd as mrhs
    old = os.environ.get("MRHS_CSR_DICT")
    if plain:
        os.environ["MRHS_CSR_DICT"] = "0"
    try:
        M = mrhs.CsrMatrix.from_csr(A)
    finally:
        if plain:
            if old is None:
                del os.environ["MRHS_CSR_DICT"]
            else:
                os.environ["MRHS_CSR_DICT"] = old
    out = {}
    scratch = torch.empty(1 << 30, dtype=torch.uint8, device="cuda") if flush else None
    for dt in dtypes:
        tdt = torch.float64 if dt == "f64" else torch.float32
        S = 8 if dt == "f64" else 4
        for m in ms:
            X = torch.empty((A.n, m), dtype=tdt, device="cuda").uniform_(-1, 1)
            Y = torch.empty_like(X)
            runs = {"warm": None}
            if flush:
                runs["flushed"] = lambda: scratch.fill_(1)
            rec = {}
            for tag, between in runs.items():
                us = event_times_us(torch, lambda: M.gspmv(X, out=Y), reps, 5, between)
                med = float(np.median(us))
                byt = M.stream_bytes(dt) + 2 * S * m * A.n
                gbs = byt / (med * 1e-6) / 1e9
                rec[tag] = {"us_median": round(med, 2), "us_p10": round(float(np.percentile(us, 10)), 2),
                            "us_p90": round(float(np.percentile(us, 90)), 2), "GBps": round(gbs, 1),
                            "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4)}
            out[f"{dt}/m{m}"] = rec if flush else rec["warm"]
            del X, Y
    M.close()
    return out


def gspmv_locality(torch, A, line=256):
    """GSpMV on A with every column index moved into its row's own line of
    ``line`` rows (same row lengths, values and bytes; every gather then hits
    rows the tile just fetched): the time the product would take if staging
    the gathered rows made every gather local."""
    import numpy as np
    from workloads.grids import CSRMatrix
    rows = np.repeat(np.arange(A.n, dtype=np.int64), np.diff(A.row_ptr))
    col = ((rows // line) * line + (A.col.astype(np.int64) % line)).astype(np.int32)
    del rows
    L = CSRMatrix(A.n, A.row_ptr, col, A.val, name=A.name + "_inline")
    return gspmv_sweep(torch, L, [8, 16], ("f64", "f32"), reps=20)


def gspmv_march(torch, A):
    """GSpMV on A as a plane march (MRHS_MARCH=1: the gathered rows of three
    planes kept in LDS windows), beside the tiled product of the main sweep."""
    old = os.environ.get("MRHS_MARCH")
    os.environ["MRHS_MARCH"] = "1"
    try:
        return gspmv_sweep(torch, A, [1, 8, 16], ("f64", "f32"), reps=20)
    finally:
        if old is None:
            os.environ.pop("MRHS_MARCH", None)
        else:
            os.environ["MRHS_MARCH"] = old


def gspmv_cube(torch):
    """GSpMV on the relabelled cube channel as generated and renumbered by
    reverse Cuthill-McKee (the permutation MRHS_CSR_REORDER applies)."""
    import paper_1711_10622_amd as mrhs
    from workloads import configs, grids
    C = configs.MATRICES["cube192"]()
    out = {"relabelled": gspmv_sweep(torch, C, [8, 16], ("f64", "f32"), reps=20)}
    Cr = grids.permute_symmetric(C, mrhs.reorder_permutation(C))
    out["rcm"] = gspmv_sweep(torch, Cr, [8, 16], ("f64", "f32"), reps=20)
    return out


def solve_pair(torch, name, m, steps, reorder=False, amg_per_iter=None):
    """binary64 and mixed block solves of one workload, its own matrix
    (renumbered by reverse Cuthill-McKee when ``reorder``), then the AMG legs."""
    import numpy as np
    import paper_1711_10622_amd as mrhs
    from workloads import configs
    wl = configs.WORKLOADS[name]
    A = wl.matrix()
    Bh = wl.rhs(A.n, m)
    t0 = time.perf_counter()
    M = mrhs.CsrMatrix.from_csr(A, reorder=reorder)
    torch.cuda.synchronize()
    create_s = time.perf_counter() - t0
    B = torch.from_numpy(Bh).to("cuda")
    X = torch.empty_like(B)
    ws = torch.empty(max(M.workspace_size(m, mixed=True), M.workspace_size(m)), dtype=torch.uint8, device="cuda")
    res = {"n": A.n, "nnz": A.nnz, "m": m, "reorder": bool(reorder), "csr_create_s": round(create_s, 3)}
    for mixed in (False, True):
        t, inf, _ = timed_solves(torch, M, B, X, ws, steps, mixed=mixed)
        res["mixed" if mixed else "fp64"] = {
            "s_per_rhs": round(t / m, 6), "iters_max": max(i["iters"] for i in inf),
            "outer_max": max(i["outer"] for i in inf), "max_relres": max(i["relres"] for i in inf)}
        log(f"{name} m={m} {'mixed' if mixed else 'fp64'}{' rcm' if reorder else ''}: {t * 1e3:.1f} ms")
    res["mixed_speedup"] = round(res["fp64"]["s_per_rhs"] / res["mixed"]["s_per_rhs"], 3)
    del M, B, X, ws
    torch.cuda.empty_cache()
    res["amg"] = amg_legs(torch, A, Bh, m, res["fp64"]["s_per_rhs"] * m,
                          per_iter_ms=amg_per_iter if amg_per_iter is not None else (1, m), steps=2, reorder=reorder)
    torch.cuda.empty_cache()
    return res


def serving(torch, n_req=300, seed=1714, mean_gap_s=0.005, budget=16 << 30, rate=None, amg=False,
            closed=False):
    """Serving run over a seeded request stream: each request picks one of the
    32^3 / 64^3 Dirichlet operators and the 128x64x64 channel with
    probability 1/3 and k ~ U{1..16} right-hand sides, solved to 1e-10 by
    mixed-precision Jacobi-BiCGStab (or, with ``amg``, AMG-preconditioned
    BiCGStab with the V-cycle in binary32); HBM budget ``budget``.  Open loop: requests arrive
    with exponential gaps of mean ``mean_gap_s`` (or scaled to ``rate``
    right-hand sides per second).  ``closed``: every request is submitted at
    once and the run measures the server's capacity.  Request blocks are
    built before the clock starts, so submitting costs only the server's own
    copy of B; latencies are stamped by the server (submit to completion)."""
    import numpy as np
    import paper_1711_10622_amd as mrhs
    from workloads import configs, rng
    names = ["dir32", "dir64", "chan128"]
    mats, pools, ids = [], [], []
    srv = mrhs.SolveServer(budget, mixed=True, amg=amg)
    for nm in names:
        wl = configs.WORKLOADS[nm]
        A = wl.matrix()
        M = mrhs.CsrMatrix.from_csr(A)
        mats.append(M)
        ids.append(srv.register(M))
        pools.append(rng.rhs_block(A.n, 32, seed, mean_zero=wl.mean_zero))
    u = rng.uniform_pm1(seed + 1, np.arange(3 * n_req, dtype=np.uint64)).reshape(n_req, 3) * 0.5 + 0.5
    gaps = -np.log1p(-np.minimum(u[:, 0], 1 - 1e-16)) * mean_gap_s
    which = np.minimum((u[:, 1] * 3).astype(int), 2)
    ks = np.minimum((u[:, 2] * 16).astype(int), 15) + 1
    rhs = int(ks.sum())
    if rate is not None:
        gaps = gaps * (rhs / gaps.sum()) / rate
    arrive = np.zeros(n_req) if closed else np.cumsum(gaps)
    # request i solves columns c0 .. c0 + k - 1 of its matrix's pool, c0 one
    # of four offsets; the distinct blocks (at most 3 x 16 x 4) are built
    # before the clock starts and shared by the requests that use them
    cache = {}
    keys = []
    for i in range(n_req):
        key = (int(which[i]), int(ks[i]), 4 * (i % 4))
        if key not in cache:
            w, k, c0 = key
            cache[key] = np.ascontiguousarray(pools[w][:, c0:c0 + k])
        keys.append(key)
    del pools
    t0 = time.perf_counter()
    pending = {}
    done = 0
    max_q = 0
    bad = 0
    i = 0
    last_poll = -1.0
    while done < n_req:
        now = time.perf_counter() - t0
        while i < n_req and arrive[i] <= now:
            tk = srv.submit(ids[which[i]], cache[keys[i]])
            pending[tk] = i
            i += 1
            if closed:
                break
        max_q = max(max_q, len(pending))
        # results are collected every 10 ms while requests still arrive, so
        # polling hundreds of outstanding tickets does not delay the arrivals
        if i >= n_req or now - last_poll >= 0.01:
            last_poll = now
            for tk in list(pending):
                r = srv.poll(tk)
                if r is not None:
                    del pending[tk]
                    done += 1
                    bad += int(r[2] != 0)
        if i < n_req and not closed:
            time.sleep(max(0.0, min(0.001, arrive[i] - (time.perf_counter() - t0))))
        elif i >= n_req:
            time.sleep(0.0005)
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    for M in mats:
        M.close()
    out = {"solver": "amg_vc32" if amg else "mixed", "mode": "closed" if closed else "open", "requests": n_req,
           "rhs": rhs, "served_rhs_per_s": round(rhs / wall, 1), "wall_s": round(wall, 3),
           "p50_ms": round(st["p50_ms"], 2), "p99_ms": round(st["p99_ms"], 2),
           "server_rhs_per_s": round(st["rhs_per_s"], 1), "max_outstanding": max_q, "not_ok": bad}
    if not closed:
        out["offered_rhs_per_s"] = round(rhs / arrive[-1], 1)
    return out


def host_cores():
    try:
        return len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        return os.cpu_count() or 1


def cpu_baseline(A, Bh, gpu_iters, threads):
    """The oracle on the host cores: every column of Bh by its own
    right-Jacobi BiCGStab (the same shadow residual as the GPU solve), one
    thread per column, ``threads`` at a time, for 2 and for 12 iterations.
    The difference is the wall time of 10 iterations of all columns; s/RHS =
    (setup + gpu_iters iterations) / m."""
    import oracle
    import paper_1711_10622_amd as mrhs
    m = Bh.shape[1]
    wall = {}
    for k in (2, 12):
        t0 = time.perf_counter()
        _, infos, _ = oracle.bicgstab(A, Bh, tol=1e-300, maxit=k, threads=threads, shadow_seed=mrhs.SHADOW_SEED)
        wall[k] = time.perf_counter() - t0
        assert all(i["iters"] == k for i in infos), infos
        log(f"oracle {k} iterations x {m} columns on {threads} threads: {wall[k]:.2f} s")
    per_iter = (wall[12] - wall[2]) / 10
    setup = max(wall[2] - 2 * per_iter, 0.0)
    value = (setup + gpu_iters * per_iter) / m
    return {"value": value, "unit": "s/RHS", "cores": threads, "kind": "oracle",
            "sample": f"all {m} right-hand sides of the same workload, one host thread per column ({threads} "
                      f"threads), binary64, run for 2 and for 12 iterations ({wall[2]:.2f} s, {wall[12]:.2f} s): "
                      f"{per_iter:.3f} s per iteration of the block, setup {setup:.2f} s; s/RHS = (setup + "
                      f"{gpu_iters} iterations, the GPU solve's count) / {m}",
            "per_iter_s": round(per_iter, 4), "iters_basis": gpu_iters}


def oracle_error(A, Bh, Xgpu, ncols, threads):
    """Per-RHS relative error (mean-free) of GPU solutions against the
    oracle's own solves of the first ncols columns."""
    import numpy as np
    import oracle
    import paper_1711_10622_amd as mrhs
    t0 = time.perf_counter()
    Xo, infos, _ = oracle.bicgstab(A, Bh[:, :ncols].copy(), tol=1e-10, maxit=20000, threads=threads,
                                   shadow_seed=mrhs.SHADOW_SEED)
    assert all(i["status"] == 0 for i in infos), infos
    out = {"oracle_s": round(time.perf_counter() - t0, 2), "oracle_iters": [i["iters"] for i in infos]}
    for tag, X in Xgpu.items():
        out[tag] = [float(np.linalg.norm(X[:, l] - Xo[:, l]) / np.linalg.norm(Xo[:, l])) for l in range(ncols)]
    return out


def memory_ceilings(torch, nbytes=2 << 30, reps=10):
    """The library's streaming kernels over nbytes (8x the 256 MB
    Infinity Cache): median GB/s of read, write and copy, plain and
    nontemporal (a copy moves 2 nbytes)."""
    import numpy as np
    import paper_1711_10622_amd as mrhs
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    a.fill_(3)
    out = {}
    for kind in ("read", "read_nt", "write", "write_nt", "copy", "copy_nt"):
        us = event_times_us(torch, lambda: mrhs.stream_probe(kind, a, b, nbytes), reps, 2)
        moved = 2 * nbytes if kind.startswith("copy") else nbytes
        med = float(np.median(us))
        out[kind] = {"GBps": round(moved / (med * 1e-6) / 1e9, 1), "us_median": round(med, 1)}
    del a, b
    torch.cuda.empty_cache()
    out["bytes"] = nbytes
    return out


def host_info():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": host_cores(), "cpu_count": os.cpu_count(), "cpu_model": model}


def cpu_gspmv(A, m, threads):
    """The oracle's GSpMV (m separate SpMVs, the matrix re-read per column) on
    one host thread and on ``threads`` threads (rows split between them)."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    from paper_1711_10622_amd import estimates as est
    from workloads import rng
    X = rng.rhs_block(A.n, m, 99)
    byt = m * est.traffic_compulsory(A.n, A.nnz, 1)
    out = {"m": m, "note": "oracle: m separate SpMVs, matrix re-read per column"}
    t0 = time.perf_counter()
    oracle.gspmv(A, X)
    dt = time.perf_counter() - t0
    out["threads_1"] = {"s": round(dt, 4), "GBps": round(byt / dt / 1e9, 2)}
    cuts = np.linspace(0, A.n, threads + 1).astype(np.int64)
    parts = [oracle.row_subset(A, np.arange(cuts[k], cuts[k + 1])) for k in range(threads)]
    with ThreadPoolExecutor(max_workers=threads) as ex:
        t0 = time.perf_counter()
        list(ex.map(lambda S: oracle.gspmv_part(S, X), parts))
        dt = time.perf_counter() - t0
    out[f"threads_{threads}"] = {"s": round(dt, 4), "GBps": round(byt / dt / 1e9, 2)}
    return out


def copy_calibration():
    """A plain 1 GiB device copy, three times: the reference reading for
    the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    nb = 1 << 30
    a = torch.empty(nb, dtype=torch.uint8, device="cuda")
    a.fill_(1)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log("copied 3 x 1 GiB")
    return 0


def gspmv_only(name):
    """Five GSpMV launches per case (binary64 and binary32, m = 8 and 16) on
    one matrix, for counter runs under rocprofv3."""
    import torch
    import paper_1711_10622_amd as mrhs
    from workloads import configs
    mrhs.load(build_if_missing=False)
    A = configs.MATRICES[name]()
    M = mrhs.CsrMatrix.from_csr(A)
    for dt in (torch.float64, torch.float32):
        for m in (8, 16):
            X = torch.empty((A.n, m), dtype=dt, device="cuda").uniform_(-1, 1)
            Y = torch.empty_like(X)
            M.gspmv(X, out=Y)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(True), torch.cuda.Event(True)
            e0.record()
            for _ in range(5):
                M.gspmv(X, out=Y)
            e1.record()
            torch.cuda.synchronize()
            log(f"gspmv {name} {str(dt)[6:]} m={m}: {e0.elapsed_time(e1) / 5 * 1e3:.1f} us")
            del X, Y
    M.close()
    return 0


def solve_only(name, mixed, steps, maxit=20000, reorder=False):
    """``steps`` block solves of one workload at its largest configured m
    (binary64, or mixed), after one untimed solve: for kernel traces and
    counter runs under rocprofv3.  A small ``maxit`` caps the iterations
    (every column stays active, so every launch moves its full bytes);
    ``reorder`` renumbers the matrix by reverse Cuthill-McKee."""
    import numpy as np
    import torch
    import paper_1711_10622_amd as mrhs
    from workloads import configs
    mrhs.load(build_if_missing=False)
    wl = configs.WORKLOADS[name]
    m = max(wl.ms)
    A = wl.matrix()
    M = mrhs.CsrMatrix.from_csr(A, reorder=reorder)
    B = torch.from_numpy(np.ascontiguousarray(wl.rhs(A.n, m))).cuda()
    X = torch.empty_like(B)
    ws = torch.empty(M.workspace_size(m, mixed), dtype=torch.uint8, device="cuda")
    ok = maxit >= 20000
    timed_solves(torch, M, B, X, ws, 1, mixed=mixed, maxit=maxit, expect_ok=ok)
    t, infos, _ = timed_solves(torch, M, B, X, ws, steps, mixed=mixed, maxit=maxit, expect_ok=ok)
    log(f"solve {name}{' (RCM)' if reorder else ''} m={m} {'mixed' if mixed else 'fp64'}: {t * 1e3:.1f} ms per solve, "
        f"iterations max {max(i['iters'] for i in infos)}, outer max {max(i['outer'] for i in infos)}")
    M.close()
    return 0


def per_iteration(torch, M, Bh, ms, reps=1):
    """Time per block iteration at a fixed count (the paper's methodology,
    Section 4.1): difference of 200- and 100-iteration runs, so setup and the
    final residual cancel; with m t_1 / t_m beside the traffic models."""
    import numpy as np
    from paper_1711_10622_amd import estimates as est
    out = {}
    n, nnz = M.n, M.nnz
    for mm in ms:
        Bm = torch.from_numpy(np.ascontiguousarray(Bh[:, :mm])).to("cuda")
        Xm = torch.empty_like(Bm)
        ws = torch.empty(M.workspace_size(mm), dtype=torch.uint8, device="cuda")
        t100, _, _ = timed_solves(torch, M, Bm, Xm, ws, reps, tol=1e-300, maxit=100, expect_ok=False)
        t200, _, _ = timed_solves(torch, M, Bm, Xm, ws, reps, tol=1e-300, maxit=200, expect_ok=False)
        out[mm] = {"ms_per_iter": (t200 - t100) / 100 * 1e3}
        del Bm, Xm, ws
    i1 = out[ms[0]]["ms_per_iter"] if ms[0] == 1 else None
    for mm, d in out.items():
        if i1:
            d["iter_gain_vs_m1"] = round(mm * i1 / d["ms_per_iter"], 3)
        d["paper_compact_5m_2m3"] = round(est.gain_compact(mm), 3)
        d["paper_full_C"] = round(est.gain_full(mm, nnz / n), 3)
        d["compulsory_bytes_model"] = round(est.gain_compulsory(n, nnz, mm), 3)
        d["ms_per_iter"] = round(d["ms_per_iter"], 4)
    torch.cuda.empty_cache()
    return out


def small_iterations(torch):
    """Time per binary64 block iteration (m = 16) on matrices small enough
    that an iteration's three kernels are bound by their fixed costs (launch,
    the grid reductions' last-workgroup tails) rather than by bytes: the
    ceiling on what merging the iteration's kernels could save."""
    import paper_1711_10622_amd as mrhs
    from workloads import configs
    out = {}
    for name in ("dir16", "dir32", "dir64", "chan128"):
        wl = configs.WORKLOADS[name]
        A = wl.matrix()
        M = mrhs.CsrMatrix.from_csr(A)
        Bh = wl.rhs(A.n, 16)
        r = per_iteration(torch, M, Bh, (16,))
        out[name] = {"n": A.n, "ms_per_iter": r[16]["ms_per_iter"],
                     "us_per_kernel": round(r[16]["ms_per_iter"] * 1e3 / 3, 1)}
        M.close()
    return out


def merged_vs_plain(torch):
    """Time per binary64 block iteration with two kernels per iteration
    (MRHS_MERGE=2: the x/r/p update fused with the next v = A p) and with
    three (MRHS_MERGE=0), at several m on a 64^3 Dirichlet operator and the
    128x64x64 channel."""
    import paper_1711_10622_amd as mrhs
    from workloads import configs
    out = {}
    old = os.environ.get("MRHS_MERGE")
    try:
        for name in ("dir64", "chan128"):
            wl = configs.WORKLOADS[name]
            A = wl.matrix()
            Bh = wl.rhs(A.n, 16)
            rec = {}
            for flag, tag in (("0", "three_kernels"), ("2", "two_kernels")):
                os.environ["MRHS_MERGE"] = flag
                M = mrhs.CsrMatrix.from_csr(A)
                r = per_iteration(torch, M, Bh, (1, 4, 8, 16))
                rec[tag] = {mm: d["ms_per_iter"] for mm, d in r.items()}
                M.close()
            out[name] = rec
    finally:
        if old is None:
            os.environ.pop("MRHS_MERGE", None)
        else:
            os.environ["MRHS_MERGE"] = old
    return out


OP_NAMES = {"OpXR": "xr_update", "OpSpmv2": "spmv_omega", "OpSpmv1": "spmv_sigma", "OpResid": "resid",
            "OpScale": "scale", "OpRestart": "restart", "OpColSum": "colsum", "OpStore": "gspmv",
            "OpCast": "cast32", "OpGcrZ": "gcr_z", "OpColDots": "gcr_dots", "OpColOrth": "gcr_orth",
            "OpColUpdate": "gcr_update", "OpFold": "fold", "OpSpmv2P": "amg_omega", "OpXRP": "amg_xr",
            "OpSForm": "amg_s", "OpVcRes": "vc_resid", "OpVcProl": "vc_prolong", "OpVcSmooth": "vc_smooth",
            "OpVcStore": "vc_store", "OpColsStore": "gcr_aw", "OpTo32": "amg_to32", "OpTo64": "amg_to64",
            "OpXRSigma": "xr_sigma"}


def kernel_class(name):
    """'void mrhs::k_stream<double, 16, mrhs::OpXR<double, 16> >(...)' -> 'xr_update/f64/m16'."""
    mo = re.search(r"mrhs::k_(?:gspmv_march|gspmv|stream)<(double|float), (\d+), mrhs::(\w+)", name)
    if not mo:
        return name.split("(")[0][:60]
    return f"{OP_NAMES.get(mo.group(3), mo.group(3))}/{'f64' if mo.group(1) == 'double' else 'f32'}/m{mo.group(2)}"


def summarize_profiles(out, workload, m):
    """Markdown summary of the rocprofv3 runs under ``out`` (kernel trace in
    trace/, FETCH_SIZE and WRITE_SIZE counters in fetch/ and write/, the 1 GiB
    copy's counters in copy_fetch/ and copy_write/) for a workload of
    configs.WORKLOADS at block width m."""
    import csv
    from workloads import configs
    A = configs.MATRICES[workload]()

    def rows(sub, suffix):
        fs = glob.glob(os.path.join(out, sub, "**", f"*{suffix}"), recursive=True)
        return list(csv.DictReader(open(fs[0]))) if fs else []

    lines = []
    st = rows("trace", "kernel_stats.csv")
    if st:
        lines += ["| kernel | calls | avg us | min us | max us | share % | algorithmic MB | GB/s at avg |",
                  "|---|---|---|---|---|---|---|---|"]
        for r in st:
            cls = kernel_class(r["Name"])
            parts = cls.split("/")
            byt = kernel_bytes(parts[0], A.n, A.nnz, int(parts[2][1:]), 8 if parts[1] == "f64" else 4,
                               summary_mat(A, parts[0], 8 if parts[1] == "f64" else 4)) \
                if len(parts) == 3 else None
            avg = float(r["AverageNs"]) / 1e3
            lines.append(f"| {cls} | {r['Calls']} | {avg:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                         f"{float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} | "
                         f"{byt / 1e6 if byt else '':{'.1f' if byt else ''}} | "
                         f"{byt / (avg * 1e-6) / 1e9 if byt else '':{'.0f' if byt else ''}} |")
    cal = {}
    for c, sub in (("FETCH_SIZE", "copy_fetch"), ("WRITE_SIZE", "copy_write")):
        vals = [float(r["Counter_Value"]) for r in rows(sub, "counter_collection.csv")
                if "copyBuffer" in r["Kernel_Name"]]
        if vals:
            cal[c] = (1 << 20) / (sum(vals) / len(vals))   # 1 GiB = 1048576 KiB
    per = {}
    for c, sub in (("FETCH_SIZE", "fetch"), ("WRITE_SIZE", "write")):
        for r in rows(sub, "counter_collection.csv"):
            per.setdefault(kernel_class(r["Kernel_Name"]), {}).setdefault(c, []).append(float(r["Counter_Value"]))
    traffic = []
    if per and len(cal) == 2:
        lines += ["", f"Counter calibration: a plain 1 GiB copy reads FETCH_SIZE x {cal['FETCH_SIZE']:.3f} and "
                      f"WRITE_SIZE x {cal['WRITE_SIZE']:.3f} = bytes / 1024.", "",
                  "| kernel | dispatches | FETCH KiB | WRITE KiB | HBM MB (scaled) | algorithmic MB | ratio |",
                  "|---|---|---|---|---|---|---|"]
        for cls, d in per.items():
            if "FETCH_SIZE" not in d or "WRITE_SIZE" not in d or not cls.count("/") == 2:
                continue
            f = sum(d["FETCH_SIZE"]) / len(d["FETCH_SIZE"])
            w = sum(d["WRITE_SIZE"]) / len(d["WRITE_SIZE"])
            hbm = (f * cal["FETCH_SIZE"] + w * cal["WRITE_SIZE"]) * 1024
            name, dt, mt = cls.split("/")
            S = 8 if dt == "f64" else 4
            byt = kernel_bytes(name, A.n, A.nnz, int(mt[1:]), S, summary_mat(A, name, S))
            ratio = f"{hbm / byt:.3f}" if byt else ""
            lines.append(f"| {cls} | {len(d['FETCH_SIZE'])} | {f:.0f} | {w:.0f} | {hbm / 1e6:.1f} | "
                         f"{byt / 1e6 if byt else '':{'.1f' if byt else ''}} | {ratio} |")
            traffic.append((cls, int(hbm)))
    if traffic:
        lines += ["", "Machine-readable lines for bench.py (used only while the kernel sources hash to this value):",
                  ""]
        dig = kernel_sources_digest()
        for cls, b in traffic:
            lines.append(f"traffic: kernel={cls} bytes_per_launch={b} sources_sha256={dig}")
    print("\n".join(lines))
    return 0


def amg_legs(torch, A, Bh, m, t_jacobi, per_iter_ms=(1, 2, 4, 8, 16), steps=1, reorder=False):
    """BiCGStab with the classical AMG preconditioner (the paper's solver,
    Section 4.1) on the same block: host setup time and hierarchy, the solve
    to 1e-10 against the Jacobi solve's time, its top kernels, and the time
    per iteration at a fixed count for several m with m t_1 / t_m (the
    quantity of Tables 2-3)."""
    import numpy as np
    import paper_1711_10622_amd as mrhs
    from paper_1711_10622_amd import estimates as est
    M = mrhs.CsrMatrix.from_csr(A, reorder=reorder)
    t0 = time.perf_counter()
    H = mrhs.AmgHierarchy(M)
    setup = time.perf_counter() - t0
    out = {"setup_s": round(setup, 2), "levels": H.levels, "operator_complexity": round(H.operator_complexity, 3),
           "device_GB": round(H.device_bytes / 1e9, 3), "rows_per_level": [H.level(l)[0] for l in range(H.levels)]}
    B = torch.from_numpy(np.ascontiguousarray(Bh[:, :m])).to("cuda")
    X = torch.empty_like(B)
    ws = torch.empty(H.workspace_size(m), dtype=torch.uint8, device="cuda")
    H.solve(B, out=X, workspace=ws)
    torch.cuda.synchronize()
    mrhs.trace_enable(True, every=TRACE_EVERY)
    t0 = time.perf_counter()
    for _ in range(steps):
        _, infos, st = H.solve(B, out=X, workspace=ws)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    tr = mrhs.trace_read()
    mrhs.trace_enable(False)
    assert st == 0, infos
    out.update({"m": m, "s_per_rhs": round(t / m, 6), "speedup_vs_jacobi": round(t_jacobi / t, 3),
                "iters": [i["iters"] for i in infos], "max_relres": max(i["relres"] for i in infos),
                "top_kernels": {k: {"launches": v["seen"], "avg_us": round(v["total_ms"] / v["launches"] * 1e3, 1)}
                                for k, v in sorted(tr.items(), key=lambda kv: -kv[1]["total_ms"] / kv[1]["launches"]
                                                   * kv[1]["seen"])[:8]}})
    # the V-cycle in binary32 (the iteration, its products and x in binary64)
    H.solve(B, out=X, workspace=ws, mixed=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _, infos32, st32 = H.solve(B, out=X, workspace=ws, mixed=True)
    torch.cuda.synchronize()
    t32 = (time.perf_counter() - t0) / steps
    assert st32 == 0, infos32
    out["vcycle_f32"] = {"s_per_rhs": round(t32 / m, 6), "speedup_vs_f64_vcycle": round(t / t32, 3),
                         "speedup_vs_jacobi": round(t_jacobi / t32, 3), "iters": [i["iters"] for i in infos32],
                         "max_relres": max(i["relres"] for i in infos32)}
    del X, B, ws
    per = {}
    for mm in per_iter_ms:
        Bm = torch.from_numpy(np.ascontiguousarray(Bh[:, :mm])).to("cuda")
        Xm = torch.empty_like(Bm)
        wsm = torch.empty(H.workspace_size(mm), dtype=torch.uint8, device="cuda")
        # 4 and 12 iterations: the preconditioned residual is still far above
        # rounding level there (about 17 iterations reach 1e-10), so no column
        # stops early on a breakdown; the faster of two runs of each
        tt = {}
        for k in (4, 12):
            H.solve(Bm, tol=1e-300, maxit=k, out=Xm, workspace=wsm)
            best = None
            for _ in range(2):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, inf, _ = H.solve(Bm, tol=1e-300, maxit=k, out=Xm, workspace=wsm)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                best = dt if best is None else min(best, dt)
            assert all(i["iters"] == k for i in inf), inf
            tt[k] = best
        per[mm] = {"ms_per_iter": round((tt[12] - tt[4]) / 8 * 1e3, 4)}
        del Bm, Xm, wsm
    if 1 in per:
        for mm, d in per.items():
            d["iter_gain_vs_m1"] = round(mm * per[1]["ms_per_iter"] / d["ms_per_iter"], 3)
            d["paper_compact_5m_2m3"] = round(est.gain_compact(mm), 3)
    out["per_iter"] = per
    H.close()
    M.close()
    torch.cuda.empty_cache()
    return out


def chan128_legs(torch, steps):
    """The 524k-row channel (its matrix, m = 16 block and workspace fit the
    256 MB Infinity Cache): binary64 solve, solves per m with the speedup per
    right-hand side, mixed; returns the legs and its first four solutions."""
    import numpy as np
    import paper_1711_10622_amd as mrhs
    from paper_1711_10622_amd import estimates as est
    from workloads import configs
    wl = configs.WORKLOADS["chan128"]
    A = wl.matrix()
    Bh = wl.rhs(A.n, 16)
    M = mrhs.CsrMatrix.from_csr(A)
    ws = torch.empty(max(M.workspace_size(16, mixed=True), M.workspace_size(16)), dtype=torch.uint8,
                     device="cuda")
    per_m = {}
    Xs = {}
    for mm in (1, 2, 4, 8, 16):
        Bm = torch.from_numpy(np.ascontiguousarray(Bh[:, :mm])).to("cuda")
        Xm = torch.empty_like(Bm)
        timed_solves(torch, M, Bm, Xm, ws, 1)
        t, inf, _ = timed_solves(torch, M, Bm, Xm, ws, steps)
        per_m[mm] = {"s_per_rhs": t / mm, "iters_max": max(i["iters"] for i in inf)}
        if mm == 16:
            Xs["fp64"] = Xm[:, :4].cpu().numpy()
            timed_solves(torch, M, Bm, Xm, ws, 1, mixed=True)
            tm, im, _ = timed_solves(torch, M, Bm, Xm, ws, steps, mixed=True)
            Xs["mixed"] = Xm[:, :4].cpu().numpy()
            mixed = {"s_per_rhs": tm / 16, "speedup_vs_fp64": round(t / tm, 3),
                     "iters_max": max(i["iters"] for i in im), "outer_max": max(i["outer"] for i in im),
                     "max_relres": max(i["relres"] for i in im)}
    amg = amg_legs(torch, A, Bh, 16, per_m[16]["s_per_rhs"] * 16, per_iter_ms=(1, 16), steps=3)
    t1 = per_m[1]["s_per_rhs"]
    for mm, d in per_m.items():
        d["gain_vs_m1"] = round(t1 / d["s_per_rhs"], 3)
        d["paper_compact_5m_2m3"] = round(est.gain_compact(mm), 3)
        d["compulsory_bytes_model"] = round(est.gain_compulsory(A.n, A.nnz, mm), 3)
        d["s_per_rhs"] = round(d["s_per_rhs"], 6)
    M.close()
    del ws
    torch.cuda.empty_cache()
    return {"per_m_fp64": per_m, "mixed_m16": mixed, "amg_m16": amg}, A, Bh, Xs


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--quick", action="store_true", help="only the timed solve (for profiling)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle legs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB copy (counter calibration under rocprofv3)")
    ap.add_argument("--solve-only", metavar="WORKLOAD",
                    help="run only --steps solves of WORKLOAD (after one warm-up), for kernel traces")
    ap.add_argument("--mixed", action="store_true", help="with --solve-only: mixed precision")
    ap.add_argument("--maxit", type=int, default=20000, help="with --solve-only: iteration cap")
    ap.add_argument("--reorder", action="store_true",
                    help="with --solve-only: renumber the matrix by reverse Cuthill-McKee")
    ap.add_argument("--gspmv-only", metavar="MATRIX",
                    help="run only five GSpMV launches per case on MATRIX (counter runs under rocprofv3)")
    ap.add_argument("--summarize", nargs=3, metavar=("OUTDIR", "WORKLOAD", "M"),
                    help="print the markdown summary of rocprofv3 runs under OUTDIR (no GPU needed)")
    args = ap.parse_args()
    if args.summarize:
        return summarize_profiles(args.summarize[0], args.summarize[1], int(args.summarize[2]))
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the design notes describe how the solve would shard).", file=sys.stderr)
        return 2
    if args.copy_calibration:
        return copy_calibration()
    if args.gspmv_only:
        return gspmv_only(args.gspmv_only)
    if args.solve_only:
        return solve_only(args.solve_only, args.mixed, args.steps, args.maxit, args.reorder)

    import numpy as np
    import torch

    import paper_1711_10622_amd as mrhs
    from workloads import configs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    mrhs.load(build_if_missing=True)
    m = 16
    wl = configs.WORKLOADS[HEADLINE]
    A = wl.matrix()
    Bh = wl.rhs(A.n, m)
    M = mrhs.CsrMatrix.from_csr(A)
    B = torch.from_numpy(Bh).to("cuda")
    X = torch.empty_like(B)
    ws = torch.empty(max(M.workspace_size(m, mixed=True), M.workspace_size(m)), dtype=torch.uint8,
                     device="cuda")
    log(f"workload {HEADLINE} n={A.n} nnz={A.nnz} m={m}")

    if args.warmup:
        timed_solves(torch, M, B, X, ws, args.warmup, label="warm-up")
    step_s, infos, trace = timed_solves(torch, M, B, X, ws, args.steps, trace=True, label="timed")
    mats = {8: M.stream_bytes("f64", True), 4: M.stream_bytes("f32", True)}
    log(f"matrix bytes per product: binary64 {mats[8]}, binary32 {mats[4]}")
    dom = dominant_kernel(trace, A.n, A.nnz, mats)
    iters = max(i["iters"] for i in infos)
    log(f"step {step_s * 1e3:.2f} ms, {iters} iterations, dominant {dom['kernel']} {dom['avg_us']:.1f} us")
    extra = {"iters": [i["iters"] for i in infos], "max_relres": max(i["relres"] for i in infos),
             "kernels": {k: {"launches": v["seen"], "timed": v["launches"],
                             "avg_us": round(v["total_ms"] / v["launches"] * 1e3, 2)}
                         for k, v in trace.items()}}
    result = {
        "metric": METRIC, "value": step_s / m, "unit": "s/RHS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": step_s * 1e3, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "chan256: stretched-channel pressure Poisson 256x192x256 (periodic x,z; Neumann y; "
                               "tanh beta=2), m=16 mean-zero U[-1,1) right-hand sides, FP64 block "
                               "Jacobi-BiCGStab to 1e-10, x0=0",
                   "n": A.n, "nnz": A.nnz, "m": m, "tol": 1e-10},
        "roofline": {"bound": "hbm", "achieved": round(dom["achieved"], 1) if dom["achieved"] else None,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(dom["achieved"] / HBM_PEAK_GBS, 4) if dom["achieved"] else None,
                     "traffic": stored_traffic(dom["class"]), "kernel": dom["kernel"],
                     "avg_us": round(dom["avg_us"], 2), "bytes_per_launch": dom["bytes_per_launch"]},
    }

    if not args.quick:
        extra["memory_ceilings"] = memory_ceilings(torch)
        log(f"memory ceilings: {extra['memory_ceilings']}")
        # mixed precision on the same block
        timed_solves(torch, M, B, X, ws, 1, mixed=True)
        Xf = torch.empty_like(B)
        timed_solves(torch, M, B, Xf, ws, 1)
        tmix, imix, trmix = timed_solves(torch, M, B, X, ws, 1, mixed=True, trace=True)
        d = (X - Xf).cpu().numpy()
        xf = Xf.cpu().numpy()
        extra["mixed"] = {"s_per_rhs": tmix / m, "speedup_vs_fp64": round(step_s / tmix, 3),
                          "iters": [i["iters"] for i in imix], "outer": [i["outer"] for i in imix],
                          "max_relres": max(i["relres"] for i in imix),
                          "rel_diff_vs_fp64_solution": [float(np.linalg.norm(d[:, l]) / np.linalg.norm(xf[:, l]))
                                                        for l in range(m)],
                          "kernels": {k: {"launches": v["seen"],
                                          "avg_us": round(v["total_ms"] / v["launches"] * 1e3, 2)}
                                      for k, v in trmix.items()}}
        log(f"mixed {tmix * 1e3:.1f} ms ({step_s / tmix:.3f}x)")
        del Xf, d, xf
        del ws, B, X
        torch.cuda.empty_cache()
        extra["per_iter_fp64"] = per_iteration(torch, M, Bh, (1, 2, 4, 7, 8, 15, 16))
        log(f"per iteration: {extra['per_iter_fp64']}")
        extra["per_iter_small"] = small_iterations(torch)
        log(f"per iteration, small matrices: {extra['per_iter_small']}")
        extra["merged_iteration"] = merged_vs_plain(torch)
        log(f"merged iteration: {extra['merged_iteration']}")
        M.close()
        extra["amg"] = amg_legs(torch, A, Bh, m, step_s)
        log(f"amg: {extra['amg']}")
        extra["gspmv_chan256"] = gspmv_sweep(torch, A, list(range(1, 17)), ("f64", "f32"), reps=20)
        extra["gspmv_chan256_plain_arrays"] = gspmv_sweep(torch, A, [1, 8, 16], ("f64", "f32"), reps=20, plain=True)
        extra["gspmv_chan256_local_gathers"] = gspmv_locality(torch, A)
        extra["gspmv_chan256_plane_march"] = gspmv_march(torch, A)
        extra["gspmv_cube192"] = gspmv_cube(torch)
        log("gspmv sweeps done")
        legs, A2, Bh2, Xs2 = chan128_legs(torch, 2)
        extra["chan128"] = legs
        log(f"chan128: {legs}")
        extra["cube192_m8"] = solve_pair(torch, "cube192", 8, 1)
        extra["cube192_m8_rcm"] = solve_pair(torch, "cube192", 8, 1, reorder=True, amg_per_iter=(8,))
        extra["projection_chan128"] = projection_step(torch)
        srv_legs = {"offered_5ms_gaps": serving(torch, n_req=300)}
        for amg in (False, True):
            tag = "amg" if amg else "mixed"
            # mixed: binary32 inner Jacobi solves; amg: the V-cycle in binary32
            # 600 requests: the AMG server's capacity run then lasts several
            # seconds (150 lasted under two and varied by 25 % between runs)
            cap = serving(torch, n_req=600, seed=1716, amg=amg, closed=True)
            srv_legs[f"{tag}_capacity"] = cap
            # 2000 requests, so the p99 latency rests on 20 of them
            srv_legs[f"{tag}_at_0.8x_capacity"] = serving(torch, n_req=2000, amg=amg,
                                                          rate=0.8 * cap["server_rhs_per_s"])
        extra["serving"] = srv_legs
        log(f"serving: {extra['serving']}")
        if not args.no_cpu:
            extra["chan128"]["error_vs_oracle_first4"] = oracle_error(A2, Bh2, Xs2, 4, 4)
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(A, Bh, iters, min(host_cores(), m))
        result["cpu_baseline"]["host"] = host_info()
    result["extra"] = extra
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
