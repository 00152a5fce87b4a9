#!/usr/bin/env python3
"""Benchmark of the block multi-RHS pressure-Poisson solve on one MI355X.

Workload (the channel case the metric is quoted on): the finite-volume
pressure operator of a 128 x 64 x 64 channel (periodic x/z, Neumann walls,
tanh beta = 2 wall stretching; n = 524,288, nnz = 3,653,632) with m = 16
mean-zero U[-1,1) right-hand sides (seed 1712), solved by block
Jacobi-BiCGStab in binary64 to a true relative residual of 1e-10 from x0 = 0.
One step = one such block solve (every kernel of the path: products,
fused vector updates, per-column dots, device-side scalar control, true
residual checks, the null-space projection and the final residual).
``value`` = seconds per right-hand side = step time / m, with the matrix,
B and the workspace already resident in HBM.

Also reported (not timed as ``value``): the same solve at m = 1, 2, 4, 8
(speedup per right-hand side next to the paper's traffic estimate), the
mixed FP32-inner/FP64-refinement solve, and the generalized SpMV sweep
m = 1..16 (FP64 and FP32) on the 256 x 192 x 256 channel (12.6M rows,
87.9M nonzeros, far larger than the 256 MB last-level cache) with GB/s and
the fraction of the 8 TB/s HBM peak.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "block-BiCGStab s/RHS to 1e-10 and GSpMV GB/s, m=1..16, FP64 vs FP32+refine"
HBM_PEAK_GBS = 8000.0


def kernel_bytes(name, n, nnz, m, S):
    """Algorithmic HBM bytes of one launch of a library kernel with all m
    columns active: each block (n x m, S bytes/element) read or written once,
    the matrix (int32 row offsets and columns, S-byte values) read once."""
    mat = 4 * (n + 1) + (4 + S) * nnz
    blk = S * m * n
    table = {
        "gspmv": mat + 2 * blk,        # read X, write Y
        "spmv_sigma": mat + 3 * blk,   # read p (gathered), r^; write v
        "spmv_omega": mat + 4 * blk,   # read r, v (gathered), r^; write t
        "xr_update": 9 * blk,          # read y, r, p, v, t, r^; write y, r, p
    }
    return table.get(name)


def dominant_kernel(trace, n, nnz):
    best = None
    for key, st in trace.items():
        name, dt, mtag, _ = key.split("/")
        if best is None or st["total_ms"] > best[1]["total_ms"]:
            best = (key, st, name, 8 if dt == "f64" else 4, int(mtag[1:]))
    key, st, name, S, m = best
    avg_ms = st["total_ms"] / st["launches"]
    byt = kernel_bytes(name, n, nnz, m, S)
    achieved = byt / (avg_ms * 1e-3) / 1e9 if byt else None
    return {
        "kernel": key, "launches": st["launches"], "avg_us": avg_ms * 1e3,
        "bytes_per_launch": byt, "achieved": achieved,
    }


def timed_solves(torch, M, B, X, ws, steps, mixed=False, trace=False):
    import paper_1711_10622_amd as mrhs
    infos = None
    torch.cuda.synchronize()
    if trace:
        mrhs.trace_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        _, infos, st = M.solve(B, tol=1e-10, maxit=20000, mixed=mixed, out=X, workspace=ws)
        if st != 0:
            raise RuntimeError(f"solve did not converge: {infos}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tr = None
    if trace:
        tr = mrhs.trace_read()
        mrhs.trace_enable(False)
    return (t1 - t0) / steps, infos, tr


def gspmv_sweep(torch, A, ms, dtypes):
    import paper_1711_10622_amd as mrhs
    from paper_1711_10622_amd import estimates as est
    M = mrhs.CsrMatrix.from_csr(A)
    out = {}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for dt in dtypes:
        tdt = torch.float64 if dt == "f64" else torch.float32
        S = 8 if dt == "f64" else 4
        for m in ms:
            X = torch.empty((A.n, m), dtype=tdt, device="cuda").uniform_(-1, 1)
            Y = torch.empty_like(X)
            for _ in range(3):
                M.gspmv(X, out=Y)
            reps = 20
            torch.cuda.synchronize()
            e0.record()
            for _ in range(reps):
                M.gspmv(X, out=Y)
            e1.record()
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) / reps * 1e3
            byt = est.traffic_compulsory(A.n, A.nnz, m, V=S, S=S)
            gbs = byt / (us * 1e-6) / 1e9
            out[f"{dt}/m{m}"] = {"us": round(us, 2), "GBps": round(gbs, 1),
                                 "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4)}
            del X, Y
    M.close()
    return out


def cpu_baseline(A, B, ncols):
    import oracle
    Bs = B[:, :ncols].copy()
    t0 = time.perf_counter()
    X, infos, _ = oracle.bicgstab(A, Bs, tol=1e-10, maxit=20000, threads=ncols)
    wall = time.perf_counter() - t0
    assert all(i["status"] == 0 for i in infos), infos
    return {"value": wall / ncols, "unit": "s/RHS", "cores": ncols, "kind": "oracle",
            "sample": f"{ncols} of the {B.shape[1]} right-hand sides of the same workload, "
                      f"one host thread per column, FP64 to 1e-10 (wall {wall:.2f} s)",
            "iters": [i["iters"] for i in infos]}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--m", type=int, default=16)
    ap.add_argument("--quick", action="store_true", help="only the timed solve (for profiling)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the design notes describe how the solve would shard).", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1711_10622_amd as mrhs
    from paper_1711_10622_amd import estimates as est
    from workloads import configs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    mrhs.load(build_if_missing=True)
    wl = configs.WORKLOADS["chan128"]
    A = wl.matrix()
    m = args.m
    Bh = wl.rhs(A.n, 16)
    M = mrhs.CsrMatrix.from_csr(A)
    B = torch.from_numpy(np.ascontiguousarray(Bh[:, :m])).to("cuda")
    X = torch.empty_like(B)
    ws = torch.empty(M.workspace_size(m, mixed=True) + M.workspace_size(m), dtype=torch.uint8, device="cuda")
    print(f"# workload chan128 n={A.n} nnz={A.nnz} m={m}", file=sys.stderr, flush=True)

    if args.warmup:
        timed_solves(torch, M, B, X, ws, args.warmup)
    step_s, infos, trace = timed_solves(torch, M, B, X, ws, args.steps, trace=True)
    dom = dominant_kernel(trace, A.n, A.nnz)
    print(f"# step {step_s * 1e3:.2f} ms, dominant {dom['kernel']} {dom['avg_us']:.1f} us", file=sys.stderr,
          flush=True)
    relres = max(i["relres"] for i in infos)
    extra = {"iters": [i["iters"] for i in infos], "max_relres": relres,
             "kernels": {k: {"launches": v["launches"], "avg_us": round(v["total_ms"] / v["launches"] * 1e3, 2)}
                         for k, v in trace.items()}}
    result = {
        "metric": METRIC, "value": step_s / m, "unit": "s/RHS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": step_s * 1e3, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "chan128: stretched-channel pressure Poisson 128x64x64 (periodic x,z; Neumann y; "
                               "tanh beta=2), FP64 block Jacobi-BiCGStab to 1e-10, x0=0",
                   "n": A.n, "nnz": A.nnz, "m": m, "tol": 1e-10},
        "roofline": {"bound": "hbm", "achieved": round(dom["achieved"], 1) if dom["achieved"] else None,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(dom["achieved"] / HBM_PEAK_GBS, 4) if dom["achieved"] else None,
                     "traffic": None, "kernel": dom["kernel"], "avg_us": round(dom["avg_us"], 2),
                     "bytes_per_launch": dom["bytes_per_launch"]},
    }

    if not args.quick:
        # per-m solve times: speedup per right-hand side vs m = 1
        per_m = {}
        for mm in (1, 2, 4, 8, 16):
            if mm == m:
                t, inf = step_s, infos
            else:
                Bm = torch.from_numpy(np.ascontiguousarray(Bh[:, :mm])).to("cuda")
                Xm = torch.empty_like(Bm)
                timed_solves(torch, M, Bm, Xm, ws, 1)
                t, inf, _ = timed_solves(torch, M, Bm, Xm, ws, 2)
            per_m[mm] = {"s_per_rhs": t / mm, "iters_max": max(i["iters"] for i in inf)}
        t1 = per_m[1]["s_per_rhs"]
        for mm, d in per_m.items():
            d["gain_vs_m1"] = round(t1 / d["s_per_rhs"], 3)
            d["paper_estimate_5m_2m3"] = round(est.gain_compact(mm), 3)
            d["s_per_rhs"] = round(d["s_per_rhs"], 6)
        extra["per_m_fp64"] = per_m
        # mixed precision at the benchmark m
        timed_solves(torch, M, B, X, ws, 1, mixed=True)
        tmix, imix, _ = timed_solves(torch, M, B, X, ws, args.steps, mixed=True)
        extra["mixed"] = {"s_per_rhs": tmix / m, "speedup_vs_fp64": round(step_s / tmix, 3),
                          "iters": [i["iters"] for i in imix], "outer": [i["outer"] for i in imix],
                          "max_relres": max(i["relres"] for i in imix)}
        del M, ws, B, X
        torch.cuda.empty_cache()
        # generalized SpMV sweep on the large channel
        L = configs.MATRICES["chan256"]()
        extra["gspmv_chan256"] = gspmv_sweep(torch, L, list(range(1, 17)), ("f64", "f32"))
        del L
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(A, Bh, 4)
    result["extra"] = extra
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
