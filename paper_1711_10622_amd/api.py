"""Python binding of libmrhs: argument marshalling only.

Device memory and streams come from PyTorch (``torch.cuda``); every step of
the computation runs in the library's HIP kernels.  Names follow the C ABI
(include/mrhs.h): ``csr_create`` -> :class:`CsrMatrix`, ``gspmv``,
``block_bicgstab``.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib


def _torch():
    import torch
    return torch


def _stream_handle(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _check_block(t, n, m, dtype, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.dim() == 1:
        t = t.view(-1, 1)
    if tuple(t.shape) != (n, m) or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous ({n}, {m}) block, got {tuple(t.shape)}")
    return t


class CsrMatrix:
    """A CRS matrix resident on the current GPU (``csr_create``)."""

    def __init__(self, n, row_ptr, col_idx, val, nullspace_const=False, reorder=False):
        lib = _lib.load()
        self._lib = lib
        self.n = int(n)
        rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
        ci = np.ascontiguousarray(col_idx, dtype=np.int32)
        va = np.ascontiguousarray(val, dtype=np.float64)
        self.nnz = int(ci.shape[0])
        self.nullspace_const = bool(nullspace_const)
        h = ctypes.c_void_p()
        flags = (_lib.CSR_NULLSPACE_CONST if nullspace_const else 0) | (_lib.CSR_REORDER if reorder else 0)
        self.reorder = bool(reorder)
        _lib.check(lib.csr_create(self.n, self.nnz, rp.ctypes.data if rp.size else None,
                                  ci.ctypes.data if ci.size else None,
                                  va.ctypes.data if va.size else None, flags, ctypes.byref(h)),
                   "csr_create")
        self._h = h

    @classmethod
    def from_csr(cls, A, nullspace_const=None, reorder=False):
        """From any object with ``n, row_ptr, col, val`` (e.g. the workload generators)."""
        if nullspace_const is None:
            nullspace_const = bool(getattr(A, "nullspace_const", False))
        return cls(A.n, A.row_ptr, A.col, A.val, nullspace_const, reorder)

    @property
    def handle(self):
        return self._h

    def device_bytes(self) -> int:
        n, nnz, b = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_size_t()
        _lib.check(self._lib.csr_info(self._h, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(b)))
        return int(b.value)

    def stream_bytes(self, dtype="f64", scaled=False) -> int:
        """Bytes one product streams from the matrix arrays (row offsets plus
        2 bytes per entry in the dictionary form, else index and value)."""
        b = ctypes.c_int64()
        dt = _lib.F64 if dtype == "f64" else _lib.F32
        _lib.check(self._lib.csr_stream_bytes(self._h, dt, 1 if scaled else 0, ctypes.byref(b)))
        return int(b.value)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.csr_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- products -------------------------------------------------------------
    def gspmv(self, X, out=None, stream=None):
        """Y = A X for an (n, m) block (float64 or float32), m in 1..16."""
        torch = _torch()
        squeeze = X.dim() == 1
        m = 1 if squeeze else int(X.shape[1])
        if X.dtype not in (torch.float64, torch.float32):
            raise TypeError("X must be float64 or float32")
        Xb = _check_block(X, self.n, m, X.dtype, "X")
        if out is None:
            out = torch.empty_like(Xb)
        Yb = _check_block(out, self.n, m, X.dtype, "out")
        dtype = _lib.F64 if X.dtype == torch.float64 else _lib.F32
        _lib.check(self._lib.gspmv_ex(self._h, dtype, ctypes.c_void_p(Xb.data_ptr()),
                                      ctypes.c_void_p(Yb.data_ptr()), m, _stream_handle(stream)),
                   "gspmv")
        return out.view(-1) if squeeze else out

    # -- solves ---------------------------------------------------------------
    def workspace_size(self, m, mixed=False) -> int:
        b = ctypes.c_size_t()
        _lib.check(self._lib.block_bicgstab_workspace_size(self._h, int(m), _lib.MIXED if mixed else 0,
                                                           ctypes.byref(b)))
        return int(b.value)

    def solve(self, B, tol=1e-10, maxit=20000, mixed=False, X0=None, out=None, workspace=None,
              stream=None):
        """Solve A X = B (``block_bicgstab_ex``).

        Returns ``(X, infos, status)``: the float64 (n, m) solution, a list
        of per-column dicts (iters, restarts, outer, status, relres) and the
        overall status (OK only if every column converged).  Argument errors
        and device failures raise :class:`MrhsError`.
        """
        torch = _torch()
        squeeze = B.dim() == 1
        m = 1 if squeeze else int(B.shape[1])
        Bb = _check_block(B, self.n, m, torch.float64, "B")
        flags = _lib.MIXED if mixed else 0
        if X0 is not None:
            X0b = _check_block(X0, self.n, m, torch.float64, "X0")
            if out is None:
                out = X0b.clone()
            else:
                out.copy_(X0b)
            flags |= _lib.X0_GIVEN
        elif out is None:
            out = torch.empty_like(Bb)
        Xb = _check_block(out, self.n, m, torch.float64, "out")
        need = self.workspace_size(m, mixed)
        if workspace is None:
            workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=Bb.device)
        elif workspace.numel() * workspace.element_size() < need:
            raise ValueError(f"workspace needs {need} bytes")
        infos = (_lib.ColInfo * m)()
        st = self._lib.block_bicgstab_ex(self._h, ctypes.c_void_p(Bb.data_ptr()),
                                         ctypes.c_void_p(Xb.data_ptr()), m, float(tol), int(maxit), flags,
                                         ctypes.c_void_p(workspace.data_ptr()), need,
                                         _stream_handle(stream), infos)
        if st not in (_lib.OK, _lib.ENOCONV, _lib.EBREAKDOWN):
            _lib.check(st, "block_bicgstab")
        return (out.view(-1) if squeeze else out), [i.as_dict() for i in infos], st


class AmgHierarchy:
    """Classical AMG hierarchy of a resident matrix (``amg_create``)."""

    def __init__(self, M: CsrMatrix, theta=0.0, max_coarse=0, max_levels=0):
        lib = _lib.load()
        self._lib = lib
        self.M = M
        h = ctypes.c_void_p()
        _lib.check(lib.amg_create(M.handle, float(theta), int(max_coarse), int(max_levels), ctypes.byref(h)),
                   "amg_create")
        self._h = h
        lv, oc, by = ctypes.c_int32(), ctypes.c_double(), ctypes.c_size_t()
        _lib.check(lib.amg_info(h, ctypes.byref(lv), ctypes.byref(oc), ctypes.byref(by)), "amg_info")
        self.levels, self.operator_complexity, self.device_bytes = int(lv.value), float(oc.value), int(by.value)

    @property
    def handle(self):
        return self._h

    def level(self, l):
        """(rows, nonzeros of A_l, nonzeros of P_l)."""
        n, na, npz = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
        _lib.check(self._lib.amg_level(self._h, int(l), ctypes.byref(n), ctypes.byref(na), ctypes.byref(npz)),
                   "amg_level")
        return int(n.value), int(na.value), int(npz.value)

    def level_arrays(self, l, what="A"):
        """Host copies of level l: ``"A"`` or ``"P"`` -> (row_ptr, col, val); ``"cf"`` -> C/F marks."""
        n, na, npz = self.level(l)
        if what == "cf":
            cf = np.empty(n, dtype=np.int32)
            _lib.check(self._lib.amg_level_copy(self._h, int(l), _lib.AMG_SPLIT, None, cf.ctypes.data, None),
                       "amg_level_copy")
            return cf
        nz = na if what == "A" else npz
        rp = np.empty(n + 1, dtype=np.int32)
        ci = np.empty(max(nz, 1), dtype=np.int32)
        va = np.empty(max(nz, 1), dtype=np.float64)
        kind = _lib.AMG_OPERATOR if what == "A" else _lib.AMG_PROLONGATION
        _lib.check(self._lib.amg_level_copy(self._h, int(l), kind, rp.ctypes.data, ci.ctypes.data, va.ctypes.data),
                   "amg_level_copy")
        return rp, ci[:nz], va[:nz]

    def vcycle(self, B, out=None, workspace=None, stream=None):
        """X = M^-1 B (one V-cycle) for an (n, m) float64 block."""
        torch = _torch()
        m = 1 if B.dim() == 1 else int(B.shape[1])
        Bb = _check_block(B, self.M.n, m, torch.float64, "B")
        if out is None:
            out = torch.empty_like(Bb)
        Xb = _check_block(out, self.M.n, m, torch.float64, "out")
        need = ctypes.c_size_t()
        _lib.check(self._lib.amg_vcycle_workspace_size(self._h, m, ctypes.byref(need)))
        if workspace is None:
            workspace = torch.empty(max(need.value, 1), dtype=torch.uint8, device=Bb.device)
        _lib.check(self._lib.amg_vcycle(self._h, ctypes.c_void_p(Bb.data_ptr()), ctypes.c_void_p(Xb.data_ptr()), m,
                                        ctypes.c_void_p(workspace.data_ptr()), need.value, _stream_handle(stream)),
                   "amg_vcycle")
        return out

    def workspace_size(self, m) -> int:
        b = ctypes.c_size_t()
        _lib.check(self._lib.block_bicgstab_amg_workspace_size(self._h, int(m), ctypes.byref(b)))
        return int(b.value)

    def solve(self, B, tol=1e-10, maxit=1000, X0=None, out=None, workspace=None, stream=None, mixed=False):
        """AMG-preconditioned block BiCGStab (``block_bicgstab_amg``); returns
        ``(X, infos, status)`` like :meth:`CsrMatrix.solve`.  ``mixed``: the
        V-cycle in binary32."""
        torch = _torch()
        m = 1 if B.dim() == 1 else int(B.shape[1])
        Bb = _check_block(B, self.M.n, m, torch.float64, "B")
        flags = _lib.MIXED if mixed else 0
        if X0 is not None:
            X0b = _check_block(X0, self.M.n, m, torch.float64, "X0")
            out = X0b.clone() if out is None else out.copy_(X0b)
            flags |= _lib.X0_GIVEN
        elif out is None:
            out = torch.empty_like(Bb)
        Xb = _check_block(out, self.M.n, m, torch.float64, "out")
        need = self.workspace_size(m)
        if workspace is None:
            workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=Bb.device)
        elif workspace.numel() * workspace.element_size() < need:
            raise ValueError(f"workspace needs {need} bytes")
        infos = (_lib.ColInfo * m)()
        st = self._lib.block_bicgstab_amg(self._h, ctypes.c_void_p(Bb.data_ptr()), ctypes.c_void_p(Xb.data_ptr()), m,
                                          float(tol), int(maxit), flags, ctypes.c_void_p(workspace.data_ptr()),
                                          need, _stream_handle(stream), infos)
        if st not in (_lib.OK, _lib.ENOCONV, _lib.EBREAKDOWN):
            _lib.check(st, "block_bicgstab_amg")
        return out, [i.as_dict() for i in infos], st

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.amg_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def reorder_permutation(A):
    """perm[new] = old of the renumbering MRHS_CSR_REORDER applies
    (``csr_reorder_permutation``, host only) for an object with ``n, row_ptr, col``."""
    rp = np.ascontiguousarray(A.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(A.col, dtype=np.int32)
    perm = np.empty(int(A.n), dtype=np.int32)
    _lib.check(_lib.load().csr_reorder_permutation(int(A.n), rp.ctypes.data, ci.ctypes.data if ci.size else None,
                                                   perm.ctypes.data), "csr_reorder_permutation")
    return perm


def gspmv(A: CsrMatrix, X, out=None, stream=None):
    return A.gspmv(X, out=out, stream=stream)


def block_bicgstab(A: CsrMatrix, B, tol=1e-10, maxit=20000, mixed=False, **kw):
    return A.solve(B, tol=tol, maxit=maxit, mixed=mixed, **kw)


def stream_probe(kind: str, src, dst, nbytes: int, stream=None):
    """One streaming pass (``mrhs_stream_probe``) over ``nbytes`` of device
    tensors ``src``/``dst`` (``kind`` in read, read_nt, write, write_nt, copy,
    copy_nt); enqueued on ``stream`` (torch's current stream by default)."""
    lib = _lib.load()
    sp = ctypes.c_void_p(src.data_ptr()) if src is not None else None
    _lib.check(lib.mrhs_stream_probe(_lib.PROBE_KINDS[kind], sp, ctypes.c_void_p(dst.data_ptr()), int(nbytes),
                                     _stream_handle(stream)), "mrhs_stream_probe")


def trace_enable(on=True, every: int = 1):
    """Start (clearing old statistics) or stop kernel timing; when on, every
    ``every``-th launch of each kernel class is timed with HIP events."""
    _lib.check(_lib.load().mrhs_trace_enable(int(every) if on else 0), "mrhs_trace_enable")


def trace_read() -> dict:
    """Per-kernel-class launch counts and durations recorded since trace_enable."""
    import json
    lib = _lib.load()
    need = ctypes.c_size_t()
    _lib.check(lib.mrhs_trace_read(None, 0, ctypes.byref(need)), "mrhs_trace_read")
    buf = ctypes.create_string_buffer(need.value + 1)
    _lib.check(lib.mrhs_trace_read(buf, need.value + 1, ctypes.byref(need)), "mrhs_trace_read")
    return json.loads(buf.value.decode())


class SolveServer:
    """Continuous-batching solve server (``solve_server_*``): host-memory
    right-hand sides in, host-memory solutions out."""

    def __init__(self, hbm_budget_bytes, mixed=False, amg=False):
        lib = _lib.load()
        self._lib = lib
        h = ctypes.c_void_p()
        flags = (_lib.SERVER_MIXED if mixed else 0) | (_lib.SERVER_AMG if amg else 0)
        _lib.check(lib.solve_server_create(int(hbm_budget_bytes), flags, ctypes.byref(h)), "solve_server_create")
        self._h = h
        self._n = {}
        self._k = {}

    def register(self, A: CsrMatrix) -> int:
        mid = ctypes.c_int32()
        _lib.check(self._lib.solve_server_register(self._h, A.handle, ctypes.byref(mid)), "solve_server_register")
        self._n[mid.value] = A.n
        return mid.value

    def submit(self, matrix_id, B, tol=1e-10, maxit=20000) -> int:
        B = np.ascontiguousarray(B, dtype=np.float64)
        if B.ndim == 1:
            B = B[:, None]
        n, k = B.shape
        if n != self._n.get(matrix_id, n):
            raise ValueError(f"B has {n} rows, matrix {matrix_id} has {self._n[matrix_id]}")
        t = ctypes.c_uint64()
        _lib.check(self._lib.solve_server_submit(self._h, int(matrix_id), B.ctypes.data, k, float(tol), int(maxit),
                                                 ctypes.byref(t)), "solve_server_submit")
        self._k[t.value] = (n, k)
        return t.value

    def poll(self, ticket):
        """None while running, else ``(X, infos, status)``."""
        n, k = self._k[ticket]
        X = np.empty((n, k), dtype=np.float64)
        infos = (_lib.ColInfo * k)()
        st = self._lib.solve_server_poll(self._h, ctypes.c_uint64(ticket), X.ctypes.data, infos)
        if st == _lib.EAGAIN:
            return None
        if st not in (_lib.OK, _lib.ENOCONV, _lib.EBREAKDOWN, _lib.EDEVICE, _lib.ENOMEM):
            _lib.check(st, "solve_server_poll")
        del self._k[ticket]
        return X, [i.as_dict() for i in infos], st

    def wait(self, ticket, timeout=600.0, interval=1e-3):
        import time
        t0 = time.monotonic()
        while True:
            r = self.poll(ticket)
            if r is not None:
                return r
            if time.monotonic() - t0 > timeout:
                raise TimeoutError(f"ticket {ticket} not done after {timeout} s")
            time.sleep(interval)

    def stats(self) -> dict:
        s = _lib.ServerStats()
        _lib.check(self._lib.solve_server_stats(self._h, ctypes.byref(s)), "solve_server_stats")
        return s.as_dict()

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.solve_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ChannelGrid:
    """Staggered channel grid of the ensemble projection step (``grid_create``):
    ``rhs`` gives the m pressure right-hand sides -(1/tau) D u*, ``correct``
    applies u -= tau G p to the m fields in place."""

    def __init__(self, nx, ny, nz, dx, dz, y_faces, solid=None):
        lib = _lib.load()
        self._lib = lib
        yf = np.ascontiguousarray(y_faces, dtype=np.float64)
        if yf.shape != (ny + 1,):
            raise ValueError(f"y_faces must hold ny + 1 = {ny + 1} coordinates")
        sd = None
        if solid is not None:
            sd = np.ascontiguousarray(solid, dtype=np.uint8)
            if sd.size != nx * ny * nz:
                raise ValueError("solid must hold nx*ny*nz cells")
        h = ctypes.c_void_p()
        _lib.check(lib.grid_create(int(nx), int(ny), int(nz), float(dx), float(dz), yf.ctypes.data,
                                   sd.ctypes.data if sd is not None else None, ctypes.byref(h)), "grid_create")
        self._h = h
        n, cells, vf = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
        _lib.check(lib.grid_info(h, ctypes.byref(n), ctypes.byref(cells), ctypes.byref(vf)), "grid_info")
        self.n, self.cells, self.v_faces = n.value, cells.value, vf.value
        self.shape = (int(nx), int(ny), int(nz))

    def _faces(self, U, V, W):
        torch = _torch()
        m = 1 if U.dim() == 1 else int(U.shape[1])
        return (m, _check_block(U, self.cells, m, torch.float64, "U"),
                _check_block(V, self.v_faces, m, torch.float64, "V"),
                _check_block(W, self.cells, m, torch.float64, "W"))

    def rhs(self, U, V, W, tau, out=None, stream=None):
        """-(1/tau) D(U, V, W) as an (n_fluid, m) block (``projection_rhs``)."""
        torch = _torch()
        m, U, V, W = self._faces(U, V, W)
        if out is None:
            out = torch.empty((self.n, m), dtype=torch.float64, device=U.device)
        B = _check_block(out, self.n, m, torch.float64, "out")
        _lib.check(self._lib.projection_rhs(self._h, ctypes.c_void_p(U.data_ptr()), ctypes.c_void_p(V.data_ptr()),
                                            ctypes.c_void_p(W.data_ptr()), float(tau),
                                            ctypes.c_void_p(B.data_ptr()), m, _stream_handle(stream)),
                   "projection_rhs")
        return out

    def correct(self, U, V, W, P, tau, stream=None):
        """U, V, W -= tau G P in place (``projection_correct``)."""
        torch = _torch()
        m, U, V, W = self._faces(U, V, W)
        Pb = _check_block(P, self.n, m, torch.float64, "P")
        _lib.check(self._lib.projection_correct(self._h, ctypes.c_void_p(U.data_ptr()),
                                                ctypes.c_void_p(V.data_ptr()), ctypes.c_void_p(W.data_ptr()),
                                                ctypes.c_void_p(Pb.data_ptr()), float(tau), m,
                                                _stream_handle(stream)),
                   "projection_correct")

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.grid_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
