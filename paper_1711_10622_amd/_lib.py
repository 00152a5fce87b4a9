"""ctypes declarations of libmrhs.so (see include/mrhs.h for the contract).

Loading fails loudly when the library is missing or cannot be loaded: there
is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmrhs.so")

OK, EAGAIN, EINVAL, ENOMEM, EDEVICE, ENOCONV, EBREAKDOWN, EBUDGET, ESHUTDOWN, ENOTFOUND = (
    0, 1, -1, -2, -3, -4, -5, -6, -7, -8)
STATUS_NAMES = {0: "OK", 1: "EAGAIN", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ENOCONV",
                -5: "EBREAKDOWN", -6: "EBUDGET", -7: "ESHUTDOWN", -8: "ENOTFOUND"}
F64, F32 = 0, 1
CSR_NULLSPACE_CONST, CSR_REORDER = 1, 2
X0_GIVEN, MIXED = 1, 2
SERVER_MIXED = 1
SERVER_AMG = 2
SHADOW_SEED = 17110622  # MRHS_SHADOW_SEED: seed of the BiCGStab shadow residual
NOALLOC_SCRATCH_BYTES = 64 << 20  # MRHS_NOALLOC_SCRATCH_BYTES

# every symbol include/mrhs.h declares
EXPORTS = (
    "mrhs_last_error", "mrhs_version", "csr_create", "csr_destroy", "csr_info", "csr_stream_bytes",
    "csr_reorder_permutation",
    "gspmv", "gspmv_ex",
    "block_bicgstab", "block_bicgstab_ex", "block_bicgstab_workspace_size", "block_bicgstab_noalloc",
    "solve_server_create", "solve_server_register", "solve_server_submit", "solve_server_poll",
    "solve_server_stats", "solve_server_destroy",
    "grid_create", "grid_destroy", "grid_info", "projection_rhs", "projection_correct",
    "mrhs_trace_enable", "mrhs_trace_read", "mrhs_stream_probe",
    "amg_create", "amg_destroy", "amg_info", "amg_level", "amg_level_copy", "amg_vcycle_workspace_size",
    "amg_vcycle", "block_bicgstab_amg_workspace_size", "block_bicgstab_amg",
)
AMG_OPERATOR, AMG_PROLONGATION, AMG_SPLIT = 0, 1, 2
PROBE_KINDS = {"read": 0, "read_nt": 1, "write": 2, "write_nt": 3, "copy": 4, "copy_nt": 5}


class ColInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("restarts", ctypes.c_int32), ("outer", ctypes.c_int32),
                ("status", ctypes.c_int32), ("relres", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerStats(ctypes.Structure):
    _fields_ = [("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("rhs_per_s", ctypes.c_double),
                ("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("queued", ctypes.c_int64),
                ("rhs_completed", ctypes.c_int64), ("admitted_bytes", ctypes.c_size_t)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class MrhsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lock = threading.Lock()
_lib = None


def _declare(lib):
    c = ctypes
    vp, i32, i64, u32, f64, sz = c.c_void_p, c.c_int32, c.c_int64, c.c_uint32, c.c_double, c.c_size_t
    lib.mrhs_last_error.restype = c.c_char_p
    lib.mrhs_last_error.argtypes = []
    lib.mrhs_version.restype = c.c_char_p
    lib.mrhs_version.argtypes = []
    sigs = {
        "csr_create": [i32, i64, vp, vp, vp, u32, c.POINTER(vp)],
        "csr_destroy": [vp],
        "csr_info": [vp, c.POINTER(i32), c.POINTER(i64), c.POINTER(sz)],
        "csr_stream_bytes": [vp, i32, i32, c.POINTER(i64)],
        "csr_reorder_permutation": [i32, vp, vp, vp],
        "gspmv": [vp, vp, vp, i32],
        "gspmv_ex": [vp, i32, vp, vp, i32, vp],
        "block_bicgstab": [vp, vp, vp, i32, f64, i32],
        "block_bicgstab_ex": [vp, vp, vp, i32, f64, i32, u32, vp, sz, vp, c.POINTER(ColInfo)],
        "block_bicgstab_workspace_size": [vp, i32, u32, c.POINTER(sz)],
        "block_bicgstab_noalloc": [vp, vp, vp, i32, f64, i32, u32, vp, c.POINTER(ColInfo)],
        "solve_server_create": [sz, u32, c.POINTER(vp)],
        "solve_server_register": [vp, vp, c.POINTER(i32)],
        "solve_server_submit": [vp, i32, vp, i32, f64, i32, c.POINTER(c.c_uint64)],
        "solve_server_poll": [vp, c.c_uint64, vp, c.POINTER(ColInfo)],
        "solve_server_stats": [vp, c.POINTER(ServerStats)],
        "solve_server_destroy": [vp],
        "grid_create": [i32, i32, i32, f64, f64, vp, vp, c.POINTER(vp)],
        "grid_destroy": [vp],
        "grid_info": [vp, c.POINTER(i32), c.POINTER(i64), c.POINTER(i64)],
        "projection_rhs": [vp, vp, vp, vp, f64, vp, i32, vp],
        "projection_correct": [vp, vp, vp, vp, vp, f64, i32, vp],
        "mrhs_trace_enable": [c.c_int],
        "mrhs_trace_read": [c.c_char_p, sz, c.POINTER(sz)],
        "mrhs_stream_probe": [i32, vp, vp, sz, vp],
        "amg_create": [vp, f64, i32, i32, c.POINTER(vp)],
        "amg_destroy": [vp],
        "amg_info": [vp, c.POINTER(i32), c.POINTER(f64), c.POINTER(sz)],
        "amg_level": [vp, i32, c.POINTER(i32), c.POINTER(i64), c.POINTER(i64)],
        "amg_level_copy": [vp, i32, i32, vp, vp, vp],
        "amg_vcycle_workspace_size": [vp, i32, c.POINTER(sz)],
        "amg_vcycle": [vp, vp, vp, i32, vp, sz, vp],
        "block_bicgstab_amg_workspace_size": [vp, i32, c.POINTER(sz)],
        "block_bicgstab_amg": [vp, vp, vp, i32, f64, i32, u32, vp, sz, vp, c.POINTER(ColInfo)],
    }
    for name, args in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = c.c_int


def load(build_if_missing: bool = True):
    """Load libmrhs.so (building it once if it has never been built)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            if not build_if_missing:
                raise RuntimeError(f"{LIB_PATH} is not built")
            from . import build as _build
            _build.build()
        lib = ctypes.CDLL(LIB_PATH)
        _declare(lib)
        _lib = lib
        return lib


def check(status: int, what: str = ""):
    if status != OK:
        msg = load().mrhs_last_error().decode(errors="replace")
        raise MrhsError(status, f"{what}: {msg}" if what else msg)
    return status
