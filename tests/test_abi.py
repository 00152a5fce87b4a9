"""The C ABI surface, without a GPU: the library loads, exports every function
include/mrhs.h declares, and rejects invalid matrices before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1711_10622_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", text)
    keywords = {"if", "while", "for", "sizeof", "return"}
    return sorted(set(n for n in names if n not in keywords))


def test_library_exports_every_declared_symbol():
    lib = _lib.load(build_if_missing=True)
    decl = declared_functions()
    assert set(decl) == set(_lib.EXPORTS), (decl, _lib.EXPORTS)
    for name in decl:
        assert hasattr(lib, name), name
    assert lib.mrhs_version().startswith(b"mrhs")


def _create(n, rp, ci, va, flags=0):
    lib = _lib.load()
    h = ctypes.c_void_p()
    rp = np.asarray(rp, dtype=np.int32)
    ci = np.asarray(ci, dtype=np.int32)
    va = np.asarray(va, dtype=np.float64)
    st = lib.csr_create(n, len(ci), rp.ctypes.data if rp.size else None, ci.ctypes.data if ci.size else None,
                        va.ctypes.data if va.size else None, flags, ctypes.byref(h))
    return st, lib.mrhs_last_error().decode()


@pytest.mark.parametrize("case", [
    ("rp0", 2, [1, 1, 2], [0, 1], [1.0, 1.0], "row_ptr[0]"),
    ("decrease", 2, [0, 2, 1], [0, 1], [1.0, 1.0], "decreases"),
    ("last", 2, [0, 1, 1], [0, 1], [1.0, 1.0], "differs from nnz"),
    ("col", 2, [0, 1, 2], [0, 2], [1.0, 1.0], "outside"),
    ("negcol", 2, [0, 1, 2], [0, -1], [1.0, 1.0], "outside"),
    ("nan", 2, [0, 1, 2], [0, 1], [1.0, float("nan")], "not finite"),
])
def test_invalid_matrices(case):
    _, n, rp, ci, va, msg = case
    st, err = _create(n, rp, ci, va)
    assert st == _lib.EINVAL and msg in err


def test_invalid_arguments_without_device():
    lib = _lib.load()
    assert lib.csr_create(-1, 0, None, None, None, 0, ctypes.byref(ctypes.c_void_p())) == _lib.EINVAL
    assert lib.csr_create(2, 0, None, None, None, 0, ctypes.byref(ctypes.c_void_p())) == _lib.EINVAL
    assert lib.csr_create(0, 0, None, None, None, 0x80, ctypes.byref(ctypes.c_void_p())) == _lib.EINVAL
    assert lib.gspmv(None, None, None, 4) == _lib.EINVAL
    assert lib.block_bicgstab(None, None, None, 4, 1e-10, 10) == _lib.EINVAL
    b = ctypes.c_size_t()
    assert lib.block_bicgstab_workspace_size(None, 4, 0, ctypes.byref(b)) == _lib.EINVAL
    sb = ctypes.c_int64()
    assert lib.csr_stream_bytes(None, _lib.F64, 0, ctypes.byref(sb)) == _lib.EINVAL
    assert lib.mrhs_trace_enable(-1) == _lib.EINVAL
    assert lib.mrhs_trace_enable(0) == _lib.OK
    h = ctypes.c_void_p()
    assert lib.solve_server_create(1 << 30, 4, ctypes.byref(h)) == _lib.EINVAL
    for flags in (0, _lib.SERVER_MIXED, _lib.SERVER_AMG, _lib.SERVER_MIXED | _lib.SERVER_AMG):
        assert lib.solve_server_create(1 << 30, flags, ctypes.byref(h)) == _lib.OK
        assert lib.solve_server_destroy(h) == _lib.OK


def test_shadow_seed_matches_header():
    text = open(os.path.join(ROOT, "include", "mrhs.h")).read()
    mo = re.search(r"#define MRHS_SHADOW_SEED (\d+)ull", text)
    assert mo and int(mo.group(1)) == _lib.SHADOW_SEED
