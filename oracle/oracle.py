"""numpy front end of the C oracle (test infrastructure only).

Matrices are passed as any object with ``nrows``, ``ncols``, ``colptr``,
``rowidx`` and ``val`` attributes (CSC, Section 2.1). Results are plain numpy
arrays. This module imports nothing from the GPU package.
"""
from __future__ import annotations

import ctypes as C
import os
from types import SimpleNamespace

import numpy as np

from . import build as _build

__all__ = [
    "OracleError", "bind", "check_csc", "opcount", "symbolic", "spgemm", "spgemm_parallel", "absprod",
    "backward", "sort_columns", "blocking", "hash_size", "csc",
]

_I32P = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_I64P = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_F64P = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_F32P = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_i32 = C.c_int32

_lib = None


class OracleError(RuntimeError):
    pass


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = _build.LIB
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
        _build.build()
    _lib = bind(path)
    return _lib


def bind(path):
    """Declare the oracle's C functions on the shared library at `path` (the
    built oracle, or a copy built from modified source by a test that checks
    its pins catch a planted mistake)."""
    lib = C.CDLL(path)
    pair = [_i32, _i32, _I32P, _I32P]
    lib.oracle_check_csc.argtypes = [_i32, _i32, _I32P, _I32P]
    lib.oracle_opcount.argtypes = [_i32, _I32P, _i32, _I32P, _I32P, _I64P]
    lib.oracle_symbolic.argtypes = pair + pair + [_I32P]
    for suffix, vp in (("f64", _F64P), ("f32", _F32P)):
        fn = getattr(lib, f"oracle_spgemm_{suffix}")
        fn.argtypes = pair + [vp] + pair + [vp] + [_I32P, _I32P, vp]
        fn = getattr(lib, f"oracle_backward_{suffix}")
        fn.argtypes = pair + [vp] + pair + [vp] + [_I32P, _I32P, vp, C.c_void_p, C.c_void_p]
    lib.oracle_absprod_f64.argtypes = pair + [_F64P] + pair + [_F64P] + [_I32P, _I32P, _F64P, _I32P]
    lib.oracle_sort_columns.argtypes = [_i32, _I64P, _I32P]
    lib.oracle_blocking.argtypes = [_i32, _I64P, _i32, _i32, _I32P, _I32P]
    lib.oracle_spgemm_f64_parallel.argtypes = pair + [_F64P] + pair + [_F64P] + [
        _I32P, C.POINTER(C.c_int64), _I32P, _F64P, _i32, C.POINTER(_i32)]
    lib.oracle_spgemm_f64_parallel.restype = C.c_int
    lib.oracle_hash_size.argtypes = [C.c_int64]
    lib.oracle_hash_size.restype = C.c_int64
    for name in ("oracle_check_csc", "oracle_opcount", "oracle_symbolic", "oracle_spgemm_f64",
                 "oracle_spgemm_f32", "oracle_backward_f64", "oracle_backward_f32",
                 "oracle_absprod_f64", "oracle_sort_columns", "oracle_blocking"):
        getattr(lib, name).restype = C.c_int
    return lib


def csc(nrows, ncols, colptr, rowidx, val=None):
    """Bundle arrays into a CSC-like namespace."""
    return SimpleNamespace(nrows=int(nrows), ncols=int(ncols),
                           colptr=np.ascontiguousarray(colptr, dtype=np.int32),
                           rowidx=np.ascontiguousarray(rowidx, dtype=np.int32),
                           val=None if val is None else np.ascontiguousarray(val))


def _pat(a):
    return [int(a.nrows), int(a.ncols), np.ascontiguousarray(a.colptr, dtype=np.int32),
            np.ascontiguousarray(a.rowidx, dtype=np.int32)]


def _rc(rc, what):
    if rc != 0:
        raise OracleError(f"{what}: oracle status {rc}")


def check_csc(a) -> int:
    return _load().oracle_check_csc(*_pat(a))


def opcount(a, b) -> np.ndarray:
    op = np.zeros(int(b.ncols), dtype=np.int64)
    _rc(_load().oracle_opcount(int(a.ncols), np.ascontiguousarray(a.colptr, dtype=np.int32),
                               int(b.ncols), np.ascontiguousarray(b.colptr, dtype=np.int32),
                               np.ascontiguousarray(b.rowidx, dtype=np.int32), op), "opcount")
    return op


def symbolic(a, b, lib=None) -> np.ndarray:
    cp = np.zeros(int(b.ncols) + 1, dtype=np.int32)
    _rc((lib or _load()).oracle_symbolic(*_pat(a), *_pat(b), cp), "symbolic")
    return cp


def spgemm(a, b, precision: str = "f64", lib=None):
    """C = A x B by Algorithm 1. ``precision`` "f64" upcasts the values and
    works in double; "f32" runs the same loops in single precision.
    Returns (colptr, rowidx, val)."""
    lib = lib or _load()
    cp = symbolic(a, b, lib)
    nnz = int(cp[-1])
    ri = np.zeros(nnz, dtype=np.int32)
    if precision == "f64":
        cv = np.zeros(nnz, dtype=np.float64)
        fn = lib.oracle_spgemm_f64
        av = np.ascontiguousarray(a.val, dtype=np.float64)
        bv = np.ascontiguousarray(b.val, dtype=np.float64)
    elif precision == "f32":
        cv = np.zeros(nnz, dtype=np.float32)
        fn = lib.oracle_spgemm_f32
        if a.val.dtype != np.float32 or b.val.dtype != np.float32:
            raise OracleError("f32 twin needs float32 inputs")
        av = np.ascontiguousarray(a.val)
        bv = np.ascontiguousarray(b.val)
    else:
        raise ValueError(precision)
    _rc(fn(*_pat(a), av, *_pat(b), bv, cp, ri, cv), "spgemm")
    return cp, ri, cv


def spgemm_parallel(a, b, nthreads: int = 0, nnz_hint: int = 0):
    """C = A x B in FP64 with whole columns spread over OpenMP threads
    (0: all host cores); identical to spgemm(a, b). Returns (colptr, rowidx,
    val, threads_used). nnz_hint sizes the outputs (0: computed first)."""
    lib = _load()
    av = np.ascontiguousarray(a.val, dtype=np.float64)
    bv = np.ascontiguousarray(b.val, dtype=np.float64)
    cp = np.zeros(int(b.ncols) + 1, dtype=np.int32)
    cap = C.c_int64(max(int(nnz_hint), 0))
    used = C.c_int32(0)
    for _ in range(2):
        ri = np.zeros(max(cap.value, 1), dtype=np.int32)
        cv = np.zeros(max(cap.value, 1), dtype=np.float64)
        rc = lib.oracle_spgemm_f64_parallel(*_pat(a), av, *_pat(b), bv, cp, C.byref(cap), ri, cv,
                                            int(nthreads), C.byref(used))
        if rc == 4 and cap.value > len(ri):
            continue  # sized now: run again with room for nnz(C)
        _rc(rc, "spgemm_parallel")
        n = int(cp[-1])
        return cp, ri[:n], cv[:n], int(used.value)
    raise OracleError("spgemm_parallel: output size changed between calls")


def absprod(a, b, c_colptr, c_rowidx, lib=None):
    """sum_k |A(i,k) B(k,j)| and the number of products, on C's pattern."""
    nnz = int(c_colptr[-1])
    s = np.zeros(nnz, dtype=np.float64)
    t = np.zeros(nnz, dtype=np.int32)
    _rc((lib or _load()).oracle_absprod_f64(*_pat(a), np.ascontiguousarray(a.val, dtype=np.float64),
                                   *_pat(b), np.ascontiguousarray(b.val, dtype=np.float64),
                                   np.ascontiguousarray(c_colptr, dtype=np.int32),
                                   np.ascontiguousarray(c_rowidx, dtype=np.int32), s, t),
        "absprod")
    return s, t


def backward(a, b, c_colptr, c_rowidx, g, precision: str = "f64", want_a=True, want_b=True,
             lib=None):
    """Gradients of <G, A x B> w.r.t. the stored values of A and B."""
    dt = np.float64 if precision == "f64" else np.float32
    fn = getattr(lib or _load(), f"oracle_backward_{precision}")
    av = np.ascontiguousarray(a.val, dtype=dt)
    bv = np.ascontiguousarray(b.val, dtype=dt)
    gv = np.ascontiguousarray(g, dtype=dt)
    if precision == "f32" and (a.val.dtype != np.float32 or b.val.dtype != np.float32
                               or np.asarray(g).dtype != np.float32):
        raise OracleError("f32 twin needs float32 inputs")
    da = np.zeros(len(av), dtype=dt) if want_a else None
    db = np.zeros(len(bv), dtype=dt) if want_b else None
    _rc(fn(*_pat(a), av, *_pat(b), bv, np.ascontiguousarray(c_colptr, dtype=np.int32),
           np.ascontiguousarray(c_rowidx, dtype=np.int32), gv,
           None if da is None else da.ctypes.data_as(C.c_void_p),
           None if db is None else db.ctypes.data_as(C.c_void_p)), "backward")
    return da, db


def sort_columns(op) -> np.ndarray:
    op = np.ascontiguousarray(op, dtype=np.int64)
    perm = np.zeros(len(op), dtype=np.int32)
    _rc(_load().oracle_sort_columns(len(op), op, perm), "sort_columns")
    return perm


def blocking(op_sorted, bmin: int, bmax: int) -> np.ndarray:
    op_sorted = np.ascontiguousarray(op_sorted, dtype=np.int64)
    starts = np.zeros(len(op_sorted) + 1, dtype=np.int32)
    nb = np.zeros(1, dtype=np.int32)
    _rc(_load().oracle_blocking(len(op_sorted), op_sorted, bmin, bmax, starts, nb), "blocking")
    return starts[: int(nb[0]) + 1].copy()


def hash_size(maxop: int) -> int:
    return int(_load().oracle_hash_size(int(maxop)))
