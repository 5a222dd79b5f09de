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
    "OracleError", "check_csc", "opcount", "symbolic", "spgemm", "absprod",
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
    lib.oracle_hash_size.argtypes = [C.c_int64]
    lib.oracle_hash_size.restype = C.c_int64
    for name in ("oracle_check_csc", "oracle_opcount", "oracle_symbolic", "oracle_spgemm_f64",
                 "oracle_spgemm_f32", "oracle_backward_f64", "oracle_backward_f32",
                 "oracle_absprod_f64", "oracle_sort_columns", "oracle_blocking"):
        getattr(lib, name).restype = C.c_int
    _lib = lib
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


def symbolic(a, b) -> np.ndarray:
    cp = np.zeros(int(b.ncols) + 1, dtype=np.int32)
    _rc(_load().oracle_symbolic(*_pat(a), *_pat(b), cp), "symbolic")
    return cp


def spgemm(a, b, precision: str = "f64"):
    """C = A x B by Algorithm 1. ``precision`` "f64" upcasts the values and
    works in double; "f32" runs the same loops in single precision.
    Returns (colptr, rowidx, val)."""
    cp = symbolic(a, b)
    nnz = int(cp[-1])
    ri = np.zeros(nnz, dtype=np.int32)
    if precision == "f64":
        cv = np.zeros(nnz, dtype=np.float64)
        fn = _load().oracle_spgemm_f64
        av = np.ascontiguousarray(a.val, dtype=np.float64)
        bv = np.ascontiguousarray(b.val, dtype=np.float64)
    elif precision == "f32":
        cv = np.zeros(nnz, dtype=np.float32)
        fn = _load().oracle_spgemm_f32
        if a.val.dtype != np.float32 or b.val.dtype != np.float32:
            raise OracleError("f32 twin needs float32 inputs")
        av = np.ascontiguousarray(a.val)
        bv = np.ascontiguousarray(b.val)
    else:
        raise ValueError(precision)
    _rc(fn(*_pat(a), av, *_pat(b), bv, cp, ri, cv), "spgemm")
    return cp, ri, cv


def absprod(a, b, c_colptr, c_rowidx):
    """sum_k |A(i,k) B(k,j)| and the number of products, on C's pattern."""
    nnz = int(c_colptr[-1])
    s = np.zeros(nnz, dtype=np.float64)
    t = np.zeros(nnz, dtype=np.int32)
    _rc(_load().oracle_absprod_f64(*_pat(a), np.ascontiguousarray(a.val, dtype=np.float64),
                                   *_pat(b), np.ascontiguousarray(b.val, dtype=np.float64),
                                   np.ascontiguousarray(c_colptr, dtype=np.int32),
                                   np.ascontiguousarray(c_rowidx, dtype=np.int32), s, t),
        "absprod")
    return s, t


def backward(a, b, c_colptr, c_rowidx, g, precision: str = "f64", want_a=True, want_b=True):
    """Gradients of <G, A x B> w.r.t. the stored values of A and B."""
    dt = np.float64 if precision == "f64" else np.float32
    fn = getattr(_load(), f"oracle_backward_{precision}")
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
