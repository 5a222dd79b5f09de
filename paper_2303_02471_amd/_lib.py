"""ctypes declarations of the C ABI in include/spgemm.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspgemm.so")

SPGEMM_F32 = 0
SPGEMM_F64 = 1
SPGEMM_VALIDATE = 1
SPGEMM_ONE_STREAM = 2
SPGEMM_NO_PLANNED_LAUNCH = 4
SPGEMM_LANE_HASH = 8
SPGEMM_RADIX_ESC = 16
SPGEMM_LANE_BLOCKED = 32
SPGEMM_LANE_SPARS = 64
SPGEMM_TUNE_LOOKUP_ONLY = 1
SPGEMM_TUNE_REFRESH = 2

STATUS = {
    0: "SPGEMM_OK", 1: "SPGEMM_ERR_NULL", 2: "SPGEMM_ERR_SHAPE", 3: "SPGEMM_ERR_CSC",
    4: "SPGEMM_ERR_DTYPE", 5: "SPGEMM_ERR_INDEX_OVERFLOW", 6: "SPGEMM_ERR_NO_MEMORY",
    7: "SPGEMM_ERR_HIP", 8: "SPGEMM_ERR_PLAN", 9: "SPGEMM_ERR_INVALID",
    10: "SPGEMM_ERR_NOT_TUNED", 11: "SPGEMM_ERR_CAPACITY", 12: "SPGEMM_ERR_SCRATCH",
}
SPGEMM_ERR_CAPACITY = 11

# every symbol include/spgemm.h declares
EXPORTS = (
    "spgemm_symbolic", "spgemm_numeric", "spgemm_multiply", "spgemm_backward", "spgemm_batched",
    "spgemm_plan_get_stats", "spgemm_plan_destroy", "spgemm_status_string", "spgemm_version",
    "spgemm_profile_enable", "spgemm_profile_read", "spgemm_profile_select",
    "spgemm_autotune", "spgemm_tune_key", "spgemm_tune_cache_load", "spgemm_tune_cache_store",
    "spgemm_set_allocator", "spgemm_batch_plan_destroy", "spgemm_multiply_noalloc",
)

# device memory callbacks of spgemm_set_allocator
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)


class SpgemmError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {STATUS.get(status, status)}")


class Csc(C.Structure):
    _fields_ = [("nrows", C.c_int32), ("ncols", C.c_int32), ("nnz", C.c_int32),
                ("colptr", C.c_void_p), ("rowidx", C.c_void_p), ("val", C.c_void_p)]


class Options(C.Structure):
    _fields_ = [("t_esc", C.c_int32), ("t_dense", C.c_int32), ("dense_rows", C.c_int32),
                ("hash_cap", C.c_int32), ("flags", C.c_uint32), ("t_split", C.c_int32),
                ("t_block", C.c_int32), ("t_lane", C.c_int32), ("b_min", C.c_int32),
                ("b_max", C.c_int32)]


class PlanStats(C.Structure):
    _fields_ = [("total_products", C.c_int64), ("nnz_c", C.c_int64), ("ncols", C.c_int32),
                ("cols_empty", C.c_int32), ("cols_esc", C.c_int32), ("cols_block", C.c_int32),
                ("esc_groups", C.c_int32), ("nprob", C.c_int32), ("later_max", C.c_int32),
                ("pad", C.c_int32), ("later_products", C.c_int64), ("cols_direct", C.c_int32),
                ("cols_hash", C.c_int32), ("cols_split", C.c_int32), ("cols_sort", C.c_int32),
                ("lane_cols", C.c_int32), ("lane_blocks", C.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class TuneReport(C.Structure):
    _fields_ = [("trials", C.c_int32), ("from_cache", C.c_int32), ("default_ms", C.c_double),
                ("best_ms", C.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class KernelTime(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_int32), ("total_ms", C.c_double)]


_lib = None


def lib() -> C.CDLL:
    """The HIP library. Raises if it was not built: there is no fallback path."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2303_02471_amd.build` (hipcc, gfx950)")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64p = C.c_void_p, C.c_int32, C.POINTER(C.c_int64)
    L.spgemm_profile_select.argtypes = [C.c_char_p]
    L.spgemm_symbolic.argtypes = [C.POINTER(Csc), C.POINTER(Csc), C.c_int, C.POINTER(Options), vp,
                                  C.POINTER(vp), vp, i64p]
    L.spgemm_numeric.argtypes = [vp, vp, vp, vp, vp, vp]
    L.spgemm_multiply.argtypes = [C.POINTER(Csc), C.POINTER(Csc), C.c_int, C.POINTER(Options), vp,
                                  C.POINTER(vp), vp, vp, vp, C.c_int64, i64p]
    L.spgemm_multiply_noalloc.argtypes = [C.POINTER(Csc), C.POINTER(Csc), C.c_int,
                                          C.POINTER(Options), vp, vp, vp, vp, C.c_int64, i64p]
    L.spgemm_multiply_noalloc.restype = C.c_int
    L.spgemm_backward.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    L.spgemm_batched.argtypes = [i32, C.POINTER(Csc), C.POINTER(Csc), C.c_int, C.POINTER(Options),
                                 vp, C.POINTER(vp), C.POINTER(vp), i64p, C.POINTER(vp),
                                 C.POINTER(vp)]
    L.spgemm_plan_get_stats.argtypes = [vp, C.POINTER(PlanStats)]
    L.spgemm_plan_destroy.argtypes = [vp]
    L.spgemm_plan_destroy.restype = None
    L.spgemm_batch_plan_destroy.argtypes = [vp]
    L.spgemm_batch_plan_destroy.restype = None
    L.spgemm_set_allocator.argtypes = [ALLOC_FN, FREE_FN, vp]
    L.spgemm_set_allocator.restype = C.c_int
    L.spgemm_status_string.argtypes = [C.c_int]
    L.spgemm_status_string.restype = C.c_char_p
    L.spgemm_profile_enable.argtypes = [C.c_int32]
    L.spgemm_profile_read.argtypes = [C.POINTER(KernelTime), C.c_int32, C.POINTER(C.c_int32)]
    L.spgemm_version.argtypes = []
    L.spgemm_version.restype = C.c_int32
    L.spgemm_autotune.argtypes = [i32, C.POINTER(Csc), C.POINTER(Csc), C.c_int, vp, C.c_char_p,
                                  C.c_uint32, C.POINTER(Options), C.POINTER(TuneReport)]
    L.spgemm_tune_key.argtypes = [i32, C.POINTER(Csc), C.POINTER(Csc), C.c_int, C.c_char_p,
                                  C.c_char_p, i32]
    L.spgemm_tune_cache_load.argtypes = [C.c_char_p, C.c_char_p, C.POINTER(Options)]
    L.spgemm_tune_cache_store.argtypes = [C.c_char_p, C.c_char_p, C.POINTER(Options), C.c_double]
    for name in ("spgemm_symbolic", "spgemm_numeric", "spgemm_multiply", "spgemm_backward",
                 "spgemm_batched",
                 "spgemm_plan_get_stats", "spgemm_profile_enable", "spgemm_profile_read",
                 "spgemm_autotune", "spgemm_tune_key", "spgemm_tune_cache_load",
                 "spgemm_tune_cache_store"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def check(status: int, what: str) -> None:
    if status != 0:
        raise SpgemmError(status, what)
