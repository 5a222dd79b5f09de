"""Python surface of the HIP library: torch tensors in, torch tensors out.

PyTorch only provides device memory and the current stream; every step of the
product runs in the library's HIP kernels, reached through the C ABI.
"""
from __future__ import annotations

import atexit
import ctypes as C
import weakref
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib

__all__ = [
    "CscTensor", "Plan", "options", "symbolic", "numeric", "matmul", "backward",
    "SpGEMMFunction", "batched_symbolic", "batched_numeric", "batched_matmul",
    "profile_enable", "profile_read", "autotune", "tune_key", "tune_cache_load",
    "tune_cache_store", "set_allocator",
]


# ---------------------------------------------------------------- plan memory
# Plans take their device memory from torch's caching allocator (on the
# stream of the call), so the library's workspace shows up in torch's memory
# statistics and reuses its cached blocks. The callbacks stay referenced here
# for the life of the process.
def _torch_alloc(nbytes, stream, ctx):
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
    except Exception:  # out of memory: the library reports SPGEMM_ERR_NO_MEMORY
        return None


def _torch_free(ptr, nbytes, stream, ctx):
    torch.cuda.caching_allocator_delete(int(ptr))


_TORCH_CALLBACKS = (_lib.ALLOC_FN(_torch_alloc), _lib.FREE_FN(_torch_free))
_installed = None  # callbacks currently installed in the library (kept alive)
_plans = weakref.WeakSet()  # live plans, closed before the interpreter exits


def set_allocator(alloc=None, free=None):
    """Device memory of plans created from now on: "torch" (the default of
    this binding: torch's caching allocator), None (the library's own
    stream-ordered hipMallocAsync), or a pair of ctypes callbacks
    (_lib.ALLOC_FN, _lib.FREE_FN) that the caller keeps alive."""
    global _installed
    if alloc == "torch":
        alloc, free = _TORCH_CALLBACKS
    if alloc is None:
        st = _lib.lib().spgemm_set_allocator(_lib.ALLOC_FN(), _lib.FREE_FN(), None)
    else:
        st = _lib.lib().spgemm_set_allocator(alloc, free, None)
    _lib.check(st, "spgemm_set_allocator")
    _installed = (alloc, free)


def _ensure_allocator():
    if _installed is None:
        set_allocator("torch")


@atexit.register
def _close_plans():
    # plans hand their memory back to torch while torch is still alive
    for p in list(_plans):
        try:
            p.close()
        except Exception:
            pass


def profile_enable(on: bool = True) -> None:
    """Start (and clear) or stop per-kernel event timing inside the library."""
    _lib.check(_lib.lib().spgemm_profile_enable(1 if on else 0), "profile_enable")


def profile_select(name: Optional[str] = None) -> None:
    """Record only the launch group `name` (None: every group)."""
    _lib.check(_lib.lib().spgemm_profile_select(name.encode() if name else None),
               "profile_select")


def profile_read() -> dict:
    """{kernel name: (launches, total ms)} recorded since profile_enable(True)."""
    buf = (_lib.KernelTime * 64)()
    n = C.c_int32(0)
    _lib.check(_lib.lib().spgemm_profile_read(buf, 64, C.byref(n)), "profile_read")
    return {buf[i].name.decode(): (int(buf[i].launches), float(buf[i].total_ms))
            for i in range(n.value)}


@dataclass
class CscTensor:
    """CSC matrix held in device tensors (int32 colptr/rowidx, float values)."""

    nrows: int
    ncols: int
    colptr: torch.Tensor
    rowidx: torch.Tensor
    val: Optional[torch.Tensor] = None

    @property
    def nnz(self) -> int:
        return int(self.rowidx.numel())

    @staticmethod
    def from_host(m, device="cuda", dtype=None) -> "CscTensor":
        """From any object with nrows/ncols/colptr/rowidx/val numpy arrays."""
        val = None
        if getattr(m, "val", None) is not None:
            v = np.asarray(m.val)
            if dtype is not None:
                v = v.astype(dtype)
            val = torch.from_numpy(np.ascontiguousarray(v)).to(device)
        return CscTensor(int(m.nrows), int(m.ncols),
                         torch.from_numpy(np.ascontiguousarray(m.colptr, dtype=np.int32)).to(device),
                         torch.from_numpy(np.ascontiguousarray(m.rowidx, dtype=np.int32)).to(device),
                         val)

    def to_host(self):
        return (self.colptr.cpu().numpy(), self.rowidx.cpu().numpy(),
                None if self.val is None else self.val.cpu().numpy())


def options(t_esc: int = 0, t_dense: int = 0, dense_rows: int = 0, hash_cap: int = 0,
            t_split: int = 0, t_block: int = 0, validate: bool = False,
            one_stream: bool = False, planned: bool = True,
            lane_hash: bool = False, radix_esc: bool = False, lane_blocked: bool = False,
            lane_spars: bool = False, t_lane: int = 0, b_min: int = 0,
            b_max: int = 0) -> _lib.Options:
    """Tuning options (zero = library default). They never change results."""
    flags = (_lib.SPGEMM_VALIDATE if validate else 0) | \
        (_lib.SPGEMM_ONE_STREAM if one_stream else 0) | \
        (0 if planned else _lib.SPGEMM_NO_PLANNED_LAUNCH) | \
        (_lib.SPGEMM_LANE_HASH if lane_hash else 0) | \
        (_lib.SPGEMM_RADIX_ESC if radix_esc else 0) | \
        (_lib.SPGEMM_LANE_BLOCKED if lane_blocked else 0) | \
        (_lib.SPGEMM_LANE_SPARS if lane_spars else 0)
    return _lib.Options(t_esc, t_dense, dense_rows, hash_cap, flags, t_split, t_block, t_lane,
                        b_min, b_max)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensors must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensors must be contiguous")
    return t.data_ptr() if t.numel() else None


def _desc(m: CscTensor, with_val: bool) -> _lib.Csc:
    if m.colptr.dtype != torch.int32 or m.rowidx.dtype != torch.int32:
        raise TypeError("colptr and rowidx must be int32")
    if m.colptr.numel() != m.ncols + 1:
        raise ValueError("colptr must hold ncols + 1 entries")
    return _lib.Csc(m.nrows, m.ncols, m.nnz, _ptr(m.colptr), _ptr(m.rowidx),
                    _ptr(m.val) if with_val else None)


def _code(dtype: torch.dtype) -> int:
    if dtype == torch.float64:
        return _lib.SPGEMM_F64
    if dtype == torch.float32:
        return _lib.SPGEMM_F32
    raise TypeError(f"unsupported value type {dtype}")


_raw_stream = getattr(torch._C, "_cuda_getCurrentRawStream", None)


def _stream(stream) -> Optional[int]:
    if stream is None:
        if _raw_stream is not None:  # the current stream's handle without a Stream object
            return _raw_stream(torch.cuda.current_device()) or None
        stream = torch.cuda.current_stream()
    return stream.cuda_stream or None


class Plan:
    """Owns a library plan and keeps the arrays it borrows alive."""

    def __init__(self):
        _ensure_allocator()
        self.handle = C.c_void_p()
        self.keep = []
        self.dtype = None
        self.nnz = None
        _plans.add(self)

    def stats(self) -> dict:
        s = _lib.PlanStats()
        _lib.check(_lib.lib().spgemm_plan_get_stats(self.handle, C.byref(s)), "plan stats")
        return s.as_dict()

    def close(self):
        if self.handle:
            _lib.lib().spgemm_plan_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def symbolic(A: CscTensor, B: CscTensor, dtype=torch.float64, opts=None,
             plan: Optional[Plan] = None, stream=None, out_colptr: Optional[torch.Tensor] = None):
    """Structure of C = A x B. Returns (plan, C_colptr, nnz(C)).

    Passing the previous plan (and its colptr as out_colptr) reuses the
    plan's device workspace: nothing is allocated on repeated calls."""
    plan = plan or Plan()
    if out_colptr is not None and (out_colptr.numel() != B.ncols + 1 or
                                   out_colptr.dtype != torch.int32):
        raise ValueError("out_colptr must be int32 with B.ncols + 1 entries")
    colptr = out_colptr if out_colptr is not None else torch.empty(
        B.ncols + 1, dtype=torch.int32, device=A.colptr.device)
    nnz = C.c_int64(0)
    da, db = _desc(A, False), _desc(B, False)
    st = _lib.lib().spgemm_symbolic(C.byref(da), C.byref(db), _code(dtype),
                                    C.byref(opts) if opts is not None else None, _stream(stream),
                                    C.byref(plan.handle), _ptr(colptr), C.byref(nnz))
    _lib.check(st, "spgemm_symbolic")
    plan.keep = [A.colptr, A.rowidx, B.colptr, B.rowidx, colptr]
    plan.dtype = dtype
    plan.nnz = int(nnz.value)
    plan.shape = (A.nrows, B.ncols)
    plan.colptr = colptr
    return plan, colptr, int(nnz.value)


def numeric(plan: Plan, A_val: torch.Tensor, B_val: torch.Tensor, C_rowidx: torch.Tensor,
            C_val: torch.Tensor, stream=None) -> None:
    for t in (A_val, B_val, C_val):
        if t.dtype != plan.dtype:
            raise TypeError("value tensors must have the plan's dtype")
    st = _lib.lib().spgemm_numeric(plan.handle, _ptr(A_val), _ptr(B_val), _ptr(C_rowidx),
                                   _ptr(C_val), _stream(stream))
    _lib.check(st, "spgemm_numeric")


def multiply(A: CscTensor, B: CscTensor, opts=None, plan: Optional[Plan] = None, out=None,
             stream=None):
    """C = A x B in one library call (symbolic, then numeric queued behind it).

    ``out`` = (colptr, rowidx, val) to reuse: rowidx / val of any capacity
    (typically the previous nnz(C)); when nnz(C) exceeds it, larger arrays are
    allocated and the numeric phase runs on them. Returns
    (plan, colptr, rowidx, val, nnz); rowidx / val hold C's entries in [:nnz]."""
    if A.val is None or B.val is None:
        raise ValueError("values required")
    dtype = A.val.dtype
    if B.val.dtype != dtype:
        raise TypeError("A and B values must have the same dtype")
    plan = plan or Plan()
    dev = A.colptr.device
    if out is not None:
        colptr, rowidx, val = out
        if colptr.numel() != B.ncols + 1:  # another shape: the pointers need their own array
            colptr = torch.empty(B.ncols + 1, dtype=torch.int32, device=dev)
    else:
        colptr = torch.empty(B.ncols + 1, dtype=torch.int32, device=dev)
        rowidx = torch.empty(0, dtype=torch.int32, device=dev)
        val = torch.empty(0, dtype=dtype, device=dev)
    if val.dtype != dtype or rowidx.dtype != torch.int32 or colptr.dtype != torch.int32:
        raise TypeError("output arrays must be int32 pointers and rows, values of A's dtype")
    cap = min(rowidx.numel(), val.numel())
    nnz = C.c_int64(0)
    da, db = _desc(A, True), _desc(B, True)
    st = _lib.lib().spgemm_multiply(C.byref(da), C.byref(db), _code(dtype),
                                    C.byref(opts) if opts is not None else None, _stream(stream),
                                    C.byref(plan.handle), _ptr(colptr), _ptr(rowidx), _ptr(val),
                                    cap, C.byref(nnz))
    if st != _lib.SPGEMM_ERR_CAPACITY:
        _lib.check(st, "spgemm_multiply")
    plan.keep = [A.colptr, A.rowidx, B.colptr, B.rowidx, colptr]
    plan.dtype = dtype
    plan.nnz = int(nnz.value)
    plan.shape = (A.nrows, B.ncols)
    plan.colptr = colptr
    if st == _lib.SPGEMM_ERR_CAPACITY:
        rowidx = torch.empty(plan.nnz, dtype=torch.int32, device=dev)
        val = torch.empty(plan.nnz, dtype=dtype, device=dev)
        numeric(plan, A.val, B.val, rowidx, val, stream)
    return plan, colptr, rowidx, val, plan.nnz


def matmul(A: CscTensor, B: CscTensor, opts=None, return_plan: bool = False):
    """C = A x B with sorted rows in every column."""
    if A.val is None or B.val is None:
        raise ValueError("values required")
    dtype = A.val.dtype
    if B.val.dtype != dtype:
        raise TypeError("A and B values must share a dtype")
    plan, colptr, nnz = symbolic(A, B, dtype, opts)
    rowidx = torch.empty(nnz, dtype=torch.int32, device=A.val.device)
    val = torch.empty(nnz, dtype=dtype, device=A.val.device)
    numeric(plan, A.val, B.val, rowidx, val)
    Cm = CscTensor(A.nrows, B.ncols, colptr, rowidx, val)
    return (Cm, plan) if return_plan else Cm


@dataclass
class CsrTensor:
    """CSR matrix held in device tensors (int32 rowptr/colidx, float values).
    Its three arrays are exactly those of the CSC form of its transpose."""

    nrows: int
    ncols: int
    rowptr: torch.Tensor
    colidx: torch.Tensor
    val: Optional[torch.Tensor] = None

    @property
    def nnz(self) -> int:
        return int(self.colidx.numel())

    def transpose_csc(self) -> CscTensor:
        """The transpose, in CSC, sharing this matrix's arrays (no copy)."""
        return CscTensor(self.ncols, self.nrows, self.rowptr, self.colidx, self.val)


def matmul_rowwise(A: CsrTensor, B: CsrTensor, opts=None) -> CsrTensor:
    """C = A x B on CSR operands, with sorted columns in every row: the
    row-wise form of Gustavson's method that Section 2.1 mentions. Row i of C
    accumulates B's row k scaled by A(i,k) over A's row i in storage order;
    that is column i of C^T = B^T x A^T, whose CSC arrays are C's CSR arrays,
    formed from the same products (a rounded product does not depend on the
    operand order) added in the same order. The column kernels therefore
    compute it unchanged, on the operands' arrays as they are."""
    if A.ncols != B.nrows:
        raise ValueError("A.ncols must equal B.nrows")
    Ct = matmul(B.transpose_csc(), A.transpose_csc(), opts)
    return CsrTensor(A.nrows, B.ncols, Ct.colptr, Ct.rowidx, Ct.val)


def backward(plan: Plan, A_val: torch.Tensor, B_val: torch.Tensor, C_rowidx: torch.Tensor,
             G_val: torch.Tensor, need_a: bool = True, need_b: bool = True, stream=None,
             out=None):
    """(dA, dB) of <G, A x B> with respect to the stored values (patterns fixed).
    ``out`` = (dA, dB) arrays to fill (either may be None to skip it)."""
    if out is not None:
        dA, dB = out
    else:
        dA = torch.empty_like(A_val) if need_a else None
        dB = torch.empty_like(B_val) if need_b else None
    st = _lib.lib().spgemm_backward(plan.handle, _ptr(A_val), _ptr(B_val), _ptr(C_rowidx),
                                    _ptr(G_val), _ptr(dA), _ptr(dB), _stream(stream))
    _lib.check(st, "spgemm_backward")
    return dA, dB


class SpGEMMFunction(torch.autograd.Function):
    """Differentiable C.val = (A x B).val with respect to A.val and B.val.

    forward(A_val, B_val, A_pattern, B_pattern, plan=None) -> (C_val, C_rowidx, C_colptr);
    only C_val carries a gradient. Sparsity patterns are fixed inputs.
    """

    @staticmethod
    def forward(ctx, A_val, B_val, A: CscTensor, B: CscTensor, plan: Optional[Plan] = None):
        dtype = A_val.dtype
        if plan is None or plan.dtype != dtype:
            plan, colptr, nnz = symbolic(A, B, dtype)
        colptr, nnz = plan.colptr, plan.nnz
        rowidx = torch.empty(nnz, dtype=torch.int32, device=A_val.device)
        val = torch.empty(nnz, dtype=dtype, device=A_val.device)
        numeric(plan, A_val.contiguous(), B_val.contiguous(), rowidx, val)
        ctx.save_for_backward(A_val, B_val, rowidx)
        ctx.plan = plan
        ctx.mark_non_differentiable(rowidx, colptr)
        return val, rowidx, colptr

    @staticmethod
    def backward(ctx, gC, _g_rowidx=None, _g_colptr=None):
        A_val, B_val, rowidx = ctx.saved_tensors
        need_a, need_b = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        dA = dB = None
        if need_a or need_b:
            dA, dB = backward(ctx.plan, A_val, B_val, rowidx, gC.contiguous(), need_a, need_b)
        return dA, dB, None, None, None


def batched_symbolic(pairs: Sequence[tuple], dtype=torch.float64, opts=None,
                     plan: Optional[Plan] = None, stream=None):
    """Size query of C_i = A_i x B_i for every pair. Returns (plan, colptrs, nnzs)."""
    n = len(pairs)
    plan = plan or Plan()
    dev = pairs[0][0].colptr.device if n else torch.device("cuda")
    colptrs = [torch.empty(b.ncols + 1, dtype=torch.int32, device=dev) for _, b in pairs]
    As = (_lib.Csc * max(n, 1))(*[_desc(a, False) for a, _ in pairs])
    Bs = (_lib.Csc * max(n, 1))(*[_desc(b, False) for _, b in pairs])
    cps = (C.c_void_p * max(n, 1))(*[_ptr(c) for c in colptrs])
    nnz = (C.c_int64 * max(n, 1))()
    st = _lib.lib().spgemm_batched(n, As, Bs, _code(dtype),
                                   C.byref(opts) if opts is not None else None, _stream(stream),
                                   C.byref(plan.handle), cps, nnz, None, None)
    _lib.check(st, "spgemm_batched (size query)")
    plan.keep = [t for a, b in pairs for t in (a.colptr, a.rowidx, b.colptr, b.rowidx)] + colptrs
    plan.dtype = dtype
    plan.colptrs = colptrs
    plan.nnzs = [int(nnz[i]) for i in range(n)]
    return plan, colptrs, plan.nnzs


def batched_numeric(plan: Plan, pairs: Sequence[tuple], rowidxs, vals, stream=None) -> None:
    n = len(pairs)
    As = (_lib.Csc * max(n, 1))(*[_desc(a, True) for a, _ in pairs])
    Bs = (_lib.Csc * max(n, 1))(*[_desc(b, True) for _, b in pairs])
    cps = (C.c_void_p * max(n, 1))(*[_ptr(c) for c in plan.colptrs])
    nnz = (C.c_int64 * max(n, 1))(*plan.nnzs)
    ris = (C.c_void_p * max(n, 1))(*[_ptr(r) for r in rowidxs])
    vs = (C.c_void_p * max(n, 1))(*[_ptr(v) for v in vals])
    st = _lib.lib().spgemm_batched(n, As, Bs, _code(plan.dtype), None, _stream(stream),
                                   C.byref(plan.handle), cps, nnz, ris, vs)
    _lib.check(st, "spgemm_batched (numeric)")


def batched_matmul(pairs: Sequence[tuple], opts=None, return_plan: bool = False):
    dtype = pairs[0][0].val.dtype
    plan, colptrs, nnzs = batched_symbolic(pairs, dtype, opts)
    dev = pairs[0][0].val.device
    rowidxs = [torch.empty(z, dtype=torch.int32, device=dev) for z in nnzs]
    vals = [torch.empty(z, dtype=dtype, device=dev) for z in nnzs]
    batched_numeric(plan, pairs, rowidxs, vals)
    out = [CscTensor(a.nrows, b.ncols, cp, ri, v)
           for (a, b), cp, ri, v in zip(pairs, colptrs, rowidxs, vals)]
    return (out, plan) if return_plan else out


def _descs(pairs: Sequence[tuple], with_val: bool):
    n = len(pairs)
    As = (_lib.Csc * max(n, 1))(*[_desc(a, with_val) for a, _ in pairs])
    Bs = (_lib.Csc * max(n, 1))(*[_desc(b, with_val) for _, b in pairs])
    return As, Bs


def autotune(pairs: Sequence[tuple], dtype=torch.float64, cache_path: Optional[str] = None,
             refresh: bool = False, lookup_only: bool = False, stream=None):
    """Tuning options for the products A_i x B_i (one pair: a single product),
    chosen by timing candidate thresholds in the library (or read from the JSON
    cache). Returns (options, report dict). The options never change results."""
    As, Bs = _descs(pairs, True)
    opts = _lib.Options()
    rep = _lib.TuneReport()
    flags = (_lib.SPGEMM_TUNE_REFRESH if refresh else 0) | \
        (_lib.SPGEMM_TUNE_LOOKUP_ONLY if lookup_only else 0)
    st = _lib.lib().spgemm_autotune(len(pairs), As, Bs, _code(dtype), _stream(stream),
                                    cache_path.encode() if cache_path else None, flags,
                                    C.byref(opts), C.byref(rep))
    _lib.check(st, "spgemm_autotune")
    return opts, rep.as_dict()


def tune_key(shapes: Sequence[tuple], dtype=torch.float64, device_tag: str = "dev") -> str:
    """Cache key of a workload given (m, k, n, nnzA, nnzB) per problem (host only)."""
    n = len(shapes)
    As = (_lib.Csc * max(n, 1))(*[_lib.Csc(m, k, za, None, None, None)
                                   for m, k, _, za, _ in shapes])
    Bs = (_lib.Csc * max(n, 1))(*[_lib.Csc(k, nn, zb, None, None, None)
                                   for _, k, nn, _, zb in shapes])
    buf = C.create_string_buffer(512)
    st = _lib.lib().spgemm_tune_key(n, As, Bs, _code(dtype), device_tag.encode(), buf, 512)
    _lib.check(st, "spgemm_tune_key")
    return buf.value.decode()


def tune_cache_load(path: str, key: str) -> Optional[_lib.Options]:
    """Cached options for `key`, or None (missing file or entry, or a file that
    does not parse)."""
    opts = _lib.Options()
    st = _lib.lib().spgemm_tune_cache_load(path.encode(), key.encode(), C.byref(opts))
    if st == 10:
        return None
    _lib.check(st, "spgemm_tune_cache_load")
    return opts


def tune_cache_store(path: str, key: str, opts: _lib.Options, ms: float) -> None:
    st = _lib.lib().spgemm_tune_cache_store(path.encode(), key.encode(), C.byref(opts), ms)
    _lib.check(st, "spgemm_tune_cache_store")
