"""The allocation-free one-call product (spgemm_multiply_noalloc) through the
C ABI, against spgemm_multiply on the same inputs and against the oracle, bit
for bit: two calls in a row (the second smaller, so stale workspace from the
first would show), FP64 and FP32, a too-small output capacity, and a problem
beyond the static scratch array (refused with SPGEMM_ERR_SCRATCH, after which
the entry point still works)."""
import ctypes as C
import sys

import numpy as np
import pytest

import oracle
from paper_2303_02471_amd import inputs as gen
from helpers import HAVE_GPU, assert_same_structure, assert_values_exact

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not HAVE_GPU, reason="needs an MI355X GPU")]

if HAVE_GPU:
    import torch
    from paper_2303_02471_amd import api, _lib


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def _noalloc(At, Bt, capacity=None, opts=None):
    """One call of the entry point; returns (status, colptr, rowidx, val, nnz)."""
    dev = At.colptr.device
    dtype = At.val.dtype
    cp = torch.full((Bt.ncols + 1,), -7, dtype=torch.int32, device=dev)
    cap = capacity if capacity is not None else 0
    ri = torch.full((max(cap, 1),), -7, dtype=torch.int32, device=dev)
    v = torch.full((max(cap, 1),), float("nan"), dtype=dtype, device=dev)
    nnz = C.c_int64(-1)
    da, db = api._desc(At, True), api._desc(Bt, True)
    st = _lib.lib().spgemm_multiply_noalloc(C.byref(da), C.byref(db), api._code(dtype),
                                           C.byref(opts) if opts is not None else None,
                                           api._stream(None), api._ptr(cp),
                                           ri.data_ptr() if cap else None,
                                           v.data_ptr() if cap else None, cap, C.byref(nnz))
    torch.cuda.synchronize()
    return st, cp, ri, v, int(nnz.value)


def _check(A, B, npdt, what, opts=None):
    At = api.CscTensor.from_host(A, dtype=npdt)
    Bt = api.CscTensor.from_host(B, dtype=npdt)
    # size: nnz(C) from the entry point itself (capacity 0)
    st, cp0, _, _, nnz = _noalloc(At, Bt, 0, opts)
    assert st in (0, _lib.SPGEMM_ERR_CAPACITY), f"{what}: status {st}"
    st, cp, ri, v, nnz2 = _noalloc(At, Bt, nnz, opts)
    assert st == 0 and nnz2 == nnz, f"{what}: status {st}"
    assert torch.equal(cp0, cp)
    got = (cp.cpu().numpy(), ri[:nnz].cpu().numpy(), v[:nnz].cpu().numpy())
    # the existing one-call entry point on the same inputs
    plan, rcp, rri, rv, rnnz = api.multiply(At, Bt, opts)
    torch.cuda.synchronize()
    assert rnnz == nnz, what
    assert np.array_equal(got[0], rcp.cpu().numpy()), f"{what}: colptr vs spgemm_multiply"
    assert np.array_equal(got[1], rri[:nnz].cpu().numpy()), f"{what}: rows vs spgemm_multiply"
    assert np.array_equal(got[2].view(np.uint8), rv[:nnz].cpu().numpy().view(np.uint8)), \
        f"{what}: values vs spgemm_multiply"
    plan.close()
    prec = "f64" if npdt == np.float64 else "f32"
    ocp, ori, ov = oracle.spgemm(A.astype(npdt), B.astype(npdt), prec)
    assert_same_structure(got[0], got[1], ocp, ori, what)
    assert_values_exact(got[2], ov, what)
    return nnz


def test_noalloc_matches_multiply_twice_second_smaller():
    _say("no-alloc entry point: two calls, second smaller")
    A1, B1 = gen.powerlaw(40_000, seed=3)
    n1 = _check(A1, B1, np.float64, "call 1 (power law n=40000)")
    A2 = gen.uniform_z(3000, 6, seed=4)
    B2 = gen.uniform_z(3000, 5, seed=5)
    n2 = _check(A2, B2, np.float64, "call 2 (n=3000)")
    assert n2 < n1
    _check(A2, B2, np.float32, "call 3 (n=3000, FP32)")


def test_noalloc_capacity_and_scratch_limit():
    _say("no-alloc entry point: capacity and scratch limit")
    A = gen.uniform_z(2000, 5, seed=6)
    B = gen.uniform_z(2000, 5, seed=7)
    At, Bt = api.CscTensor.from_host(A), api.CscTensor.from_host(B)
    ocp, ori, ov = oracle.spgemm(A, B)
    st, cp, _, _, nnz = _noalloc(At, Bt, int(ocp[-1]) - 1)
    assert st == _lib.SPGEMM_ERR_CAPACITY and nnz == ocp[-1]
    assert np.array_equal(cp.cpu().numpy(), ocp)
    # 16 M products in columns of 1600 (expanded, 12 B each in FP64) need
    # more than the 128 MiB array
    Ab = gen.uniform_z(10_000, 40, seed=8)
    Abt = api.CscTensor.from_host(Ab)
    st, _, _, _, _ = _noalloc(Abt, Abt, 1)
    assert st == 12, f"status {st}"
    msg = _lib.lib().spgemm_status_string(12)
    assert b"scratch" in msg
    # the entry point still works afterwards
    _check(A, B, np.float64, "after the refused problem")


@pytest.mark.parametrize("kw", [dict(radix_esc=True), dict(lane_blocked=True),
                                dict(lane_blocked=True, lane_spars=True)])
def test_noalloc_option_paths(kw):
    """The optional accumulators through the allocation-free entry point: the
    radix ESC of the heavy columns, the lane blocks with per-lane hash tables
    and with dense per-lane accumulators (their slabs carved from the array)."""
    _say(f"no-alloc entry point with {kw}")
    if kw.get("lane_spars"):
        A = gen.uniform_z(2560, 5, seed=11)
        B = gen.uniform_z(4000, 6, seed=12, nrows=2560)
    else:
        A, B = gen.powerlaw(30_000, seed=13)
    _check(A, B, np.float64, f"{kw}", api.options(**kw))
    _check(A, B, np.float32, f"{kw} FP32", api.options(**kw))
