"""CPU checks of the C ABI: the library loads and exports every declared symbol.

No compute call is made here (there is no GPU in this environment); calls that
only touch host state (status strings, version, argument checks that fail
before any device work) are exercised.
"""
import ctypes as C
import os
import re

import pytest

from paper_2303_02471_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spgemm.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(spgemm_[a-z_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2303_02471_amd import build
        build.build()
    return _lib.lib()


def test_header_declares_the_boundary():
    names = _declared_functions()
    for must in ("spgemm_symbolic", "spgemm_numeric", "spgemm_batched", "spgemm_backward"):
        assert must in names
    assert set(names) == set(_lib.EXPORTS)


def test_every_declared_symbol_exported(L):
    for name in _declared_functions():
        assert hasattr(L, name), name


def test_status_strings_and_version(L):
    assert L.spgemm_version() == 10000
    for code in range(12):
        s = L.spgemm_status_string(code)
        assert isinstance(s, bytes) and len(s) > 0
    assert L.spgemm_status_string(0) == b"ok"
    assert L.spgemm_status_string(11) != b"unknown status"
    assert L.spgemm_status_string(99) == b"unknown status"


def test_null_and_invalid_arguments_rejected_on_host(L):
    """Argument checks that return before any device work."""
    plan = C.c_void_p()
    nnz = C.c_int64()
    a = _lib.Csc(4, 4, 0, None, None, None)
    # NULL plan pointer / NULL descriptors
    assert L.spgemm_symbolic(None, None, 1, None, None, None, None, None) == 1
    assert L.spgemm_symbolic(C.byref(a), C.byref(a), 1, None, None, C.byref(plan), None,
                             C.byref(nnz)) == 1
    # one-call product: NULL outputs, negative capacity, NULL rows with capacity
    dummy = C.c_void_p(1)
    assert L.spgemm_multiply(C.byref(a), C.byref(a), 1, None, None, C.byref(plan), None, None,
                             None, 0, C.byref(nnz)) == 1
    assert L.spgemm_multiply(C.byref(a), C.byref(a), 1, None, None, C.byref(plan), dummy, None,
                             None, -1, C.byref(nnz)) == 9
    assert L.spgemm_multiply(C.byref(a), C.byref(a), 1, None, None, C.byref(plan), dummy, None,
                             None, 5, C.byref(nnz)) == 1
    # numeric / backward / stats on a NULL plan
    assert L.spgemm_numeric(None, None, None, None, None, None) == 8
    assert L.spgemm_backward(None, None, None, None, None, None, None, None) == 8
    st = _lib.PlanStats()
    assert L.spgemm_plan_get_stats(None, C.byref(st)) == 8
    L.spgemm_plan_destroy(None)  # no-op


def test_options_validated_on_host(L):
    """Out-of-range tuning values are refused before the device is touched."""
    fake = C.c_int32(0)
    a = _lib.Csc(4, 4, 0, C.addressof(fake), None, None)
    plan = C.c_void_p()
    nnz = C.c_int64()
    for bad in (_lib.Options(2, 0, 0, 0, 0), _lib.Options(512, 0, 0, 0, 0),
                _lib.Options(0, 0, -1, 0, 0), _lib.Options(0, 0, 0, 8, 0),
                _lib.Options(0, 0, 0, 2_000_000, 0), _lib.Options(0, -1, 0, 0, 0),
                _lib.Options(0, 0, 0, 0, 0, -2),
                _lib.Options(0, 0, 0, 0, 0, 0, -2)):
        st = L.spgemm_symbolic(C.byref(a), C.byref(a), 1, C.byref(bad), None, C.byref(plan),
                               C.addressof(fake), C.byref(nnz))
        assert st == 9, (bad.t_esc, bad.t_dense, bad.dense_rows, bad.hash_cap)
    # unknown dtype
    st = L.spgemm_symbolic(C.byref(a), C.byref(a), 7, None, None, C.byref(plan),
                           C.addressof(fake), C.byref(nnz))
    assert st == 4
    # shape mismatch
    b = _lib.Csc(5, 4, 0, C.addressof(fake), None, None)
    st = L.spgemm_symbolic(C.byref(a), C.byref(b), 1, None, None, C.byref(plan),
                           C.addressof(fake), C.byref(nnz))
    assert st == 2


def test_rowwise_operands_map_to_the_transposed_column_problem():
    """CSR arrays are the CSC arrays of the transpose: the row-wise call hands
    B^T x A^T to the column path with the arrays as they are, and refuses
    operands whose inner sizes differ before any library call."""
    import torch
    from paper_2303_02471_amd import api
    rp = torch.tensor([0, 1, 3], dtype=torch.int32)
    ci = torch.tensor([2, 0, 1], dtype=torch.int32)
    v = torch.tensor([1.0, 2.0, 3.0], dtype=torch.float64)
    A = api.CsrTensor(2, 3, rp, ci, v)
    t = A.transpose_csc()
    assert (t.nrows, t.ncols) == (3, 2) and t.nnz == A.nnz == 3
    assert t.colptr is rp and t.rowidx is ci and t.val is v
    B = api.CsrTensor(4, 5, torch.zeros(5, dtype=torch.int32), torch.zeros(0, dtype=torch.int32),
                      torch.zeros(0, dtype=torch.float64))
    with pytest.raises(ValueError):
        api.matmul_rowwise(A, B)


def test_set_allocator_arguments_checked_on_host(L):
    """spgemm_set_allocator takes both callbacks or neither (host only)."""
    f = _lib.ALLOC_FN(lambda n, s, c: None)
    g = _lib.FREE_FN(lambda p, n, s, c: None)
    assert L.spgemm_set_allocator(f, _lib.FREE_FN(), None) == 1
    assert L.spgemm_set_allocator(_lib.ALLOC_FN(), g, None) == 1
    assert L.spgemm_set_allocator(f, g, None) == 0
    # back to the library's own stream-ordered allocator
    assert L.spgemm_set_allocator(_lib.ALLOC_FN(), _lib.FREE_FN(), None) == 0
    L.spgemm_batch_plan_destroy(None)  # no-op
    from paper_2303_02471_amd import api
    api._installed = None  # the binding installs its own again on the next plan
