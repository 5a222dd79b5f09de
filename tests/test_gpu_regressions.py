"""GPU regression tests for specific failure modes, each against the oracle.

* Rows at the 2^20 boundary: 32-bit sort keys (row << 12 | position) are
  used only while every key stays below the all-ones padding key.
* A lane-hash launch planned from an earlier call's (smaller) column count.
* A numeric tile whose column window holds no stored B entry (a long run of
  empty B columns inside one product tile).
* The workgroup hash / direct-index accumulator forced at the dense-bin size
  (n = 4096, 40 per column) and at the forward/backward size (8 per column).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2303_02471_amd import inputs as gen
from helpers import (HAVE_GPU, assert_same_structure, assert_values_exact, check_f64, check_f32,
                     gpu_product)

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not HAVE_GPU, reason="needs an MI355X GPU")]

if HAVE_GPU:
    import torch
    from paper_2303_02471_amd import api


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def _rows_2pow20():
    """A with exactly 2^20 rows and two columns: column 0 holds rows 0..3,
    column 1 the 4096 rows 2^20 - 4096 .. 2^20 - 1 (the last stored last).
    B(:,0) = [0, 1] gives a column of 4100 products (windowed sort: its upper
    row window holds exactly 4096 products, the last on row 2^20 - 1 at window
    position 4095); B(:,1) = [1] gives 4096 products (workgroup sort of 4096,
    the last on row 2^20 - 1 at position 4095)."""
    m = 1 << 20
    rng = np.random.default_rng(20)
    rows = np.concatenate([np.arange(4), np.arange(m - 4096, m)]).astype(np.int32)
    A = gen.CSC(m, 2, np.array([0, 4, 4100], np.int32), rows, rng.uniform(-1, 1, 4100))
    B = gen.CSC(2, 2, np.array([0, 2, 3], np.int32), np.array([0, 1, 1], np.int32),
                rng.uniform(-1, 1, 3))
    return A, B


@pytest.mark.parametrize("opts", [None, dict(t_esc=4), dict(t_split=100)])
def test_rows_at_2pow20(opts):
    _say(f"2^20 rows, opts={opts}")
    A, B = _rows_2pow20()
    o = api.options(**opts) if opts else None
    cp, ri, v = check_f64(A, B, o, "2^20 rows")
    assert cp.tolist() == [0, 4100, 8196]
    assert ri[4099] == (1 << 20) - 1 and ri[-1] == (1 << 20) - 1
    check_f32(A, B, o, "2^20 rows f32")
    # one row fewer (2^20 - 1 rows, 32-bit keys): the same shape of columns
    m2 = (1 << 20) - 1
    rows2 = np.concatenate([np.arange(4), np.arange(m2 - 4096, m2)]).astype(np.int32)
    A2 = gen.CSC(m2, 2, A.colptr, rows2, A.val)
    check_f64(A2, B, o, "2^20 - 1 rows")


def test_lane_hash_planned_grid_covers_more_columns():
    """The lane-per-column launch of a planned pass is sized from the previous
    call's column counts; a second call on the same plan with the same product
    total and no new non-empty sub-bin, but many more columns in one lane
    sub-bin, must still cover every column (no redo is triggered)."""
    _say("lane hash planned grid")
    n, m = 200, 5000
    rng = np.random.default_rng(7)

    def make(ops_a):
        # B(:,j) selects one A column with ops_a[j] rows: Op_j = ops_a[j]
        a_cp = np.zeros(n + 1, np.int64)
        a_cp[1:] = np.cumsum(ops_a)
        ari = np.concatenate([rng.choice(m, int(z), replace=False) for z in ops_a]).astype(np.int32)
        A = gen.CSC(m, n, a_cp.astype(np.int32), ari, rng.uniform(-1, 1, int(a_cp[-1])))
        B = gen.CSC(n, n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32),
                    rng.uniform(-1, 1, n))
        return A, B

    # call 1: 10 columns of 4 products (lane sub-bin 0) and 45 of 8 (sub-bin 1)
    ops1 = np.zeros(n, np.int64)
    ops1[:10] = 4
    ops1[10:55] = 8
    # call 2: the same total (400) as 100 columns of 4: only sub-bin 0
    ops2 = np.zeros(n, np.int64)
    ops2[:100] = 4
    A1, B1 = make(ops1)
    A2, B2 = make(ops2)
    opts = api.options(lane_hash=True)
    At, Bt = api.CscTensor.from_host(A1), api.CscTensor.from_host(B1)
    plan, colptr, ri, v, nnz = api.multiply(At, Bt, opts)
    out = (colptr, ri, v)
    torch.cuda.synchronize()
    ocp, ori, ov = oracle.spgemm(A1, B1)
    assert nnz == ocp[-1]
    assert_same_structure(colptr.cpu().numpy(), ri[:nnz].cpu().numpy(), ocp, ori, "call 1")
    assert_values_exact(v[:nnz].cpu().numpy(), ov, "call 1")
    At2, Bt2 = api.CscTensor.from_host(A2), api.CscTensor.from_host(B2)
    for r in range(2):
        _, _, _, _, nnz2 = api.multiply(At2, Bt2, opts, plan=plan, out=out)
        torch.cuda.synchronize()
        ocp, ori, ov = oracle.spgemm(A2, B2)
        assert nnz2 == ocp[-1]
        assert_same_structure(colptr.cpu().numpy(), ri[:nnz2].cpu().numpy(), ocp, ori,
                              f"call 2.{r}")
        assert_values_exact(v[:nnz2].cpu().numpy(), ov, f"call 2.{r}")
    plan.close()


@pytest.mark.parametrize("opts", [None, dict(t_split=300)])
def test_numeric_window_without_b_entries(opts):
    """n = 2000 with B's columns 10..700 empty: inside one product tile, column
    windows of 256 columns hold no stored B entry at all (their bounds in LDS
    must not be overwritten before every wave has read them)."""
    _say(f"empty B column run, opts={opts}")
    A = gen.uniform_z(2000, 6, seed=11)
    B = gen.uniform_z(2000, 7, seed=12)
    counts = np.diff(B.colptr.astype(np.int64))
    counts[10:701] = 0
    keep = np.repeat(counts > 0, np.diff(B.colptr.astype(np.int64)))
    cp = np.zeros(B.ncols + 1, np.int64)
    cp[1:] = np.cumsum(counts)
    Be = gen.CSC(B.nrows, B.ncols, cp.astype(np.int32), B.rowidx[keep], B.val[keep])
    o = api.options(**opts) if opts else None
    check_f64(A, Be, o, "empty B column run")
    # a heavier A so the run sits inside product tiles of its neighbours
    A2 = gen.uniform_z(2000, 40, seed=13)
    check_f64(A2, Be, o, "empty B column run, 40 per column")


@pytest.mark.parametrize("opts", [dict(t_block=-1), dict(t_block=-1, hash_cap=64),
                                  dict(t_block=-1, dense_rows=1, hash_cap=256)])
def test_block_accumulator_dense_bin_size(opts):
    """The workgroup LDS accumulator (direct-indexed windows, and hash windows
    when the row span does not fit) on every non-ESC column of the dense-bin
    workload: A x A, n = 4096, 40 rows per column (1600 products per column),
    FP64 and FP32."""
    _say(f"block accumulator n=4096 z=40 {opts}")
    A = gen.uniform_z(4096, 40, seed=0)
    o = api.options(**opts)
    cp, ri, v = check_f64(A, A, o, "n=4096 z=40 block")
    (_, _, _), plan, _ = gpu_product(A, A, o, return_plan=True)
    st = plan.stats()
    plan.close()
    assert st["cols_block"] == 4096, st
    if opts.get("dense_rows") == 1:
        assert st["cols_hash"] > 0, st
    check_f32(A, A, o, "n=4096 z=40 block f32")


@pytest.mark.parametrize("opts", [dict(t_block=-1, t_esc=4), dict(t_block=-1, t_esc=32,
                                                                   hash_cap=32)])
def test_block_accumulator_forward_backward_size(opts):
    """The same accumulator on the forward/backward workload's shape: n =
    100,000, 8 per column (64 products per column), FP32; with t_esc = 4 every
    column goes to it."""
    _say(f"block accumulator n=100000 z=8 {opts}")
    A = gen.uniform_z(100_000, 8, seed=1, dist="normal", dtype=np.float32)
    B = gen.uniform_z(100_000, 8, seed=2, dist="normal", dtype=np.float32)
    o = api.options(**opts)
    check_f32(A, B, o, "n=1e5 z=8 block")
    (_, _, _), plan, _ = gpu_product(A.astype(np.float32), B.astype(np.float32), o,
                                     dtype=np.float32, return_plan=True)
    st = plan.stats()
    plan.close()
    assert st["cols_block"] > 0, st


def test_one_call_product_after_structure_change():
    """A one-call product on a plan that has run before starts its numeric
    phase at the previous structure's column positions. Here the second call
    keeps every column's product count, bin and the product total, but one
    column's two selected A columns now share all their rows (fewer output
    entries): the counts differ, the call is redone, and the result equals
    the oracle's. Then the first inputs again."""
    _say("one-call product, structure change with equal product counts")
    rng = np.random.default_rng(23)
    A = gen.uniform_z(2000, 6, seed=21)
    ri = A.rowidx.copy()
    ri[A.colptr[1]:A.colptr[2]] = ri[A.colptr[0]:A.colptr[1]]  # column 1 = column 0's rows
    A = gen.CSC(A.nrows, A.ncols, A.colptr, ri, A.val)
    B1 = gen.uniform_z(2000, 5, seed=22)
    # column 7 of B: A columns 0 and 2 (12 distinct rows), then 0 and 1 (6)
    def with_col7(B, rows):
        cp = B.colptr.astype(np.int64)
        cols = [B.rowidx[cp[j]:cp[j + 1]] for j in range(B.ncols)]
        vals = [B.val[cp[j]:cp[j + 1]] for j in range(B.ncols)]
        cols[7] = np.array(rows, np.int32)
        vals[7] = rng.uniform(-1, 1, len(rows))
        ncp = np.zeros(B.ncols + 1, np.int64)
        ncp[1:] = np.cumsum([len(c) for c in cols])
        return gen.CSC(B.nrows, B.ncols, ncp.astype(np.int32), np.concatenate(cols),
                       np.concatenate(vals))
    Ba, Bb = with_col7(B1, [0, 2]), with_col7(B1, [0, 1])
    At = api.CscTensor.from_host(A)
    plan, out = None, None
    for step, B in enumerate((Ba, Ba, Bb, Bb, Ba)):
        Bt = api.CscTensor.from_host(B)
        plan, colptr, ri_, v, nnz = api.multiply(At, Bt, plan=plan, out=out)
        out = (colptr, ri_, v)
        torch.cuda.synchronize()
        ocp, ori, ov = oracle.spgemm(A, B)
        assert nnz == int(ocp[-1]), f"step {step}"
        assert_same_structure(colptr.cpu().numpy(), ri_[:nnz].cpu().numpy(), ocp, ori,
                              f"step {step}")
        assert_values_exact(v[:nnz].cpu().numpy(), ov, f"step {step}")
    plan.close()


def test_one_call_heavy_windows_outgrow_the_plan():
    """One-call products on a reused plan whose heavy columns (above 1024
    products) need more row windows than the previous call planned: the heavy
    plan maps only the windows the scratch holds and asks for a redo, which
    grows the scratch. Then the smaller structure again. Every result equals
    the oracle's."""
    _say("one-call product, heavy windows outgrow the plan")
    A = gen.uniform_z(4000, 20, seed=31)
    B_small = gen.uniform_z(30, 60, seed=32, nrows=4000)   # 1200 products: 2 windows per column
    B_large = gen.uniform_z(30, 200, seed=33, nrows=4000)  # 4000 products: 5 windows per column
    At = api.CscTensor.from_host(A)
    plan, out = None, None
    for B in (B_small, B_small, B_large, B_large, B_small):
        Bt = api.CscTensor.from_host(B)
        plan, colptr, ri_, v, nnz = api.multiply(At, Bt, plan=plan, out=out)
        out = (colptr, ri_, v)
        torch.cuda.synchronize()
        ocp, ori, ov = oracle.spgemm(A, B)
        assert_same_structure(colptr.cpu().numpy(), ri_[:nnz].cpu().numpy(), ocp, ori, "heavy windows")
        assert_values_exact(v[:nnz].cpu().numpy(), ov, "heavy windows")
    plan.close()
