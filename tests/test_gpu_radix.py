"""GPU parity of the global radix ESC (Section 4) for the heavy columns
(option SPGEMM_RADIX_ESC), element by element against the oracle.

Cases: power-law inputs with heavy columns of every size class; heavy columns
dense in a few rows (long runs of one row: the ordered sums of Algorithm 1);
a column alone above the 10,000-product group threshold; a single-row A (no
row digits at all); rows at 2^21 (the radix length switches from 5 to 6);
a planned relaunch on a changed structure; FP32.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2303_02471_amd import inputs as gen
from helpers import (HAVE_GPU, assert_same_structure, assert_values_exact, check_f32, check_f64)

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not HAVE_GPU, reason="needs an MI355X GPU")]

if HAVE_GPU:
    import torch
    from paper_2303_02471_amd import api


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def _opts(**kw):
    return api.options(radix_esc=True, **kw)


def _clustered(m, ncols_a, z, ncols_b, zb, seed, span=None):
    """A: ncols_a columns of z distinct rows drawn from the first `span` rows
    (few distinct rows: many products per output entry); B: ncols_b columns
    of zb distinct entries. Values N(0,1)."""
    rng = np.random.default_rng(seed)
    span = span or m
    a_rows = np.concatenate([np.sort(rng.choice(span, z, replace=False)) for _ in range(ncols_a)])
    A = gen.CSC(m, ncols_a, (np.arange(ncols_a + 1) * z).astype(np.int32), a_rows.astype(np.int32),
                rng.standard_normal(ncols_a * z))
    b_rows = np.concatenate([np.sort(rng.choice(ncols_a, zb, replace=False))
                             for _ in range(ncols_b)])
    B = gen.CSC(ncols_a, ncols_b, (np.arange(ncols_b + 1) * zb).astype(np.int32),
                b_rows.astype(np.int32), rng.standard_normal(ncols_b * zb))
    return A, B


@pytest.mark.parametrize("one_stream", [False, True])
def test_powerlaw_heavy_columns(one_stream):
    _say(f"radix powerlaw n=100000 one_stream={one_stream}")
    A, B = gen.powerlaw(100_000, seed=3)
    check_f64(A, B, _opts(one_stream=one_stream), "radix powerlaw")


def test_long_runs_in_few_rows():
    """Heavy columns whose products fall on 300 rows: every output entry sums
    ~20 products, in B's stored order then A's."""
    _say("radix long runs")
    A, B = _clustered(5000, 60, 250, 40, 25, seed=11, span=300)
    cp, ri, v = check_f64(A, B, _opts(), "radix long runs")
    assert np.diff(cp).min() > 0
    check_f32(A, B, _opts(), "radix long runs f32")


def test_column_above_group_threshold():
    """One B column selects 48 A columns of 250 rows (12,000 products, a group
    of its own); neighbours of 1,250 products share groups."""
    _say("radix column above the group threshold")
    rng = np.random.default_rng(5)
    A, _ = _clustered(40_000, 60, 250, 1, 1, seed=5)
    cols = [np.sort(rng.choice(60, 48, replace=False))] + \
           [np.sort(rng.choice(60, 5, replace=False)) for _ in range(30)]
    b_cp = np.concatenate([[0], np.cumsum([len(c) for c in cols])]).astype(np.int32)
    B = gen.CSC(60, len(cols), b_cp, np.concatenate(cols).astype(np.int32),
                rng.standard_normal(int(b_cp[-1])))
    check_f64(A, B, _opts(), "radix 12000-product column")


def test_single_row():
    """A has one row: every heavy column is one entry summing all its products
    (no row digits; the sort runs on the column digits only)."""
    _say("radix single row")
    rng = np.random.default_rng(9)
    k, n = 3000, 12
    A = gen.CSC(1, k, np.arange(k + 1, dtype=np.int32), np.zeros(k, np.int32),
                rng.standard_normal(k))
    cols = [np.sort(rng.choice(k, 1100 + 97 * j, replace=False)) for j in range(n)]
    b_cp = np.concatenate([[0], np.cumsum([len(c) for c in cols])]).astype(np.int32)
    B = gen.CSC(k, n, b_cp, np.concatenate(cols).astype(np.int32), rng.standard_normal(int(b_cp[-1])))
    cp, ri, v = check_f64(A, B, _opts(), "radix single row")
    assert np.array_equal(np.diff(cp), np.ones(n))


def test_rows_at_2pow21():
    """2^21 + 5 rows: 22 row bits take four rounds of 6 bits instead of five
    of 5 (the radix length the group picks)."""
    _say("radix rows 2^21")
    A, B = _clustered((1 << 21) + 5, 40, 400, 25, 6, seed=21)
    check_f64(A, B, _opts(), "radix 2^21 rows")


def test_planned_relaunch_changed_structure():
    """A plan reused on another structure of the same shapes: the launch
    planned from the first call's sizes must be redone, and both results
    match the oracle."""
    _say("radix planned relaunch")
    A1, B1 = _clustered(8000, 50, 300, 30, 9, seed=31)
    A2, B2 = _clustered(8000, 50, 300, 30, 6, seed=32)  # fits the first call's arrays
    opts = _opts()
    At, Bt = api.CscTensor.from_host(A1), api.CscTensor.from_host(B1)
    plan, colptr, ri, v, nnz = api.multiply(At, Bt, opts)
    torch.cuda.synchronize()
    ocp, ori, ov = oracle.spgemm(A1, B1)
    assert_same_structure(colptr.cpu().numpy(), ri[:nnz].cpu().numpy(), ocp, ori, "first")
    assert_values_exact(v[:nnz].cpu().numpy(), ov, "first")
    At2, Bt2 = api.CscTensor.from_host(A2), api.CscTensor.from_host(B2)
    plan, colptr2, ri2, v2, nnz2 = api.multiply(At2, Bt2, opts, plan=plan, out=(colptr, ri, v))
    torch.cuda.synchronize()
    ocp, ori, ov = oracle.spgemm(A2, B2)
    assert_same_structure(colptr2.cpu().numpy(), ri2[:nnz2].cpu().numpy(), ocp, ori, "second")
    assert_values_exact(v2[:nnz2].cpu().numpy(), ov, "second")
    plan.close()


def test_f32_powerlaw():
    _say("radix powerlaw f32")
    A, B = gen.powerlaw(50_000, seed=4)
    check_f32(A, B, _opts(), "radix powerlaw f32")
