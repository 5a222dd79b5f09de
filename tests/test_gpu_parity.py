"""Parity of the HIP path with the CPU oracle (element by element).

Structure (column pointers, ascending rows) must be identical; FP64 values
must be bit-identical (and so inside the stated 1e-12 relative tolerance);
FP32 values must equal the oracle's single-precision twin and stay inside the
float32 rounding bound of the double oracle.
"""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2303_02471_amd import inputs as gen
from helpers import (HAVE_GPU, assert_same_structure, assert_values_exact, check_f32, check_f64,
                     gpu_product)

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not HAVE_GPU, reason="needs an MI355X GPU")]


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def _fig1():
    here = os.path.join(os.path.dirname(__file__), "golden", "fig1_gustavson_4x4.txt")
    mats, cur = {}, None
    for line in open(here):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line in ("A", "B", "C"):
            cur = line
            mats[cur] = []
        else:
            mats[cur].append([float(x) for x in line.split()])
    return {k: np.array(v) for k, v in mats.items()}


def test_figure1_on_gpu():
    _say("figure 1 4x4")
    m = _fig1()
    A, B = gen.from_dense(m["A"]), gen.from_dense(m["B"])
    cp, ri, v = gpu_product(A, B)
    d = np.zeros((4, 4))
    d[ri, np.repeat(np.arange(4), np.diff(cp))] = v
    assert np.array_equal(d, m["C"])
    assert cp.tolist() == [0, 3, 6, 9, 13]


def test_tiny_random_many():
    rng = np.random.default_rng(123)
    for trial in range(150):
        m, k, n = (int(x) for x in rng.integers(1, 40, size=3))
        dist = "int" if trial % 2 else "uniform"
        A = gen.random_tiny(rng, m, k, float(rng.choice([0.05, 0.2, 0.5, 1.0])), dist)
        B = gen.random_tiny(rng, k, n, float(rng.choice([0.05, 0.2, 0.5, 1.0])), dist)
        _say(f"tiny trial {trial} m={m} k={k} n={n} nnzA={A.nnz} nnzB={B.nnz}")
        check_f64(A, B, what=f"tiny {trial}")


def test_config1_diag_plus_random():
    _say("diag+4 random n=1000")
    A = gen.diag_plus_random(1000, 4, seed=0)
    check_f64(A, A, what="config 1")


def test_laplacian_squared():
    _say("laplacian 64x64 squared")
    L = gen.laplacian_2d(64)
    cp, ri, v = check_f64(L, L, what="laplacian")
    assert int(cp[-1]) == 51972


def test_dense_bin_n4096_z40():
    _say("n=4096 z=40 (dense accumulator)")
    A = gen.uniform_z(4096, 40, seed=0)
    check_f64(A, A, what="n4096 z40")


def test_powerlaw_reduced():
    _say("power law n=50000")
    A, B = gen.powerlaw(50_000, seed=1)
    check_f64(A, B, what="powerlaw 50k")


@pytest.mark.parametrize("opts", [
    dict(t_esc=4), dict(t_esc=16, hash_cap=128), dict(t_esc=256, hash_cap=16, t_block=-1),
    dict(t_dense=100000, t_block=-1), dict(dense_rows=1, t_block=600), dict(t_esc=4, dense_rows=64),
    dict(t_split=-1), dict(t_split=1), dict(t_esc=4, t_split=300, hash_cap=64, t_block=-1),
    dict(t_esc=16, t_split=1, t_dense=100000, t_block=1000), dict(hash_cap=16, t_dense=100000),
    dict(t_esc=4, hash_cap=16, dense_rows=1, t_block=-1), dict(t_block=-1), dict(t_block=512),
    dict(t_block=4096, hash_cap=300), dict(lane_hash=True), dict(lane_hash=True, t_esc=16),
    dict(one_stream=True), dict(one_stream=True, t_esc=32), dict(one_stream=True, lane_hash=True)])
def test_forced_bins_identical(opts):
    """Any split of the work between accumulators gives the same bits (the
    t = 0 / t = infinity limits of Section 3.3 and everything between)."""
    from paper_2303_02471_amd import api
    _say(f"forced bins {opts}")
    rng = np.random.default_rng(5)
    cases = [gen.uniform_z(3000, 12, seed=3), gen.powerlaw(20_000, seed=2)[0],
             gen.random_tiny(rng, 300, 300, 0.2, "uniform")]
    for A in cases:
        ocp, ori, ov = oracle.spgemm(A, A)
        cp, ri, v = gpu_product(A, A, api.options(**opts))
        assert_same_structure(cp, ri, ocp, ori, str(opts))
        assert_values_exact(v, ov, str(opts))


def test_input_order_free():
    _say("shuffled storage order")
    A = gen.uniform_z(2000, 9, seed=4)
    B = gen.uniform_z(2000, 7, seed=5)
    ocp, ori, ov = oracle.spgemm(A, B)
    As, Bs = gen.shuffle_within_columns(A, 1), gen.shuffle_within_columns(B, 2)
    ocp2, ori2, ov2 = oracle.spgemm(As, Bs)
    cp, ri, v = gpu_product(As, Bs)
    assert_same_structure(cp, ri, ocp, ori, "shuffled")
    assert_values_exact(v, ov2, "shuffled")


def test_rectangular_and_empty():
    rng = np.random.default_rng(9)
    for (m, k, n) in [(1, 1, 1), (7, 300, 5), (500, 3, 800), (1000, 1000, 1), (3, 5, 0),
                      (0, 5, 3), (4, 0, 6)]:
        _say(f"rect m={m} k={k} n={n}")
        A = gen.random_tiny(rng, m, k, 0.3, "uniform") if m and k else gen.CSC(
            m, k, np.zeros(k + 1, np.int32), np.zeros(0, np.int32), np.zeros(0))
        B = gen.random_tiny(rng, k, n, 0.3, "uniform") if k and n else gen.CSC(
            k, n, np.zeros(n + 1, np.int32), np.zeros(0, np.int32), np.zeros(0))
        check_f64(A, B, what=f"rect {m}x{k}x{n}")


def test_empty_columns_and_empty_a_columns():
    _say("empty columns in A and B")
    rng = np.random.default_rng(3)
    A = gen.random_tiny(rng, 200, 150, 0.02, "uniform")  # many empty A columns
    B = gen.random_tiny(rng, 150, 180, 0.05, "uniform")
    check_f64(A, B, what="empties")


def test_deterministic_reruns():
    _say("determinism")
    A, B = gen.powerlaw(30_000, seed=7)
    r1 = gpu_product(A, B)
    r2 = gpu_product(A, B)
    for x, y in zip(r1, r2):
        assert np.array_equal(x, y)


def test_f32_config_small():
    _say("f32 n=20000 z=8")
    A = gen.uniform_z(20_000, 8, seed=11, dist="normal", dtype=np.float32)
    B = gen.uniform_z(20_000, 8, seed=12, dist="normal", dtype=np.float32)
    rel = check_f32(A, B, what="f32")
    print("max rel err f32 vs f64 oracle", rel)


def test_f32_dense_and_hash():
    _say("f32 dense + hash")
    A = gen.uniform_z(4096, 40, seed=1, dtype=np.float32)
    check_f32(A, A, what="f32 dense")
    P, Q = gen.powerlaw(20_000, seed=3, dtype=np.float32)
    check_f32(P, Q, what="f32 powerlaw")


def test_stats_reported():
    from paper_2303_02471_amd import api
    _say("plan stats")
    A, B = gen.powerlaw(20_000, seed=5)
    _, plan, _ = gpu_product(A, B, return_plan=True)
    st = plan.stats()
    op = oracle.opcount(A, B)
    assert st["total_products"] == int(op.sum())
    assert st["ncols"] == 20_000
    assert st["cols_empty"] == int((op == 0).sum())
    assert st["cols_empty"] + st["cols_esc"] + st["cols_sort"] + st["cols_block"] == 20_000
    assert st["cols_esc"] == int(((op > 0) & (op <= 256)).sum())
    assert st["cols_sort"] == int((op > 256).sum())
    assert st["cols_block"] == 0
    # every workgroup column has at least one row window
    assert st["cols_direct"] + st["cols_hash"] >= st["cols_block"]
    nnz_c = int(oracle.symbolic(A, B)[-1])
    assert st["nnz_c"] == nnz_c
    # products beyond the first of every output entry
    assert st["later_products"] == int(op.sum()) - nnz_c


def _csc_from_columns(m, cols, rng, dtype=np.float64):
    """CSC with the given row lists per column (storage order kept), U[-1, 1]."""
    counts = np.array([len(c) for c in cols], dtype=np.int64)
    cp = np.zeros(len(cols) + 1, dtype=np.int64)
    np.cumsum(counts, out=cp[1:])
    ri = np.concatenate([np.asarray(c, dtype=np.int64) for c in cols]) if len(cols) else \
        np.zeros(0, np.int64)
    val = rng.uniform(-1.0, 1.0, size=len(ri)).astype(dtype)
    return gen.CSC(m, len(cols), cp.astype(np.int32), ri.astype(np.int32), val)


@pytest.mark.parametrize("opts", [dict(), dict(t_block=4096), dict(t_block=4096, t_dense=100000),
                                  dict(t_block=4096, hash_cap=512)])
def test_heavy_columns_streamed(opts):
    """Heavy columns (up to 24000 products): the row-windowed sort by default;
    with t_block the hash accumulator, whose columns above its register
    capacity stream their rows again for every pass. With many repeated rows
    (20000 products over 20000 rows) most products are later products."""
    from paper_2303_02471_amd import api
    _say(f"heavy streamed columns {opts}")
    rng = np.random.default_rng(11)
    A = gen.uniform_z(20000, 40, seed=11)
    degs = [8] * 200 + [100, 200, 310, 500, 600, 600]
    cols = [rng.choice(20000, size=d, replace=False) for d in degs]
    B = _csc_from_columns(20000, cols, rng)
    ocp, ori, ov = oracle.spgemm(A, B)
    (cp, ri, v), plan, _ = gpu_product(A, B, api.options(**opts), return_plan=True)
    assert_same_structure(cp, ri, ocp, ori, str(opts))
    assert_values_exact(v, ov, str(opts))
    st = plan.stats()
    plan.close()
    assert st["later_max"] >= 2


def test_clustered_rows_split():
    """Rows packed at the end of a wide row span crowd a few home slots of the
    order-preserving hash: the window overruns its table and is split in
    halves until the rows fit; results are unchanged."""
    from paper_2303_02471_amd import api
    _say("clustered rows: window splits")
    rng = np.random.default_rng(12)
    m = 100_000
    acols = []
    for _ in range(2000):
        rows = np.concatenate([rng.choice(np.arange(m - 300, m), size=40, replace=False), [0]])
        rng.shuffle(rows)
        acols.append(rows)
    A = _csc_from_columns(m, acols, rng)
    B = _csc_from_columns(2000, [rng.choice(2000, size=60, replace=False) for _ in range(200)],
                          rng)
    ocp, ori, ov = oracle.spgemm(A, B)
    for opts in (dict(t_block=-1), dict(t_block=-1, t_dense=100000)):
        (cp, ri, v), plan, _ = gpu_product(A, B, api.options(**opts), return_plan=True)
        assert_same_structure(cp, ri, ocp, ori, f"clustered {opts}")
        assert_values_exact(v, ov, f"clustered {opts}")
        st = plan.stats()
        plan.close()
        assert st["cols_split"] > 0


def test_repeated_row_heavy_column():
    """One row reached by more than 4096 products of a column: the windowed
    sort splits its row window down to that single row, which is one entry
    whose products take their occurrence indices in product order."""
    _say("one row in 4500 products of a column")
    rng = np.random.default_rng(13)
    m = 50_000
    acols = []
    for _ in range(5000):
        rows = np.concatenate([[5], rng.choice(np.arange(10, m), size=2, replace=False)])
        rng.shuffle(rows)
        acols.append(rows)
    A = _csc_from_columns(m, acols, rng)
    B = _csc_from_columns(5000, [rng.choice(5000, size=d, replace=False)
                                 for d in (4500, 3000, 7, 1600)], rng)
    check_f64(A, B, what="repeated row")


def test_planned_launch_and_retry():
    """A plan that has run before launches its symbolic phase from the previous
    sizes; when the device finds other sizes (another product count, or the
    same count spread over other bins) the phase is redone. Results always
    equal the oracle's."""
    import torch
    from paper_2303_02471_amd import api
    _say("planned symbolic launches, reuse and retry")
    rng = np.random.default_rng(17)
    A = gen.uniform_z(1000, 10, seed=7)
    # two columns of 100 products; then 190 + 10 products (same total, other
    # bins); then another product count; then the first pair again
    B1 = _csc_from_columns(1000, [rng.choice(1000, 10, replace=False) for _ in range(2)], rng)
    B2 = _csc_from_columns(1000, [rng.choice(1000, 19, replace=False),
                                  rng.choice(1000, 1, replace=False)], rng)
    B3 = gen.uniform_z(1000, 6, seed=8, nrows=1000)
    At = api.CscTensor.from_host(A)
    plan = None
    for B in (B1, B1, B2, B3, B1, B1):
        Bt = api.CscTensor.from_host(B)
        plan, colptr, nnz = api.symbolic(At, Bt, torch.float64, None, plan=plan)
        ri = torch.empty(nnz, dtype=torch.int32, device="cuda")
        v = torch.empty(nnz, dtype=torch.float64, device="cuda")
        api.numeric(plan, At.val, Bt.val, ri, v)
        torch.cuda.synchronize()
        ocp, ori, ov = oracle.spgemm(A, B)
        assert_same_structure(colptr.cpu().numpy(), ri.cpu().numpy(), ocp, ori, "planned")
        assert_values_exact(v.cpu().numpy(), ov, "planned")
    plan.close()


@pytest.mark.parametrize("opts", [dict(), dict(t_esc=8), dict(t_block=300), dict(t_split=300),
                                  dict(lane_hash=True), dict(one_stream=True)])
def test_wide_rows(opts):
    """More than 2^24 - 1 rows: the sort bins and the wavefront sort-merge use
    64-bit keys. Columns reach every accumulator (up to about 11,000 products),
    rows spread over the whole range with some at its top and one row shared
    by many A columns (later products)."""
    from paper_2303_02471_amd import api
    _say(f"wide rows m=2^24+1000 {opts}")
    rng = np.random.default_rng(19)
    m = (1 << 24) + 1000
    acols = []
    for kk in range(3000):
        ln = int(rng.choice([1, 2, 3, 5, 8, 40]))
        rows = rng.choice(m - 1, size=ln, replace=False)
        if kk % 3 == 0:
            rows[0] = m - 1 - int(rng.integers(0, 64))  # near the top of the range
        if kk % 10 == 0:
            rows = np.concatenate([rows[rows != m - 1], [m - 1]])  # one shared row
        rng.shuffle(rows)
        acols.append(np.unique(rows) if kk % 7 == 0 else rows)
    A = _csc_from_columns(m, acols, rng)
    degs = [1, 2, 4, 8, 16, 32, 64, 120, 400, 900, 1500, 3000]
    B = _csc_from_columns(3000, [rng.choice(3000, size=d, replace=False) for d in degs * 2], rng)
    ocp, ori, ov = oracle.spgemm(A, B)
    (cp, ri, v), plan, _ = gpu_product(A, B, api.options(**opts), return_plan=True)
    assert_same_structure(cp, ri, ocp, ori, f"wide {opts}")
    assert_values_exact(v, ov, f"wide {opts}")
    st = plan.stats()
    plan.close()
    assert st["later_max"] >= 1


def test_multiply_one_call():
    """spgemm_multiply: the numeric phase queued behind a planned symbolic one
    from the previous sizes, redone when the sizes read back differ (another
    product count, the same count over other bins, the same bins with other
    output counts so other later-product counts); C arrays too small give the
    capacity status and leave the plan ready. Every result equals the oracle's."""
    import torch
    from paper_2303_02471_amd import api
    _say("one-call multiply: queued numeric, redo, capacity")
    rng = np.random.default_rng(23)
    A = gen.uniform_z(1000, 10, seed=9)
    B1 = _csc_from_columns(1000, [rng.choice(1000, 10, replace=False) for _ in range(2)], rng)
    B2 = _csc_from_columns(1000, [rng.choice(1000, 19, replace=False),
                                  rng.choice(1000, 1, replace=False)], rng)
    B4 = _csc_from_columns(1000, [rng.choice(1000, 10, replace=False) for _ in range(2)], rng)
    B3 = gen.uniform_z(1000, 6, seed=8, nrows=1000)
    At = api.CscTensor.from_host(A)
    plan, out = None, None
    seq = [B1, B1, B4, B2, B3, B3, B1]
    for step, B in enumerate(seq):
        Bt = api.CscTensor.from_host(B)
        if step == 5:
            # new values on the same pattern, through the queued numeric phase
            At.val.mul_(-0.5)
            A = gen.CSC(A.nrows, A.ncols, A.colptr, A.rowidx, A.val * -0.5)
        plan, colptr, ri, v, nnz = api.multiply(At, Bt, None, plan=plan, out=out)
        torch.cuda.synchronize()
        ocp, ori, ov = oracle.spgemm(A, B)
        assert nnz == int(ocp[-1])
        assert_same_structure(colptr.cpu().numpy(), ri[:nnz].cpu().numpy(), ocp, ori, f"step {step}")
        assert_values_exact(v[:nnz].cpu().numpy(), ov, f"step {step}")
        out = (colptr, ri, v)
    # arrays one entry short: capacity status, the binding allocates and the
    # numeric phase fills the new arrays; the next call runs normally again
    Bt = api.CscTensor.from_host(B1)
    plan, colptr, ri, v, nnz = api.multiply(At, Bt, None, plan=plan, out=out)
    short = (colptr, ri[:nnz - 1].clone(), v[:nnz - 1].clone())
    plan, colptr, ri2, v2, nnz2 = api.multiply(At, Bt, None, plan=plan, out=short)
    assert ri2.numel() == nnz2 == nnz
    ocp, ori, ov = oracle.spgemm(A, B1)
    assert_same_structure(colptr.cpu().numpy(), ri2.cpu().numpy(), ocp, ori, "capacity")
    assert_values_exact(v2.cpu().numpy(), ov, "capacity")
    plan, colptr, ri3, v3, nnz3 = api.multiply(At, Bt, None, plan=plan, out=(colptr, ri2, v2))
    torch.cuda.synchronize()
    assert_values_exact(v3[:nnz3].cpu().numpy(), ov, "after capacity")
    st = plan.stats()
    plan.close()
    assert st["later_max"] >= 1


def test_rowwise_csr_product():
    """The row-wise form on CSR operands (Section 2.1). Bit for bit equal to the
    oracle's row-wise sums, i.e. the column oracle on C^T = B^T x A^T whose CSC
    arrays are C's CSR arrays; its structure is that of the column-wise product
    and its values agree with the column-wise oracle within the stated
    tolerance (the same terms, added in another order)."""
    import torch
    from paper_2303_02471_amd import api
    rng = np.random.default_rng(21)
    for (m, k, n, dens) in [(300, 200, 250, 0.05), (7, 500, 40, 0.2), (1, 1, 1, 1.0),
                            (600, 80, 3, 0.3)]:
        _say(f"row-wise CSR m={m} k={k} n={n}")
        at = gen.random_tiny(rng, k, m, dens, "normal")  # CSC of A^T = CSR of A
        bt = gen.random_tiny(rng, n, k, dens, "normal")  # CSC of B^T = CSR of B
        ta, tb = api.CscTensor.from_host(at), api.CscTensor.from_host(bt)
        A = api.CsrTensor(m, k, ta.colptr, ta.rowidx, ta.val)
        B = api.CsrTensor(k, n, tb.colptr, tb.rowidx, tb.val)
        C = api.matmul_rowwise(A, B)
        torch.cuda.synchronize()
        rp, ci, v = C.rowptr.cpu().numpy(), C.colidx.cpu().numpy(), C.val.cpu().numpy()
        orp, oci, ov = oracle.spgemm(bt, at)
        assert_same_structure(rp, ci, orp, oci, f"row-wise {m}x{k}x{n}")
        assert_values_exact(v, ov, f"row-wise {m}x{k}x{n}")
        # against the column-wise oracle of A x B, transposed on the host
        a = gen.CSC(m, k, *_csc_of_transpose(at))
        b = gen.CSC(k, n, *_csc_of_transpose(bt))
        ccp, cri, cv = oracle.spgemm(a, b)
        dense_r = np.zeros((m, n))
        for i in range(m):
            dense_r[i, ci[rp[i]:rp[i + 1]]] = v[rp[i]:rp[i + 1]]
        dense_c = np.zeros((m, n))
        mask_c = np.zeros((m, n), bool)
        for j in range(n):
            dense_c[cri[ccp[j]:ccp[j + 1]], j] = cv[ccp[j]:ccp[j + 1]]
            mask_c[cri[ccp[j]:ccp[j + 1]], j] = True
        mask_r = np.zeros((m, n), bool)
        for i in range(m):
            mask_r[i, ci[rp[i]:rp[i + 1]]] = True
        assert np.array_equal(mask_r, mask_c), "row-wise structure differs from column-wise"
        assert np.allclose(dense_r, dense_c, rtol=1e-12, atol=1e-12)


def _csc_of_transpose(t):
    """(colptr, rowidx, val) of the CSC form of the transpose of CSC matrix t
    (entries of each output column in ascending row order)."""
    cols = np.repeat(np.arange(t.ncols), np.diff(t.colptr))
    order = np.lexsort((cols, t.rowidx))
    counts = np.bincount(t.rowidx, minlength=t.nrows)
    cp = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    return cp, cols[order].astype(np.int32), np.asarray(t.val)[order]
