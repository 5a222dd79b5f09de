"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these compares the oracle with itself: each check uses a printed
example (Figures 1 and 2), a closed form, an identity, or an independent
brute-force / library computation on small inputs.
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from paper_2303_02471_amd import inputs as gen


def _read_fig1(path):
    mats, cur = {}, None
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line in ("A", "B", "C"):
            cur = line
            mats[cur] = []
            continue
        mats[cur].append([float(x) for x in line.split()])
    return {k: np.array(v) for k, v in mats.items()}


def _pattern(a):
    d = np.zeros((a.nrows, a.ncols), dtype=np.int64)
    col = np.repeat(np.arange(a.ncols), np.diff(a.colptr.astype(np.int64)))
    d[a.rowidx.astype(np.int64), col] = 1
    return d


def _dense_from_oracle(m, n, cp, ri, v):
    d = np.zeros((m, n))
    col = np.repeat(np.arange(n), np.diff(cp.astype(np.int64)))
    d[ri.astype(np.int64), col] = v
    return d


def _assert_sorted_columns(cp, ri):
    for j in range(len(cp) - 1):
        seg = ri[cp[j]:cp[j + 1]]
        assert np.all(np.diff(seg) > 0), f"column {j} not strictly ascending"


# --------------------------------------------------------------------------- Figure 1

def test_figure1_worked_example(golden_dir):
    m = _read_fig1(os.path.join(golden_dir, "fig1_gustavson_4x4.txt"))
    A, B = gen.from_dense(m["A"]), gen.from_dense(m["B"])
    cp, ri, v = oracle.spgemm(A, B)
    assert np.array_equal(_dense_from_oracle(4, 4, cp, ri, v), m["C"])
    # structure: column 0 has no product landing on row 2, column 1 none on
    # row 1, column 2 none on row 3, column 3 is full
    assert cp.tolist() == [0, 3, 6, 9, 13]
    assert ri.tolist() == [0, 1, 3, 0, 2, 3, 0, 1, 2, 0, 1, 2, 3]
    # Op_j of Section 3.1 on this example
    assert oracle.opcount(A, B).tolist() == [3, 4, 4, 6]
    # column 1 is 1 * A(:,0) + 3 * A(:,2) as the figure draws it
    col1 = 1 * m["A"][:, 0] + 3 * m["A"][:, 2]
    assert np.array_equal(col1, m["C"][:, 1])


def test_figure1_input_order_free(golden_dir):
    m = _read_fig1(os.path.join(golden_dir, "fig1_gustavson_4x4.txt"))
    A, B = gen.from_dense(m["A"]), gen.from_dense(m["B"])
    for seed in range(5):
        cp, ri, v = oracle.spgemm(gen.shuffle_within_columns(A, seed),
                                  gen.shuffle_within_columns(B, seed + 100))
        assert np.array_equal(_dense_from_oracle(4, 4, cp, ri, v), m["C"])


# --------------------------------------------------------------------------- Figure 2

def _read_kv(path):
    out = {}
    for line in open(path):
        line = line.strip()
        if line and not line.startswith("#"):
            k, *vals = line.split()
            out[k] = [int(x) for x in vals]
    return out


def test_figure2_block_costs(golden_dir):
    f = _read_kv(os.path.join(golden_dir, "fig2_block_costs.txt"))
    ops = np.array(f["ops"], dtype=np.int64)
    # SPA: one vector instruction per stored B entry
    assert sum(f["bnnz"]) == f["spa_instructions"][0]
    # the columns are already in decreasing order: sorting keeps them
    assert oracle.sort_columns(ops).tolist() == list(range(6))

    def cost(starts):
        return sum(int(ops[s:e].max()) for s, e in zip(starts[:-1], starts[1:]))

    one = oracle.blocking(ops, 6, 6)
    assert one.tolist() == [0, 6] and cost(one) == f["spars_one_block"][0]
    two = oracle.blocking(ops, 3, 3)
    assert two.tolist() == [0, 3, 6] and cost(two) == f["spars_two_blocks_of_3"][0]


def test_blocking_rule_brute_force():
    """Blocking Algorithm (Section 3.1) against a direct reading of its three steps."""
    rng = np.random.default_rng(7)
    for _ in range(300):
        n = int(rng.integers(1, 40))
        ops = np.sort(rng.integers(0, 6, size=n))[::-1].astype(np.int64)
        bmin = int(rng.integers(1, 6))
        bmax = int(rng.integers(bmin, 10))
        starts = oracle.blocking(ops, bmin, bmax).tolist()
        # independent reading: every block has >= min(bmin, remaining) columns,
        # <= bmax columns; columns beyond the first bmin share the first's Op;
        # a block stops growing only at bmax, at n, or at a different Op
        assert starts[0] == 0 and starts[-1] == n
        for s, e in zip(starts[:-1], starts[1:]):
            size = e - s
            assert min(bmin, n - s) <= size <= bmax
            assert all(ops[t] == ops[s] for t in range(s + bmin, e))
            if e < n and size >= bmin and size < bmax:
                assert ops[e] != ops[s]


def test_sort_columns_stable_decreasing():
    rng = np.random.default_rng(3)
    op = rng.integers(0, 5, size=500).astype(np.int64)
    perm = oracle.sort_columns(op)
    assert np.array_equal(perm, np.lexsort((np.arange(500), -op)))


@pytest.mark.parametrize("maxop,h", [(1, 2), (2, 4), (3, 4), (15, 16), (16, 32), (1000, 1024),
                                     (1024, 2048), (0, 0)])
def test_hash_size_rule(maxop, h):
    """Section 3.2: H = 2^k with 2^(k-1) <= max Op < 2^k."""
    assert oracle.hash_size(maxop) == h
    if h:
        assert h // 2 <= maxop < h


# --------------------------------------------------------------------------- brute force

@pytest.mark.parametrize("dist", ["int", "uniform"])
def test_brute_force_tiny(dist):
    """Thousands of tiny random pairs against dense products done in numpy."""
    rng = np.random.default_rng(11 if dist == "int" else 12)
    for trial in range(1500):
        m, k, n = (int(x) for x in rng.integers(0, 9, size=3))
        dens = float(rng.choice([0.0, 0.15, 0.4, 0.8, 1.0]))
        A = gen.random_tiny(rng, m, k, dens, dist)
        B = gen.random_tiny(rng, k, n, float(rng.choice([0.0, 0.2, 0.5, 1.0])), dist)
        cp, ri, v = oracle.spgemm(A, B)
        _assert_sorted_columns(cp, ri)
        # structure = boolean product of the stored patterns
        pat = (_pattern(A) @ _pattern(B)) > 0
        got = np.zeros((m, n), dtype=bool)
        col = np.repeat(np.arange(n), np.diff(cp.astype(np.int64)))
        got[ri.astype(np.int64), col] = True
        assert np.array_equal(got, pat), trial
        # nnz per column from the symbolic pass
        assert np.array_equal(np.diff(oracle.symbolic(A, B)), pat.sum(axis=0))
        dense = gen.to_dense(A) @ gen.to_dense(B)
        mine = _dense_from_oracle(m, n, cp, ri, v)
        if dist == "int":
            assert np.array_equal(mine, dense), trial  # exact in any order
        else:
            s, t = oracle.absprod(A, B, cp, ri)
            bound = (t + 1) * 2.0 ** -52 * s
            assert np.all(np.abs(v - dense[ri, col]) <= bound + 1e-300), trial
        # Op_j = number of products
        op = oracle.opcount(A, B)
        assert np.array_equal(op, (_pattern(A).sum(axis=0) @ _pattern(B)).astype(np.int64))


def test_against_scipy_medium():
    """Medium random pairs against an independent library product."""
    rng = np.random.default_rng(5)
    for _ in range(20):
        m, k, n = (int(x) for x in rng.integers(50, 400, size=3))
        A = gen.random_tiny(rng, m, k, float(rng.uniform(0.005, 0.05)), "uniform")
        B = gen.random_tiny(rng, k, n, float(rng.uniform(0.005, 0.05)), "uniform")
        cp, ri, v = oracle.spgemm(A, B)
        sa = sp.csc_matrix((A.val, A.rowidx, A.colptr), shape=(m, k))
        sb = sp.csc_matrix((B.val, B.rowidx, B.colptr), shape=(k, n))
        pa = sp.csc_matrix((np.ones(A.nnz), A.rowidx, A.colptr), shape=(m, k))
        pb = sp.csc_matrix((np.ones(B.nnz), B.rowidx, B.colptr), shape=(k, n))
        pc = (pa @ pb).tocsc()
        pc.sort_indices()
        assert np.array_equal(pc.indptr, cp) and np.array_equal(pc.indices, ri)
        sc = (sa @ sb).toarray()
        col = np.repeat(np.arange(n), np.diff(cp))
        s, t = oracle.absprod(A, B, cp, ri)
        assert np.all(np.abs(v - sc[ri, col]) <= (t + 1) * 2.0 ** -52 * s + 1e-300)


# --------------------------------------------------------------------------- invariants

def _oracle_dense(A, B):
    cp, ri, v = oracle.spgemm(A, B)
    return _dense_from_oracle(A.nrows, B.ncols, cp, ri, v), cp, ri


def test_identity_and_permutation_factors():
    rng = np.random.default_rng(9)
    A = gen.random_tiny(rng, 60, 70, 0.08, "uniform")
    dA = gen.to_dense(A)
    d, cp, ri = _oracle_dense(A, gen.identity(70))
    assert np.array_equal(d, dA)                              # A I = A (values exact: x*1)
    d, _, _ = _oracle_dense(gen.identity(60), A)
    assert np.array_equal(d, dA)                              # I A = A
    perm = rng.permutation(70)
    d, _, _ = _oracle_dense(A, gen.permutation(perm))
    assert np.array_equal(d, dA[:, perm])                     # A P selects columns
    perm2 = rng.permutation(60)
    d, _, _ = _oracle_dense(gen.permutation(perm2), A)
    P = np.zeros((60, 60))
    P[perm2, np.arange(60)] = 1
    assert np.array_equal(d, P @ dA)                          # P A permutes rows


def _transpose(a):
    return gen.from_dense(gen.to_dense(a).T) if a.nnz else gen.CSC(
        a.ncols, a.nrows, np.zeros(a.nrows + 1, np.int32), np.zeros(0, np.int32), np.zeros(0))


def test_transpose_identity():
    """(AB)^T = B^T A^T: structure exact, values exact on integer inputs."""
    rng = np.random.default_rng(21)
    for _ in range(30):
        m, k, n = (int(x) for x in rng.integers(1, 40, size=3))
        A = gen.random_tiny(rng, m, k, 0.2, "int")
        B = gen.random_tiny(rng, k, n, 0.2, "int")
        # explicit zeros would vanish in a dense round trip: drop them first
        A = gen.from_dense(gen.to_dense(A))
        B = gen.from_dense(gen.to_dense(B))
        d1, cp1, ri1 = _oracle_dense(A, B)
        d2, cp2, ri2 = _oracle_dense(_transpose(B), _transpose(A))
        assert np.array_equal(d1.T, d2)
        p1 = np.zeros((m, n), bool)
        p1[ri1, np.repeat(np.arange(n), np.diff(cp1))] = True
        p2 = np.zeros((n, m), bool)
        p2[ri2, np.repeat(np.arange(m), np.diff(cp2))] = True
        assert np.array_equal(p1.T, p2)


def test_explicit_zeros_and_cancellation_kept():
    """Stored zeros and cancelling sums stay structural (SPA flags ignore values)."""
    # A(:,0) = [1, 1], A(:,1) = [1, 1]; B(:,0) = [1, -1] -> C(:,0) = [0, 0], both stored
    A = gen.CSC(2, 2, np.array([0, 2, 4], np.int32), np.array([0, 1, 1, 0], np.int32),
                np.array([1.0, 1.0, 1.0, 1.0]))
    B = gen.CSC(2, 1, np.array([0, 2], np.int32), np.array([0, 1], np.int32),
                np.array([1.0, -1.0]))
    cp, ri, v = oracle.spgemm(A, B)
    assert cp.tolist() == [0, 2] and ri.tolist() == [0, 1] and v.tolist() == [0.0, 0.0]
    # a stored zero in B still creates structure
    B0 = gen.CSC(2, 1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([0.0]))
    cp, ri, v = oracle.spgemm(A, B0)
    assert ri.tolist() == [0, 1] and v.tolist() == [0.0, 0.0]


def test_empty_and_degenerate_shapes():
    for (m, k, n) in [(0, 0, 0), (3, 0, 4), (0, 5, 2), (4, 3, 0), (1, 1, 1)]:
        A = gen.CSC(m, k, np.zeros(k + 1, np.int32), np.zeros(0, np.int32), np.zeros(0))
        B = gen.CSC(k, n, np.zeros(n + 1, np.int32), np.zeros(0, np.int32), np.zeros(0))
        cp, ri, v = oracle.spgemm(A, B)
        assert cp.tolist() == [0] * (n + 1) and len(ri) == 0


def test_invalid_inputs_rejected():
    good = gen.identity(3)
    bad_start = gen.CSC(3, 3, np.array([1, 1, 2, 3], np.int32), np.arange(3, dtype=np.int32), np.ones(3))
    dup = gen.CSC(3, 1, np.array([0, 2], np.int32), np.array([1, 1], np.int32), np.ones(2))
    oob = gen.CSC(3, 1, np.array([0, 1], np.int32), np.array([3], np.int32), np.ones(1))
    dec = gen.CSC(3, 2, np.array([0, 2, 1], np.int32), np.array([0, 1], np.int32), np.ones(2))
    for b in (bad_start, dup, oob, dec):
        assert oracle.check_csc(b) != 0
        with pytest.raises(oracle.OracleError):
            oracle.spgemm(good, b)
        with pytest.raises(oracle.OracleError):
            oracle.spgemm(b if b.ncols == 3 else gen.identity(3), good) if b.ncols == 3 else \
                oracle.spgemm(gen.identity(3), b)
    with pytest.raises(oracle.OracleError):
        oracle.spgemm(gen.identity(3), gen.identity(4))  # shape mismatch


# --------------------------------------------------------------------------- closed forms

def test_constant_z_opcount():
    """Section 5.2: Z non-zeros in every column of A and B give Op_j = Z^2."""
    for z in (2, 4, 5, 8):
        A = gen.uniform_z(300, z, seed=z)
        assert np.all(oracle.opcount(A, A) == z * z)
    A = gen.diag_plus_random(1000, 4, seed=0)
    assert np.all(oracle.opcount(A, A) == 25)


def test_laplacian_squared_closed_form():
    """L = 4I - Adj on a 64 x 64 grid: L^2 = 16 I - 8 Adj + Adj^2, i.e. diagonal
    16 + deg(v), axis neighbours -8, diagonal neighbours +2, axis distance-2
    neighbours +1; every node within graph distance 2 is stored."""
    g = 64
    L = gen.laplacian_2d(g)
    cp, ri, v = oracle.spgemm(L, L)
    n = g * g
    expect = {}
    for y in range(g):
        for x in range(g):
            vtx = x + g * y
            deg = (x > 0) + (x < g - 1) + (y > 0) + (y < g - 1)
            for dy in range(-2, 3):
                for dx in range(-2, 3):
                    if abs(dx) + abs(dy) > 2:
                        continue
                    xx, yy = x + dx, y + dy
                    if not (0 <= xx < g and 0 <= yy < g):
                        continue
                    w = xx + g * yy
                    dist = abs(dx) + abs(dy)
                    if dist == 0:
                        val = 16 + deg
                    elif dist == 1:
                        val = -8
                    elif dx != 0 and dy != 0:
                        val = 2
                    else:
                        val = 1
                    expect[(w, vtx)] = float(val)
    assert int(cp[-1]) == len(expect) == 51972
    col = np.repeat(np.arange(n), np.diff(cp))
    got = {(int(i), int(j)): float(x) for i, j, x in zip(ri, col, v)}
    assert got == expect


# --------------------------------------------------------------------------- gradients

def test_backward_finite_differences():
    """L(A,B) = <G, AB> is bilinear, so a central difference in one stored value
    is its derivative up to rounding."""
    n, z = 200, 8
    A = gen.uniform_z(n, z, seed=1, dist="normal")
    B = gen.uniform_z(n, z, seed=2, dist="normal")
    cp, ri, v = oracle.spgemm(A, B)
    G = gen.gradient_values(int(cp[-1]), seed=3, dtype=np.float64)
    dA, dB = oracle.backward(A, B, cp, ri, G)
    h = 2.0 ** -10

    def loss(a, b):
        c = oracle.spgemm(a, b)
        assert np.array_equal(c[0], cp) and np.array_equal(c[1], ri)
        return float(np.dot(G, c[2]))

    rng = np.random.default_rng(4)
    for which, M, grad in (("A", A, dA), ("B", B, dB)):
        for q in rng.choice(M.nnz, size=60, replace=False):
            vp, vm = M.val.copy(), M.val.copy()
            vp[q] += h
            vm[q] -= h
            Mp = gen.CSC(M.nrows, M.ncols, M.colptr, M.rowidx, vp)
            Mm = gen.CSC(M.nrows, M.ncols, M.colptr, M.rowidx, vm)
            if which == "A":
                fd = (loss(Mp, B) - loss(Mm, B)) / (2 * h)
            else:
                fd = (loss(A, Mp) - loss(A, Mm)) / (2 * h)
            assert abs(fd - grad[q]) <= 1e-9 * max(1.0, abs(grad[q])), (which, q, fd, grad[q])


def test_backward_dense_reference():
    """dA = (G B^T) on A's pattern, dB = (A^T G) on B's pattern, in dense numpy."""
    rng = np.random.default_rng(8)
    for _ in range(40):
        m, k, n = (int(x) for x in rng.integers(1, 30, size=3))
        A = gen.random_tiny(rng, m, k, 0.3, "uniform")
        B = gen.random_tiny(rng, k, n, 0.3, "uniform")
        cp, ri, v = oracle.spgemm(A, B)
        G = rng.standard_normal(int(cp[-1]))
        dA, dB = oracle.backward(A, B, cp, ri, G)
        Gd = _dense_from_oracle(m, n, cp, ri, G)
        ref_a = Gd @ gen.to_dense(B).T
        ref_b = gen.to_dense(A).T @ Gd
        colA = np.repeat(np.arange(k), np.diff(A.colptr))
        colB = np.repeat(np.arange(n), np.diff(B.colptr))
        np.testing.assert_allclose(dA, ref_a[A.rowidx, colA], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(dB, ref_b[B.rowidx, colB], rtol=1e-12, atol=1e-12)


def test_f32_twin_matches_f64_within_bound():
    """The single-precision twin stays within the rounding bound of the double oracle."""
    A = gen.uniform_z(500, 8, seed=1, dist="normal", dtype=np.float32)
    B = gen.uniform_z(500, 8, seed=2, dist="normal", dtype=np.float32)
    cp, ri, v64 = oracle.spgemm(A, B, "f64")
    cp2, ri2, v32 = oracle.spgemm(A, B, "f32")
    assert np.array_equal(cp, cp2) and np.array_equal(ri, ri2)
    s, t = oracle.absprod(A, B, cp, ri)
    u = 2.0 ** -24
    assert np.all(np.abs(v32.astype(np.float64) - v64) <= (t + 1) * u * s * 1.01 + 1e-30)


# --------------------------------------------------------------------------- parallel oracle

@pytest.mark.parametrize("nthreads", [1, 3, 0])
def test_parallel_oracle_identical(nthreads):
    """The OpenMP oracle spreads whole columns over threads (each column still
    Algorithm 1 on one thread): output identical bit for bit, including
    empty columns, rectangular shapes and a size hint that is too small."""
    cases = [gen.powerlaw(20000, seed=5), (gen.uniform_z(3000, 7, seed=1),
                                           gen.uniform_z(3000, 9, seed=2))]
    for A, B in cases:
        ref = oracle.spgemm(A, B)
        for hint in (0, 5):
            cp, ri, v, used = oracle.spgemm_parallel(A, B, nthreads, nnz_hint=hint)
            assert used >= 1 and (nthreads == 0 or used == nthreads)
            assert np.array_equal(cp, ref[0]) and np.array_equal(ri, ref[1])
            assert np.array_equal(v.view(np.uint64), ref[2].view(np.uint64))
    A = gen.from_dense(np.array([[1.0, 0.0], [0.0, 0.0], [2.0, 3.0]]))
    B = gen.from_dense(np.array([[0.0, 1.0, 0.0], [0.0, 2.0, 0.0]]))
    ref = oracle.spgemm(A, B)
    cp, ri, v, _ = oracle.spgemm_parallel(A, B, nthreads)
    assert np.array_equal(cp, ref[0]) and np.array_equal(ri, ref[1]) and np.array_equal(v, ref[2])
