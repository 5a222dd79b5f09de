"""Seeded synthetic CSC workloads shared by the tests, the benchmark and the oracle's checks.

This module only draws matrices. It holds none of the product's arithmetic: no
operation count, no accumulation, no output structure. Every generator returns
plain numpy arrays in CSC form (int32 ``colptr``/``rowidx``, float values) so
that the HIP path and the CPU oracle are fed byte-identical inputs.

The workload shapes follow the paper's evaluation (Section 5): square matrices,
C = A x A for the single-matrix cases, a fixed number Z of uniformly placed
non-zeros per column for the synthetic law of Section 5.2, and sparsity levels
spanning the sparse and dense ends of Table 1 (about 2 to 30 non-zeros per
column). The paper's SuiteSparse matrices are not reproduced; the power-law
workload stands in for their high-variance columns.

Row indices inside a column are distinct and stored in the order they were
drawn (CSC leaves the order inside a column free, Section 2.1).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

__all__ = [
    "CSC",
    "uniform_z",
    "diag_plus_random",
    "laplacian_2d",
    "powerlaw",
    "batched_problems",
    "gradient_values",
    "random_tiny",
    "shuffle_within_columns",
    "to_dense",
    "from_dense",
    "identity",
    "permutation",
]


@dataclass
class CSC:
    """A sparse matrix in compressed sparse column form (Section 2.1)."""

    nrows: int
    ncols: int
    colptr: np.ndarray  # int32[ncols + 1]
    rowidx: np.ndarray  # int32[nnz]
    val: np.ndarray     # float32 or float64 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.colptr[-1])

    def astype(self, dtype) -> "CSC":
        return CSC(self.nrows, self.ncols, self.colptr, self.rowidx,
                   np.ascontiguousarray(self.val.astype(dtype)))


def _colptr_from_counts(counts: np.ndarray) -> np.ndarray:
    cp = np.zeros(len(counts) + 1, dtype=np.int64)
    np.cumsum(counts, out=cp[1:])
    if cp[-1] > np.iinfo(np.int32).max:
        raise ValueError("nnz exceeds int32")
    return cp.astype(np.int32)


def _distinct_rows(rng: np.random.Generator, nrows: int, counts: np.ndarray,
                   exclude: np.ndarray | None = None) -> np.ndarray:
    """Draw counts[j] distinct rows in [0, nrows) for every column j.

    Rows are drawn uniformly; duplicates inside a column (and the excluded row
    of that column, if given) are redrawn until none remain. The result keeps
    the draw order inside each column.
    """
    counts = np.asarray(counts, dtype=np.int64)
    if np.any(counts > nrows - (0 if exclude is None else 1)):
        raise ValueError("more rows requested than available")
    n = len(counts)
    nnz = int(counts.sum())
    col = np.repeat(np.arange(n, dtype=np.int64), counts)
    rows = rng.integers(0, nrows, size=nnz, dtype=np.int64)
    todo = np.arange(nnz, dtype=np.int64)
    while True:
        # a position is bad if it repeats an earlier position of its column,
        # or hits the excluded row
        key = col * nrows + rows
        order = np.argsort(key, kind="stable")
        sk = key[order]
        dup = np.zeros(nnz, dtype=bool)
        dup[order[1:][sk[1:] == sk[:-1]]] = True
        if exclude is not None:
            dup |= rows == exclude[col]
        bad = np.nonzero(dup)[0]
        if len(bad) == 0:
            break
        rows[bad] = rng.integers(0, nrows, size=len(bad), dtype=np.int64)
        todo = bad
    del todo
    return rows.astype(np.int32)


def uniform_z(n: int, z: int, seed: int, *, nrows: int | None = None,
              dist: str = "uniform", dtype=np.float64,
              rng: np.random.Generator | None = None) -> CSC:
    """Section 5.2's synthetic law: every column holds exactly z uniformly placed rows.

    ``dist`` selects the value law: "uniform" draws from U[-1, 1], "normal"
    from N(0, 1).
    """
    rng = np.random.default_rng(seed) if rng is None else rng
    m = n if nrows is None else nrows
    counts = np.full(n, z, dtype=np.int64)
    rows = _distinct_rows(rng, m, counts)
    vals = _values(rng, len(rows), dist)
    return CSC(m, n, _colptr_from_counts(counts), rows, vals.astype(dtype))


def _values(rng: np.random.Generator, size: int, dist: str) -> np.ndarray:
    if dist == "uniform":
        return rng.uniform(-1.0, 1.0, size=size)
    if dist == "normal":
        return rng.standard_normal(size=size)
    if dist == "int":
        # small integers: every summation order gives the same exact result
        return rng.integers(-8, 9, size=size).astype(np.float64)
    raise ValueError(dist)


def diag_plus_random(n: int = 1000, extra: int = 4, seed: int = 0) -> CSC:
    """n x n: column j holds its diagonal plus ``extra`` distinct random off-diagonal rows.

    The diagonal comes first in each column, followed by the drawn rows; all
    values are U[-1, 1].
    """
    rng = np.random.default_rng(seed)
    counts = np.full(n, extra, dtype=np.int64)
    off = _distinct_rows(rng, n, counts, exclude=np.arange(n))
    rows = np.empty(n * (extra + 1), dtype=np.int32)
    rows2 = rows.reshape(n, extra + 1)
    rows2[:, 0] = np.arange(n)
    rows2[:, 1:] = off.reshape(n, extra)
    vals = rng.uniform(-1.0, 1.0, size=len(rows))
    return CSC(n, n, _colptr_from_counts(np.full(n, extra + 1)), rows, vals)


def laplacian_2d(g: int = 64) -> CSC:
    """5-point Laplacian on a g x g grid with Dirichlet boundary.

    Node (x, y) is column x + g*y; the diagonal is 4 and each grid neighbour
    is -1. Rows inside a column are stored in ascending order.
    """
    n = g * g
    cols = []
    for y in range(g):
        for x in range(g):
            nb = []
            if y > 0:
                nb.append(x + g * (y - 1))
            if x > 0:
                nb.append(x - 1 + g * y)
            nb.append(x + g * y)
            if x < g - 1:
                nb.append(x + 1 + g * y)
            if y < g - 1:
                nb.append(x + g * (y + 1))
            cols.append(nb)
    counts = np.array([len(c) for c in cols], dtype=np.int64)
    rows = np.concatenate([np.array(c, dtype=np.int32) for c in cols])
    j = np.repeat(np.arange(n), counts)
    vals = np.where(rows == j, 4.0, -1.0)
    return CSC(n, n, _colptr_from_counts(counts), rows, vals)


def zipf_degrees(rng: np.random.Generator, n: int, exponent: float = 2.0,
                 dmax: int = 2000) -> np.ndarray:
    """Column degrees from a truncated power law P(d) proportional to d^-exponent on [1, dmax]."""
    d = np.arange(1, dmax + 1, dtype=np.float64)
    p = d ** (-exponent)
    cdf = np.cumsum(p)
    cdf /= cdf[-1]
    u = rng.random(n)
    return (np.searchsorted(cdf, u, side="right") + 1).astype(np.int64)


def powerlaw(n: int = 1_000_000, seed: int = 0, exponent: float = 2.0,
             dmax: int = 2000, dtype=np.float64) -> tuple[CSC, CSC]:
    """Two independent n x n matrices with power-law column degrees, uniform rows, N(0,1) values.

    A is drawn first and B after it from the same generator stream.
    """
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(2):
        deg = np.minimum(zipf_degrees(rng, n, exponent, dmax), n)
        rows = _distinct_rows(rng, n, deg)
        vals = rng.standard_normal(len(rows)).astype(dtype)
        out.append(CSC(n, n, _colptr_from_counts(deg), rows, vals))
    return out[0], out[1]


def batched_problems(count: int = 512, seed: int = 0, nmin: int = 500,
                     nmax: int = 20000, zmin: int = 2, zmax: int = 40,
                     dtype=np.float64) -> list[tuple[CSC, CSC]]:
    """``count`` independent square pairs (A_i, B_i).

    n_i is log-uniform in [nmin, nmax]; each problem draws one z_i uniformly
    from {zmin..zmax} and gives every column of A_i and B_i exactly z_i
    uniform rows; values are U[-1, 1].
    """
    rng = np.random.default_rng(seed)
    ns = np.rint(np.exp(rng.uniform(np.log(nmin), np.log(nmax), size=count))).astype(np.int64)
    zs = rng.integers(zmin, zmax + 1, size=count)
    probs = []
    for n, z in zip(ns, zs):
        a = uniform_z(int(n), int(min(z, n)), 0, rng=rng, dtype=dtype)
        b = uniform_z(int(n), int(min(z, n)), 0, rng=rng, dtype=dtype)
        probs.append((a, b))
    return probs


def gradient_values(nnz: int, seed: int, dtype=np.float32) -> np.ndarray:
    """Upstream gradient values G ~ N(0, 1), one per stored entry of C."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(nnz).astype(dtype)


def random_tiny(rng: np.random.Generator, m: int, n: int, density: float,
                dist: str = "uniform", dtype=np.float64) -> CSC:
    """Small random CSC matrix with Bernoulli(density) pattern; may have empty columns."""
    mask = rng.random((m, n)) < density
    counts = mask.sum(axis=0).astype(np.int64)
    rows = []
    for j in range(n):
        r = np.nonzero(mask[:, j])[0]
        rng.shuffle(r)  # storage order inside a column is free
        rows.append(r)
    rowidx = (np.concatenate(rows) if rows else np.zeros(0)).astype(np.int32)
    vals = _values(rng, len(rowidx), dist).astype(dtype)
    return CSC(m, n, _colptr_from_counts(counts), rowidx, vals)


def shuffle_within_columns(a: CSC, seed: int) -> CSC:
    """The same matrix with the storage order inside every column permuted."""
    rng = np.random.default_rng(seed)
    ri = a.rowidx.copy()
    v = a.val.copy()
    cp = a.colptr
    for j in range(a.ncols):
        s, e = int(cp[j]), int(cp[j + 1])
        if e - s > 1:
            p = rng.permutation(e - s) + s
            ri[s:e] = a.rowidx[p]
            v[s:e] = a.val[p]
    return CSC(a.nrows, a.ncols, cp, ri, v)


def to_dense(a: CSC) -> np.ndarray:
    d = np.zeros((a.nrows, a.ncols), dtype=np.float64)
    col = np.repeat(np.arange(a.ncols), np.diff(a.colptr.astype(np.int64)))
    d[a.rowidx.astype(np.int64), col] = a.val
    return d


def from_dense(d: np.ndarray, dtype=np.float64) -> CSC:
    m, n = d.shape
    counts = (d != 0).sum(axis=0)
    rows = [np.nonzero(d[:, j])[0] for j in range(n)]
    rowidx = (np.concatenate(rows) if n else np.zeros(0)).astype(np.int32)
    vals = np.concatenate([d[r, j] for j, r in enumerate(rows)]) if n else np.zeros(0)
    return CSC(m, n, _colptr_from_counts(counts), rowidx, vals.astype(dtype))


def identity(n: int, dtype=np.float64) -> CSC:
    return CSC(n, n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32),
               np.ones(n, dtype=dtype))


def permutation(perm: np.ndarray, dtype=np.float64) -> CSC:
    """P with P[perm[j], j] = 1."""
    n = len(perm)
    return CSC(n, n, np.arange(n + 1, dtype=np.int32), np.asarray(perm, dtype=np.int32),
               np.ones(n, dtype=dtype))
