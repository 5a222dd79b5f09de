"""Pins of the oracle's summation order and rounding (Algorithm 1, Section 2.2).

Bit-exact parity of the GPU path rests on the oracle adding every product to
the running value of its output entry in Algorithm 1's order: stored B
entries of the column in storage order, starting from the zero that
SPA_values is initialised with, each product and each sum rounded on its own.
The hand-worked cases in tests/golden/summation_order.txt are built so that
the expected bits come out only in that order (their comments give what the
other orders produce), and likewise for the stated orders of the two
gradients and for the float-per-step FP32 twin.

The second half plants each plausible mistake in a copy of the oracle's
source (on the CPU), builds it, and checks that at least one golden case
fails for it -- so the pins are known to catch that mistake.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from oracle import build as obuild


def _parse(path):
    cases, cur = [], None
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        key, *vals = line.split()
        if key == "case":
            cur = {"name": vals[0]}
        elif key == "end":
            cases.append(cur)
            cur = None
        else:
            cur[key] = vals
    return cases


def _floats(vals, dt):
    return np.array([float.fromhex(v) for v in vals], dtype=dt)


def _ints(vals):
    return np.array([int(v) for v in vals], dtype=np.int32)


def _mat(c, p, dt):
    nrows, ncols = (int(x) for x in c[p])
    return oracle.csc(nrows, ncols, _ints(c[p + "_colptr"]), _ints(c[p + "_rowidx"]),
                      _floats(c[p + "_val"], dt))


def _bits(x):
    x = np.asarray(x)
    return x.view(np.uint64 if x.dtype == np.float64 else np.uint32)


@pytest.fixture(scope="module")
def cases(golden_dir):
    return _parse(os.path.join(golden_dir, "summation_order.txt"))


def _check_case(c, lib=None):
    """Raises AssertionError when the oracle (or `lib`) disagrees with the
    case's hand-worked bits."""
    dt = np.float64 if c["dtype"][0] == "f64" else np.float32
    prec = c["dtype"][0]
    A, B = _mat(c, "a", dt), _mat(c, "b", dt)
    cp, ri, v = oracle.spgemm(A, B, prec, lib=lib)
    assert np.array_equal(cp, _ints(c["c_colptr"])), f"{c['name']}: colptr"
    assert np.array_equal(ri, _ints(c["c_rowidx"])), f"{c['name']}: rowidx"
    want = _floats(c["c_val"], dt)
    assert np.array_equal(_bits(v), _bits(want)), f"{c['name']}: C {v} != {want}"
    if "g_val" in c:
        g = _floats(c["g_val"], dt)
        da, db = oracle.backward(A, B, cp, ri, g, prec, lib=lib)
        if "da_val" in c:
            w = _floats(c["da_val"], dt)
            assert np.array_equal(_bits(da), _bits(w)), f"{c['name']}: dA {da} != {w}"
        if "db_val" in c:
            w = _floats(c["db_val"], dt)
            assert np.array_equal(_bits(db), _bits(w)), f"{c['name']}: dB {db} != {w}"
    if "abs_val" in c:
        s, t = oracle.absprod(A, B, cp, ri, lib=lib)
        w = _floats(c["abs_val"], np.float64)
        assert np.array_equal(_bits(s), _bits(w)), f"{c['name']}: abs {s} != {w}"
        assert np.array_equal(t, _ints(c["abs_terms"])), f"{c['name']}: terms {t}"


def test_golden_cases_present(cases):
    names = {c["name"] for c in cases}
    assert {"b_stored_order", "two_entries_interleaved", "negative_zero_product",
            "f32_rounds_every_step", "f32_product_rounding", "f32_product_before_sum",
            "backward_db_a_stored_order", "backward_da_columns_ascending", "backward_f32_steps",
            "absprod_mixed_signs", "figure1_abs_terms"} <= names


@pytest.mark.parametrize("name", [
    "b_stored_order", "two_entries_interleaved", "negative_zero_product",
    "f32_rounds_every_step", "f32_product_rounding", "f32_product_before_sum",
    "backward_db_a_stored_order", "backward_da_columns_ascending", "backward_f32_steps",
    "absprod_mixed_signs", "figure1_abs_terms"])
def test_summation_order_golden(cases, name):
    """Algorithm 1 (Section 2.2): the hand-worked bits of each case."""
    (c,) = [x for x in cases if x["name"] == name]
    _check_case(c)


def test_golden_values_independent_of_oracle(cases):
    """The product's expected bits, re-derived by a plain Python loop in
    Algorithm 1's order with numpy scalars of the case's type (a second,
    independent reading of the order the golden comments work by hand), and
    the sign of every expected zero is +0 (SPA_values starts at +0)."""
    for c in cases:
        dt = np.float64 if c["dtype"][0] == "f64" else np.float32
        A, B = _mat(c, "a", dt), _mat(c, "b", dt)
        want_cp, want_ri, want_v = _ints(c["c_colptr"]), _ints(c["c_rowidx"]), \
            _floats(c["c_val"], dt)
        for j in range(B.ncols):
            acc = {}
            for p in range(B.colptr[j], B.colptr[j + 1]):
                k = B.rowidx[p]
                for q in range(A.colptr[k], A.colptr[k + 1]):
                    i = int(A.rowidx[q])
                    prod = dt(A.val[q]) * dt(B.val[p])
                    acc[i] = dt(acc.get(i, dt(0.0)) + prod)
            rows = sorted(acc)
            assert rows == want_ri[want_cp[j]:want_cp[j + 1]].tolist(), c["name"]
            got = np.array([acc[i] for i in rows], dtype=dt)
            assert np.array_equal(_bits(got), _bits(want_v[want_cp[j]:want_cp[j + 1]])), \
                c["name"]


# --------------------------------------------------------------------------- planted mistakes

def _src():
    return open(obuild.SRC).read()


# (name, replacements: list of (old, new[, occurrences]) in oracle.c) -- each
# is a plausible mistake in the order or rounding of the sums
MUTANTS = [
    # B's column walked backwards in the FP64 product
    ("b_reversed_f64", [(
        "        for (int32_t p = b_colptr[j]; p < b_colptr[j + 1]; ++p) {      /* B(k,j) */",
        "        for (int32_t p = b_colptr[j + 1] - 1; p >= b_colptr[j]; --p) {  /* B(k,j) */")]),
    # B's column walked backwards in the FP32 twin
    ("b_reversed_f32", [(
        "            float bkj = b_val[p];",
        "            p = b_colptr[j] + b_colptr[j + 1] - 1 - p; float bkj = b_val[p];"), (
        "                    spa_indices[counter++] = i;\n                }\n            }\n"
        "        }\n        if (counter != c_colptr[j + 1] - c_colptr[j]) {\n"
        "            free(spa_values); free(spa_flags); free(spa_indices);\n"
        "            return ORACLE_EBADCSC;\n        }\n        qsort",
        "                    spa_indices[counter++] = i;\n                }\n            }\n"
        "            p = b_colptr[j] + b_colptr[j + 1] - 1 - p;\n"
        "        }\n        if (counter != c_colptr[j + 1] - c_colptr[j]) {\n"
        "            free(spa_values); free(spa_flags); free(spa_indices);\n"
        "            return ORACLE_EBADCSC;\n        }\n        qsort")]),
    # the first product of an entry assigned instead of added to zero (-0 kept)
    ("first_assigned", [(
        "                spa_values[i] = spa_values[i] + tmp_val;\n                if (spa_flags[i] == 0) {",
        "                spa_values[i] = spa_flags[i] ? spa_values[i] + tmp_val : tmp_val;\n"
        "                if (spa_flags[i] == 0) {", 2)]),
    # the FP32 twin accumulating in double and rounding once at the end
    ("f32_double_accumulator", [(
        "    float *spa_values = (float *)calloc(m, sizeof(float));",
        "    double *spa_values = (double *)calloc(m, sizeof(double));")]),
    # the FP32 twin forming its products in double
    ("f32_double_products", [(
        "                float tmp_val = a_val[q] * bkj;",
        "                double tmp_val = (double)a_val[q] * (double)bkj;")]),
    # dB summed over A's column backwards
    ("db_reversed", [(
        "                for (int32_t q = a_colptr[k]; q < a_colptr[k + 1]; ++q) {             \\\n"
        "                    int32_t at = find_in_column(c_colptr, c_rowidx, j, a_rowidx[q]);  \\",
        "                for (int32_t q = a_colptr[k + 1] - 1; q >= a_colptr[k]; --q) {        \\\n"
        "                    int32_t at = find_in_column(c_colptr, c_rowidx, j, a_rowidx[q]);  \\")]),
    # dA summed over B's row with columns descending
    ("da_reversed", [(
        "                for (int32_t r = rowptr[k]; r < rowptr[k + 1]; ++r) {                 \\",
        "                for (int32_t r = rowptr[k + 1] - 1; r >= rowptr[k]; --r) {            \\")]),
    # the absolute sums without the absolute value of B
    ("abs_signed", [(
        "            double bkj = b_val[p] < 0 ? -b_val[p] : b_val[p];",
        "            double bkj = b_val[p];")]),
    # term count off by one per entry
    ("abs_terms_skip_first", [(
        "                cnt[i] += 1;",
        "                cnt[i] += acc[i] != aik * bkj;")]),
]


@pytest.fixture(scope="module")
def mutant_dir():
    d = tempfile.mkdtemp(prefix="oracle_mutants_")
    yield d
    shutil.rmtree(d, ignore_errors=True)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.parametrize("name,edits", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(cases, mutant_dir, name, edits):
    src = _src()
    for old, new, *count in edits:
        want = count[0] if count else 1
        assert src.count(old) == want, f"{name}: the oracle source changed; update the mutant"
        src = src.replace(old, new)
    cdir = os.path.join(mutant_dir, name)
    os.makedirs(cdir, exist_ok=True)
    shutil.copy(os.path.join(os.path.dirname(obuild.SRC), "oracle.h"), cdir)
    cfile = os.path.join(cdir, "oracle.c")
    open(cfile, "w").write(src)
    so = os.path.join(cdir, "liboracle_mutant.so")
    flags = [f for f in obuild.CFLAGS if f != "-Werror"]
    subprocess.run(["gcc", *flags, "-o", so, cfile], check=True, capture_output=True)
    lib = oracle.bind(so)
    caught = []
    for c in cases:
        try:
            _check_case(c, lib=lib)
        except (AssertionError, oracle.OracleError):
            caught.append(c["name"])
    assert caught, f"no golden case catches the planted mistake {name}"
