"""Shared helpers for the GPU parity tests: run the HIP path, compare with the oracle."""
from __future__ import annotations

import numpy as np

import oracle

try:
    import torch
    HAVE_GPU = torch.cuda.is_available()
except Exception:  # pragma: no cover
    torch = None
    HAVE_GPU = False


def gpu_product(A, B, opts=None, dtype=np.float64, return_plan=False):
    """C = A x B on the GPU; returns host arrays (colptr, rowidx, val)."""
    from paper_2303_02471_amd import api
    At = api.CscTensor.from_host(A, dtype=dtype)
    Bt = api.CscTensor.from_host(B, dtype=dtype)
    Cm, plan = api.matmul(At, Bt, opts, return_plan=True)
    torch.cuda.synchronize()
    out = Cm.to_host()
    if return_plan:
        return out, plan, (At, Bt, Cm)
    plan.close()
    return out


def assert_same_structure(cp, ri, ocp, ori, what=""):
    assert np.array_equal(cp, ocp), f"{what}: column pointers differ"
    assert np.array_equal(ri, ori), f"{what}: row indices differ"


def assert_values_exact(v, ov, what=""):
    """Bit-identical up to the sign of zero (the ordered accumulation matches
    Algorithm 1's order, so every value is the same rounded number)."""
    bad = np.nonzero(v != ov)[0]
    assert len(bad) == 0, f"{what}: {len(bad)} values differ, first at {bad[:5]}: " \
                          f"{v[bad[:5]]} vs {ov[bad[:5]]}"


def assert_rel_1e12(v, ov, A, B, cp, ri):
    """The stated FP64 tolerance: |c - o| <= 1e-12 |o|, and for o == 0,
    |c| <= 1e-12 * sum_k |A_ik B_kj|."""
    s, _ = oracle.absprod(A, B, cp, ri)
    ref = np.where(ov != 0, np.abs(ov), s)
    assert np.all(np.abs(v - ov) <= 1e-12 * ref), "relative error above 1e-12"


def check_f64(A, B, opts=None, what=""):
    ocp, ori, ov = oracle.spgemm(A, B)
    cp, ri, v = gpu_product(A, B, opts, np.float64)
    assert_same_structure(cp, ri, ocp, ori, what)
    assert_values_exact(v, ov, what)
    assert_rel_1e12(v, ov, A, B, ocp, ori)
    return cp, ri, v


def f32_bound(A, B, cp, ri):
    """Error bound of a float32 evaluation against the exact sum: every product
    and every addition rounds once (unit roundoff 2^-24), so
    |c - exact| <= (terms + 1) * 2^-24 * sum |A_ik B_kj| to first order; the
    factor 1.01 covers the second-order terms."""
    s, t = oracle.absprod(A, B, cp, ri)
    return 1.01 * (t + 1) * 2.0 ** -24 * s


def check_f32(A, B, opts=None, what=""):
    A32, B32 = A.astype(np.float32), B.astype(np.float32)
    ocp, ori, ov32 = oracle.spgemm(A32, B32, "f32")
    _, _, ov64 = oracle.spgemm(A32, B32, "f64")
    cp, ri, v = gpu_product(A32, B32, opts, np.float32)
    assert_same_structure(cp, ri, ocp, ori, what)
    assert_values_exact(v, ov32, what)  # same order, same float rounding
    err = np.abs(v.astype(np.float64) - ov64)
    assert np.all(err <= f32_bound(A32, B32, ocp, ori) + 1e-38), what
    nz = ov64 != 0
    return float(np.max(err[nz] / np.abs(ov64[nz]))) if nz.any() else 0.0
