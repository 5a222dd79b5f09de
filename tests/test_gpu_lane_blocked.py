"""GPU parity of the lane-per-column blocks (option SPGEMM_LANE_BLOCKED):
the light columns sorted by decreasing Op_j and cut by the Blocking
Algorithm (Section 3.1), one column per lane stepping one product at a time
(Algorithm 3) into a per-lane hash table (HASH, Section 3.2) or dense
accumulator (SPARS). Every case compares C element by element with the
oracle; the number of blocks is compared with the oracle's Blocking
Algorithm on the same sorted loads.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2303_02471_amd import _lib, inputs as gen
from helpers import (HAVE_GPU, assert_same_structure, assert_values_exact, check_f32, check_f64,
                     gpu_product)

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not HAVE_GPU, reason="needs an MI355X GPU")]

if HAVE_GPU:
    import torch
    from paper_2303_02471_amd import api


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def _lane_ops(A, B, t):
    """Op_j of the columns the lane blocks take (0 < Op_j <= t rounded up to a
    power of two), sorted decreasing."""
    t2 = 4
    while t2 < t:
        t2 *= 2
    op = oracle.opcount(A, B)
    sel = op[(op > 0) & (op <= t2)]
    return np.sort(sel)[::-1]


def _check_blocks(A, B, opts, t=64, bmin=16, bmax=64):
    (cp, ri, v), plan, _ = gpu_product(A, B, opts, np.float64, return_plan=True)
    st = plan.stats()
    plan.close()
    ops = _lane_ops(A, B, t)
    assert st["lane_cols"] == len(ops)
    starts = oracle.blocking(ops, bmin, bmax)
    assert st["lane_blocks"] == len(starts) - 1, (st["lane_blocks"], len(starts) - 1)
    ocp, ori, ov = oracle.spgemm(A, B)
    assert_same_structure(cp, ri, ocp, ori, "lane blocks")
    assert_values_exact(v, ov, "lane blocks")


@pytest.mark.parametrize("spars", [False, True])
@pytest.mark.parametrize("z", [2, 4, 6, 8])
def test_constant_z_2560(z, spars):
    """The paper's synthetic matrices: n = 2560, Z entries per column."""
    _say(f"lane blocks n=2560 z={z} spars={spars}")
    A = gen.uniform_z(2560, z, seed=100 + z)
    B = gen.uniform_z(2560, z, seed=200 + z)
    o = api.options(lane_blocked=True, lane_spars=spars)
    _check_blocks(A, B, o)
    check_f32(A, B, o, f"lane blocks z={z} f32")


@pytest.mark.parametrize("bmin,bmax", [(1, 1), (5, 7), (16, 64), (64, 64), (3, 40)])
def test_blocking_parameters(bmin, bmax):
    """Mixed loads (many Op values, short runs): spanning blocks, remainders
    and full blocks of every kind."""
    _say(f"lane blocks bmin={bmin} bmax={bmax}")
    A, B = gen.powerlaw(20_000, seed=7)
    o = api.options(lane_blocked=True, b_min=bmin, b_max=bmax)
    _check_blocks(A, B, o, bmin=bmin, bmax=bmax)


@pytest.mark.parametrize("t", [1, 4, 16, 33, 64])
def test_thresholds(t):
    _say(f"lane blocks t={t}")
    A, B = gen.powerlaw(20_000, seed=8)
    o = api.options(lane_blocked=True, t_lane=t)
    _check_blocks(A, B, o, t=t)


def test_powerlaw_1e5_hash_and_spars_refused():
    """HASH blocks on the power-law input; SPARS needs at most 4096 rows."""
    _say("lane blocks powerlaw n=100000")
    A, B = gen.powerlaw(100_000, seed=9)
    check_f64(A, B, api.options(lane_blocked=True), "lane blocks powerlaw")
    with pytest.raises(_lib.SpgemmError) as e:
        gpu_product(A, B, api.options(lane_spars=True))
    assert e.value.status == 9


def test_repeated_rows_in_lane_columns():
    """Columns whose products meet the same rows many times (A with 3 rows):
    the ordered sums of Algorithm 1 in both accumulators."""
    _say("lane blocks repeated rows")
    rng = np.random.default_rng(4)
    k, n = 400, 3000
    A = gen.CSC(3, k, (np.arange(k + 1) * 2).astype(np.int32),
                np.tile(np.array([0, 2], np.int32), k), rng.standard_normal(2 * k))
    zb = rng.integers(1, 30, n)
    b_cp = np.concatenate([[0], np.cumsum(zb)]).astype(np.int32)
    b_ri = np.concatenate([np.sort(rng.choice(k, z, replace=False)) for z in zb]).astype(np.int32)
    B = gen.CSC(k, n, b_cp, b_ri, rng.standard_normal(int(b_cp[-1])))
    for spars in (False, True):
        o = api.options(lane_blocked=True, lane_spars=spars)
        check_f64(A, B, o, f"repeated rows spars={spars}")
        check_f32(A, B, o, f"repeated rows spars={spars} f32")


def test_planned_relaunch_changed_structure():
    """A plan reused on another structure with the same shapes: the numeric
    phase run at the first structure's positions must be redone."""
    _say("lane blocks planned relaunch")
    A1 = gen.uniform_z(2560, 5, seed=1)
    B1 = gen.uniform_z(2560, 5, seed=2)
    A2 = gen.uniform_z(2560, 4, seed=3)
    B2 = gen.uniform_z(2560, 4, seed=4)
    for spars in (False, True):
        opts = api.options(lane_blocked=True, lane_spars=spars)
        At, Bt = api.CscTensor.from_host(A1), api.CscTensor.from_host(B1)
        plan, colptr, ri, v, nnz = api.multiply(At, Bt, opts)
        torch.cuda.synchronize()
        ocp, ori, ov = oracle.spgemm(A1, B1)
        assert_same_structure(colptr.cpu().numpy(), ri[:nnz].cpu().numpy(), ocp, ori, "first")
        assert_values_exact(v[:nnz].cpu().numpy(), ov, "first")
        At2, Bt2 = api.CscTensor.from_host(A2), api.CscTensor.from_host(B2)
        plan, colptr2, ri2, v2, nnz2 = api.multiply(At2, Bt2, opts, plan=plan,
                                                   out=(colptr, ri, v))
        torch.cuda.synchronize()
        ocp, ori, ov = oracle.spgemm(A2, B2)
        assert_same_structure(colptr2.cpu().numpy(), ri2[:nnz2].cpu().numpy(), ocp, ori, "second")
        assert_values_exact(v2[:nnz2].cpu().numpy(), ov, "second")
        plan.close()
