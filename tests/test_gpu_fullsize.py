"""Parity at the full workload sizes, in the launch configuration the benchmark
times (options chosen by the autotuner, as bench.py does).

* C = A x B, power-law n = 1,000,000 (FP64): every column, rows and values,
  against the oracle (a few seconds of CPU).
* 512 independent problems in one batched call (FP64 and FP32): every
  column of every problem against the oracle (1.8e9 products; the problems
  are compared on a pool of host threads).
* Forward and backward at n = 100,000, 8 per column, FP32: sampled gradient
  entries against the oracle's gradients.
"""
import os
import sys
import tempfile

import numpy as np
import pytest

import oracle
from paper_2303_02471_amd import inputs as gen
from helpers import HAVE_GPU, assert_same_structure, assert_values_exact

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not HAVE_GPU, reason="needs an MI355X GPU")]


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def _columns(m, cols):
    """CSC with the columns `cols` of m (storage order kept)."""
    cp = m.colptr.astype(np.int64)
    counts = cp[cols + 1] - cp[cols]
    ncp = np.zeros(len(cols) + 1, dtype=np.int64)
    np.cumsum(counts, out=ncp[1:])
    idx = np.concatenate([np.arange(cp[c], cp[c + 1]) for c in cols]) if len(cols) else \
        np.zeros(0, np.int64)
    return gen.CSC(m.nrows, len(cols), ncp.astype(np.int32), m.rowidx[idx], m.val[idx])


def _compare_columns(cp, ri, v, cols, ocp, ori, ov, what):
    """GPU columns `cols` of (cp, ri, v) against the oracle's product with the
    same columns (ocp, ori, ov), bit for bit."""
    for t, c in enumerate(cols):
        a, b = int(cp[c]), int(cp[c + 1])
        oa, ob = int(ocp[t]), int(ocp[t + 1])
        assert b - a == ob - oa, f"{what}: column {c} length"
        assert np.array_equal(ri[a:b], ori[oa:ob]), f"{what}: column {c} rows"
        assert np.array_equal(v[a:b], ov[oa:ob]), f"{what}: column {c} values"


def test_powerlaw_1e6_full():
    import torch
    from paper_2303_02471_amd import api
    _say("power law n=1e6 FP64, autotuned options, whole output")
    A, B = gen.powerlaw(1_000_000, seed=0)
    At, Bt = api.CscTensor.from_host(A), api.CscTensor.from_host(B)
    with tempfile.TemporaryDirectory() as td:
        opts, _ = api.autotune([(At, Bt)], torch.float64, cache_path=os.path.join(td, "t.json"))
    Cm, plan = api.matmul(At, Bt, opts, return_plan=True)
    torch.cuda.synchronize()
    cp, ri, v = Cm.to_host()
    plan.close()
    ocp, ori, ov = oracle.spgemm(A, B)
    assert_same_structure(cp, ri, ocp, ori, "powerlaw 1e6")
    assert_values_exact(v, ov, "powerlaw 1e6")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batched_512_full(dtype):
    """Every column of every one of the 512 problems against the oracle (FP64,
    or the FP32 twin), bit for bit. The problems are compared as they finish on
    a pool of host threads (the oracle's C calls release the interpreter lock),
    each reading its own problem's output back, so host memory stays bounded."""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    from paper_2303_02471_amd import api
    _say(f"512 problems, one batched call, {dtype}, every column")
    npdt = np.float64 if dtype == "f64" else np.float32
    tdt = torch.float64 if dtype == "f64" else torch.float32
    probs = gen.batched_problems(512, seed=0)
    if dtype == "f32":
        probs = [(a.astype(np.float32), b.astype(np.float32)) for a, b in probs]
    pairs = [(api.CscTensor.from_host(a, dtype=npdt), api.CscTensor.from_host(b, dtype=npdt))
             for a, b in probs]
    opts, _ = api.autotune(pairs, tdt)
    outs = api.batched_matmul(pairs, opts)
    torch.cuda.synchronize()
    del pairs

    def one(i):
        a, b = probs[i]
        cp, ri, v = outs[i].to_host()
        ocp, ori, ov = oracle.spgemm(a, b, dtype)
        ok = (np.array_equal(cp, ocp) and np.array_equal(ri, ori) and np.array_equal(v, ov))
        return i, ok, int(ocp[-1])

    workers = min(16, os.cpu_count() or 4)
    bad, total = [], 0
    with ThreadPoolExecutor(workers) as ex:
        for i, ok, nz in ex.map(one, range(len(probs))):
            total += nz
            if not ok:
                bad.append(i)
    _say(f"compared {len(probs)} problems, {total} entries")
    assert not bad, f"problems differing from the oracle: {bad[:10]}"
    del outs
    torch.cuda.empty_cache()


def test_forward_backward_100k_f32_sampled():
    import torch
    from paper_2303_02471_amd import api
    _say("forward + backward n=100000, 8 per column, FP32")
    n, z = 100_000, 8
    A = gen.uniform_z(n, z, seed=1, dist="normal", dtype=np.float32)
    B = gen.uniform_z(n, z, seed=2, dist="normal", dtype=np.float32)
    At, Bt = api.CscTensor.from_host(A), api.CscTensor.from_host(B)
    Cm, plan = api.matmul(At, Bt, return_plan=True)
    G = gen.gradient_values(Cm.nnz, seed=3, dtype=np.float32)
    dA, dB = api.backward(plan, At.val, Bt.val, Cm.rowidx, torch.from_numpy(G).cuda())
    torch.cuda.synchronize()
    cp, ri, v = Cm.to_host()
    plan.close()
    ocp, ori, ov = oracle.spgemm(A, B, "f32")
    assert_same_structure(cp, ri, ocp, ori, "fwd 100k")
    assert_values_exact(v, ov, "fwd 100k")
    odA, odB = oracle.backward(A, B, ocp, ori, G, "f32")
    assert np.array_equal(dA.cpu().numpy(), odA), "dA"
    assert np.array_equal(dB.cpu().numpy(), odB), "dB"
