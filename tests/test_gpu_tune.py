"""Autotuner on the GPU: the chosen options give the oracle's bits, and the
choice is served from the JSON cache the second time."""
import json
import sys

import numpy as np
import pytest

import oracle
from paper_2303_02471_amd import inputs as gen
from helpers import HAVE_GPU, assert_same_structure, assert_values_exact, gpu_product

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not HAVE_GPU, reason="needs an MI355X GPU")]


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def test_autotune_single_cached(tmp_path):
    import torch
    from paper_2303_02471_amd import api
    _say("autotune power law n=30000")
    A, B = gen.powerlaw(30_000, seed=7)
    At, Bt = api.CscTensor.from_host(A), api.CscTensor.from_host(B)
    path = str(tmp_path / "tune.json")
    opts, rep = api.autotune([(At, Bt)], torch.float64, cache_path=path)
    assert rep["from_cache"] == 0 and rep["trials"] >= 2
    assert rep["best_ms"] <= rep["default_ms"]
    doc = json.load(open(path))
    assert len(doc["entries"]) == 1
    ocp, ori, ov = oracle.spgemm(A, B)
    cp, ri, v = gpu_product(A, B, opts)
    assert_same_structure(cp, ri, ocp, ori, "tuned")
    assert_values_exact(v, ov, "tuned")
    opts2, rep2 = api.autotune([(At, Bt)], torch.float64, cache_path=path)
    assert rep2["from_cache"] == 1 and rep2["trials"] == 0
    for f in ("t_esc", "t_dense", "dense_rows", "hash_cap", "t_split", "t_block"):
        assert getattr(opts2, f) == getattr(opts, f)
    # lookup only with an unknown workload: not tuned, nothing timed
    C = gen.uniform_z(5000, 3, seed=1)
    Ct = api.CscTensor.from_host(C)
    with pytest.raises(Exception) as ei:
        api.autotune([(Ct, Ct)], torch.float64, cache_path=path, lookup_only=True)
    assert "NOT_TUNED" in str(ei.value)


def test_autotune_batched():
    import torch
    from paper_2303_02471_amd import api
    _say("autotune batched 12 problems")
    probs = gen.batched_problems(12, seed=3, nmax=4000)
    pairs = [(api.CscTensor.from_host(a), api.CscTensor.from_host(b)) for a, b in probs]
    opts, rep = api.autotune(pairs, torch.float64)
    assert rep["trials"] >= 2
    out = api.batched_matmul(pairs, opts)
    torch.cuda.synchronize()
    for (a, b), cm in zip(probs, out):
        ocp, ori, ov = oracle.spgemm(a, b)
        cp, ri, v = cm.to_host()
        assert_same_structure(cp, ri, ocp, ori, "batched tuned")
        assert_values_exact(v, ov, "batched tuned")
