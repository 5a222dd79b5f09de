"""Plan memory through the caller's allocator (spgemm_set_allocator).

A counting allocator (delegating to torch's caching allocator) is installed
through the C ABI; every device allocation a plan makes in its symbolic,
numeric, one-call, batched and backward calls must reach it, and every one
must come back through its free with the same size and stream by the time the
plans are destroyed. Outputs stay equal to the oracle's.
"""
import ctypes as C
import sys

import numpy as np
import pytest

import oracle
from paper_2303_02471_amd import inputs as gen
from helpers import HAVE_GPU, assert_same_structure, assert_values_exact

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not HAVE_GPU, reason="needs an MI355X GPU")]

if HAVE_GPU:
    import torch
    from paper_2303_02471_amd import api, _lib


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


class Counting:
    def __init__(self):
        self.live = {}
        self.allocs = 0
        self.frees = 0
        self.bad_frees = []
        self.alloc_cb = _lib.ALLOC_FN(self._alloc)
        self.free_cb = _lib.FREE_FN(self._free)

    def _alloc(self, nbytes, stream, ctx):
        ptr = torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
        self.live[int(ptr)] = (int(nbytes), int(stream or 0))
        self.allocs += 1
        return ptr

    def _free(self, ptr, nbytes, stream, ctx):
        key = int(ptr)
        got = (int(nbytes), int(stream or 0))
        if self.live.get(key) != got:
            self.bad_frees.append((key, got, self.live.get(key)))
        self.live.pop(key, None)
        self.frees += 1
        torch.cuda.caching_allocator_delete(key)


def test_counting_allocator_sees_every_plan_allocation():
    _say("counting allocator")
    cnt = Counting()
    api.set_allocator(cnt.alloc_cb, cnt.free_cb)
    try:
        A = gen.uniform_z(3000, 6, seed=1)
        B = gen.uniform_z(3000, 7, seed=2)
        At, Bt = api.CscTensor.from_host(A), api.CscTensor.from_host(B)
        # symbolic + numeric
        Cm, plan = api.matmul(At, Bt, return_plan=True)
        assert cnt.allocs > 0
        ocp, ori, ov = oracle.spgemm(A, B)
        cp, ri, v = Cm.to_host()
        assert_same_structure(cp, ri, ocp, ori, "matmul")
        assert_values_exact(v, ov, "matmul")
        # backward (builds its view: another allocation)
        before = cnt.allocs
        G = torch.from_numpy(gen.gradient_values(Cm.nnz, seed=3, dtype=np.float64)).cuda()
        api.backward(plan, At.val, Bt.val, Cm.rowidx, G)
        torch.cuda.synchronize()
        assert cnt.allocs > before
        # the same plan on a larger problem: its buffers grow (old ones freed)
        A2 = gen.uniform_z(6000, 9, seed=4)
        B2 = gen.uniform_z(6000, 9, seed=5)
        At2, Bt2 = api.CscTensor.from_host(A2), api.CscTensor.from_host(B2)
        frees_before = cnt.frees
        p2, cp2, nnz2 = api.symbolic(At2, Bt2, torch.float64, plan=plan)
        assert cnt.frees > frees_before
        r2 = torch.empty(nnz2, dtype=torch.int32, device="cuda")
        v2 = torch.empty(nnz2, dtype=torch.float64, device="cuda")
        api.numeric(p2, At2.val, Bt2.val, r2, v2)
        torch.cuda.synchronize()
        ocp, ori, ov = oracle.spgemm(A2, B2)
        assert_same_structure(cp2.cpu().numpy(), r2.cpu().numpy(), ocp, ori, "grown")
        assert_values_exact(v2.cpu().numpy(), ov, "grown")
        # one-call product on a side stream, and a batched plan
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            p3, c3, ri3, v3, nnz3 = api.multiply(At, Bt)
        s.synchronize()
        outs, bplan = api.batched_matmul([(At, Bt), (At2, Bt2)], return_plan=True)
        torch.cuda.synchronize()
        assert_values_exact(outs[1].val.cpu().numpy(), ov, "batched")
        assert cnt.live, "plans hold memory while alive"
        for p in (plan, p3, bplan):
            p.close()
        torch.cuda.synchronize()
        assert not cnt.live, f"{len(cnt.live)} allocations never freed"
        assert not cnt.bad_frees, cnt.bad_frees[:3]
        assert cnt.allocs == cnt.frees
    finally:
        api.set_allocator("torch")


class Refusing(Counting):
    """Grants the first `grant` requests, refuses every later one (NULL)."""

    def __init__(self, grant):
        super().__init__()
        self.grant = grant
        self.refused = 0

    def _alloc(self, nbytes, stream, ctx):
        if self.allocs >= self.grant:
            self.refused += 1
            return None
        return super()._alloc(nbytes, stream, ctx)


def _symbolic_allocations(At, Bt):
    """Allocations one symbolic call makes on a fresh plan."""
    cnt = Counting()
    api.set_allocator(cnt.alloc_cb, cnt.free_cb)
    try:
        plan = api.Plan()
        api.symbolic(At, Bt, torch.float64, plan=plan)
        torch.cuda.synchronize()
        plan.close()
        torch.cuda.synchronize()
    finally:
        api.set_allocator("torch")
    return cnt.allocs


@pytest.mark.parametrize("which", ["first", "last"])
def test_refused_allocation_gives_no_memory(which):
    """An allocator that runs out (at the symbolic call's first request, or at
    its last one: the rest of the plan's workspace already in place) makes the
    call return SPGEMM_ERR_NO_MEMORY; everything granted comes back through
    free once the plan is gone, and the library works again with the default
    allocator."""
    A = gen.uniform_z(3000, 6, seed=1)
    B = gen.uniform_z(3000, 7, seed=2)
    At, Bt = api.CscTensor.from_host(A), api.CscTensor.from_host(B)
    n = _symbolic_allocations(At, Bt)
    assert n >= 2, n
    grant = 0 if which == "first" else n - 1
    _say(f"refusing allocator after {grant} of {n} grants")
    ref = Refusing(grant)
    api.set_allocator(ref.alloc_cb, ref.free_cb)
    try:
        plan = api.Plan()
        with pytest.raises(_lib.SpgemmError) as e:
            api.symbolic(At, Bt, torch.float64, plan=plan)
        assert e.value.status == 6, e.value
        assert ref.refused >= 1
        plan.close()
        torch.cuda.synchronize()
        assert not ref.live, f"{len(ref.live)} granted allocations never freed"
        assert not ref.bad_frees, ref.bad_frees[:3]
    finally:
        api.set_allocator("torch")
    Cm = api.matmul(At, Bt)
    ocp, ori, ov = oracle.spgemm(A, B)
    cp, ri, v = Cm.to_host()
    assert_same_structure(cp, ri, ocp, ori, "after the refusals")
    assert_values_exact(v, ov, "after the refusals")
