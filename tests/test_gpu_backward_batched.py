"""GPU parity of the gradient kernels, the batched path, plan reuse, HIP-graph
replay of the batched numeric phase, and the device-side input checks."""
import sys

import numpy as np
import pytest

import oracle
from paper_2303_02471_amd import inputs as gen
from helpers import (HAVE_GPU, assert_same_structure, assert_values_exact, f32_bound,
                     gpu_product)

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not HAVE_GPU, reason="needs an MI355X GPU")]

if HAVE_GPU:
    import torch
    from paper_2303_02471_amd import api
    from paper_2303_02471_amd._lib import SpgemmError


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def _grads_gpu(A, B, G, dtype):
    At = api.CscTensor.from_host(A, dtype=dtype)
    Bt = api.CscTensor.from_host(B, dtype=dtype)
    Cm, plan = api.matmul(At, Bt, return_plan=True)
    Gt = torch.from_numpy(np.ascontiguousarray(G.astype(dtype))).cuda()
    dA, dB = api.backward(plan, At.val, Bt.val, Cm.rowidx, Gt)
    torch.cuda.synchronize()
    return Cm, dA.cpu().numpy(), dB.cpu().numpy()


def test_backward_f64_matches_oracle():
    _say("backward f64 n=2000 z=8")
    A = gen.uniform_z(2000, 8, seed=1, dist="normal")
    B = gen.uniform_z(2000, 8, seed=2, dist="normal")
    cp, ri, _ = oracle.spgemm(A, B)
    G = gen.gradient_values(int(cp[-1]), seed=3, dtype=np.float64)
    odA, odB = oracle.backward(A, B, cp, ri, G)
    _, dA, dB = _grads_gpu(A, B, G, np.float64)
    assert_values_exact(dA, odA, "dA")
    assert_values_exact(dB, odB, "dB")


def test_backward_powerlaw_f64():
    _say("backward f64 power law n=20000")
    A, B = gen.powerlaw(20_000, seed=4)
    cp, ri, _ = oracle.spgemm(A, B)
    G = gen.gradient_values(int(cp[-1]), seed=5, dtype=np.float64)
    odA, odB = oracle.backward(A, B, cp, ri, G)
    _, dA, dB = _grads_gpu(A, B, G, np.float64)
    assert_values_exact(dA, odA, "dA")
    assert_values_exact(dB, odB, "dB")


def test_backward_f32_config5():
    """n = 100,000, 8 per column, FP32: equal to the oracle's float twin and
    inside the float32 rounding bound of the double oracle."""
    _say("backward f32 n=100000 z=8")
    A = gen.uniform_z(100_000, 8, seed=1, dist="normal", dtype=np.float32)
    B = gen.uniform_z(100_000, 8, seed=2, dist="normal", dtype=np.float32)
    cp, ri, _ = oracle.spgemm(A, B, "f32")
    G = gen.gradient_values(int(cp[-1]), seed=3, dtype=np.float32)
    o32A, o32B = oracle.backward(A, B, cp, ri, G, "f32")
    o64A, o64B = oracle.backward(A, B, cp, ri, G.astype(np.float64), "f64")
    _, dA, dB = _grads_gpu(A, B, G, np.float32)
    assert_values_exact(dA, o32A, "dA f32")
    assert_values_exact(dB, o32B, "dB f32")
    # |sum of t terms in float - exact| <= (t + 1) u sum|terms|, u = 2^-24
    abs_dA, _ = oracle.backward(gen.CSC(A.nrows, A.ncols, A.colptr, A.rowidx, np.abs(A.val)),
                              gen.CSC(B.nrows, B.ncols, B.colptr, B.rowidx, np.abs(B.val)),
                              cp, ri, np.abs(G).astype(np.float64), "f64")
    za = np.diff(A.colptr)
    nbrow = np.bincount(B.rowidx, minlength=B.nrows)
    termsA = nbrow[np.repeat(np.arange(A.ncols), za)]
    assert np.all(np.abs(dA.astype(np.float64) - o64A) <= 1.01 * (termsA + 1) * 2.0 ** -24 * abs_dA
                  + 1e-38)


def test_autograd_function_and_finite_differences():
    _say("autograd + central differences n=200")
    n, z = 200, 8
    A = gen.uniform_z(n, z, seed=1, dist="normal")
    B = gen.uniform_z(n, z, seed=2, dist="normal")
    At, Bt = api.CscTensor.from_host(A), api.CscTensor.from_host(B)
    a = At.val.clone().requires_grad_(True)
    b = Bt.val.clone().requires_grad_(True)
    cval, rowidx, colptr = api.SpGEMMFunction.apply(a, b, At, Bt)
    G = torch.from_numpy(gen.gradient_values(cval.numel(), seed=3, dtype=np.float64)).cuda()
    loss = (cval * G).sum()
    loss.backward()
    ga, gb = a.grad.cpu().numpy(), b.grad.cpu().numpy()
    cp, ri, _ = oracle.spgemm(A, B)
    odA, odB = oracle.backward(A, B, cp, ri, G.cpu().numpy())
    assert_values_exact(ga, odA, "autograd dA")
    assert_values_exact(gb, odB, "autograd dB")
    # central differences through the GPU forward (bilinear: exact up to rounding)
    h = 2.0 ** -10
    _, plan = api.matmul(At, Bt, return_plan=True)
    cbuf = torch.empty(plan.nnz, dtype=torch.float64, device="cuda")
    rbuf = torch.empty(plan.nnz, dtype=torch.int32, device="cuda")

    def L(av, bv):
        api.numeric(plan, av, bv, rbuf, cbuf)
        return float((cbuf * G).sum())

    rng = np.random.default_rng(0)
    for q in rng.choice(A.nnz, 20, replace=False):
        vp, vm = At.val.clone(), At.val.clone()
        vp[q] += h
        vm[q] -= h
        fd = (L(vp, Bt.val) - L(vm, Bt.val)) / (2 * h)
        assert abs(fd - ga[q]) <= 1e-9 * max(1.0, abs(ga[q]))
    for q in rng.choice(B.nnz, 20, replace=False):
        vp, vm = Bt.val.clone(), Bt.val.clone()
        vp[q] += h
        vm[q] -= h
        fd = (L(At.val, vp) - L(At.val, vm)) / (2 * h)
        assert abs(fd - gb[q]) <= 1e-9 * max(1.0, abs(gb[q]))


def _batch(count, seed, nmax=3000):
    rng = np.random.default_rng(seed)
    probs = gen.batched_problems(count, seed=seed, nmin=50, nmax=nmax)
    # add an empty problem and a rectangular one
    probs.append((gen.CSC(0, 0, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0)),
                  gen.CSC(0, 0, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0))))
    probs.append((gen.random_tiny(rng, 40, 70, 0.1, "uniform"),
                  gen.random_tiny(rng, 70, 33, 0.1, "uniform")))
    return probs


def test_batched_matches_oracle_and_single_path():
    _say("batched 40 problems")
    probs = _batch(38, seed=3)
    pairs = [(api.CscTensor.from_host(a), api.CscTensor.from_host(b)) for a, b in probs]
    outs = api.batched_matmul(pairs)
    torch.cuda.synchronize()
    for i, ((a, b), o) in enumerate(zip(probs, outs)):
        cp, ri, v = o.to_host()
        ocp, ori, ov = oracle.spgemm(a, b)
        assert_same_structure(cp, ri, ocp, ori, f"problem {i}")
        assert_values_exact(v, ov, f"problem {i}")
        if a.ncols and b.ncols:
            scp, sri, sv = gpu_product(a, b)
            assert np.array_equal(scp, cp) and np.array_equal(sri, ri) and np.array_equal(sv, v)


def test_batched_plan_reuse_other_counts():
    """One batch plan reused for batches of 3, 12 and 2 problems: the host
    mirror of the header and per-problem totals grows once and is then reused;
    every batch equals the oracle."""
    plan = None
    for k, seed in ((1, 11), (10, 12), (0, 13)):
        probs = _batch(k, seed=seed, nmax=1500)
        _say(f"batch plan reuse: {len(probs)} problems, seed {seed}")
        pairs = [(api.CscTensor.from_host(a), api.CscTensor.from_host(b)) for a, b in probs]
        plan, colptrs, nnzs = api.batched_symbolic(pairs, torch.float64, plan=plan)
        ris = [torch.empty(z, dtype=torch.int32, device="cuda") for z in nnzs]
        vals = [torch.empty(z, dtype=torch.float64, device="cuda") for z in nnzs]
        api.batched_numeric(plan, pairs, ris, vals)
        torch.cuda.synchronize()
        for i, (a, b) in enumerate(probs):
            ocp, ori, ov = oracle.spgemm(a, b)
            assert_same_structure(colptrs[i].cpu().numpy(), ris[i].cpu().numpy(), ocp, ori,
                                  f"batch of {len(probs)}, problem {i}")
            assert_values_exact(vals[i].cpu().numpy(), ov, f"batch of {len(probs)}, problem {i}")


def test_batched_f32():
    _say("batched f32")
    probs = [(a.astype(np.float32), b.astype(np.float32)) for a, b in _batch(12, seed=8)]
    pairs = [(api.CscTensor.from_host(a), api.CscTensor.from_host(b)) for a, b in probs]
    outs = api.batched_matmul(pairs)
    for i, ((a, b), o) in enumerate(zip(probs, outs)):
        cp, ri, v = o.to_host()
        ocp, ori, ov = oracle.spgemm(a, b, "f32")
        assert_same_structure(cp, ri, ocp, ori, f"problem {i}")
        assert_values_exact(v, ov, f"f32 problem {i}")


def test_plan_reuse_new_values():
    _say("plan reuse with new values")
    A = gen.uniform_z(5000, 10, seed=1)
    B = gen.uniform_z(5000, 10, seed=2)
    At, Bt = api.CscTensor.from_host(A), api.CscTensor.from_host(B)
    Cm, plan = api.matmul(At, Bt, return_plan=True)
    rng = np.random.default_rng(1)
    for r in range(3):
        av = rng.standard_normal(A.nnz)
        bv = rng.standard_normal(B.nnz)
        api.numeric(plan, torch.from_numpy(av).cuda(), torch.from_numpy(bv).cuda(), Cm.rowidx,
                    Cm.val)
        _, _, ov = oracle.spgemm(gen.CSC(A.nrows, A.ncols, A.colptr, A.rowidx, av),
                                 gen.CSC(B.nrows, B.ncols, B.colptr, B.rowidx, bv))
        assert_values_exact(Cm.val.cpu().numpy(), ov, f"reuse {r}")
    # symbolic again into the same plan (workspace reused) gives the same structure
    p2, cp2, nnz2 = api.symbolic(At, Bt, torch.float64, plan=plan, out_colptr=plan.colptr)
    assert nnz2 == Cm.nnz


def test_batched_numeric_graph_replay():
    """Capture the batched numeric phase in a HIP graph; replay it several times
    with new values copied into the captured inputs and eager work in between;
    every replay equals the oracle's product on that replay's values."""
    _say("graph replay of batched numeric")
    rng = np.random.default_rng(55)
    probs = _batch(10, seed=5, nmax=2000)
    pairs = [(api.CscTensor.from_host(a), api.CscTensor.from_host(b)) for a, b in probs]
    outs, plan = api.batched_matmul(pairs, return_plan=True)
    torch.cuda.synchronize()
    ris = [o.rowidx for o in outs]
    vals = [torch.zeros_like(o.val) for o in outs]
    api.batched_numeric(plan, pairs, ris, vals)  # uploads the pointer table once
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            api.batched_numeric(plan, pairs, ris, vals)
    torch.cuda.current_stream().wait_stream(s)
    for r in range(4):
        new_probs = []
        for (a, b), (at, bt) in zip(probs, pairs):
            av = rng.uniform(-1, 1, a.nnz)
            bv = rng.uniform(-1, 1, b.nnz)
            at.val.copy_(torch.from_numpy(av))
            bt.val.copy_(torch.from_numpy(bv))
            new_probs.append((gen.CSC(a.nrows, a.ncols, a.colptr, a.rowidx, av),
                              gen.CSC(b.nrows, b.ncols, b.colptr, b.rowidx, bv)))
        for v in vals:
            v.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i, ((a, b), v, ri) in enumerate(zip(new_probs, vals, ris)):
            ocp, ori, ov = oracle.spgemm(a, b)
            assert np.array_equal(ri.cpu().numpy(), ori), f"replay {r} problem {i}: rows"
            assert_values_exact(v.cpu().numpy(), ov, f"replay {r} problem {i}")
        # eager work between replays
        _ = gpu_product(*probs[0])


def _bad_case(kind):
    A = gen.uniform_z(300, 4, seed=1)
    B = gen.uniform_z(300, 4, seed=2)
    if kind == "b_row_out_of_range":
        ri = B.rowidx.copy()
        ri[17] = 300
        B = gen.CSC(B.nrows, B.ncols, B.colptr, ri, B.val)
    elif kind == "a_row_out_of_range":
        ri = A.rowidx.copy()
        ri[5] = -3
        A = gen.CSC(A.nrows, A.ncols, A.colptr, ri, A.val)
    elif kind == "b_colptr_decreasing":
        cp = B.colptr.copy()
        cp[10], cp[11] = cp[11], cp[10]
        B = gen.CSC(B.nrows, B.ncols, cp, B.rowidx, B.val)
    elif kind == "b_colptr_last":
        cp = B.colptr.copy()
        cp[-1] -= 1
        B = gen.CSC(B.nrows, B.ncols, cp, B.rowidx, B.val)
    elif kind == "a_without_columns":
        # A has no columns (its column pointers are one entry), B stores
        # entries: every row of B is out of range
        A = gen.CSC(300, 0, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0))
        cp = np.array([0, 2, 2, 3], np.int32)
        B = gen.CSC(0, 3, cp, np.zeros(3, np.int32), np.ones(3))
    return A, B


@pytest.mark.parametrize("kind", ["b_row_out_of_range", "a_row_out_of_range",
                                  "b_colptr_decreasing", "b_colptr_last", "a_without_columns"])
def test_device_input_checks(kind):
    """Malformed inputs are reported (SPGEMM_ERR_CSC) by the kernels' own
    range checks, which run before any index is used as an address."""
    _say(f"device check {kind}")
    A, B = _bad_case(kind)
    At, Bt = api.CscTensor.from_host(A), api.CscTensor.from_host(B)
    with pytest.raises(SpgemmError) as ei:
        api.symbolic(At, Bt, torch.float64)
    assert ei.value.status == 3


def test_validate_flag_detects_repeated_rows():
    _say("validate flag")
    A = gen.uniform_z(100, 3, seed=1)
    ri = A.rowidx.copy()
    ri[1] = ri[0]  # repeated row in column 0
    Ad = gen.CSC(A.nrows, A.ncols, A.colptr, ri, A.val)
    At = api.CscTensor.from_host(Ad)
    with pytest.raises(SpgemmError) as ei:
        api.symbolic(At, At, torch.float64, api.options(validate=True))
    assert ei.value.status == 3
    # without the flag the library still runs (memory-safe) and keeps rows ascending
    cp, ri2, v = gpu_product(Ad, Ad)
    for j in range(len(cp) - 1):
        assert np.all(np.diff(ri2[cp[j]:cp[j + 1]]) > 0)


def test_forward_backward_graph_replay():
    """Numeric forward and backward of one plan captured in a HIP graph; the
    graph is replayed with new values of A, B and G copied into the captured
    inputs, eager work in between; every replay's C, dA and dB equal the
    oracle's on that replay's values (FP32 twin, bit for bit)."""
    _say("graph replay of numeric forward + backward, FP32 n=3000")
    rng = np.random.default_rng(31)
    A = gen.uniform_z(3000, 6, seed=31, dist="normal", dtype=np.float32)
    B = gen.uniform_z(3000, 6, seed=32, dist="normal", dtype=np.float32)
    At, Bt = api.CscTensor.from_host(A), api.CscTensor.from_host(B)
    Cm, plan = api.matmul(At, Bt, return_plan=True)
    G = torch.from_numpy(gen.gradient_values(Cm.nnz, seed=33, dtype=np.float32)).cuda()
    dA, dB = torch.empty_like(At.val), torch.empty_like(Bt.val)
    api.backward(plan, At.val, Bt.val, Cm.rowidx, G, out=(dA, dB))  # builds the view
    torch.cuda.synchronize()
    ocp = Cm.colptr.cpu().numpy()
    ori = Cm.rowidx.cpu().numpy()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            api.numeric(plan, At.val, Bt.val, Cm.rowidx, Cm.val)
            api.backward(plan, At.val, Bt.val, Cm.rowidx, G, out=(dA, dB))
    torch.cuda.current_stream().wait_stream(s)
    for r in range(4):
        av = rng.standard_normal(A.nnz).astype(np.float32)
        bv = rng.standard_normal(B.nnz).astype(np.float32)
        gv = rng.standard_normal(Cm.nnz).astype(np.float32)
        At.val.copy_(torch.from_numpy(av))
        Bt.val.copy_(torch.from_numpy(bv))
        G.copy_(torch.from_numpy(gv))
        Cm.val.zero_()
        dA.zero_()
        dB.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        An = gen.CSC(A.nrows, A.ncols, A.colptr, A.rowidx, av)
        Bn = gen.CSC(B.nrows, B.ncols, B.colptr, B.rowidx, bv)
        wcp, wri, wv = oracle.spgemm(An, Bn, "f32")
        assert np.array_equal(ocp, wcp) and np.array_equal(ori, wri), f"replay {r}: structure"
        assert_values_exact(Cm.val.cpu().numpy(), wv, f"replay {r}: C")
        odA, odB = oracle.backward(An, Bn, wcp, wri, gv, "f32")
        assert_values_exact(dA.cpu().numpy(), odA, f"replay {r}: dA")
        assert_values_exact(dB.cpu().numpy(), odB, f"replay {r}: dB")
        # eager work between replays
        _ = gpu_product(A, B, dtype=np.float32)
    plan.close()
