#!/usr/bin/env python
"""Benchmark of the column-wise sparse product C = A x B on one MI355X.

A step is one pass of the whole hot path over one synthetic input: the
symbolic phase (product counts, accumulator binning, distinct-row counts,
column-pointer scan, one device-to-host copy of nnz(C)) and the numeric
phase (rows and values of C) -- i.e. C = A x B from scratch, excluding
allocation (the paper's protocol, Section 5.1).

Default workload: A, B square n = 1,000,000 with power-law column degrees
(truncated Zipf, exponent 2.0, degrees 1..2000, uniform rows, N(0,1) values,
seed 0), FP64, C = A x B. Inputs are resident in HBM before timing starts.

The single JSON line carries the metric (GFLOP/s = 2 x products / s), the
roofline of the dominant kernel (event-timed inside the timed region), the
oracle's CPU rate on the same workload, and two side measurements named by the
metric: forward+backward against forward on the n = 100,000 / 8-per-column
FP32 workload, and one batched launch set against a per-matrix loop.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
METRIC = "SpGEMM GFLOP/s + HBM GB/s vs peak; batched & fwd+bwd speedup vs plain"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--pilot-steps", type=int, default=5,
                    help="untimed steps with every kernel event-timed (per-kernel breakdown)")
    ap.add_argument("--n", type=int, default=1_000_000, help="columns of the power-law workload")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-runs", type=int, default=4)
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--t-esc", type=int, default=0, help="library option (0 = default)")
    ap.add_argument("--hash-cap", type=int, default=0, help="library option (0 = default)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="library defaults instead of autotuned thresholds")
    ap.add_argument("--one-stream", action="store_true",
                    help="library option: no overlap of accumulator kinds (per-kernel timings)")
    ap.add_argument("--cold-steps", type=int, default=5,
                    help="single steps timed after writing a 512 MiB buffer (caches flushed), "
                         "beside as many single warm steps")
    ap.add_argument("--configs", action="store_true",
                    help="only the small configurations (A*A n=1000 diagonal+4; Laplacian^2 "
                         "64x64; A*A n=4096 40/col): GPU one-call product and the oracle on 1 "
                         "and N host threads; prints one JSON line")
    ap.add_argument("--radix-esc", action="store_true",
                    help="library option: columns above 1024 products on the global radix ESC "
                         "(Section 4) instead of row windows")
    ap.add_argument("--accumulators", action="store_true",
                    help="every accumulator kind on the dense-bin, fixed-degree and power-law "
                         "workloads (one stream, event-timed launch groups); then exit")
    ap.add_argument("--lane-sweep", action="store_true",
                    help="only the lane-per-column hash accumulator against the wavefront "
                         "sort-merge on constant-Z inputs (Z in 2,4,5,6,8,10; n 2560 and "
                         "262144); prints one JSON line")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--tune-cache", default=None,
                    help="autotuner cache file (default: a temporary one); profiled runs "
                         "pass the timed run's file to reuse its options")
    ap.add_argument("--record-traffic", nargs=4,
                    metavar=("FETCH_DIR", "WRITE_DIR", "CAL_FETCH_DIR", "CAL_WRITE_DIR"),
                    help="no GPU: turn rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE output of this "
                         "benchmark and of --copy-calibration into profiles/traffic.json")
    ap.add_argument("--traffic-kernel", default="numeric",
                    help="launch group whose traffic --record-traffic records")
    return ap.parse_args()


def lane_sweep(reps=20):
    """C = A x B with every column of A and B holding exactly Z rows (Op = Z^2
    per column), the synthetic law of the paper's crossover study (Section
    5.2). A is 2560 x 2560; B has 2560 rows and n columns: n = 2560 (the
    paper's size) and n = 262144 (enough columns to fill the GPU while the
    rows stay within a dense per-lane accumulator). Each case runs the light
    columns through four accumulators on one stream: the wavefront sort-merge
    (default), the lane-per-column hash on the product space
    (SPGEMM_LANE_HASH), and the sorted, blocked lane columns of Section 3.1
    with a per-lane hash (SPGEMM_LANE_BLOCKED, HASH) or a per-lane dense
    accumulator (SPGEMM_LANE_SPARS, SPARS). Per one-call product: wall time
    and the event-timed accumulator groups."""
    import numpy as np
    import torch
    sys.path.insert(0, ROOT)
    from paper_2303_02471_amd import api, inputs as gen
    kinds = (("esc", {}), ("lane_hash", {"lane_hash": True}),
             ("blocked_hash", {"lane_blocked": True}),
             ("blocked_spars", {"lane_blocked": True, "lane_spars": True}))
    groups = ("esc_symbolic", "esc_numeric", "wave_symbolic", "wave_numeric", "lane_symbolic",
              "numeric")
    rows = []
    for n in (2560, 262144):
        for z in (2, 4, 5, 6, 8, 10):
            A = gen.uniform_z(2560, z, seed=41)
            B = gen.uniform_z(n, z, seed=42, nrows=2560)
            At, Bt = api.CscTensor.from_host(A), api.CscTensor.from_host(B)
            row = {"m": 2560, "n": n, "z": z, "op_per_column": z * z}
            ref = None
            for kind, kw in kinds:
                opts = api.options(one_stream=True, **kw)
                plan, colptr, ri, v, nnz = api.multiply(At, Bt, opts)
                out = (colptr, ri, v)
                for _ in range(3):
                    api.multiply(At, Bt, opts, plan=plan, out=out)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    api.multiply(At, Bt, opts, plan=plan, out=out)
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t0) * 1e3 / reps
                api.profile_select(None)
                api.profile_enable(True)
                for _ in range(3):
                    api.multiply(At, Bt, opts, plan=plan, out=out)
                torch.cuda.synchronize()
                api.profile_enable(False)
                prof = api.profile_read()
                acc = sum(prof[g][1] / prof[g][0] for g in groups if g in prof and prof[g][0])
                got = (colptr.cpu().numpy(), ri[:nnz].cpu().numpy(), v[:nnz].cpu().numpy())
                if ref is None:
                    ref = got
                same = all(np.array_equal(g, r) for g, r in zip(got, ref))
                st = plan.stats()
                row[kind] = {"ms": round(ms, 4), "accumulator_ms": round(acc, 4),
                             "same_output": bool(same), "lane_blocks": st["lane_blocks"]}
                plan.close()
            log(f"n={n} z={z}: " + " ".join(f"{k} {row[k]['ms']:.3f}/{row[k]['accumulator_ms']:.3f}"
                                           for k, _ in kinds))
            rows.append(row)
    # fixed block sizes (b_min = b_max, as in the paper's synthetic study,
    # where every block reaches b_max), n = 262144
    bmax_rows = []
    n = 262144
    for z in (2, 5, 8):
        A = gen.uniform_z(2560, z, seed=41)
        B = gen.uniform_z(n, z, seed=42, nrows=2560)
        At, Bt = api.CscTensor.from_host(A), api.CscTensor.from_host(B)
        for kind, kw in kinds[2:]:
            for bmax in (8, 16, 32, 64):
                opts = api.options(one_stream=True, b_min=bmax, b_max=bmax, **kw)
                plan, colptr, ri, v, nnz = api.multiply(At, Bt, opts)
                out = (colptr, ri, v)
                for _ in range(3):
                    api.multiply(At, Bt, opts, plan=plan, out=out)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    api.multiply(At, Bt, opts, plan=plan, out=out)
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t0) * 1e3 / reps
                bmax_rows.append({"z": z, "kind": kind, "b_max": bmax, "ms": round(ms, 4),
                                  "lane_blocks": plan.stats()["lane_blocks"]})
                plan.close()
            log(f"b_max sweep z={z} {kind}: " +
                " ".join(f"{r['b_max']}:{r['ms']:.3f}" for r in bmax_rows[-4:]))
    print(json.dumps({"lane_sweep": rows, "bmax_sweep": bmax_rows}), flush=True)


def host_threads():
    """Threads the N-thread oracle uses: OMP_NUM_THREADS when set (the GPU
    box sets it to its CPU share), else every host core."""
    try:
        n = int(os.environ.get("OMP_NUM_THREADS", "0"))
    except ValueError:
        n = 0
    return n if n > 0 else (os.cpu_count() or 1)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def accumulator_compare(reps=20):
    """Every accumulator kind of the library on the dense-bin configuration (A x A,
    n = 4096, 40 rows per column: 1600 products per column, FP64), the
    fixed-degree product of the forward+backward configuration (A x B,
    n = 100,000, 8 per column: 64 products per column, FP32) and the power-law
    product at n = 100,000 (FP64). Per kind: the one-call product on a reused
    plan (median of `reps` synchronised calls), the event time of every launch
    group, and the output compared with the default kind's (which is checked
    against the oracle). The kinds: the direct-gather sort-merge (default);
    the workgroup hash accumulator with direct indexing of row windows that
    fit (Section 3.2 HASH with the SPA of Section 2.2) for every column above
    4 products (t_esc = 4, t_block = -1); the same without direct indexing;
    the lane-per-column hash on the product space (SPGEMM_LANE_HASH); the
    sorted, blocked lane columns of Section 3.1 with HASH and (at most 4096
    rows) SPARS; the global radix ESC of Section 4 for the heavy columns."""
    import numpy as np
    import torch
    import oracle
    sys.path.insert(0, ROOT)
    from paper_2303_02471_amd import api, inputs as gen
    pl = gen.powerlaw(100_000, seed=5)
    cases = (("2b: A*A n=4096 40/col FP64", gen.uniform_z(4096, 40, seed=0), None),
             ("5: A*B n=100000 8/col FP32",
              gen.uniform_z(100_000, 8, seed=1, dist="normal", dtype=np.float32),
              gen.uniform_z(100_000, 8, seed=2, dist="normal", dtype=np.float32)),
             ("power-law A*B n=100000 FP64", pl[0], pl[1]))
    kinds = (("direct sort-merge (default)", {}),
             ("hash + direct-indexed windows", {"t_esc": 4, "t_block": -1}),
             ("hash only", {"t_esc": 4, "t_block": -1, "t_dense": 100000}),
             ("lane hash (product space)", {"lane_hash": True}),
             ("blocked lanes, HASH", {"lane_blocked": True}),
             ("blocked lanes, SPARS", {"lane_blocked": True, "lane_spars": True}),
             ("radix ESC for heavy columns", {"radix_esc": True}))
    plan_groups = ("classify", "tally", "place", "heavy_plan", "scan", "product_offsets")
    out = []
    for name, A, B in cases:
        B = A if B is None else B
        At, Bt = api.CscTensor.from_host(A), api.CscTensor.from_host(B)
        ocp, ori, ov = oracle.spgemm(A, B, "f32" if A.val.dtype == np.float32 else "f64")
        ref = None
        row = {"workload": name, "products": None, "kinds": {}}
        for kind, kw in kinds:
            if kw.get("lane_spars") and A.nrows > 4096:
                continue
            opts = api.options(one_stream=True, **kw)
            plan, colptr, ri, v, nnz = api.multiply(At, Bt, opts)
            o = (colptr, ri, v)
            for _ in range(3):
                api.multiply(At, Bt, opts, plan=plan, out=o)
            torch.cuda.synchronize()
            ts = []
            for _ in range(reps):
                c0 = time.perf_counter()
                api.multiply(At, Bt, opts, plan=plan, out=o)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - c0)
            api.profile_select(None)
            api.profile_enable(True)
            for _ in range(3):
                api.multiply(At, Bt, opts, plan=plan, out=o)
            torch.cuda.synchronize()
            api.profile_enable(False)
            prof = api.profile_read()
            groups = {g: round(t / c, 4) for g, (c, t) in prof.items() if c}
            acc = sum(t for g, t in groups.items() if g not in plan_groups)
            got = (colptr.cpu().numpy(), ri[:nnz].cpu().numpy(), v[:nnz].cpu().numpy())
            if ref is None:
                ref = got
                row["equals_oracle"] = bool(np.array_equal(got[0], ocp) and np.array_equal(got[1], ori)
                                            and np.array_equal(got[2], ov))
            row["products"] = int(plan.stats()["total_products"])
            row["kinds"][kind] = {"ms": round(statistics.median(ts) * 1e3, 4),
                                  "accumulator_ms": round(acc, 4), "groups_ms": groups,
                                  "same_output": bool(all(np.array_equal(g, r) for g, r in zip(got, ref)))}
            plan.close()
        log(name + ": " + ", ".join(f"{k} {d['ms']:.3f}/{d['accumulator_ms']:.3f}"
                                    for k, d in row["kinds"].items()))
        out.append(row)
    print(json.dumps({"accumulators": out}), flush=True)


def configs_table(reps=50):
    """The small configurations, each C = A x A in FP64: A n=1000 with its
    diagonal and 4 random rows per column; the 5-point Laplacian on 64 x 64;
    A n=4096 with 40 random rows per column. Per configuration: the one-call
    product on the GPU (plan and output arrays reused; median of `reps`
    synchronised calls and the pipelined mean), GFLOP/s (2 x products),
    compulsory GB/s (|A| + |A| + |C|), the oracle on one thread and on N
    threads (median of 3), and the output compared with the oracle's."""
    import numpy as np
    import torch
    import oracle
    sys.path.insert(0, ROOT)
    from paper_2303_02471_amd import api, inputs as gen
    cases = (("1: A*A n=1000 diag+4", gen.diag_plus_random(1000, 4, seed=0)),
             ("2a: Laplacian^2 64x64", gen.laplacian_2d(64)),
             ("2b: A*A n=4096 40/col", gen.uniform_z(4096, 40, seed=0)))
    nthr = host_threads()
    out = []
    for name, A in cases:
        At = api.CscTensor.from_host(A)
        plan, colptr, ri, v, nnz = api.multiply(At, At)
        o = (colptr, ri, v)
        for _ in range(5):
            api.multiply(At, At, plan=plan, out=o)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            c0 = time.perf_counter()
            api.multiply(At, At, plan=plan, out=o)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - c0)
        c0 = time.perf_counter()
        for _ in range(reps):
            api.multiply(At, At, plan=plan, out=o)
        torch.cuda.synchronize()
        tpipe = (time.perf_counter() - c0) / reps
        ops = int(plan.stats()["total_products"])
        got = (colptr.cpu().numpy(), ri[:nnz].cpu().numpy(), v[:nnz].cpu().numpy())
        plan.close()
        t1, tn = [], []
        for _ in range(3):
            c0 = time.perf_counter()
            ref = oracle.spgemm(A, A)
            t1.append(time.perf_counter() - c0)
            c0 = time.perf_counter()
            _, _, _, used = oracle.spgemm_parallel(A, A, nthreads=nthr, nnz_hint=nnz)
            tn.append(time.perf_counter() - c0)
        same = all(np.array_equal(g, r) for g, r in zip(got, ref))
        tg = statistics.median(ts)
        comp = 2 * csc_bytes(A.ncols, A.nnz, 8) + csc_bytes(A.ncols, nnz, 8)
        row = {"config": name, "products": ops, "nnz_c": int(nnz),
               "gpu_ms": round(tg * 1e3, 4), "gpu_pipelined_ms": round(tpipe * 1e3, 4),
               "gflops": round(2 * ops / tg / 1e9, 3),
               "compulsory_GBps": round(comp / tg / 1e9, 2),
               "compulsory_frac": round(comp / tg / 1e9 / HBM_PEAK_GBS, 5),
               "oracle_1thread_ms": round(statistics.median(t1) * 1e3, 3),
               "oracle_nthread_ms": round(statistics.median(tn) * 1e3, 3), "threads": used,
               "output_equals_oracle": bool(same)}
        log(str(row))
        out.append(row)
    print(json.dumps({"configs": out, "nproc": os.cpu_count(), "cpu_model": cpu_model()}),
          flush=True)


def copy_calibration():
    """A plain device-to-device copy of exactly 1 GiB, three times: the
    FETCH_SIZE / WRITE_SIZE counters of this kernel against its 1 GiB read and
    1 GiB write give the scale factor of the HBM byte counters."""
    import torch
    n = 1 << 30
    src = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n, "launches": 3}), flush=True)


# launch group -> kernel symbol (FP64 runs)
# launch groups whose HBM traffic --record-traffic can record: the kernels of
# one launch of the group (their per-dispatch traffic adds up)
KERNEL_SYMBOL = {"heavy_numeric": ("k_heavy_expand<double, true>",
                                   "k_acc_window<unsigned int, double, true>"),
                 "wave_numeric": ("k_acc_wave<unsigned int, double, 16, 1024, true>",
                                  "k_acc_wave<unsigned int, double, 8, 512, true>",
                                  "k_acc_wave<unsigned int, double, 4, 128, true>",
                                  "k_acc_wave<unsigned int, double, 4, 256, true>"),
                 "esc_numeric": ("k_acc_lane<unsigned int, double, 4, true>",
                                 "k_acc_lane<unsigned int, double, 8, true>",
                                 "k_acc_wave<unsigned int, double, 4, 16, true>",
                                 "k_acc_wave<unsigned int, double, 4, 32, true>",
                                 "k_acc_wave<unsigned int, double, 4, 64, true>"),
                 "numeric": ("k_numeric<double>",), "expand": ("k_expand",)}


def _src_digest():
    """Digest of the library sources: traffic counters taken on other sources
    are stale."""
    import glob
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2303_02471_amd", "csrc")
    for f in sorted(glob.glob(os.path.join(csrc, "*"))):
        h.update(os.path.basename(f).encode())
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def _pmc_rows(d):
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        rows += list(csv.DictReader(open(f)))
    return rows


def _per_dispatch(rows, counter, symbol):
    v = [float(r["Counter_Value"]) for r in rows
         if r["Counter_Name"] == counter and symbol in r["Kernel_Name"]]
    return sum(v) / len(v) if v else None, len(v)


def record_traffic(args):
    """HBM-side bytes per launch of one kernel from two rocprofv3 --pmc runs
    (FETCH_SIZE, WRITE_SIZE, KiB per dispatch), each scaled by what the same
    counter reads for a plain 1 GiB device copy."""
    fdir, wdir, cfdir, cwdir = args.record_traffic
    syms = KERNEL_SYMBOL[args.traffic_kernel]
    frows, wrows = _pmc_rows(fdir), _pmc_rows(wdir)
    fetch = write = 0.0
    nf, nw = [], []
    for sym in syms:
        f1, n1 = _per_dispatch(frows, "FETCH_SIZE", sym)
        w1, n2 = _per_dispatch(wrows, "WRITE_SIZE", sym)
        if f1 is None or w1 is None:
            raise SystemExit(f"no {sym} dispatch in the counter runs")
        fetch += f1
        write += w1
        nf.append(n1)
        nw.append(n2)
    sym = list(syms)
    cfetch, _ = _per_dispatch(_pmc_rows(cfdir), "FETCH_SIZE", "copyBuffer")
    cwrite, _ = _per_dispatch(_pmc_rows(cwdir), "WRITE_SIZE", "copyBuffer")
    gib_kib = float(1 << 20)
    fs, ws = gib_kib / cfetch, gib_kib / cwrite
    out = {"kernel_key": args.traffic_kernel, "kernel_symbol": sym,
           "workload": f"powerlaw_n{args.n}",
           "fetch_kib_per_dispatch": round(fetch, 1), "write_kib_per_dispatch": round(write, 1),
           "dispatches": [nf, nw],
           "copy_calibration": {"copy_bytes": 1 << 30, "fetch_kib": cfetch, "write_kib": cwrite,
                                "fetch_scale": round(fs, 4), "write_scale": round(ws, 4)},
           "hbm_bytes_per_launch": int(round((fetch * fs + write * ws) * 1024)),
           "source_digest": _src_digest()}
    # one entry per launch group
    path = os.path.join(ROOT, "profiles", "traffic.json")
    allg = {}
    if os.path.exists(path):
        old = json.load(open(path))
        allg = old.get("groups", {}) if "groups" in old else {}
    allg[args.traffic_kernel] = out
    with open(path, "w") as f:
        json.dump({"groups": allg}, f, indent=1)
    print(json.dumps(out))


def csc_bytes(n, nnz, vb):
    return 4 * (n + 1) + (4 + vb) * nnz


def per_column_work(A, B, t_esc=256, t_block=2 ** 31 - 1):
    """Host accounting of the per-column work and of the accumulator each
    column goes to (the library's rule), for algorithmic byte counts."""
    import numpy as np
    za = np.diff(A.colptr.astype(np.int64))
    nb = np.diff(B.colptr.astype(np.int64))
    colB = np.repeat(np.arange(B.ncols), nb)
    op = np.bincount(colB, weights=za[B.rowidx], minlength=B.ncols).astype(np.int64)
    esc_max = 4
    while esc_max < t_esc:
        esc_max *= 2
    esc = (op > 0) & (op <= esc_max)
    blk = (op > esc_max) & (op > t_block)
    srt = (op > esc_max) & ~blk
    # direct-gather accumulators by stream: lane bins and wavefront groups of
    # at most 64 products (esc); wavefront groups above 64 and one-column
    # waves up to 1024 products (wave); heavy columns above (heavy)
    return op, nb, {"esc": esc & (op <= 64), "wave": (esc & (op > 64)) | (srt & (op <= 1024)),
                    "heavy": srt & (op > 1024),
                    "sort512": srt & (op <= 512), "sort1k": srt & (op > 512) & (op <= 1024),
                    "sort2k": srt & (op > 1024) & (op <= 2048),
                    "sort4k": srt & (op > 2048) & (op <= 4096), "wsort": srt & (op > 4096),
                    "block512": blk & (op <= 512), "block1k": blk & (op > 512) & (op <= 1024),
                    "block2k": blk & (op > 1024) & (op <= 2048),
                    "block4k": blk & (op > 2048) & (op <= 4096), "block_xl": blk & (op > 4096)}


def kernel_bytes(op, nb, nnzc, sel, vb):
    """Algorithmic bytes of the accumulator kernels over the columns `sel`.
    numeric: B column pointer 4 per column, B entry (4+vb) + A column pointer
    pair 8 per stored B entry, (4+vb) per product (A row and value), C column
    pointer 4 per column, (4+vb) per output entry. symbolic: 4 per column, 12
    per stored B entry, 4 per product, 4 per column (the count)."""
    s_nb, s_op, s_nnz, ncol = int(nb[sel].sum()), int(op[sel].sum()), int(nnzc[sel].sum()), int(sel.sum())
    num = 4 * ncol + (4 + vb + 8) * s_nb + (4 + vb) * s_op + 4 * ncol + (4 + vb) * s_nnz
    sym = 4 * ncol + 12 * s_nb + 4 * s_op + 4 * ncol
    return num, sym


def main():
    args = parse()
    if args.record_traffic:
        record_traffic(args)
        return
    if args.copy_calibration:
        copy_calibration()
        return
    if args.lane_sweep:
        lane_sweep()
        return
    if args.configs:
        configs_table()
        return
    if args.accumulators:
        accumulator_compare()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU only; multi-GPU sharding "
                          "is not implemented", "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2303_02471_amd import api
    from paper_2303_02471_amd import inputs as gen

    assert torch.cuda.is_available(), "needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    # ------------------------------------------------------------ workload
    t0 = time.time()
    A, B = gen.powerlaw(args.n, seed=0)
    log(f"generated n={args.n} nnzA={A.nnz} nnzB={B.nnz} in {time.time() - t0:.1f}s")
    At, Bt = api.CscTensor.from_host(A), api.CscTensor.from_host(B)
    vb = 8
    tuning = None
    if args.no_autotune or args.t_esc or args.hash_cap or args.radix_esc:
        opts = api.options(t_esc=args.t_esc, hash_cap=args.hash_cap, one_stream=args.one_stream,
                           radix_esc=args.radix_esc)
    else:
        # thresholds chosen by the library's autotuner (outside the timed region;
        # the options never change results)
        with tempfile.TemporaryDirectory() as td:
            opts, trep = api.autotune([(At, Bt)], torch.float64,
                                      cache_path=args.tune_cache or os.path.join(td, "tune.json"))
        if args.one_stream:
            opts.flags |= 2
        tuning = {"t_esc": opts.t_esc, "t_block": opts.t_block, "t_split": opts.t_split,
                  "hash_cap": opts.hash_cap,
                  "dense_rows": opts.dense_rows, "trials": trep["trials"],
                  "default_ms": round(trep["default_ms"], 4), "tuned_ms": round(trep["best_ms"], 4)}
        log(f"autotune: {tuning}")
    plan, colptr, nnz = api.symbolic(At, Bt, torch.float64, opts)
    rowidx = torch.empty(nnz, dtype=torch.int32, device=dev)
    val = torch.empty(nnz, dtype=torch.float64, device=dev)
    stats = plan.stats()
    total_op = stats["total_products"]
    log(f"plan: {stats}")

    def step():
        # one library call: symbolic, then numeric queued behind it on the
        # output arrays of the first call (their capacity is nnz(C))
        api.multiply(At, Bt, opts, plan=plan, out=(colptr, rowidx, val))

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("warmup done")

    # pilot (untimed): every launch group event-timed, for the per-kernel
    # breakdown and to name the dominant kernel
    api.profile_select(None)
    api.profile_enable(True)
    for _ in range(args.pilot_steps):
        step()
    torch.cuda.synchronize()
    api.profile_enable(False)
    pilot = api.profile_read()
    dom = max(pilot.items(), key=lambda kv: kv[1][1])[0]

    # timed region: the whole step, with HIP events around the dominant
    # kernel's launches only (on the stream they run on)
    api.profile_select(dom)
    api.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    api.profile_enable(False)
    prof_dom = api.profile_read()
    api.profile_select(None)
    ms = (t1 - t0) * 1e3 / args.steps
    gflops = 2.0 * total_op / (ms * 1e-3) / 1e9
    log(f"timed {args.steps} steps: {ms:.3f} ms/step, {gflops:.1f} GFLOP/s")

    # ------------------------------------------------------------ roofline of the dominant kernel
    nnzc = np.diff(colptr.cpu().numpy().astype(np.int64))
    t_block = {0: 2 ** 31 - 1, -1: 0}.get(opts.t_block, opts.t_block)
    op, nb, bins = per_column_work(A, B, t_esc=opts.t_esc or 256, t_block=t_block)
    kbytes = {}
    for name in bins:
        num, sym = kernel_bytes(op, nb, nnzc, bins[name], vb)
        kbytes[f"{name}_numeric"] = num
        kbytes[f"{name}_symbolic"] = sym
    # one numeric launch does every column (tiles and chunks of large ones)
    kbytes["numeric"] = kernel_bytes(op, nb, nnzc, op > 0, vb)[0]
    heavy_prod = int(op[bins["heavy"]].sum())
    kbytes["heavy_plan"] = 4 * int(bins["heavy"].sum())
    # expansion: (A column start, length) per stored B entry, A row read and
    # product row written per product
    kbytes["expand"] = 8 * B.nnz + 8 * int(op.sum())
    kbytes["classify"] = 4 * (B.ncols + 1) + 12 * B.nnz + 12 * B.ncols
    kbytes["place"] = 8 * B.ncols
    kbytes["product_offsets"] = 4 * B.ncols + 8 * B.ncols
    kbytes["scan"] = 4 * B.ncols + 4 * (B.ncols + 1) + 8 * B.ncols
    kernels = {}
    for name, (launches, tot) in pilot.items():
        avg = tot / launches
        kb = kbytes.get(name)
        kernels[name] = {"avg_ms": round(avg, 4), "launches": launches,
                         "GBps": None if kb is None or avg <= 0 else round(kb / (avg * 1e-3) / 1e9, 1)}
    dom_launches, dom_total = prof_dom[dom]
    dom_avg_s = dom_total / dom_launches * 1e-3
    achieved = kbytes[dom] / dom_avg_s / 1e9
    traffic = None
    tfile = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tfile):
        tj = json.load(open(tfile)).get("groups", {}).get(dom, {})
        if tj.get("workload") == f"powerlaw_n{args.n}" and tj.get("source_digest") == _src_digest():
            traffic = tj.get("hbm_bytes_per_launch")
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "algorithmic_bytes": int(kbytes[dom]),
                "avg_launch_ms": round(dom_avg_s * 1e3, 4), "launches_timed": dom_launches}
    compulsory = csc_bytes(A.ncols, A.nnz, vb) + csc_bytes(B.ncols, B.nnz, vb) + \
        csc_bytes(B.ncols, nnz, vb)
    log(f"dominant kernel {dom}: {achieved:.0f} GB/s")

    # ------------------------------------------------------------ cold steps
    # Single steps, each after a 512 MiB buffer is written (twice the MALL,
    # many times the L2s): the inputs come from HBM. The same number of single
    # warm steps (no flush, same synchronisation) is timed beside them.
    cold = None
    if args.cold_steps > 0:
        flush = torch.empty(512 << 20, dtype=torch.uint8, device=dev)

        def single(flushed):
            if flushed:
                flush.fill_(1)
            torch.cuda.synchronize()
            api.profile_select(dom)
            api.profile_enable(True)
            c0 = time.perf_counter()
            step()
            torch.cuda.synchronize()
            t = time.perf_counter() - c0
            api.profile_enable(False)
            launches, tot = api.profile_read()[dom]
            api.profile_select(None)
            return t * 1e3, tot / launches

        warm1 = [single(False) for _ in range(args.cold_steps)]
        cold1 = [single(True) for _ in range(args.cold_steps)]
        cms = statistics.median(x[0] for x in cold1)
        cdom = statistics.median(x[1] for x in cold1)
        cold = {"ms_per_step": round(cms, 4), "value": round(2.0 * total_op / (cms * 1e-3) / 1e9, 2),
                "warm_single_ms_per_step": round(statistics.median(x[0] for x in warm1), 4),
                "flush_bytes": 512 << 20, "steps": args.cold_steps,
                "hbm_compulsory_frac": round(compulsory / (cms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "dominant_avg_launch_ms": round(cdom, 4),
                "dominant_warm_single_ms": round(statistics.median(x[1] for x in warm1), 4),
                "dominant_frac": round(kbytes[dom] / (cdom * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        del flush
        log(f"cold single steps: {cold}")

    # ------------------------------------------------------------ CPU baseline (the oracle)
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        times = []
        for r in range(args.cpu_runs):
            c0 = time.perf_counter()
            ref = oracle.spgemm(A, B)
            times.append(time.perf_counter() - c0)
            log(f"oracle run {r}: {times[-1]:.2f}s")
        # the timed steps' output against the oracle's, bit for bit
        torch.cuda.synchronize()
        got = (colptr.cpu().numpy(), rowidx[:nnz].cpu().numpy(), val[:nnz].cpu().numpy())
        same = all(np.array_equal(g, o) for g, o in zip(got, ref))
        log(f"output of the timed steps equals the oracle's: {same}")
        tmed = statistics.median(times)
        # the same oracle with whole columns spread over host threads
        nthr = host_threads()
        ptimes, used, psame = [], 0, True
        for r in range(args.cpu_runs):
            c0 = time.perf_counter()
            pcp, pri, pv, used = oracle.spgemm_parallel(A, B, nthreads=nthr, nnz_hint=nnz)
            ptimes.append(time.perf_counter() - c0)
            psame &= all(np.array_equal(g, o) for g, o in zip((pcp, pri, pv), ref))
            log(f"oracle on {used} threads, run {r}: {ptimes[-1]:.2f}s")
        pmed = statistics.median(ptimes)
        cpu = {"value": round(2.0 * total_op / tmed / 1e9, 5), "unit": "GFLOP/s", "cores": 1,
               "kind": "oracle",
               "sample": f"full workload (symbolic + numeric), median of {args.cpu_runs} "
                         f"single-thread runs, {tmed:.2f} s each",
               "output_equals_oracle": bool(same),
               "threads": {"value": round(2.0 * total_op / pmed / 1e9, 5), "unit": "GFLOP/s",
                           "cores": used, "seconds": round(pmed, 3),
                           "sample": f"full workload, median of {args.cpu_runs} runs, whole "
                                     f"columns over {used} OpenMP threads",
                           "equals_single_thread": bool(psame)},
               "nproc": os.cpu_count(), "cpu_model": cpu_model()}

    # ------------------------------------------------------------ side measurements
    extras = {}
    if not args.no_extras:
        extras["fwd_bwd"] = fwd_bwd(api, gen, np, torch)
        extras["batched"] = batched(api, gen, np, torch, args.batch_count,
                                    tune=not args.no_autotune)

    out = {
        "metric": METRIC, "value": round(gflops, 2), "unit": "GFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"C=A*B, A and B n={args.n} square CSC, power-law column degrees "
                               "(Zipf 2.0, max 2000), uniform rows, N(0,1), FP64, seed 0",
                   "n": args.n, "nnz_a": A.nnz, "nnz_b": B.nnz, "products": int(total_op),
                   "nnz_c": int(nnz), "parallelism": "single GPU"},
        "hbm_compulsory_GBps": round(compulsory / (ms * 1e-3) / 1e9, 1),
        "hbm_compulsory_frac": round(compulsory / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "roofline": roofline,
        "cold": cold,
        "tuning": tuning,
        "kernels": kernels,
        "cpu_baseline": cpu,
    }
    out.update(extras)
    print(json.dumps(out), flush=True)


def fwd_bwd(api, gen, np, torch, n=100_000, z=8, reps=20):
    """t(numeric forward + backward) / t(numeric forward) on a fixed pattern."""
    A = gen.uniform_z(n, z, seed=1, dist="normal", dtype=np.float32)
    B = gen.uniform_z(n, z, seed=2, dist="normal", dtype=np.float32)
    At, Bt = api.CscTensor.from_host(A), api.CscTensor.from_host(B)
    Cm, plan = api.matmul(At, Bt, return_plan=True)
    G = torch.from_numpy(gen.gradient_values(Cm.nnz, seed=3, dtype=np.float32)).cuda()
    dA, dB = torch.empty_like(At.val), torch.empty_like(Bt.val)

    def fwd():
        api.numeric(plan, At.val, Bt.val, Cm.rowidx, Cm.val)

    def fb():
        fwd()
        api.backward(plan, At.val, Bt.val, Cm.rowidx, G)

    def timeit(fn):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / reps

    tf, tfb = timeit(fwd), timeit(fb)
    # the same step captured once in a HIP graph and replayed (fixed pattern,
    # the values read from the captured arrays at every replay)
    api.backward(plan, At.val, Bt.val, Cm.rowidx, G, out=(dA, dB))
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    cs = torch.cuda.Stream()
    cs.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cs):
        with torch.cuda.graph(g, stream=cs):
            fwd()
            api.backward(plan, At.val, Bt.val, Cm.rowidx, G, out=(dA, dB))
    torch.cuda.current_stream().wait_stream(cs)
    tg = timeit(g.replay)
    log(f"fwd {tf:.3f} ms, fwd+bwd {tfb:.3f} ms, fwd+bwd graph replay {tg:.3f} ms")
    return {"workload": f"n={n}, {z} per column, FP32", "fwd_ms": round(tf, 4),
            "fwd_bwd_ms": round(tfb, 4), "fwd_bwd_over_fwd": round(tfb / tf, 3),
            "fwd_bwd_graph_ms": round(tg, 4), "fwd_bwd_graph_over_fwd": round(tg / tf, 3)}


def batched(api, gen, np, torch, count, reps=5, tune=True):
    """One batched launch set against a loop of per-matrix calls, same kernels
    and options (autotuned on the batch); numeric also replayed as a HIP graph."""
    probs = gen.batched_problems(count, seed=0)
    pairs = [(api.CscTensor.from_host(a), api.CscTensor.from_host(b)) for a, b in probs]
    opts = api.autotune(pairs, torch.float64)[0] if tune else None
    outs, bplan = api.batched_matmul(pairs, opts, return_plan=True)
    nnzs = bplan.nnzs
    rowidxs = [o.rowidx for o in outs]
    vals = [o.val for o in outs]
    plans = []
    for (a, b), o in zip(pairs, outs):
        _, p = api.matmul(a, b, opts, return_plan=True)
        plans.append(p)

    def t_batched():
        bplan2, cps, _ = api.batched_symbolic(pairs, torch.float64, opts, plan=bplan)
        api.batched_numeric(bplan, pairs, rowidxs, vals)

    def t_loop():
        for (a, b), p, ri, v in zip(pairs, plans, rowidxs, vals):
            api.symbolic(a, b, torch.float64, opts, plan=p, out_colptr=p.colptr)
            api.numeric(p, a.val, b.val, ri, v)

    def t_batched_num():
        api.batched_numeric(bplan, pairs, rowidxs, vals)

    def t_loop_num():
        for (a, b), p, ri, v in zip(pairs, plans, rowidxs, vals):
            api.numeric(p, a.val, b.val, ri, v)

    def timeit(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / reps

    tb, tl = timeit(t_batched), timeit(t_loop)
    tbn, tln = timeit(t_batched_num), timeit(t_loop_num)
    # numeric phase captured once in a HIP graph and replayed
    t_batched_num()
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(graph, stream=stream):
            api.batched_numeric(bplan, pairs, rowidxs, vals, stream=stream)
    tgn = timeit(graph.replay)
    log(f"batched {tb:.2f} ms vs loop {tl:.2f} ms; numeric {tbn:.2f} vs {tln:.2f}; "
        f"numeric graph replay {tgn:.2f}")
    # per size decile (problems ranked by products): the decile's problems as
    # one batched call against the loop of their single calls
    ops = np.array([p.stats()["total_products"] for p in plans], dtype=np.int64)
    deciles = []
    for d, idx in enumerate(np.array_split(np.argsort(ops, kind="stable"), 10)):
        sub = [pairs[i] for i in idx]
        souts, sbplan = api.batched_matmul(sub, opts, return_plan=True)
        sri = [o.rowidx for o in souts]
        sv = [o.val for o in souts]

        def t_sub_batched():
            api.batched_symbolic(sub, torch.float64, opts, plan=sbplan)
            api.batched_numeric(sbplan, sub, sri, sv)

        def t_sub_loop():
            for i in idx:
                a, b = pairs[i]
                api.symbolic(a, b, torch.float64, opts, plan=plans[i], out_colptr=plans[i].colptr)
                api.numeric(plans[i], a.val, b.val, rowidxs[i], vals[i])

        sb, sl = timeit(t_sub_batched), timeit(t_sub_loop)
        deciles.append({"decile": d, "problems": len(idx),
                        "products": int(ops[idx].sum()),
                        "products_per_problem": [int(ops[idx].min()), int(ops[idx].max())],
                        "batched_ms": round(sb, 3), "loop_ms": round(sl, 3),
                        "speedup": round(sl / sb, 3)})
        sbplan.close()
    log("batched speed-up per size decile: " +
        " ".join(f"{x['decile']}:{x['speedup']:.2f}" for x in deciles))
    return {"workload": f"{count} problems, n log-uniform [500, 20000], 2..40 per column, FP64",
            "products": int(sum(p.stats()["total_products"] for p in plans)),
            "nnz_c": int(sum(nnzs)),
            "batched_ms": round(tb, 3), "per_matrix_loop_ms": round(tl, 3),
            "speedup": round(tl / tb, 3),
            "numeric_batched_ms": round(tbn, 3), "numeric_loop_ms": round(tln, 3),
            "numeric_speedup": round(tln / tbn, 3),
            "numeric_graph_ms": round(tgn, 3), "numeric_graph_speedup": round(tln / tgn, 3),
            "deciles": deciles}


if __name__ == "__main__":
    main()
