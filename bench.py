"""Benchmark: useful FP64 GFLOP/s of the filtered block-sparse multiply.

One step = one full multiply C = A.B of the banded workload (2000 x 2000
blocks of sizes {5,13,23}, band probability 0.5*exp(-|i-j|/40), values
N(0,1)*exp(-|i-j|/20), filter eps 1e-8): block norms, symbolic phase with the
single size readback, and the numeric kernels.  Inputs are resident in HBM
before timing starts.  Prints one JSON line, which also carries the
roofline of the dominant numeric kernel (timed live with HIP events on the
library's stream), the split-precision forms on the same workload and the
64-problem batch (FP64 and bf16x3, replayed from a HIP graph), each with its
error against FP64, the tall-skinny multiply, the rank-3 contraction
(forward and forward + backward, with the forward's fraction of the HBM
roofline) and the CPU oracle's rate on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-extra]
       python bench.py --traffic-from FETCH_CSV WRITE_CSV --copy-bytes N
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "useful FP64 GFLOP/s of block-sparse C+=A·B; % FP64 roofline; split vs FP64"
PEAK_FP64 = 78.6e12       # MI355X dense FP64 (vector and matrix core), FLOP/s
PEAK_HBM = 8.0e12         # MI355X HBM3E, B/s
KERNEL_SRC = os.path.join(ROOT, "paper_1910_13555_amd", "csrc", "bsm_numeric_core.h")
SEQUENTIAL = False   # --sequential: numeric kernel families one after another
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "numeric_traffic_banded.json")
TUNED = os.path.join(ROOT, "paper_1910_13555_amd", "tuned", "banded.json")
# numeric kernel families (bsm_ctx_launch_times order) and their names in profiler output
FAMILIES = ["FP64 4x4x4, tiles <= 16 wide", "FP64 4x4x4, 24 wide", "FP64 4x4x4, 32 wide",
            "FP64 16x16x4, 16 x 16", "FP64 16x16x4, 32 wide"]
KERNEL_NAME = "bsm::k_numeric<false, false, false, {}>"


def kernel_source_hash() -> str:
    """Hash of the numeric kernels' source and of the tile-class table that
    decides which classes each kernel family serves: the recorded traffic of
    a family holds only while both are unchanged."""
    h = hashlib.sha256()
    for path in (KERNEL_SRC, TUNED):
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def recorded_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    runs, or None if the kernel source changed since they were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch", {}).get(kernel)


def kernel_of(c, v):
    """Kernel family of tile class c under variant v (mirrors the library's table)."""
    if v == 0:
        return 2 if (c // 4 == 3 or c % 4 == 3) else (1 if (c // 4 == 2 or c % 4 == 2) else 0)
    return 3 if (c // 4 < 2 and c % 4 < 2) else 4


def family_flops(plan, A, B, variants):
    """Useful flops of each numeric kernel family: 2*mt*nt*K per product and
    output tile (tiles of at most 32 x 32; class from the padded tile shape)."""
    import numpy as np
    a, b, c = plan.export_stack()
    _, ac, _ = A.pattern.export()
    cr, cc, _ = plan.c_pattern().export()
    rs = np.asarray(A.row_sizes, np.int64)
    ks = np.asarray(A.col_sizes, np.int64)
    cs = np.asarray(B.col_sizes, np.int64)
    M, N, K = rs[cr[c]], cs[cc[c]], ks[ac[a]]
    fam_of_cls = np.array([kernel_of(k, int(variants[k])) for k in range(16)])
    out = np.zeros(5)
    if len(M) == 0:
        return out
    for tr in range(int((M.max() + 31) // 32)):
        mt = np.clip(M - 32 * tr, 0, 32)
        for tc in range(int((N.max() + 31) // 32)):
            nt = np.clip(N - 32 * tc, 0, 32)
            ok = (mt > 0) & (nt > 0)
            cls = ((mt[ok] + 7) // 8 - 1) * 4 + (nt[ok] + 7) // 8 - 1
            np.add.at(out, fam_of_cls[cls], 2.0 * mt[ok] * nt[ok] * K[ok])
    return out


def compulsory_bytes(plan, A, B, beta):
    """Touched A and B blocks read once, C_out written once (C_in read if beta != 0)."""
    import numpy as np
    a, b, _ = plan.export_stack()
    _, _, aoff = A.pattern.export()
    _, _, boff = B.pattern.export()
    alen = np.diff(np.append(aoff, A.pattern.nvals))
    blen = np.diff(np.append(boff, B.pattern.nvals))
    return 8 * (int(alen[np.unique(a)].sum()) + int(blen[np.unique(b)].sum()) + plan.info["c_nvals"])


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(d, nrows=1000):
    """The CPU oracle (block loop, numpy/BLAS) timed on a bounded sample of
    output block rows (every second one by default), with BLAS on all the
    threads its pool uses (the host's cores unless OMP_NUM_THREADS or the like
    limit them; that count is reported) and again on one thread."""
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import blocksparse as ob
    A = ob.BlockSparse.from_workload(d["A"])
    B = ob.BlockSparse.from_workload(d["B"])
    n = len(d["A"]["row_sizes"])
    rows = set(range(0, n, max(1, n // nrows)))

    def blas_threads():   # what the BLAS pools will actually use
        t = [p["num_threads"] for p in threadpool_info() if p.get("user_api") == "blas"]
        return max(t) if t else 1

    cores = blas_threads()
    res = {}
    for threads in (cores, 1):
        with threadpool_limits(threads):
            assert blas_threads() == threads
            t0 = time.perf_counter()
            _, trip = ob.multiply(A, B, eps=d["eps"], rows=rows)
            res[threads] = time.perf_counter() - t0
    f = ob.flop_count(A, B, trip)
    return {"value": f / res[cores] / 1e9, "unit": "GFLOP/s", "cores": cores, "kind": "oracle",
            "sample": f"{len(rows)} of {n} output block rows of the same workload "
                      f"({len(trip)} products, {f / 1e9:.3f} GFLOP), block-loop oracle, "
                      f"BLAS on {cores} threads {res[cores]:.1f} s, on 1 thread {res[1]:.1f} s",
            "single_thread_value": f / res[1] / 1e9, "cpu_model": cpu_model()}


def traffic_from_counters(fetch_csv, write_csv, copy_bytes):
    """HBM bytes per launch of each numeric kernel from two rocprofv3 --pmc runs
    (FETCH_SIZE, WRITE_SIZE; KiB per dispatch), each scaled by what the same
    counter read for the plain copy of copy_bytes in the same run.  Writes the
    result next to the committed profiles, keyed by the kernel source hash."""
    import csv
    from collections import defaultdict

    def per_kernel(path, counter):
        vals = defaultdict(list)
        with open(path) as f:
            for row in csv.DictReader(f):
                if row.get("Counter_Name") == counter:
                    vals[row["Kernel_Name"]].append(float(row["Counter_Value"]))
        return vals

    rec = {"kernel_source_sha256_16": kernel_source_hash(), "copy_bytes": copy_bytes,
           "counters": {}, "hbm_bytes_per_launch": {}}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        pk = per_kernel(path, counter)
        # the runtime's device copy kernel; the largest dispatch is the calibration copy
        copies = [max(v) for k, v in pk.items() if "copyBuffer" in k]
        if not copies:
            raise SystemExit(f"{path}: no copy kernel rows for {counter}")
        scale = copy_bytes / (max(copies) * 1024.0)
        mine = {k.split("(")[0].replace("void ", ""): sum(v) / len(v) for k, v in pk.items() if "k_numeric" in k}
        rec["counters"][counter] = {"copy_kib": max(copies), "scale": scale, "kib_per_dispatch": mine}
        for k, v in mine.items():
            rec["hbm_bytes_per_launch"][k] = rec["hbm_bytes_per_launch"].get(k, 0.0) + v * 1024.0 * scale
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec["hbm_bytes_per_launch"]))


def rel_err(x, ref):
    import torch
    den = torch.linalg.vector_norm(ref).item()
    num = torch.linalg.vector_norm(x - ref).item()
    return num / den if den > 0 else num


def time_events(fn, reps, stream):
    """Average GPU time (ms) of fn() over reps calls, HIP events on the launch stream."""
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def roofline_section(bsm, ctx, plan, A, B, out, reps):
    """Dominant numeric kernel: its useful flops per launch over its launch
    time, both measured here (HIP events recorded by the library around each
    of its launches, on its stream).  The families run one after another for
    this measurement, so each launch time is that kernel's own."""
    import numpy as np
    flops = family_flops(plan, A, B, bsm.bsm_tune_get())
    ctx.set_concurrent(False)
    ctx.set_timing(True)
    times = np.zeros(5)
    for _ in range(reps):
        plan.execute(1.0, A.values, B.values, 0.0, None, out)
        times += np.asarray(ctx.launch_times())
    ctx.set_timing(False)
    ctx.set_concurrent(not SEQUENTIAL)
    times /= reps
    k = int(np.argmax(times))
    achieved = flops[k] / (times[k] * 1e-3)
    name = KERNEL_NAME.format(k)
    return {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64, "traffic": recorded_traffic(name),
            "kernel": name, "family": FAMILIES[k], "launch_ms": float(times[k]),
            "algorithmic_flops_per_launch": float(flops[k]),
            "families_ms": [round(float(t), 4) for t in times],
            "families_gflop": [round(float(f) / 1e9, 4) for f in flops]}


def split_section(bsm, ctx, A, B, eps, ref, reps, stream):
    """Split-precision numeric phase on the same workload: rate and error vs the FP64 result."""
    import torch
    res = {}
    for scheme in ("bf16x3", "bf16x6"):
        plan = bsm.bsm_multiply_plan(ctx, A.pattern, A.values, B.pattern, B.values, None, eps,
                                     precision=scheme)
        out = torch.empty(plan.info["c_nvals"], dtype=torch.float64, device=ref.device)
        plan.execute(1.0, A.values, B.values, 0.0, None, out)
        ms = time_events(lambda: plan.execute(1.0, A.values, B.values, 0.0, None, out), reps, stream)
        res[scheme] = {"numeric_ms": ms, "useful_gflops": plan.info["flops"] / (ms * 1e-3) / 1e9,
                       "rel_frob_err_vs_fp64": rel_err(out, ref)}
        del plan, out
    return res


def batched_section(bsm, reps, stream):
    """The 64-problem batch: one merged launch per kernel family replayed from
    a HIP graph, in FP64 and again in bf16x3 (error vs the FP64 batch)."""
    import torch
    import workloads
    probs = workloads.batched()
    ctx = bsm.default_context()
    tuned = os.path.join(ROOT, "paper_1910_13555_amd", "tuned", "batched.json")
    if os.path.exists(tuned):
        bsm.bsm_tune_load(tuned)          # the autotuner's table for this workload
    mats = [(bsm.BlockSparseMatrix.from_workload(p["A"], ctx=ctx),
             bsm.BlockSparseMatrix.from_workload(p["B"], ctx=ctx)) for p in probs]
    a = [m[0].values for m in mats]
    b = [m[1].values for m in mats]
    res = {"workload": "batched_64", "problems": len(probs)}
    ref = None
    for prec in ("fp64", "bf16x3"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plans = [bsm.bsm_multiply_plan(ctx, A.pattern, A.values, B.pattern, B.values, None, p["eps"],
                                       precision=prec) for (A, B), p in zip(mats, probs)]
        torch.cuda.synchronize()
        plan_s = time.perf_counter() - t0
        flops = sum(pl.info["flops"] for pl in plans)
        batch = bsm.bsm_batch_create(ctx, plans)
        outs = batch.execute(1.0, a, b, use_graph=True)
        ms = time_events(lambda: batch.execute(1.0, a, b, out=outs, use_graph=True), reps, stream)
        ent = {"graph_ms": ms, "useful_gflops": flops / (ms * 1e-3) / 1e9, "plan_s": plan_s,
               "products": sum(pl.info["nprod"] for pl in plans), "useful_gflop": flops / 1e9}
        if prec == "fp64":
            ent["pct_fp64_peak"] = 100.0 * flops / (ms * 1e-3) / PEAK_FP64
            ref = outs
        else:
            num = sum(torch.linalg.vector_norm(o - r).item() ** 2 for o, r in zip(outs, ref))
            den = sum(torch.linalg.vector_norm(r).item() ** 2 for r in ref)
            ent["rel_frob_err_vs_fp64"] = (num / den) ** 0.5
        res[prec] = ent
        batch.close()
        del batch, plans
        if prec != "fp64":
            del outs
    del ref
    torch.cuda.empty_cache()
    res["tuning"] = bsm.bsm_tune_get()
    if os.path.exists(TUNED):
        bsm.bsm_tune_load(TUNED)
    return res


def tall_skinny_section(bsm, reps, stream):
    """The tall-skinny case (Sec. 3.1 shape): full multiply (plan + numeric) and
    the numeric phase alone, C_in dense with beta = 1 accumulated in place."""
    import torch
    import workloads
    d = workloads.tall_skinny()
    ctx = bsm.default_context()
    tuned = os.path.join(ROOT, "paper_1910_13555_amd", "tuned", "tall_skinny.json")
    if os.path.exists(tuned):
        bsm.bsm_tune_load(tuned)          # the autotuner's table for this workload
    A = bsm.BlockSparseMatrix.from_workload(d["A"], ctx=ctx)
    B = bsm.BlockSparseMatrix.from_workload(d["B"], ctx=ctx)
    Cm = bsm.BlockSparseMatrix.from_workload(d["C"], ctx=ctx)
    cin = Cm.values.clone()

    def full():
        plan = bsm.bsm_multiply_plan(ctx, A.pattern, A.values, B.pattern, B.values, Cm.pattern, d["eps"])
        plan.execute(d["alpha"], A.values, B.values, d["beta"], cin, cin)
        return plan

    plan = full()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plans = [full() for _ in range(reps)]
    torch.cuda.synchronize()
    full_ms = (time.perf_counter() - t0) * 1e3 / reps
    del plans
    ms = time_events(lambda: plan.execute(d["alpha"], A.values, B.values, d["beta"], cin, cin), reps, stream)
    F = plan.info["flops"]
    # bound by HBM: touched A and B blocks read once, the C blocks that get
    # products read and written once (the others are left untouched in place)
    import numpy as np
    a, b, c = plan.export_stack()
    lens = lambda pat, n: np.diff(np.append(pat.export()[2], n))
    comp = 8 * (int(lens(A.pattern, A.pattern.nvals)[np.unique(a)].sum())
                + int(lens(B.pattern, B.pattern.nvals)[np.unique(b)].sum())
                + 2 * int(lens(plan.c_pattern(), plan.info["c_nvals"])[np.unique(c)].sum()))
    res = {"workload": d["name"], "products": plan.info["nprod"], "useful_gflop": F / 1e9,
           "ms_per_multiply": full_ms, "gflops": F / (full_ms * 1e-3) / 1e9,
           "numeric_ms": ms, "numeric_gflops": F / (ms * 1e-3) / 1e9,
           "numeric_compulsory_mb": comp / 1e6, "numeric_hbm_frac": comp / (ms * 1e-3) / PEAK_HBM,
           "run": bsm.bsm_tune_get_run(), "group": bsm.bsm_tune_get_group()}
    if os.path.exists(TUNED):
        bsm.bsm_tune_load(TUNED)
    return res


def rank3_section(bsm, reps, stream):
    """The rank-3 contraction T[mu,nu,P] M[nu,lambda] -> R[mu,lambda,P] (Sec. 4):
    forward (plan + numeric) and the autograd backward."""
    import numpy as np
    import torch
    import workloads
    d = workloads.rank3()
    ctx = bsm.default_context()
    sz = d["sizes"]
    T = bsm.BlockSparseTensor.from_lists([sz["mu"], sz["nu"], sz["P"]], d["T_idx"], d["T_values"], ctx=ctx)
    Mi = np.stack([d["M_rows"], d["M_cols"]], 1).astype(np.int32)
    M = bsm.BlockSparseTensor.from_lists([sz["nu"], sz["lam"]], Mi, d["M_values"], ctx=ctx)
    T.values.requires_grad_(True)
    M.values.requires_grad_(True)
    out = bsm.contract("mnP,nl->mlP", T, M)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        out = bsm.contract("mnP,nl->mlP", T, M)
    torch.cuda.synchronize()
    fwd_ms = (time.perf_counter() - t0) * 1e3 / reps
    F = out.plan.info["flops"]
    g = torch.ones_like(out.values)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        T.values.grad = None
        M.values.grad = None
        out = bsm.contract("mnP,nl->mlP", T, M)
        out.values.backward(g)
    torch.cuda.synchronize()
    fb_ms = (time.perf_counter() - t0) * 1e3 / reps
    # the forward is bound by HBM: R written once (beta = 0) and T, M read once
    comp = 8.0 * (out.values.numel() + T.values.numel() + M.values.numel())
    res = {"workload": d["name"], "products": out.plan.info["nprod"], "useful_gflop_forward": F / 1e9,
           "forward_ms": fwd_ms, "forward_gflops": F / (fwd_ms * 1e-3) / 1e9,
           "forward_compulsory_gb": comp / 1e9,
           "forward_hbm_frac": comp / (fwd_ms * 1e-3) / PEAK_HBM,
           "forward_backward_ms": fb_ms, "forward_backward_gflops": 3 * F / (fb_ms * 1e-3) / 1e9}
    r_values = out.values.numel()
    del out, g
    T.values.grad = None
    M.values.grad = None
    ctx.release_cache()          # the one-piece runs' buffers
    torch.cuda.empty_cache()
    res["chunked"] = rank3_chunked(bsm, T, M, F, r_values)
    return res


def rank3_chunked(bsm, T, M, F, r_values, budget=16 << 30):
    """The same contraction and its gradient streamed in chunks of the tall
    first mode under a device-memory budget for each chunk (two chunks in
    flight on two streams): each chunk's output is reduced (<1, R_c>) and
    its gradient (ones) handed back, so R is never held whole.  The device
    memory in use beyond the inputs and their gradients is sampled (free
    memory) at every chunk of a first run that starts from empty caches; the
    second run is timed."""
    import torch
    Tv, Mv = T.values.detach(), M.values.detach()
    Tt = bsm.BlockSparseTensor(T.pattern, Tv)
    Mt = bsm.BlockSparseTensor(M.pattern, Mv)
    dT, dM = torch.empty_like(Tv), torch.empty_like(Mv)
    used = []

    def consume(c, Rc, stream):
        used.append(free0 - torch.cuda.mem_get_info()[0])
        Rc.values.sum()
        return torch.ones_like(Rc.values)

    # run 1 from empty caches: the growth of device memory in use is the
    # chunked run's working set (torch's and the library's caches grow to
    # it and keep it); run 2 reuses those caches and is timed
    torch.cuda.synchronize()
    bsm.release_chunk_contexts()
    torch.cuda.empty_cache()
    free0 = torch.cuda.mem_get_info()[0]
    bounds = bsm.contract_chunked("mnP,nl->mlP", Tt, Mt, budget, consume, dT1=dT, dT2=dM)
    torch.cuda.synchronize()
    peak = max(used + [free0 - torch.cuda.mem_get_info()[0]])
    t0 = time.perf_counter()
    bounds = bsm.contract_chunked("mnP,nl->mlP", Tt, Mt, budget, consume, dT1=dT, dT2=dM)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    bsm.release_chunk_contexts()
    return {"chunks": len(bounds) - 1, "budget_gb": budget / 2 ** 30, "forward_backward_ms": ms,
            "forward_backward_gflops": 3 * F / (ms * 1e-3) / 1e9,
            "working_set_gb": peak / 2 ** 30,
            "unchunked_output_and_gradient_gb": 16.0 * r_values / 2 ** 30}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--sequential", action="store_true",
                    help="numeric kernel families one after another (default: concurrent on side streams)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the split-precision and batched sections")
    ap.add_argument("--rank3", action="store_true",
                    help="run the rank-3 contraction (13.5 GB tensor; about a minute of setup) also "
                         "with --no-extra (the default run includes it)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="first run one plain device-to-device copy of this many bytes "
                         "(calibrates HBM byte counters of a profiler run)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="no benchmark: turn two rocprofv3 counter CSVs (taken with --copy-bytes) "
                         "into the recorded HBM traffic of the numeric kernels")
    args = ap.parse_args()
    if args.traffic_from:
        traffic_from_counters(args.traffic_from[0], args.traffic_from[1], args.copy_bytes)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              f"(asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1910_13555_amd as bsm
    import workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if os.path.exists(TUNED):
        bsm.bsm_tune_load(TUNED)          # tile-class variants chosen by the autotuner
    dev = torch.device("cuda:0")
    d = workloads.banded()
    A = bsm.BlockSparseMatrix.from_workload(d["A"])
    B = bsm.BlockSparseMatrix.from_workload(d["B"])
    ctx = A.pattern.ctx
    global SEQUENTIAL
    SEQUENTIAL = args.sequential
    ctx.set_concurrent(not SEQUENTIAL)
    eps = d["eps"]
    stream = torch.cuda.current_stream(dev)
    if args.copy_bytes > 0:
        src = torch.ones(args.copy_bytes // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def step(ev=None):
        plan = bsm.bsm_multiply_plan(ctx, A.pattern, A.values, B.pattern, B.values, None, eps)
        out = torch.empty(plan.info["c_nvals"], dtype=torch.float64, device=dev)
        if ev is not None:
            ev[0].record(stream)
        plan.execute(1.0, A.values, B.values, 0.0, None, out)
        if ev is not None:
            ev[1].record(stream)
        return plan, out

    # a 512 MB write before each timed step evicts the 256 MB last-level
    # cache, which would otherwise hold the 233 MB of A and B from the step
    # before (the write itself is outside the timed region)
    evict = torch.empty(512 << 20, dtype=torch.uint8, device=dev)
    for _ in range(args.warmup):
        plan, out = step()
        plan = None
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    per_step = []
    plan = None
    for k in range(args.steps):
        plan = None     # the previous step's plan returns its memory to the library's cache
        evict.fill_(k & 0xff)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan, out = step(evs[k])
        torch.cuda.synchronize()
        per_step.append((time.perf_counter() - t0) * 1e3)
    ms_step = sum(per_step) / args.steps
    numeric_ms = sum(e0.elapsed_time(e1) for e0, e1 in evs) / args.steps
    info = plan.info
    # per-phase device times (library events on its stream): median of five
    # more steps, each after the cache eviction
    ctx.set_timing(True)
    ph = []
    for k in range(5):
        evict.fill_(k + 1)
        torch.cuda.synchronize()
        plan2, out2 = step()
        ph.append(ctx.phase_times())
        del plan2, out2
    phases = [round(sorted(p[i] for p in ph)[2], 4) for i in range(4)]
    ctx.set_timing(False)
    # the same steps back to back without the eviction (operands left in the
    # Infinity Cache by the previous step), for comparison with measurements
    # taken that way
    plan2 = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        plan2 = None
        plan2, out2 = step()
    torch.cuda.synchronize()
    ms_warm = (time.perf_counter() - t0) * 1e3 / args.steps
    del plan2, out2, evict

    # numeric phase alone (plan reuse, as in repeated multiplies with a fixed pattern)
    reuse_ms = time_events(lambda: plan.execute(1.0, A.values, B.values, 0.0, None, out), args.steps,
                           stream)

    F = info["flops"]
    Bytes = compulsory_bytes(plan, A, B, 0.0)
    t_roof = max(F / PEAK_FP64, Bytes / PEAK_HBM)
    res = {
        "metric": METRIC,
        "value": F / (ms_step * 1e-3) / 1e9,
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "ms_per_step_median": float(sorted(per_step)[len(per_step) // 2]),
        "ms_per_step_min": float(min(per_step)),
        "ms_per_step_back_to_back_no_eviction": ms_warm,
        "phase_ms": {"norms": phases[0], "symbolic": phases[1], "step_lists": phases[2], "numeric": phases[3]},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": d["name"], "block_rows": 2000, "block_sizes": [5, 13, 23],
                   "pattern": "P(i,j)=0.5*exp(-|i-j|/40)", "filter_eps": eps,
                   "products": info["nprod"], "candidates": info["ncand"],
                   "c_blocks": info["c_nblk"], "useful_gflop": F / 1e9,
                   "compulsory_bytes": Bytes},
        "pct_fp64_roofline": 100.0 * t_roof * 1e3 / ms_step,
        "t_roof_ms": t_roof * 1e3,
        "numeric_ms": numeric_ms,
        "numeric_only_gflops": F / (reuse_ms * 1e-3) / 1e9,
        "roofline": roofline_section(bsm, ctx, plan, A, B, out, args.steps),
        "tuning": bsm.bsm_tune_get(),
        "concurrent_families": not SEQUENTIAL,
    }
    if not args.no_extra:
        res["split"] = split_section(bsm, ctx, A, B, eps, out, args.steps, stream)
        del plan, out
        torch.cuda.empty_cache()
        res["batched"] = batched_section(bsm, max(2, args.steps // 4), stream)
        res["tall_skinny"] = tall_skinny_section(bsm, max(2, args.steps // 4), stream)
    if args.rank3 or not args.no_extra:
        tuned = os.path.join(ROOT, "paper_1910_13555_amd", "tuned", "rank3.json")
        if os.path.exists(tuned):
            bsm.bsm_tune_load(tuned)      # the autotuner's table for this workload
        try:
            res["rank3"] = rank3_section(bsm, 3, stream)
            res["rank3"]["tuning"] = bsm.bsm_tune_get()
            res["rank3"]["run"] = bsm.bsm_tune_get_run()
        except (RuntimeError, MemoryError) as e:   # reported, not fatal to the main line
            res["rank3"] = {"error": str(e)[:300]}
        torch.cuda.empty_cache()
        bsm.bsm_tune_load(TUNED)
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(d)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
