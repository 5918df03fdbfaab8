"""Benchmark: RU-QLP throughput on one MI355X.

One step = one full decomposition (Gaussian sketch, 2q+2 products with A,
2q+2 CholeskyQR2 factorizations, L = R^T) of the 8000 x 8000 float32 gapped
workload, k = 200, p = 10, q = 1, with A already resident in HBM.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                    [--no-cpu-baseline] [--copy-calibration]

Prints one JSON line.  `value` is algorithmic GFLOP/s = F_alg / time, with
F_alg = 2 m n d (2q + 2) + sum over the QRs of (4 r d^2 - 4 d^3 / 3).
`roofline` is for the dominant kernel (the dense product on the matrix
cores), timed with HIP events recorded by the library on the launch stream
during the timed steps.  `cpu_baseline` times the float64 oracle on the host.
"""

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {  # MI355X published dense peaks
    "bf16_mfma_tflops": 2500.0,
    "f32_mfma_tflops": 157.3,
    "f64_mfma_tflops": 78.6,
    "hbm_gbs": 8000.0,
}

WORKLOADS = {
    "dense8000": dict(kind="dense", m=8000, n=8000, k=200, p=10, q=1, dtype="f32", spectrum="gapped"),
    "dense8000_q0": dict(kind="dense", m=8000, n=8000, k=200, p=10, q=0, dtype="f32", spectrum="gapped"),
    "small_fp64": dict(kind="dense", m=1000, n=800, k=20, p=5, q=0, dtype="f64", spectrum="geometric"),
    "csr100k": dict(kind="csr", m=100000, n=50000, k=100, p=10, q=1, dtype="f32", density=1e-3),
    # the same 8000^2 workload in the paper's own row-sketch orientation (Algorithm 1 as printed)
    "paper_dense8000": dict(kind="dense", m=8000, n=8000, k=200, p=10, q=1, dtype="f32", spectrum="gapped",
                            paper=True),
    # a batch of 64 uneven requests of the serving stream (float32, q = 1)
    # the same 8000^2 workload in the SVD-like form of Remark 1
    "svd_dense8000": dict(kind="dense", m=8000, n=8000, k=200, p=10, q=1, dtype="f32", spectrum="gapped",
                          svd=True),
    "batch64": dict(kind="batch", count=64, q=1, dtype="f32"),
    # the serving stream: 4096 Poisson-arrival requests over 64 distinct matrices
    "serve4096": dict(kind="serve", count=4096, pool=64, q=1, dtype="f32", slots=8, tick=2, budget_gb=8.0),
    # bfloat16 products with float32 accumulation, float64 Gram and Cholesky
    "bf16_20000x15000": dict(kind="dense", m=20000, n=15000, k=500, p=20, q=1, dtype="f32",
                             spectrum="polynomial", bf16=True),
}


def f_alg(m, n, k, p, q):
    d = k + p
    qr = lambda r: 4.0 * r * d * d - 4.0 * d ** 3 / 3.0  # noqa: E731
    prods = 2.0 * m * n * d * (2 * q + 2)
    qrs = qr(m) * (q + 1) + qr(n) * (q + 1)
    return prods + qrs


def f_alg_paper(m, n, k, p, q):
    """F_alg of the row-sketch orientation: the same products and tall QRs
    plus the d x d QR of R^T and the product P-bar P-tilde."""
    d = k + p
    return f_alg(m, n, k, p, q) + (4.0 * d ** 3 - 4.0 * d ** 3 / 3.0) + 2.0 * n * d * d


def f_alg_csr(nnz, m, n, k, p, q):
    d = k + p
    qr = lambda r: 4.0 * r * d * d - 4.0 * d ** 3 / 3.0  # noqa: E731
    return 2.0 * nnz * d * (2 * q + 2) + qr(m) * (q + 1) + qr(n) * (q + 1)


# source files that define each timed kernel class (for the traffic and
# MFMA records); the bfloat16 workloads time the bfloat16 product kernel
KERNEL_SOURCES = {
    "gemm_nn": ["k_gemm.hip", "common.h", "kernels.h"],
    "gemm_tn": ["k_gemm.hip", "common.h", "kernels.h"],
    "spmm": ["k_csr.hip", "common.h", "kernels.h"],
}
BF16_GEMM_SOURCES = ["k_bf16.hip", "common.h", "kernels.h"]


# workloads whose timed products are the same kernels on the same shapes as
# another workload's, so that they share its counter records
RECORD_ALIAS = {"dense8000_q0": "dense8000"}


def kernel_source_hash(kernel, workload):
    names = KERNEL_SOURCES[kernel]
    if workload.startswith("bf16") and kernel in ("gemm_nn", "gemm_tn"):
        names = BF16_GEMM_SOURCES
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(ROOT, "paper_2209_12464_amd", "csrc", name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(workload, kernel, path=None):
    """HBM bytes per launch of `kernel` from the rocprofv3 FETCH_SIZE and
    WRITE_SIZE runs recorded in profiles/traffic.json, if they were taken on
    the kernel's current sources; else None."""
    path = path or os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    ent = rec.get(RECORD_ALIAS.get(workload, workload), {}).get(kernel)
    if not ent or ent.get("source_hash") != kernel_source_hash(kernel, workload):
        return None
    return ent.get("bytes_per_launch")


def load_mfma_record(workload, kernel, path=None):
    """MFMA utilization (fraction of SIMD cycles with the matrix core busy)
    and shader clock of `kernel` from the rocprofv3 SQ_VALU_MFMA_BUSY_CYCLES /
    GRBM_GUI_ACTIVE run recorded in profiles/mfma.json, if taken on the
    kernel's current sources; else (None, None)."""
    path = path or os.path.join(ROOT, "profiles", "mfma.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None, None
    ent = rec.get(RECORD_ALIAS.get(workload, workload), {}).get(kernel)
    if not ent or ent.get("source_hash") != kernel_source_hash(kernel, workload):
        return None, None
    return ent.get("mfma_util"), ent.get("clock_ghz")


def record_mfma(workload, pmc_csv, simds=1024, xcds=8, path=None):
    """MFMA utilization per dispatch of the timed product kernels from a
    rocprofv3 counter CSV holding SQ_VALU_MFMA_BUSY_CYCLES (summed over all
    SIMDs) and GRBM_GUI_ACTIVE (summed over the XCDs): busy / (active / xcds
    * simds); stored in profiles/mfma.json with the kernel's source hash,
    together with the shader clock the dispatches ran at (active cycles per
    XCD over the dispatch's duration)."""
    import csv
    busy = read_counter(pmc_csv, "SQ_VALU_MFMA_BUSY_CYCLES")
    active = read_counter(pmc_csv, "GRBM_GUI_ACTIVE")
    dur, mops_name = {}, None
    with open(pmc_csv) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] == "GRBM_GUI_ACTIVE":
                dur.setdefault(r["Kernel_Name"], []).append(
                    (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9)
            elif r["Counter_Name"].startswith("SQ_INSTS_VALU_MFMA_MOPS_"):
                mops_name = r["Counter_Name"]
    mops = read_counter(pmc_csv, mops_name) if mops_name else {}
    path = path or os.path.join(ROOT, "profiles", "mfma.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        rec = {}
    out = {}
    for name, bv in busy.items():
        if name not in active:
            continue
        if "rqlp::gemm_bf16_kernel" in name:
            # one kernel for both products: dispatches alternate A X, A^T X
            parts = (("gemm_nn", slice(0, None, 2)), ("gemm_tn", slice(1, None, 2)))
        else:
            cls = kernel_class(name)
            if cls is None:
                continue
            parts = ((cls, slice(None)),)
        for cls, sl in parts:
            b, a = bv[sl], active[name][sl]
            util = [x / (y / xcds * simds) for x, y in zip(b, a)]
            ent = {"mfma_util": float(np.mean(util)), "dispatches": len(util),
                   "busy_cycles": float(np.mean(b)), "gui_active_per_xcd": float(np.mean(a)) / xcds,
                   "source_hash": kernel_source_hash(cls, workload)}
            if name in dur:
                ent["clock_ghz"] = float(np.mean([y / xcds / t for y, t in zip(a, dur[name][sl])])) / 1e9
            if name in mops:
                ent["mfma_flops"] = float(np.mean(mops[name][sl])) * 512.0
                ent["mfma_mops_counter"] = mops_name
            out[cls] = ent
    rec[workload] = out
    with open(path, "w") as f:
        json.dump(rec, f, indent=1, sort_keys=True)
    print(json.dumps({workload: out}, indent=1), flush=True)


def make_inputs(w, seed):
    import workloads
    if w["kind"] == "dense":
        if w["spectrum"] == "gapped":
            c = workloads.cfg_gapped_fp32(seed=seed, m=w["m"], n=w["n"], q=w["q"])
            return c["A"]
        if w["spectrum"] == "polynomial":
            return workloads.cfg_poly_bf16(seed=seed, m=w["m"], n=w["n"])["A"]
        c = workloads.cfg_small_fp64(seed=seed)
        return c["A"]
    c = workloads.cfg_sparse(seed=seed, m=w["m"], n=w["n"], density=w["density"])
    return c


METRIC_NAMES = {
    "dense8000": "RU-QLP GFLOP/s (8000^2 FP32, k=200, p=10, q=1)",
    "bf16_20000x15000": "RU-QLP GFLOP/s (20000x15000, k=500, p=20, q=1, BF16 products + FP32 accumulation)",
    "paper_dense8000": "RU-QLP GFLOP/s (8000^2 FP32, k=200, p=10, q=1, row-sketch orientation of Algorithm 1)",
    "svd_dense8000": "RU-QLP SVD-like form GFLOP/s (8000^2 FP32, k=200, p=10, q=1, Remark 1)",
}


def _recon_stats(torch, A, factors_a, factors_b=None, rows=2048):
    """||A - Q L V^T||_F / ||A||_F of factors_a and, if factors_b is given,
    ||Qa La Va^T - Qb Lb Vb^T||_F / ||A||_F, in float64 on the device, by row
    blocks (measurement only, outside any timed region)."""
    Qa, La, Va = (x.double() for x in factors_a)
    LVa = La @ Va.T
    if factors_b is not None:
        Qb, Lb, Vb = (x.double() for x in factors_b)
        LVb = Lb @ Vb.T
    nA2 = e2 = dd2 = 0.0
    for r0 in range(0, A.shape[0], rows):
        Ab = A[r0:r0 + rows].double()
        Ra = Qa[r0:r0 + rows] @ LVa
        nA2 += float((Ab * Ab).sum())
        e2 += float(((Ab - Ra) ** 2).sum())
        if factors_b is not None:
            dd2 += float(((Ra - Qb[r0:r0 + rows] @ LVb) ** 2).sum())
    return np.sqrt(e2 / nA2), (np.sqrt(dd2 / nA2) if factors_b is not None else None)


def compare_with_fp32(rqlp, ctx, A, k, p, q, args, out_bf16, ws_fp32_steps):
    """The plain float32 form on the same GPU and input: its time per step,
    both reconstruction errors and their difference Delta."""
    import torch
    m, n = A.shape
    d = k + p
    ws = rqlp.alloc_workspace(rqlp.workspace_size(m, n, k, p, q, A.dtype), A.device)
    out = tuple(torch.empty_like(x) for x in out_bf16)
    f32 = lambda: rqlp.decompose(A, k, p, q, seed=args.seed, ctx=ctx, workspace=ws, out=out)  # noqa: E731
    for _ in range(max(1, args.warmup)):
        f32()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(ws_fp32_steps):
        f32()
    torch.cuda.synchronize()
    ms32 = (time.perf_counter() - t0) * 1e3 / ws_fp32_steps
    e_bf, delta = _recon_stats(torch, A, out_bf16, out)
    e_32, _ = _recon_stats(torch, A, out)
    del ws
    return {"fp32_ms_per_step": ms32, "e_bf16": e_bf, "e_fp32": e_32, "delta_bf16_vs_fp32": delta,
            "d": d}


def run_serve_bench(args, w, rqlp, torch, dev):
    """Serving stream: first all requests at once (saturated throughput),
    then Poisson arrivals at 0.5, 0.8 and 0.95 of that rate, with p50 / p99
    of completion - arrival.  Request i decomposes pool matrix i % pool with
    its own seed and its own output buffers."""
    import workloads
    pool = workloads.serving_requests(w["pool"], args.seed)
    As = [torch.from_numpy(workloads.request_matrix(r, np.float32)).to(dev) for r in pool]
    n_req, q = w["count"], w["q"]
    req = [(i % w["pool"], 1000 + i) for i in range(n_req)]
    outs = []
    for j, _ in req:
        r = pool[j]
        d = r["k"] + r["p"]
        outs.append((torch.empty((r["m"], d), device=dev), torch.empty((d, d), device=dev),
                     torch.empty((r["n"], d), device=dev)))
    flops = sum(f_alg(pool[j]["m"], pool[j]["n"], pool[j]["k"], pool[j]["p"], q) for j, _ in req)
    ctx = rqlp.Context(0)
    slots = args.slots or w["slots"]
    tick = args.tick or w["tick"]
    srv = rqlp.Server(int(w["budget_gb"] * 2 ** 30), slots=slots, ctx=ctx, max_tick=tick)

    def run(arrivals):
        """Submit request i at arrivals[i] (seconds from the start); return
        (wall seconds, completion - arrival per request)."""
        cnt = len(arrivals)
        done_at = np.zeros(cnt)
        tick = {}
        i = ndone = 0
        t0 = time.perf_counter()
        while ndone < cnt:
            now = time.perf_counter() - t0
            while i < cnt and arrivals[i] <= now:
                j, seed = req[i]
                r = pool[j]
                tick[srv.submit(As[j], r["k"], r["p"], q, seed, outs[i])] = i
                i += 1
            fin, _, _ = srv.poll()
            if fin:
                now = time.perf_counter() - t0
                for t in fin:
                    done_at[tick[t]] = now
                ndone += len(fin)
        return time.perf_counter() - t0, done_at - np.asarray(arrivals)

    run(np.zeros(min(n_req, 256)))  # warm-up
    torch.cuda.synchronize()
    wall, lat = run(np.zeros(n_req))
    sat_rps = n_req / wall
    rng = np.random.default_rng(args.seed)
    levels = []
    rates = [frac * sat_rps for frac in (0.5, 0.8, 0.95)]
    rates += [float(x) for x in args.serve_rps.split(",") if x.strip()]
    for lam in rates:
        arr = np.cumsum(rng.exponential(1.0 / lam, size=n_req))
        arr -= arr[0]
        wl, lt = run(arr)
        levels.append({"load": lam / sat_rps, "offered_rps": lam, "achieved_rps": n_req / wl,
                       "p50_ms": float(np.percentile(lt, 50) * 1e3), "p99_ms": float(np.percentile(lt, 99) * 1e3)})
    srv.close()
    roof = products_roofline(rqlp, ctx, As, pool, q, torch)
    res = {
        "metric": f"RU-QLP served GFLOP/s at saturation ({n_req} requests, FP32, q={q}); p50/p99 latency",
        "value": flops / wall / 1e9, "unit": "GFLOP/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": wall * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "requests": n_req, "distinct_matrices": w["pool"], "q": q,
                   "slots": slots, "max_tick": tick, "hbm_budget_gb": w["budget_gb"], "m_range": [512, 8192],
                   "n_range": [256, 4096], "k_range": [8, 256], "p": 10},
        "saturated": {"requests_per_s": sat_rps, "p50_ms": float(np.percentile(lat, 50) * 1e3),
                      "p99_ms": float(np.percentile(lat, 99) * 1e3)},
        "latency_by_load": levels,
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = oracle_on_problems(pool, [a.cpu().numpy() for a in As], q)
    print(json.dumps(res), flush=True)


def products_roofline(rqlp, ctx, As, reqs, q, torch):
    """Products with A of the given problems, event-timed one problem after
    another: achieved TFLOP/s against the float32 MFMA peak."""
    ctx.set_timing(True, classes=["gemm_nn", "gemm_tn"])
    for A, r in zip(As, reqs):
        rqlp.decompose(A, r["k"], r["p"], q, seed=r["seed"], ctx=ctx)
    torch.cuda.synchronize()
    g_ms = sum(ctx.timing(c)[0] for c in ("gemm_nn", "gemm_tn"))
    ctx.set_timing(False)
    g_flops = sum(2.0 * r["m"] * r["n"] * (r["k"] + r["p"]) * (2 * q + 2) for r in reqs)
    achieved = g_flops / (g_ms * 1e-3) / 1e12
    return {"bound": "mfma", "achieved": achieved, "peak": PEAK["f32_mfma_tflops"], "unit": "TFLOP/s",
            "frac": achieved / PEAK["f32_mfma_tflops"], "traffic": None,
            "kernel": "gemm_nn+gemm_tn (problems one by one)"}


def oracle_on_problems(reqs, hostAs, q, budget_s=15.0):
    """The float64 oracle on the problems in order until about budget_s."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    done, f_done, t_done = 0, 0.0, 0.0
    for r, a in zip(reqs, hostAs):
        t0 = time.perf_counter()
        oracle.ruqlp(a.astype(np.float64), r["k"], r["p"], q, r["seed"], omega_dtype="f32")
        t_done += time.perf_counter() - t0
        f_done += f_alg(r["m"], r["n"], r["k"], r["p"], q)
        done += 1
        if t_done > budget_s:
            break
    return {"value": f_done / t_done / 1e9, "unit": "GFLOP/s", "cores": int(threads), "kind": "oracle",
            "sample": f"the first {done} distinct problems of the workload", "seconds": t_done}


def run_batch_bench(args, w, rqlp, torch, dev):
    """One step = one rqlp_decompose_batched call over the whole batch, with
    graph replay on (the batch repeats).  Also timed: the same batch without
    graphs, and the problems decomposed one after another."""
    import workloads
    reqs = workloads.serving_requests(w["count"], args.seed)
    hostAs = [workloads.request_matrix(r, np.float32) for r in reqs]
    As = [torch.from_numpy(a).to(dev) for a in hostAs]
    params = [(r["k"], r["p"], w["q"], r["seed"]) for r in reqs]
    flops = sum(f_alg(r["m"], r["n"], r["k"], r["p"], w["q"]) for r in reqs)
    ctx = rqlp.Context(0)
    shapes = [(r["m"], r["n"], r["k"], r["p"], w["q"]) for r in reqs]
    ws = rqlp.alloc_workspace(rqlp.workspace_size_batched(shapes, torch.float32), dev)
    outs = rqlp.decompose_batched(As, params, ctx=ctx, workspace=ws)

    def timed(fn, steps):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    # one step: the batch as grouped launches (every phase of every problem
    # in one launch per kernel variant, argument tables cached on the device)
    ms = timed(lambda: rqlp.decompose_batched(As, params, ctx=ctx, workspace=ws, outs=outs), args.steps)
    ungrouped_ms = graph_ms = seq_ms = None
    if not args.no_compare:
        # for comparison: every problem's sequence on its own lane stream,
        # eager and replayed from a captured graph
        ctx.set_batch_grouping(False)
        ungrouped_ms = timed(lambda: rqlp.decompose_batched(As, params, ctx=ctx, workspace=ws, outs=outs),
                             args.steps)
        ctx.set_batch_grouping(True)
        ctx.set_graphs(True)
        graph_ms = timed(lambda: rqlp.decompose_batched(As, params, ctx=ctx, workspace=ws, outs=outs), args.steps)
        ctx.set_graphs(False)
        solo_ws = rqlp.alloc_workspace(max(rqlp.workspace_size(r["m"], r["n"], r["k"], r["p"], w["q"],
                                                               torch.float32) for r in reqs), dev)

        def sequential():
            for A, (k, p, q, seed), o in zip(As, params, outs):
                rqlp.decompose(A, k, p, q, seed=seed, ctx=ctx, workspace=solo_ws, out=o)
        seq_ms = timed(sequential, max(1, args.steps // 4))
    roof = products_roofline(rqlp, ctx, As, [dict(r, seed=s_) for r, (_, _, _, s_) in zip(reqs, params)], w["q"],
                             torch)
    res = {
        "metric": f"RU-QLP GFLOP/s (batch of {w['count']} uneven requests, FP32, q={w['q']})",
        "value": flops / (ms * 1e-3) / 1e9, "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "count": w["count"], "q": w["q"], "flops_per_step": flops,
                   "m_range": [512, 8192], "n_range": [256, 4096], "k_range": [8, 256], "p": 10},
        "lanes_eager_ms": ungrouped_ms, "lanes_graph_replay_ms": graph_ms, "sequential_ms": seq_ms,
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = oracle_on_problems(reqs, hostAs, w["q"])
    print(json.dumps(res), flush=True)


def cpu_baseline(w, A_host, seed, flops):
    """Time the float64 oracle on this host on one decomposition (or, for
    the sparse workload, the same)."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    t0 = time.perf_counter()
    if w["kind"] == "dense" and w.get("bf16"):
        # the full 20000 x 15000 oracle takes minutes on a few cores: time the
        # same recipe at half of every dimension (m, n, k, p) instead
        import workloads
        mh, nh, kh, ph = w["m"] // 2, w["n"] // 2, w["k"] // 2, w["p"] // 2
        Ah = workloads.cfg_poly_bf16(seed=seed, m=mh, n=nh)["A"].astype(np.float64)
        flops = f_alg(mh, nh, kh, ph, w["q"])
        t0 = time.perf_counter()
        oracle.ruqlp(Ah, kh, ph, w["q"], seed, omega_dtype="bf16", operand_dtype="bf16")
        dt = time.perf_counter() - t0
        return {"value": flops / dt / 1e9, "unit": "GFLOP/s", "cores": int(threads), "kind": "oracle",
                "sample": (f"one decomposition of the same recipe at half size ({mh}x{nh}, k={kh}, p={ph}, "
                           f"q={w['q']}), bfloat16 operand rounding emulated"), "seconds": dt}
    elif w["kind"] == "dense" and w.get("svd"):
        oracle.ruqlp_svd(A_host.astype(np.float64), w["k"], w["p"], w["q"], seed, omega_dtype="f32")
        sample = f"one full SVD-like decomposition of the same {w['m']}x{w['n']} workload (q={w['q']})"
    elif w["kind"] == "dense" and w.get("paper"):
        oracle.ruqlp_paper(A_host.astype(np.float64), w["k"], w["p"], w["q"], seed, omega_dtype="f32")
        sample = f"one full decomposition of the same {w['m']}x{w['n']} workload (q={w['q']}), row-sketch orientation"
    elif w["kind"] == "dense":
        oracle.ruqlp(A_host.astype(np.float64), w["k"], w["p"], w["q"], seed,
                     omega_dtype="f32" if w["dtype"] == "f32" else "f64")
        sample = f"one full decomposition of the same {w['m']}x{w['n']} workload (q={w['q']})"
    else:
        c = A_host
        oracle.ruqlp_csr(c["rowptr"], c["colidx"], c["vals"], c["m"], c["n"], w["k"], w["p"], w["q"], seed,
                         omega_dtype="f32")
        sample = f"one full decomposition of the same {w['m']}x{w['n']} CSR workload (q={w['q']})"
    dt = time.perf_counter() - t0
    return {"value": flops / dt / 1e9, "unit": "GFLOP/s", "cores": int(threads), "kind": "oracle",
            "sample": sample, "seconds": dt}


def copy_calibration(nbytes=1 << 30, reps=5):
    """A plain device-to-device copy of known size, for scaling the
    FETCH_SIZE / WRITE_SIZE counters of a profiled run."""
    import torch
    n = nbytes // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": nbytes, "reps": reps}), flush=True)


def kernel_class(name):
    """Timed kernel class of a profiled kernel name (None if untimed)."""
    if name.startswith("void rqlp::gemm_kernel<"):
        trans = name.split("<", 1)[1].split(",")[2].strip()
        return "gemm_tn" if trans == "true" else "gemm_nn"
    if "rqlp::spmm_kernel" in name:
        return "spmm"
    return None


def read_counter(csv_path, counter):
    """{kernel name: [per-dispatch values]} of one counter from a rocprofv3
    counter_collection.csv."""
    import csv
    out = {}
    with open(csv_path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] == counter:
                out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return out


def record_traffic(workload, fetch_csv, write_csv, cal_fetch_csv, cal_write_csv, cal_bytes, path=None):
    """Scale the FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the timed
    kernels by what the same counters read for a plain copy of cal_bytes per
    dispatch, and store bytes per launch in profiles/traffic.json."""
    def scale(csv_path, counter):
        vals = [v for name, vs in read_counter(csv_path, counter).items() if "copyBuffer" in name for v in vs]
        return cal_bytes / (1024.0 * float(np.median(vals)))
    f_fetch = scale(cal_fetch_csv, "FETCH_SIZE")
    f_write = scale(cal_write_csv, "WRITE_SIZE")
    fetch = read_counter(fetch_csv, "FETCH_SIZE")
    write = read_counter(write_csv, "WRITE_SIZE")
    path = path or os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        rec = {}
    # the bfloat16 product is one kernel for both forms; a decomposition
    # launches it as A X, A^T X, A X, A^T X, ... so dispatches alternate
    split = {}
    for name in fetch:
        if name not in write:
            continue
        if "rqlp::gemm_bf16_kernel" in name:
            for cls, sl in (("gemm_nn", slice(0, None, 2)), ("gemm_tn", slice(1, None, 2))):
                split[cls] = (fetch[name][sl], write[name][sl])
        else:
            cls = kernel_class(name)
            if cls is not None:
                split[cls] = (fetch[name], write[name])
    out = {}
    for cls, (fv, wv) in split.items():
        fb = float(np.mean(fv)) * 1024.0 * f_fetch
        wb = float(np.mean(wv)) * 1024.0 * f_write
        out[cls] = {"bytes_per_launch": fb + wb, "fetch_bytes": fb, "write_bytes": wb,
                    "fetch_scale": f_fetch, "write_scale": f_write, "dispatches": len(fv),
                    "source_hash": kernel_source_hash(cls, workload)}
    rec[workload] = out
    with open(path, "w") as f:
        json.dump(rec, f, indent=1, sort_keys=True)
    print(json.dumps({workload: out}, indent=1), flush=True)


def time_svd_small(rqlp, ctx, A, k, p, q, seed, torch, reps=10):
    """Time of the d x d SVD alone (rqlp_svd_small on this workload's L)."""
    _, L, _ = rqlp.decompose(A, k, p, q, seed=seed, ctx=ctx)
    ws = rqlp.alloc_workspace(int(rqlp._lib().rqlp_svd_workspace_size(k + p)), A.device)
    out = rqlp.svd_small(L, ctx=ctx, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        rqlp.svd_small(L, ctx=ctx, workspace=ws, out=out)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / reps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="dense8000", choices=sorted(WORKLOADS))
    ap.add_argument("--seed", type=int, default=2024)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--slots", type=int, default=0, help="serving: tick streams (default: the workload's)")
    ap.add_argument("--tick", type=int, default=0, help="serving: requests per tick (default: the workload's)")
    ap.add_argument("--serve-rps", type=str, default="",
                    help="serving: extra Poisson arrival rates in requests/s (comma list), run after the load fractions")
    ap.add_argument("--no-compare", action="store_true",
                    help="bfloat16 workload: skip the float32 comparison run; batch workload: time the "
                         "grouped form only (no lane, graph or one-by-one runs)")
    ap.add_argument("--no-svd-split", action="store_true",
                    help="SVD-like workload: skip the separate timing of the small SVD")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB device copy (x5), to scale FETCH_SIZE / WRITE_SIZE")
    ap.add_argument("--record-traffic", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "CAL_FETCH_CSV", "CAL_WRITE_CSV"),
                    help="write profiles/traffic.json for --workload from rocprofv3 counter CSVs (no GPU use)")
    ap.add_argument("--record-mfma", metavar="PMC_CSV",
                    help="write profiles/mfma.json for --workload from a rocprofv3 counter CSV (no GPU use)")
    args = ap.parse_args()

    if args.record_traffic:
        record_traffic(args.workload, *args.record_traffic, cal_bytes=float(1 << 30))
        return
    if args.record_mfma:
        record_mfma(args.workload, args.record_mfma)
        return

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; use --gpus 1"}), flush=True)
        sys.exit(2)

    import torch
    from paper_2209_12464_amd import rqlp

    if args.copy_calibration:
        copy_calibration()
        return

    w = WORKLOADS[args.workload]
    dev = torch.device("cuda", 0)
    try:
        if w["kind"] == "batch":
            run_batch_bench(args, w, rqlp, torch, dev)
        elif w["kind"] == "serve":
            run_serve_bench(args, w, rqlp, torch, dev)
        else:
            run_single_bench(args, w, rqlp, torch, dev)
    finally:
        # destroy servers and contexts (device sync, stream and buffer
        # teardown) while the HIP runtime is certainly still up
        torch.cuda.synchronize()
        rqlp.close_all()


def run_single_bench(args, w, rqlp, torch, dev):
    """One decomposition per step of a dense or CSR workload."""
    host = make_inputs(w, args.seed)
    ctx = rqlp.Context(0)
    k, p, q = w["k"], w["p"], w["q"]
    d = k + p
    bf16 = bool(w.get("bf16"))
    if w["kind"] == "dense":
        A = torch.from_numpy(host).to(dev)
        m, n = A.shape
        out = (torch.empty((m, d), dtype=A.dtype, device=dev), torch.empty((d, d), dtype=A.dtype, device=dev),
               torch.empty((n, d), dtype=A.dtype, device=dev))
        svd_small_ms = None
        if w.get("svd"):
            # the decomposition's work plus the two products Q U-bar and V V-bar
            # (the small SVD's iteration count depends on the input: not counted)
            flops = f_alg(m, n, k, p, q) + 2.0 * (m + n) * d * d
            ws = rqlp.alloc_workspace(rqlp.workspace_size_svd(m, n, k, p, q, A.dtype), dev)
            out = (torch.empty((m, d), dtype=A.dtype, device=dev), torch.empty((d,), dtype=A.dtype, device=dev),
                   torch.empty((n, d), dtype=A.dtype, device=dev))
            step = lambda: rqlp.decompose_svd(A, k, p, q, seed=args.seed, ctx=ctx, workspace=ws,  # noqa: E731
                                              out=out)
            if not args.no_svd_split:
                svd_small_ms = time_svd_small(rqlp, ctx, A, k, p, q, args.seed, torch)
        elif w.get("paper"):
            flops = f_alg_paper(m, n, k, p, q)
            ws = rqlp.alloc_workspace(int(rqlp._lib().rqlp_workspace_size_paper(m, n, k, p, q, rqlp._prec(A.dtype))),
                                      dev)
            step = lambda: rqlp.decompose_paper(A, k, p, q, seed=args.seed, ctx=ctx, workspace=ws,  # noqa: E731
                                                out=out)
        else:
            flops = f_alg(m, n, k, p, q)
            ws = rqlp.alloc_workspace(rqlp.workspace_size(m, n, k, p, q, A.dtype, bf16=bf16), dev)
            step = lambda: rqlp.decompose(A, k, p, q, seed=args.seed, ctx=ctx, workspace=ws, out=out,  # noqa: E731
                                          bf16=bf16)
        dom = ["gemm_nn", "gemm_tn"]
        # algorithmic flops per step of each product class: q + 1 products
        # with A each way, plus the small d-column products of the paper
        # orientation (P = P-bar P-tilde) and of the SVD-like form (Q U-bar,
        # V V-bar), which run as the same kernel
        big = (q + 1) * 2.0 * m * n * d
        small = 2.0 * (m + n) * d * d if w.get("svd") else (2.0 * n * d * d if w.get("paper") else 0.0)
        dom_flops = {"gemm_nn": big + small, "gemm_tn": big}
        dtype_name = "bf16" if bf16 else ("f32" if A.dtype == torch.float32 else "f64")
    else:
        c = host
        m, n = c["m"], c["n"]
        rp, ci, vv = (torch.from_numpy(c[x]).to(dev) for x in ("rowptr", "colidx", "vals"))
        nnz = ci.numel()
        flops = f_alg_csr(nnz, m, n, k, p, q)
        ws = rqlp.alloc_workspace(rqlp.workspace_size_csr(m, n, nnz, k, p, q, vv.dtype), dev)
        out = (torch.empty((m, d), dtype=vv.dtype, device=dev), torch.empty((d, d), dtype=vv.dtype, device=dev),
               torch.empty((n, d), dtype=vv.dtype, device=dev))
        step = lambda: rqlp.decompose_csr(rp, ci, vv, m, n, k, p, q, seed=args.seed, ctx=ctx, workspace=ws,  # noqa: E731
                                          out=out)
        dom = ["spmm"]
        dtype_name = "f32"

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # only the dominant kernel classes are event-timed: every timed launch
    # adds two event records to the stream
    ctx.set_timing(True, classes=dom)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    per_kernel = {}
    for name in rqlp.KERNEL_CLASSES:
        ms, cnt = ctx.timing(name)
        if cnt:
            per_kernel[name] = {"avg_ms": ms / cnt, "launches": cnt, "total_ms": ms}
    ctx.set_timing(False)
    info = ctx.info()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = flops / (ms_per_step * 1e-3) / 1e9

    roofline = None
    dom_present = [k_ for k_ in dom if k_ in per_kernel]
    if dom_present:
        kname = max(dom_present, key=lambda x: per_kernel[x]["total_ms"])
        avg_s = per_kernel[kname]["avg_ms"] * 1e-3
        if w["kind"] == "dense":
            peak = PEAK[{"bf16": "bf16_mfma_tflops", "f32": "f32_mfma_tflops"}.get(dtype_name, "f64_mfma_tflops")]
            step_s = per_kernel[kname]["total_ms"] * 1e-3 / args.steps
            achieved = dom_flops[kname] / step_s / 1e12
            traffic = load_traffic(args.workload, kname)
            util, clock = load_mfma_record(args.workload, kname)
            roofline = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                        "frac": achieved / peak, "traffic": traffic, "kernel": kname,
                        "mfma_util": util, "clock_ghz": clock,
                        "timed": "product kernel and its split-K reduction, HIP events on the launch stream"}
        else:
            # gather-inclusive bytes of one A X product: indices+values, row
            # pointers, one gathered X row per entry, the output rows
            es = 4
            byts = nnz * (4 + es) + (m + 1) * 4 + nnz * d * es + m * d * es
            # compulsory bytes: every input read once (A, row pointers, X) and Y written
            comp = nnz * (4 + es) + (m + 1) * 4 + n * d * es + m * d * es
            achieved = byts / avg_s / 1e9
            traffic = load_traffic(args.workload, kname)
            roofline = {"bound": "hbm", "achieved": achieved, "peak": PEAK["hbm_gbs"], "unit": "GB/s",
                        "frac": achieved / PEAK["hbm_gbs"], "traffic": traffic, "kernel": kname,
                        "achieved_is": "effective bandwidth counting every gathered X row (gather-inclusive bytes)",
                        "compulsory_gbs": comp / avg_s / 1e9,
                        "compulsory_frac": comp / avg_s / 1e9 / PEAK["hbm_gbs"],
                        "compulsory_bytes": comp, "gather_inclusive_bytes": byts}

    vs_fp32 = None
    if bf16 and not args.no_compare:
        vs_fp32 = compare_with_fp32(rqlp, ctx, A, k, p, q, args, out, ws_fp32_steps=args.steps)

    res = {
        "metric": METRIC_NAMES.get(args.workload, f"RU-QLP GFLOP/s ({args.workload})"),
        "value": value,
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype_name,
        "data": "synthetic",
        "config": {"workload": args.workload, "m": m, "n": n, "k": k, "p": p, "q": q,
                   "flops_per_step": flops},
        "roofline": roofline,
        "kernels": per_kernel,
        **({"vs_fp32_same_gpu": vs_fp32} if vs_fp32 else {}),
        **({"svd_small_ms": svd_small_ms} if w["kind"] == "dense" and w.get("svd") else {}),
        "info": info,
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(w, host, args.seed, flops)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
