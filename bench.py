"""Benchmark: Katz queries/sec at 1e-6 relative residual, LRC-Katz vs plain GPU CG,
on one MI355X.

Workload (default): Chung-Lu power-law graph, 1,000,000 nodes, exponent 2.5,
mean degree 20 (seeded, synthetic), damping c = beta * lambda_max in
{0.1, 0.5, 0.9}, rank 32, FP64, one query node per solve.  A step is one query
solved through the whole path (right-hand side, Schur RHS, PCG on S, block
back-solve, FP64 residual check, unpermute into a device buffer).  The headline
value is LRC queries/sec at c = 0.5; CG at the same c, latency percentiles,
iterations and the other c values are reported beside it.

Prints ONE JSON line.  Options: --gpus (1 only), --steps, --warmup, --c,
--scale (node-count factor for quick runs), --no-cpu (skip the oracle leg),
--copy-calib (adds a plain 1 GiB device copy, to calibrate rocprofv3 byte
counters), --profile-kernels (HIP-event kernel timing in a repeat of the timed
steps; on by default).
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

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of the SpMM kernel's source (its section of solver.hip, between the
    SpMM and column-lane-map markers) and of kernels.h."""
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_1912_06525_amd", "csrc", "solver.hip")) as fh:
        src = fh.read()
    a = src.index("// ------------------------------------------------------------------- SpMM")
    b = src.index("// ------------------------------------------------------- column-lane maps")
    h.update(src[a:b].encode())
    with open(os.path.join(ROOT, "paper_1912_06525_amd", "csrc", "kernels.h"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str, workload: str, achieved_bytes_per_launch: float):
    """HBM bytes per launch from the committed rocprofv3 PMC summary, or None
    when absent or taken on a different kernel source."""
    p = os.path.join(ROOT, "profiles", "pmc_%s_%s.json" % (kernel, workload))
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f)
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--c", type=str, default="0.1,0.5,0.9")
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--rank", type=int, default=32)
    ap.add_argument("--max-block", type=int, default=64)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-profile-kernels", action="store_true")
    ap.add_argument("--copy-calib", action="store_true")
    ap.add_argument("--workload", type=str, default="cl1m",
                    help="cl1m (default, one query per solve), lnsbm4m (256 FP64 RHS), cl8m (512 mixed RHS)")
    ap.add_argument("--batch", type=int, default=0, help="override the workload's batch size")
    ap.add_argument("--host-output", action="store_true",
                    help="one-query workload: deliver scores to pinned host memory (PCIe-inclusive rate; "
                         "the result line then says so in config.output)")
    ap.add_argument("--precision", type=str, default="fp64", choices=["fp64", "mixed"],
                    help="one-query workload: FP64 path (the configuration's) or the precision form")
    ap.add_argument("--u-precision", type=int, default=0, help="low-rank factor storage (0 auto, 1 FP64, 2 FP32, 3 BF16)")
    ap.add_argument("--concurrency", type=int, default=2,
                    help="one-query workload: also time this many host threads solving independent single "
                         "queries at once (each on its own workspace stream); 0 or 1 to skip")
    ap.add_argument("--pairs", type=int, default=0,
                    help="pairwise queries on the 1M-node graph: this many distinct sources per step, "
                         "16 destinations each")
    ap.add_argument("--sparse-katz", type=str, default="",
                    help="Sparse-Katz on the 1M-node graph: 'nq,s,T' (queries per call, list length, modular nodes)")
    ap.add_argument("--serve", action="store_true", help="serving mode on --workload (default dcsbm16m)")
    ap.add_argument("--requests", type=int, default=200, help="requests per offered-load point (serving)")
    ap.add_argument("--workers", type=int, default=4)
    ap.add_argument("--max-batch-cols", type=int, default=64)
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(queries would shard across GPUs with a replicated index)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import katz_inputs as ki
    import paper_1912_06525_amd as K

    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.serve:
        return run_serving(args)
    if args.pairs:
        return run_pairs(args)
    if args.sparse_katz:
        return run_sparse_katz(args)
    if args.workload != "cl1m":
        return run_batched(args)

    t0 = time.time()
    w = ki.workload("cl1m", scale=args.scale)
    g = w.graph
    log("graph: n=%d nnz=%d (%.1fs)" % (g.n, g.nnz, time.time() - t0))
    cs = [float(x) for x in args.c.split(",")]
    head_c = 0.5 if 0.5 in cs else cs[0]
    tol = 1e-6
    queries = w.queries
    results = {}
    roofline = None
    kernel_table = None
    if args.host_output:
        # scores delivered to pinned host memory: the PCIe-inclusive rate
        out = torch.empty((1, g.n), dtype=torch.float64, pin_memory=True)
    else:
        out = torch.empty((1, g.n), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream

    def run(idx, method, steps, offset, check_every=0):
        lat, its, res = [], [], []
        for s in range(steps):
            q = queries[(offset + s) % len(queries)]
            t = time.perf_counter()
            _, st = idx.query([q], out=out, tol=tol, method=method, stream=stream,
                              check_every=check_every or int(os.environ.get("KATZ_CHECK_EVERY", "0")))
            lat.append(time.perf_counter() - t)
            its.append(st[0]["iters"])
            res.append(st[0]["rel_residual"])
            if st[0]["status"] != 0:
                raise RuntimeError("query %d did not converge: %r" % (q, st[0]))
        return lat, its, res

    for c in cs:
        tb = time.time()
        idx = K.KatzIndex.from_graph(g, beta_frac=c, rank=args.rank, max_block=args.max_block, device=0,
                                     u_precision=args.u_precision,
                                     precision=K.KATZ_PREC_MIXED if args.precision == "mixed" else K.KATZ_PREC_FP64)
        info = idx.info
        log("c=%.2f index: n1=%d n2=%d blocks=%d sigma1=%.4f sigma_r+1=%.5f build %.1fs"
            % (c, info.n1, info.n2, info.nblocks, info.sigma_max, info.sigma_next, time.time() - tb))
        entry = {"n1": info.n1, "n2": info.n2, "nblocks": info.nblocks, "build_s": round(info.build_seconds, 2),
                 "beta": info.beta, "lambda_max": info.lambda_max}
        for name, method in (("lrc", K.KATZ_METHOD_LRC), ("cg", K.KATZ_METHOD_CG)):
            run(idx, method, args.warmup, 0)
            torch.cuda.synchronize()
            t = time.perf_counter()
            lat, its, res = run(idx, method, args.steps, args.warmup)
            torch.cuda.synchronize()
            el = time.perf_counter() - t
            lat_ms = np.array(lat) * 1e3
            entry[name] = {"qps": args.steps / el, "ms_per_query": el * 1e3 / args.steps,
                           "p50_ms": float(np.percentile(lat_ms, 50)), "p99_ms": float(np.percentile(lat_ms, 99)),
                           "iters_median": float(np.median(its)), "iters_max": int(np.max(its)),
                           "max_rel_residual": float(np.max(res))}
            log("  %s: %.1f q/s, %.3f ms/query, iters median %g" % (name, entry[name]["qps"],
                                                                    entry[name]["ms_per_query"],
                                                                    entry[name]["iters_median"]))
            if c == head_c and args.concurrency > 1 and not args.host_output:
                # independent one-query solves from several host threads at once
                import threading
                per = max(1, args.steps // args.concurrency) * 2
                outs = [torch.empty((1, g.n), dtype=torch.float64, device=dev) for _ in range(args.concurrency)]
                errs = []

                # one caller stream per thread (default priority): on a shared stream
                # each call would be ordered after the others
                strs = [torch.cuda.Stream(device=dev) for _ in range(args.concurrency)]

                def worker(tid):
                    try:
                        for s2 in range(per):
                            q = queries[(tid * per + s2) % len(queries)]
                            _, st2 = idx.query([q], out=outs[tid], tol=tol, method=method,
                                               stream=strs[tid].cuda_stream)
                            if st2[0]["status"] != 0:
                                errs.append(q)
                    except Exception as e:  # reported below
                        errs.append(repr(e))
                ths = [threading.Thread(target=worker, args=(i,)) for i in range(args.concurrency)]
                torch.cuda.synchronize()
                t = time.perf_counter()
                for th in ths:
                    th.start()
                for th in ths:
                    th.join()
                torch.cuda.synchronize()
                el = time.perf_counter() - t
                if errs:
                    raise RuntimeError("concurrent solves failed: %r" % errs[:3])
                entry[name]["concurrent_qps"] = per * args.concurrency / el
                entry[name]["concurrency"] = args.concurrency
                log("  %s: %.1f q/s with %d concurrent one-query solves" % (name, per * args.concurrency / el,
                                                                          args.concurrency))
            if c == head_c and not args.no_profile_kernels:
                # repeat of the timed steps with HIP-event timing of every hot kernel
                # launch; convergence is polled every iteration here so that no
                # launch runs after a query has converged (each timed launch works)
                K.katz_profile_reset()
                K.katz_profile_enable(True)
                run(idx, method, args.steps, args.warmup, check_every=1)
                torch.cuda.synchronize()
                K.katz_profile_enable(False)
                tab = [r for r in K.katz_profile_read() if r["launches"] > 0]
                for r in tab:
                    r["avg_us"] = 1e3 * r["total_ms"] / r["launches"]
                    r["alg_bytes_per_launch"] = r["alg_bytes"] / r["launches"]
                    r["achieved_GBs"] = r["alg_bytes"] / (r["total_ms"] * 1e-3) / 1e9
                entry[name]["kernels"] = tab
                if name == "lrc":
                    kernel_table = tab
        if c == head_c:
            head_idx_info = entry
            if not args.no_cpu:
                cpu = cpu_baseline(g, idx, queries, tol, out, stream, K)
                entry["cpu"] = cpu
        results["c=%g" % c] = entry
        idx.close()

    if args.copy_calib:
        x = torch.empty(2 ** 27, dtype=torch.float64, device=dev)   # 1 GiB
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()

    head = results["c=%g" % head_c]
    copy_gbs = measured_copy_bandwidth(torch, dev)
    log("measured device copy bandwidth: %.0f GB/s (read + write of a 1 GiB copy)" % copy_gbs)
    if kernel_table:
        dom = max(kernel_table, key=lambda r: r["total_ms"])
        wl = "cl1m" if args.scale == 1.0 else "cl1m_s%g" % args.scale
        traffic = load_traffic(dom["name"], wl, dom["alg_bytes_per_launch"])
        roofline = {"bound": "hbm", "kernel": dom["name"], "achieved": round(dom["achieved_GBs"], 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(dom["achieved_GBs"] / HBM_PEAK_GBS, 4),
                    "traffic": traffic, "avg_launch_us": round(dom["avg_us"], 2),
                    "alg_bytes_per_launch": dom["alg_bytes_per_launch"],
                    "measured_copy_GBs": round(copy_gbs, 1),
                    "frac_of_measured_copy": round(dom["achieved_GBs"] / copy_gbs, 4),
                    "traffic_GBs": round(traffic / (dom["avg_us"] * 1e-6) / 1e9, 1) if traffic else None}
    value = head["lrc"]["qps"]
    line = {
        "metric": "Katz queries/sec at 1e-6 rel. residual, LRC-Katz vs CG, 1 MI355X; p99 ms",
        "value": round(value, 2),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["lrc"]["ms_per_query"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+bf16/f64",
        "data": "synthetic",
        "config": {"workload": "Chung-Lu power-law graph, %d nodes, exponent 2.5, mean degree 20, "
                               "c = beta*lambda_max = %g, rank %d, %s, 1 query per solve"
                               % (g.n, head_c, args.rank,
                                  "FP64" if args.precision == "fp64" else "FP32 inner solves + FP64 refinement"),
                   "n": g.n, "nnz": g.nnz, "c": head_c, "rank": args.rank, "batch": 1, "tol": tol,
                   "output": "pinned host memory (PCIe-inclusive)" if args.host_output else "device memory"},
        "p99_ms": round(head["lrc"]["p99_ms"], 4),
        "p50_ms": round(head["lrc"]["p50_ms"], 4),
        "cg_qps": round(head["cg"]["qps"], 2),
        "lrc_over_cg": round(value / head["cg"]["qps"], 3),
        "concurrent": {"threads": args.concurrency,
                       "lrc_qps": round(head["lrc"].get("concurrent_qps", 0.0), 2),
                       "cg_qps": round(head["cg"].get("concurrent_qps", 0.0), 2)} if args.concurrency > 1 else None,
        "roofline": roofline,
        "cpu_baseline": head.get("cpu", {}).get("baseline"),
        "results": results,
    }
    print(json.dumps(line), flush=True)


def run_batched(args):
    """Batched workloads: one step = one batch of B queries solved together."""
    import numpy as np
    import torch

    import katz_inputs as ki
    import paper_1912_06525_amd as K

    dev = torch.device("cuda:0")
    t0 = time.time()
    w = ki.workload(args.workload, scale=args.scale)
    g = w.graph
    B = args.batch or w.batch
    log("graph %s: n=%d nnz=%d (%.1fs)" % (args.workload, g.n, g.nnz, time.time() - t0))
    cs = [float(x) for x in args.c.split(",")] if args.c != "0.1,0.5,0.9" else list(w.c)
    prec = K.KATZ_PREC_MIXED if w.precision == "mixed" else K.KATZ_PREC_FP64
    rank = args.rank if args.rank != 32 else w.rank
    tol = w.tol
    queries = ki.sample_queries(g, B * (args.steps + args.warmup), 3003)
    if args.copy_calib:
        # plain 1 GiB copies: the reference that scales the PMC byte counters
        x = torch.empty(2 ** 27, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    out = torch.empty((B, g.n), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    results = {}
    kernel_table = None
    for c in cs:
        tb = time.time()
        idx = K.KatzIndex.from_graph(g, beta_frac=c, rank=rank, max_block=args.max_block, device=0,
                                     labels=g.labels, precision=prec)
        info = idx.info
        log("c=%.2f index: n1=%d n2=%d blocks=%d sigma1=%.4f sigma_r+1=%.5f build %.1fs dev %.1f GB"
            % (c, info.n1, info.n2, info.nblocks, info.sigma_max, info.sigma_next, time.time() - tb,
               info.device_bytes / 1e9))
        entry = {"n1": info.n1, "n2": info.n2, "build_s": round(info.build_seconds, 2)}
        for name, method in (("lrc", K.KATZ_METHOD_LRC), ("cg", K.KATZ_METHOD_CG)):
            def step(s):
                q = queries[s * B:(s + 1) * B]
                t = time.perf_counter()
                _, st = idx.query(q, out=out, tol=tol, method=method, stream=stream)
                bad = [x for x in st if x["status"] != 0]
                if bad:
                    raise RuntimeError("no convergence: %r" % bad[:2])
                return time.perf_counter() - t, st
            for s in range(args.warmup):
                step(s)
            torch.cuda.synchronize()
            t = time.perf_counter()
            lat, its, sw = [], [], []
            for s in range(args.steps):
                dt, st = step(args.warmup + s)
                lat.append(dt)
                its += [x["iters"] for x in st]
                sw += [x["sweeps"] for x in st]
            torch.cuda.synchronize()
            el = time.perf_counter() - t
            entry[name] = {"qps": B * args.steps / el, "ms_per_batch": 1e3 * el / args.steps,
                           "iters_median": float(np.median(its)), "sweeps_median": float(np.median(sw))}
            log("  %s: %.1f q/s, %.1f ms/batch of %d, iters median %g, sweeps %g"
                % (name, entry[name]["qps"], entry[name]["ms_per_batch"], B, entry[name]["iters_median"],
                   entry[name]["sweeps_median"]))
            if not args.no_profile_kernels:
                K.katz_profile_reset()
                K.katz_profile_enable(True)
                step(args.warmup)
                torch.cuda.synchronize()
                K.katz_profile_enable(False)
                tab = [r for r in K.katz_profile_read() if r["launches"] > 0]
                for r in tab:
                    r["avg_us"] = 1e3 * r["total_ms"] / r["launches"]
                    r["achieved_GBs"] = r["alg_bytes"] / (r["total_ms"] * 1e-3) / 1e9
                    r["alg_bytes_per_launch"] = r["alg_bytes"] / r["launches"]
                    log("    %-22s %5d x %9.1f us  %8.1f GB/s" % (r["name"], r["launches"], r["avg_us"],
                                                                r["achieved_GBs"]))
                entry[name]["kernels"] = tab
                if name == "lrc" and c == cs[0]:
                    kernel_table = tab
        results["c=%g" % c] = entry
        idx.close()
    head = results["c=%g" % cs[0]]
    roofline = None
    if kernel_table:
        dom = max(kernel_table, key=lambda r: r["total_ms"])
        wl = args.workload if args.scale == 1.0 else "%s_s%g" % (args.workload, args.scale)
        traffic = load_traffic(dom["name"], "%s_b%d_c%g" % (wl, B, cs[0]), dom["alg_bytes_per_launch"])
        roofline = {"bound": "hbm", "kernel": dom["name"], "achieved": round(dom["achieved_GBs"], 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(dom["achieved_GBs"] / HBM_PEAK_GBS, 4),
                    "traffic": traffic, "avg_launch_us": round(dom["avg_us"], 2),
                    "alg_bytes_per_launch": dom["alg_bytes_per_launch"],
                    "traffic_GBs": round(traffic / (dom["avg_us"] * 1e-6) / 1e9, 1) if traffic else None}
    line = {"metric": "Katz queries/sec at 1e-6 rel. residual, LRC-Katz vs CG, 1 MI355X; p99 ms",
            "value": round(head["lrc"]["qps"], 2), "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(head["lrc"]["ms_per_batch"], 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32+bf16/f64" if prec == K.KATZ_PREC_MIXED else "f64", "data": "synthetic",
            "config": {"workload": "%s, %d nodes, batch %d, rank %d, c %s" % (args.workload, g.n, B, rank, cs),
                       "n": g.n, "nnz": g.nnz, "batch": B},
            "cg_qps": round(head["cg"]["qps"], 2), "lrc_over_cg": round(head["lrc"]["qps"] / head["cg"]["qps"], 3),
            "roofline": roofline, "cpu_baseline": None, "results": results}
    print(json.dumps(line), flush=True)


def run_pairs(args):
    """Pairwise Katz scores K[dst, src] on the 1M-node Chung-Lu graph: a step is
    `pairs` distinct sources x 16 destinations, solved as one batch."""
    import numpy as np
    import torch

    import katz_inputs as ki
    import paper_1912_06525_amd as K

    w = ki.workload("cl1m", scale=args.scale)
    g = w.graph
    c = float(args.c.split(",")[0]) if args.c != "0.1,0.5,0.9" else 0.5
    idx = K.KatzIndex.from_graph(g, beta_frac=c, rank=args.rank, max_block=args.max_block, device=0)
    rng = np.random.default_rng(6006)
    S, D = args.pairs, 16
    res = {}
    for name, method in (("lrc", K.KATZ_METHOD_LRC), ("cg", K.KATZ_METHOD_CG)):
        def step(s):
            src = np.repeat(ki.sample_queries(g, S, 7000 + s), D)
            dst = rng.integers(0, g.n, size=len(src)).astype(np.int32)
            t = time.perf_counter()
            _, st = idx.pair_scores(src, dst, tol=1e-6, method=method)
            if any(x["status"] != 0 for x in st):
                raise RuntimeError("no convergence")
            return time.perf_counter() - t
        for s in range(args.warmup):
            step(s)
        torch.cuda.synchronize()
        lat = [step(args.warmup + s) for s in range(args.steps)]
        el = sum(lat)
        res[name] = {"pairs_per_s": S * D * args.steps / el, "ms_per_step": 1e3 * el / args.steps}
        log("  %s: %.0f pairs/s (%d sources x %d destinations per step, %.1f ms)"
            % (name, res[name]["pairs_per_s"], S, D, res[name]["ms_per_step"]))
    line = {"metric": "pairwise Katz scores/sec at 1e-6 rel. residual, 1 MI355X", "value": round(res["lrc"]["pairs_per_s"], 1),
            "unit": "pairs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(res["lrc"]["ms_per_step"], 3), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "Chung-Lu power-law graph, %d nodes, c = %g, rank %d, %d sources x 16 "
                                   "destinations per step" % (g.n, c, args.rank, S)},
            "cg_pairs_per_s": round(res["cg"]["pairs_per_s"], 1)}
    print(json.dumps(line), flush=True)


def run_sparse_katz(args):
    """Sparse-Katz requests (Algorithm 3) on the 1M-node Chung-Lu graph: a step is
    one call with nq query nodes, each re-ranking its top-s list by the
    correlation with T modular nodes."""
    import torch

    import katz_inputs as ki
    import paper_1912_06525_amd as K

    nq, S, T = (int(x) for x in args.sparse_katz.split(","))
    w = ki.workload("cl1m", scale=args.scale)
    g = w.graph
    c = float(args.c.split(",")[0]) if args.c != "0.1,0.5,0.9" else 0.5
    idx = K.KatzIndex.from_graph(g, beta_frac=c, rank=args.rank, max_block=args.max_block, device=0)
    res = {}
    for name, method in (("lrc", K.KATZ_METHOD_LRC), ("cg", K.KATZ_METHOD_CG)):
        def step(s):
            q = ki.sample_queries(g, nq, 8000 + s)
            t = time.perf_counter()
            _, _, st = idx.sparse_katz(q, S, T, tol=1e-6, method=method)
            if any(x["status"] != 0 for x in st):
                raise RuntimeError("no convergence")
            return time.perf_counter() - t
        for s in range(args.warmup):
            step(s)
        torch.cuda.synchronize()
        lat = [step(args.warmup + s) for s in range(args.steps)]
        el = sum(lat)
        res[name] = {"requests_per_s": nq * args.steps / el, "ms_per_step": 1e3 * el / args.steps}
        log("  %s: %.1f requests/s (%d per call, s=%d, T=%d, %.1f ms per call)"
            % (name, res[name]["requests_per_s"], nq, S, T, res[name]["ms_per_step"]))
    line = {"metric": "Sparse-Katz link-prediction requests/sec at 1e-6 rel. residual, 1 MI355X",
            "value": round(res["lrc"]["requests_per_s"], 2), "unit": "requests/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(res["lrc"]["ms_per_step"], 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "Chung-Lu power-law graph, %d nodes, c = %g, rank %d, %d queries per call, "
                                   "s = %d, T = %d" % (g.n, c, args.rank, nq, S, T)},
            "cg_requests_per_s": round(res["cg"]["requests_per_s"], 2)}
    print(json.dumps(line), flush=True)


def run_serving(args):
    """Serving: Poisson arrivals of top-100 link-prediction requests of
    round(2^u) query nodes, u ~ U[0, 9]; saturation throughput, then offered
    loads of 0.5 / 0.8 / 0.95 x saturation with p50 / p99 latency."""
    import threading

    import numpy as np
    import torch

    import katz_inputs as ki
    import paper_1912_06525_amd as K

    wl = args.workload if args.workload != "cl1m" else "dcsbm16m"
    t0 = time.time()
    w = ki.workload(wl, scale=args.scale)
    g = w.graph
    log("graph %s: n=%d nnz=%d (%.1fs)" % (wl, g.n, g.nnz, time.time() - t0))
    c = 0.5
    rank = args.rank if args.rank != 32 else w.rank
    prec = K.KATZ_PREC_MIXED if w.precision == "mixed" else K.KATZ_PREC_FP64
    tb = time.time()
    idx = K.KatzIndex.from_graph(g, beta_frac=c, rank=rank, max_block=args.max_block, device=0,
                                 labels=g.labels, precision=prec)
    log("index: n2=%d build %.1fs" % (idx.info.n2, time.time() - tb))
    rng = np.random.default_rng(4005)
    pool = ki.sample_queries(g, min(g.n // 2, 200000), 4006)
    results = {}
    for method_name, method in (("lrc", K.KATZ_METHOD_LRC), ("cg", K.KATZ_METHOD_CG)):
        srv = K.KatzServer(idx, workers=args.workers, max_batch=args.max_batch_cols, k=100, tol=1e-6,
                           method=method)
        info = srv.info()
        log("server %s: %d workers x %d columns (%.2f GB per column)" % (method_name, info["workers"], info["capacity"],
                                                                         info["bytes_per_column"] / 1e9))

        def make_req():
            size = int(round(2 ** rng.uniform(0, 9)))
            return pool[rng.integers(0, len(pool), size=size)]

        # warm-up (workspaces, graphs)
        for t in [srv.submit(make_req()) for _ in range(args.workers * 2)]:
            srv.poll(t)
        # saturation: a burst of requests, completion rate in queries/s
        reqs = [make_req() for _ in range(args.requests)]
        tt = time.perf_counter()
        tks = [srv.submit(r) for r in reqs]
        lats = [srv.poll(t)[3] for t in tks]
        el = time.perf_counter() - tt
        nq = sum(len(r) for r in reqs)
        sat = nq / el
        entry = {"saturation_qps": sat, "burst_requests": len(reqs), "mean_request_size": nq / len(reqs)}
        log("  %s saturation: %.1f queries/s (%d requests, %d queries, %.1fs)" % (method_name, sat, len(reqs), nq, el))
        for load in (0.5, 0.8, 0.95):
            reqs = [make_req() for _ in range(args.requests)]
            mean_q = np.mean([len(r) for r in reqs])
            rate = load * sat / mean_q                       # requests per second
            gaps = rng.exponential(1.0 / rate, size=len(reqs))
            tks = []
            tt = time.perf_counter()
            nxt = tt
            for r, gp in zip(reqs, gaps):
                nxt += gp
                d = nxt - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                tks.append(srv.submit(r))
            lat = np.array([srv.poll(t)[3] for t in tks])
            el = time.perf_counter() - tt
            nq = sum(len(r) for r in reqs)
            entry["load_%g" % load] = {"offered_qps": load * sat, "achieved_qps": nq / el,
                                       "p50_ms": float(np.percentile(lat, 50)),
                                       "p99_ms": float(np.percentile(lat, 99))}
            log("  %s load %.2f: offered %.1f q/s, achieved %.1f q/s, p50 %.1f ms, p99 %.1f ms"
                % (method_name, load, load * sat, nq / el, np.percentile(lat, 50), np.percentile(lat, 99)))
        results[method_name] = entry
        srv.close()
    head = results["lrc"]
    line = {"metric": "Katz queries/sec at 1e-6 rel. residual, LRC-Katz vs CG, 1 MI355X; p99 ms",
            "value": round(head["saturation_qps"], 2), "unit": "queries/s", "n_gpus": 1, "steps": args.requests,
            "warmup": args.workers * 2, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32+bf16/f64" if prec == K.KATZ_PREC_MIXED else "f64",
            "data": "synthetic",
            "config": {"workload": "serving, %s, %d nodes, top-100 requests of 1-512 nodes" % (wl, g.n),
                       "n": g.n, "nnz": g.nnz, "workers": args.workers, "max_batch": args.max_batch_cols},
            "p99_ms": round(head["load_0.8"]["p99_ms"], 3), "cg_qps": round(results["cg"]["saturation_qps"], 2),
            "roofline": None, "cpu_baseline": None, "results": results}
    print(json.dumps(line), flush=True)


def measured_copy_bandwidth(torch, dev, nbytes=1 << 30, reps=5):
    """Device-to-device copy rate (bytes read + written per second, GB/s) of
    a plain 1 GiB copy, best of `reps`, timed with HIP events."""
    x = torch.empty(nbytes // 8, dtype=torch.float64, device=dev)
    y = torch.empty_like(x)
    y.copy_(x)
    best = 0.0
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        y.copy_(x)
        b.record()
        b.synchronize()
        best = max(best, 2 * nbytes / (a.elapsed_time(b) * 1e-3) / 1e9)
    del x, y
    torch.cuda.empty_cache()
    return best


def cpu_baseline(g, idx, queries, tol, out, stream, K):
    """Times the CPU oracle (never tuned) on a bounded sample of the queries and
    checks the GPU's scores for those queries against it (full-size parity)."""
    import numpy as np

    import oracle
    info = idx.info
    sample = [int(q) for q in queries[:4]]
    # the oracle's own lambda_max (outside the timed region) and the same c
    lam = oracle.lambda_max(oracle.csr_matrix(g.n, g.row_ptr, g.col))
    t = time.perf_counter()
    ref = oracle.katz_oracle(g.n, g.row_ptr, g.col, sample, c=info.c, lam=lam, validate=False)
    el = time.perf_counter() - t
    errs = []
    for j, q in enumerate(sample):
        sc, st = idx.query([q], tol=tol)
        k = ref["k"][:, j]
        errs.append(float(np.linalg.norm(sc[0] - k) / np.linalg.norm(k)))
    bound = tol * (1 + info.c) / (1 - info.c)
    log("  cpu oracle: %d queries in %.1fs; GPU rel err max %.2e (bound %.2e)" % (len(sample), el, max(errs), bound))
    return {"baseline": {"value": round(len(sample) / el, 4), "unit": "queries/s", "cores": 1, "kind": "oracle",
                         "sample": "%d queries of the same graph and c, truncated Neumann series to a 1e-13 tail "
                                   "bound (scipy CSR SpMV, single thread)" % len(sample)},
            "gpu_rel_err_max": max(errs), "err_bound": bound, "oracle_terms": ref["terms"].tolist()}


if __name__ == "__main__":
    main()
