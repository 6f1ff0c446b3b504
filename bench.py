"""Benchmark: Katz queries/sec at 1e-6 relative residual, LRC-Katz vs plain GPU CG,
on one MI355X.

Workload (default): Chung-Lu power-law graph, 1,000,000 nodes, exponent 2.5,
mean degree 20 (seeded, synthetic), damping c = beta * lambda_max in
{0.1, 0.5, 0.9}, rank 32, FP64, one query node per solve.  A step is one query
solved through the whole path (right-hand side, Schur RHS, PCG on S, block
back-solve, FP64 residual check, unpermute into a device buffer).  The headline
value is LRC queries/sec at c = 0.5; CG at the same c, latency percentiles,
iterations and the other c values are reported beside it.

Two batched legs follow in the same run and are reported inside `results`
(`legs`): the 4M-node lognormal SBM with 256 queries per solve in FP64
(c = 0.5, rank 32) and the 8M-node Chung-Lu graph with 512 queries per solve
in the precision form (c = 0.9, rank 64).  Each reports LRC and CG
queries/sec, its dominant kernel's roofline and the error of sampled columns
against the oracle.

CPU side (rank 0 only): the oracle's multi-core Neumann series and a
multi-core FP64 CPU CG (oracle/katz_cpu.c) on bounded samples of each
workload, with the host's core count, CPU model and thread placement.  The
GPU's sampled errors must lie within the residual's bound; the line carries
`parity_ok` and the run exits with status 3 when it is false.

Prints ONE JSON line.  Options: --gpus (1 only), --steps, --warmup, --c,
--scale (node-count factor for quick runs), --no-cpu (skip the CPU legs),
--legs (batched legs to run, default "c3,c4"; "" for none), --copy-calib
(adds a plain 1 GiB device copy, to calibrate rocprofv3 byte counters),
--no-profile-kernels (skip the HIP-event kernel timing in a repeat of the
timed steps).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

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
    ap.add_argument("--partition", type=str, default="bfs", choices=["bfs", "louvain"],
                    help="one-query workload: initial parts of the partition (bfs: one part cut into BFS chunks, "
                         "the build's default; louvain: katz_communities capped at max_block)")
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
    ap.add_argument("--methods", type=str, default="lrc,cg", help="serving: methods to run (lrc, cg)")
    ap.add_argument("--burst", type=int, default=0, help="serving: requests of the saturation burst (default --requests)")
    ap.add_argument("--max-batch-cols", type=int, default=64)
    ap.add_argument("--legs", type=str, default="c3,c4",
                    help="batched legs after the one-query headline: c3 (4M-node SBM, 256 FP64 columns), "
                         "c4 (8M-node Chung-Lu, 512 columns, precision form); empty for none")
    ap.add_argument("--ablation", action="store_true",
                    help="the paper's regime and ablations: Table 1-shaped Chung-Lu graphs at alpha = "
                         "1/(lambda_max + 1) (LRC, the PCGNR recurrence, CG; ranks 5 and 25), and L = chol / "
                         "IC(0) / I on community graphs where the dense factor fits")
    ap.add_argument("--latency-queries", type=int, default=500,
                    help="one-query workload: queries per c and method in the latency pass (p50/p99; "
                         "500: the p99 is about the fifth-slowest query, not the slowest)")
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
    if args.ablation:
        return run_ablation(args)
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
    # warm-up, timed and latency queries all distinct (a seeded prefix: more
    # latency queries leave the timed ones unchanged)
    queries = ki.sample_queries(g, max(100, args.latency_queries + args.steps + args.warmup), 2002)
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

    labels = None
    if args.partition == "louvain":
        tb = time.time()
        labels, passes = K.katz_communities(g.n, g.row_ptr, g.col, cap=args.max_block, passes=8)
        log("communities: %d in %d passes (%.1fs)" % (int(labels.max()) + 1, passes, time.time() - tb))
    for c in cs:
        tb = time.time()
        idx = K.KatzIndex.from_graph(g, beta_frac=c, rank=args.rank, max_block=args.max_block, device=0,
                                     u_precision=args.u_precision, labels=labels,
                                     precision=K.KATZ_PREC_MIXED if args.precision == "mixed" else K.KATZ_PREC_FP64)
        info = idx.info
        log("c=%.2f index: n1=%d n2=%d blocks=%d sigma1=%.4f sigma_r+1=%.5f build %.1fs"
            % (c, info.n1, info.n2, info.nblocks, info.sigma_max, info.sigma_next, time.time() - tb))
        entry = {"n1": info.n1, "n2": info.n2, "nblocks": info.nblocks, "build_s": round(info.build_seconds, 2),
                 "build_phases": build_phases(info), "beta": info.beta, "lambda_max": info.lambda_max}
        for name, method in (("lrc", K.KATZ_METHOD_LRC), ("cg", K.KATZ_METHOD_CG)):
            run(idx, method, args.warmup, 0)
            torch.cuda.synchronize()
            t = time.perf_counter()
            lat, its, res = run(idx, method, args.steps, args.warmup)
            torch.cuda.synchronize()
            el = time.perf_counter() - t
            # latency pass: p50 / p99 over further queries (outside the timed steps)
            nl = max(args.latency_queries, args.steps)
            lat2, its2, res2 = run(idx, method, nl, args.warmup + args.steps)
            lat_ms = np.array(lat2) * 1e3
            entry[name] = {"qps": args.steps / el, "ms_per_query": el * 1e3 / args.steps,
                           "p50_ms": float(np.percentile(lat_ms, 50)), "p99_ms": float(np.percentile(lat_ms, 99)),
                           "latency_queries": nl,
                           "iters_median": float(np.median(its + its2)),
                           "iters_p99": float(np.percentile(its + its2, 99)), "iters_max": int(np.max(its + its2)),
                           "max_rel_residual": float(np.max(res + res2))}
            log("  %s: %.1f q/s, %.3f ms/query, p50 %.3f p99 %.3f max %.3f ms over %d, iters median %g"
                % (name, entry[name]["qps"], entry[name]["ms_per_query"], entry[name]["p50_ms"],
                   entry[name]["p99_ms"], float(np.max(lat_ms)), nl, entry[name]["iters_median"]))
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
                # an untimed round first: each thread's workspace, its captured
                # iteration graphs and the device caches are in place before timing
                ths = [threading.Thread(target=worker, args=(i,)) for i in range(args.concurrency)]
                for th in ths:
                    th.start()
                for th in ths:
                    th.join()
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
                tab = kernel_rows(K)
                entry[name]["kernels"] = tab
                entry[name]["path_roofline"] = path_roofline(tab, args.steps, entry[name]["qps"])
                if name == "lrc":
                    kernel_table = tab
        if c == head_c and not args.no_cpu:
            entry["cpu"] = cpu_leg_one_query(g, idx, queries, tol, K)
        results["c=%g" % c] = entry
        idx.close()

    if args.copy_calib:
        x = torch.empty(2 ** 27, dtype=torch.float64, device=dev)   # 1 GiB
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        del x, y

    head = results["c=%g" % head_c]
    del out
    torch.cuda.empty_cache()
    copy_gbs = measured_copy_bandwidth(torch, dev)
    log("measured device copy bandwidth: %.0f GB/s (read + write of a 1 GiB copy)" % copy_gbs)
    if kernel_table:
        wl = "cl1m" if args.scale == 1.0 else "cl1m_s%g" % args.scale
        roofline = roofline_of(kernel_table, wl, copy_gbs)

    legs = {}
    for leg in [x for x in args.legs.split(",") if x]:
        legs[leg] = run_leg(leg, args, torch, K, ki, dev, copy_gbs)
    if legs:
        results["legs"] = legs

    value = head["lrc"]["qps"]
    cpu = head.get("cpu")
    parity = [head["cpu"]["parity_ok"]] if cpu else []
    parity += [lg["parity_ok"] for lg in legs.values() if "parity_ok" in lg]
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
                   "output": "pinned host memory (PCIe-inclusive)" if args.host_output else "device memory",
                   "partition": args.partition},
        "p99_ms": round(head["lrc"]["p99_ms"], 4),
        "p50_ms": round(head["lrc"]["p50_ms"], 4),
        "latency_queries": head["lrc"]["latency_queries"],
        "cg_qps": round(head["cg"]["qps"], 2),
        "lrc_over_cg": round(value / head["cg"]["qps"], 3),
        "concurrent": {"threads": args.concurrency,
                       "lrc_qps": round(head["lrc"].get("concurrent_qps", 0.0), 2),
                       "cg_qps": round(head["cg"].get("concurrent_qps", 0.0), 2)} if args.concurrency > 1 else None,
        "roofline": roofline,
        "path_roofline": {m: head[m].get("path_roofline") for m in ("lrc", "cg")},
        "iters": {m: {"median": head[m]["iters_median"], "p99": head[m]["iters_p99"]} for m in ("lrc", "cg")},
        "cpu_baseline": cpu["baseline"] if cpu else None,
        "parity_ok": all(parity) if parity else None,
        "legs": {k: {"lrc_qps": v["lrc"]["qps"], "cg_qps": v["cg"]["qps"], "lrc_over_cg": v["lrc_over_cg"],
                     "roofline_frac": (v.get("roofline") or {}).get("frac"),
                     "path_frac": {m: (v[m].get("path_roofline") or {}).get("frac") for m in ("lrc", "cg")},
                     "max_rel_err_vs_oracle": v.get("max_rel_err_vs_oracle")} for k, v in legs.items()},
        "results": results,
    }
    print(json.dumps(line), flush=True)
    if parity and not all(parity):
        log("PARITY FAILURE: a sampled GPU result lies outside its residual bound against the oracle")
        sys.exit(3)


def kernel_rows(K):
    """The profiled kernel table (HIP events) with per-launch figures."""
    tab = [r for r in K.katz_profile_read() if r["launches"] > 0]
    for r in tab:
        r["avg_us"] = 1e3 * r["total_ms"] / r["launches"]
        r["alg_bytes_per_launch"] = r["alg_bytes"] / r["launches"]
        r["achieved_GBs"] = r["alg_bytes"] / (r["total_ms"] * 1e-3) / 1e9
    return tab


def path_roofline(tab, queries, qps):
    """Path-level roofline: the algorithmic bytes of every profiled kernel per
    query (the profiled pass solved `queries` queries), and queries/s as a
    fraction of 8 TB/s over those bytes."""
    per_query = sum(r["alg_bytes"] for r in tab) / max(1, queries)
    return {"alg_bytes_per_query": per_query,
            "roof_qps": HBM_PEAK_GBS * 1e9 / per_query if per_query > 0 else None,
            "frac": round(qps * per_query / (HBM_PEAK_GBS * 1e9), 4) if per_query > 0 else None}


def roofline_of(tab, workload_key, copy_gbs):
    """Roofline object of the kernel with the largest total time."""
    dom = max(tab, key=lambda r: r["total_ms"])
    traffic = load_traffic(dom["name"], workload_key, dom["alg_bytes_per_launch"])
    return {"bound": "hbm", "kernel": dom["name"], "achieved": round(dom["achieved_GBs"], 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(dom["achieved_GBs"] / HBM_PEAK_GBS, 4),
            "traffic": traffic, "avg_launch_us": round(dom["avg_us"], 2),
            "alg_bytes_per_launch": dom["alg_bytes_per_launch"],
            "measured_copy_GBs": round(copy_gbs, 1) if copy_gbs else None,
            "frac_of_measured_copy": round(dom["achieved_GBs"] / copy_gbs, 4) if copy_gbs else None,
            "traffic_GBs": round(traffic / (dom["avg_us"] * 1e-6) / 1e9, 1) if traffic else None}


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


# Table 1 of the paper: network, nodes, average degree (the stand-ins are
# Chung-Lu graphs with exponent 2.5 and these sizes; the networks themselves
# are not available).
TABLE1 = [("DBLP_lcc", 93156, 3.82), ("Arxiv_lcc", 86376, 11.98), ("Email-Enron", 36692, 10.02),
          ("Gowalla", 196591, 9.67), ("Flickr", 513969, 12.41), ("Hollywood-2009", 1139905, 99.13),
          ("PPI_Data", 12976, 7.6916), ("DBLP_2006-2008", 179266, 4.2693)]


def run_ablation(args):
    """NEXT-3: (1) Table 1-shaped Chung-Lu graphs at the paper's damping
    alpha = 1 / (lambda_max + 1), one query per solve, FP64, L = I, ranks 5
    and 25: PCG on S (LRC-Katz), the PCGNR recurrence of Algorithm 2 (step
    corrected) and plain CG; iterations and queries/s.  (2) The factor L of
    the preconditioner (eq. RMatrix): dense chol(M22), its zero-fill
    incomplete factor IC(0) and I, on community graphs whose separator fits
    the dense factor (2,000 and 5,000 nodes), c in {0.5, 0.9, 0.99}, ranks 0
    and 16."""
    import torch

    import katz_inputs as ki
    import paper_1912_06525_amd as K

    dev = torch.device("cuda:0")
    steps = max(4, min(args.steps, 20))
    tol = 1e-6

    def measure(idx, g, method, qs):
        out = torch.empty((1, g.n), dtype=torch.float64, device=dev)
        stream = torch.cuda.current_stream(dev).cuda_stream
        for q in qs[:3]:   # warm-up (autotuned launch shape, captured iteration chunks)
            idx.query([int(q)], out=out, tol=tol, method=method, stream=stream)
        torch.cuda.synchronize()
        its = []
        t = time.perf_counter()
        for q in qs:
            _, st = idx.query([int(q)], out=out, tol=tol, method=method, stream=stream)
            if st[0]["status"] != 0:
                raise RuntimeError("no convergence: %r" % st[0])
            its.append(st[0]["iters"])
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        return {"qps": round(len(qs) / el, 1), "iters_median": float(np.median(its)), "iters_max": int(max(its))}

    regime = {}
    for name, n, deg in TABLE1:
        n = max(1000, int(round(n * args.scale)))
        t0 = time.time()
        g = ki.chung_lu(n, 2.5, deg, seed=1100)
        # lambda_max from a host-only index of the same graph (the library's own Lanczos)
        lam = K.KatzIndex.from_graph(g, beta_frac=0.5, rank=0, max_block=args.max_block, device=-1).info.lambda_max
        beta = 1.0 / (lam + 1.0)
        qs = ki.sample_queries(g, steps, 1200)
        entry = {"n": g.n, "nnz": g.nnz, "mean_degree": round(g.nnz / g.n, 2), "lambda_max": lam,
                 "alpha": beta, "c": lam / (lam + 1.0)}
        for rank in (5, 25):
            idx = K.KatzIndex.from_graph(g, beta=beta, rank=rank, max_block=args.max_block, device=0,
                                         l_kind=K.KATZ_L_IDENTITY)
            e = {"n2": idx.info.n2, "sigma_r": idx.info.sigma_max, "build_s": round(idx.info.build_seconds, 2)}
            for mname, m in (("lrc", K.KATZ_METHOD_LRC), ("pcgnr", K.KATZ_METHOD_PCGNR), ("cg", K.KATZ_METHOD_CG)):
                if mname == "cg" and rank != 5:
                    continue
                e[mname] = measure(idx, g, m, qs)
            entry["rank%d" % rank] = e
            idx.close()
        entry["cg"] = entry["rank5"].pop("cg")
        log("%-15s n=%d nnz=%d c=%.5f: LRC r5 %s / r25 %s, PCGNR r5 %s, CG %s (%.0fs)"
            % (name, g.n, g.nnz, entry["c"], entry["rank5"]["lrc"], entry["rank25"]["lrc"],
               entry["rank5"]["pcgnr"], entry["cg"], time.time() - t0))
        regime[name] = entry
        torch.cuda.empty_cache()

    factors = {}
    for nblk in (10, 25):
        g = ki.sbm([200] * nblk, 0.05, 0.001, seed=1001)
        qs = ki.sample_queries(g, steps, 2001)
        for c in (0.5, 0.9, 0.99):
            key = "sbm%dk_c%g" % (nblk * 200 // 1000, c)
            factors[key] = {"n": g.n, "nnz": g.nnz}
            for lname, lk in (("chol", K.KATZ_L_CHOL), ("ic0", K.KATZ_L_IC0), ("identity", K.KATZ_L_IDENTITY)):
                for rank in (0, 16):
                    idx = K.KatzIndex.from_graph(g, beta_frac=c, rank=rank, labels=g.labels, max_block=200,
                                                 device=0, l_kind=lk)
                    e = measure(idx, g, K.KATZ_METHOD_LRC, qs)
                    e["n2"] = idx.info.n2
                    factors[key]["%s_r%d" % (lname, rank)] = e
                    idx.close()
            factors[key]["cg"] = measure(K.KatzIndex.from_graph(g, beta_frac=c, rank=0, labels=g.labels,
                                                                max_block=200, device=0), g, K.KATZ_METHOD_CG, qs)
            log("%s: %s" % (key, {k: (v["iters_median"], v["qps"]) for k, v in factors[key].items()
                                  if isinstance(v, dict)}))
    line = {"metric": "ablations: iterations and Katz queries/sec at 1e-6 rel. residual, 1 MI355X",
            "value": None, "unit": "queries/s", "n_gpus": 1, "steps": steps, "warmup": 1, "ms_per_step": None,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "Table 1-shaped Chung-Lu graphs (exponent 2.5) at alpha = 1/(lambda_max+1); "
                                   "SBMs of 200-node communities for the factor comparison", "scale": args.scale},
            "paper_regime": regime, "factor_comparison": factors}
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
    log("index: n2=%d build %.1fs %s" % (idx.info.n2, time.time() - tb, build_phases(idx.info)))
    rng = np.random.default_rng(4005)
    pool = ki.sample_queries(g, min(g.n // 2, 200000), 4006)
    results = {}
    for method_name, method in (("lrc", K.KATZ_METHOD_LRC), ("cg", K.KATZ_METHOD_CG)):
        if method_name not in args.methods.split(","):
            continue
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
        reqs = [make_req() for _ in range(args.burst or args.requests)]
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
    head = results.get("lrc") or results["cg"]
    line = {"metric": "Katz queries/sec at 1e-6 rel. residual, LRC-Katz vs CG, 1 MI355X; p99 ms",
            "value": round(head["saturation_qps"], 2), "unit": "queries/s", "n_gpus": 1, "steps": args.requests,
            "warmup": args.workers * 2, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32+bf16/f64" if prec == K.KATZ_PREC_MIXED else "f64",
            "data": "synthetic",
            "config": {"workload": "serving, %s, %d nodes, top-100 requests of 1-512 nodes" % (wl, g.n),
                       "n": g.n, "nnz": g.nnz, "workers": args.workers, "max_batch": args.max_batch_cols,
                       "requests_per_load_point": args.requests},
            "build_s": round(idx.info.build_seconds, 2), "build_phases": build_phases(idx.info),
            "p99_ms": round(head["load_0.8"]["p99_ms"], 3),
            "cg_qps": round(results["cg"]["saturation_qps"], 2) if "cg" in results else None,
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


def host_info():
    """Host cores, CPU model and thread placement of the CPU legs."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = os.cpu_count()
    bind = os.environ.get("OMP_PROC_BIND"), os.environ.get("OMP_PLACES"), os.environ.get("GOMP_CPU_AFFINITY")
    pin = ("OMP_PROC_BIND=%s OMP_PLACES=%s GOMP_CPU_AFFINITY=%s" % bind) if any(bind) else \
        "none: OpenMP threads placed by the OS scheduler"
    return {"nproc": os.cpu_count(), "affinity_cpus": aff, "cpu_model": model,
            "omp_num_threads_env": os.environ.get("OMP_NUM_THREADS"), "pinning": pin}


def cpu_threads():
    """OpenMP threads for the CPU legs: every CPU this process may use."""
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:
        return max(1, os.cpu_count() or 1)


def _errs(kh, k):
    nk = float(np.linalg.norm(k))
    return float(np.linalg.norm(kh - k)) / nk, float(np.max(np.abs(kh - k))) / nk


def cpu_leg_one_query(g, idx, queries, tol, K, nsample=8):
    """CPU side of the one-query workload, after the GPU timing: the oracle's
    multi-core series and the multi-core CPU CG, each on `nsample` queries of
    the same graph and c, and the GPU's error on those queries against the
    oracle.  The oracle is evaluated at the index's beta; its tail bound uses
    c from the oracle's own lambda_max (which must agree with the index's)."""
    import oracle
    info = idx.info
    sample = [int(q) for q in queries[:nsample]]
    thr = cpu_threads()
    lam = oracle.lambda_max_mt(g.n, g.row_ptr, g.col, threads=thr)["lambda"]
    c_or = info.beta * lam
    t = time.perf_counter()
    ser = oracle.katz_series_mt(g.n, g.row_ptr, g.col, sample, info.beta, c_or * (1 + 1e-6), tol=1e-13, threads=thr)
    el_or = time.perf_counter() - t
    # the single-threaded Python oracle (scipy SpMV) on 2 of the queries, as an extra
    t = time.perf_counter()
    ref1 = oracle.katz_oracle(g.n, g.row_ptr, g.col, sample[:2], beta=info.beta, lam=lam, validate=False)
    el_1 = time.perf_counter() - t
    # CPU CG, one query per solve like the GPU headline
    t = time.perf_counter()
    cg_its = []
    for q in sample:
        r = oracle.cg_mt(g.n, g.row_ptr, g.col, [q], info.beta, tol=tol, threads=thr)
        if not r["converged"]:
            raise RuntimeError("CPU CG did not converge on query %d" % q)
        cg_its.append(int(r["iters"][0]))
    el_cg = time.perf_counter() - t
    errs = []
    for j, q in enumerate(sample):
        for method in (K.KATZ_METHOD_LRC, K.KATZ_METHOD_CG):
            sc, st = idx.query([q], tol=tol, method=method)
            errs.append(_errs(sc[0], ser["k"][:, j]))
    e1 = max(_errs(ref1["k"][:, j], ser["k"][:, j])[0] for j in range(2))
    bound = tol * (1 + c_or) / (1 - c_or) + 1e-13
    ok = all(e[0] <= bound and e[1] <= bound for e in errs)
    log("  cpu: oracle series %d queries in %.1fs (%d threads), 1-core oracle 2 in %.1fs, CPU CG %d in %.1fs "
        "(iters %s); GPU rel err max %.2e (bound %.2e)" % (len(sample), el_or, ser["threads"], el_1, len(sample),
                                                           el_cg, cg_its, max(e[0] for e in errs), bound))
    hi = host_info()
    base = {"value": round(len(sample) / el_or, 4), "unit": "queries/s", "cores": ser["threads"], "kind": "oracle",
            "sample": "%d queries of the same graph and c in one multi-column truncated Neumann series to a "
                      "1e-13 tail bound (oracle/katz_cpu.c, OpenMP)" % len(sample),
            "host": hi,
            "cpu_cg": {"value": round(len(sample) / el_cg, 4), "unit": "queries/s", "cores": thr,
                       "kind": "FP64 CG, one query per solve, OpenMP CSR SpMV, stop at true residual %g" % tol,
                       "iters": cg_its},
            "oracle_1core": {"value": round(2 / el_1, 4), "unit": "queries/s", "cores": 1,
                             "kind": "Python oracle (scipy CSR SpMV), truncated series to a 1e-13 tail bound",
                             "max_rel_diff_vs_multicore_oracle": e1},
            "gpu_err_vs_oracle": [{"query": q, "lrc_rel_err": errs[2 * j][0], "lrc_max_entry_err": errs[2 * j][1],
                                   "cg_rel_err": errs[2 * j + 1][0], "cg_max_entry_err": errs[2 * j + 1][1]}
                                  for j, q in enumerate(sample)],
            "err_bound": bound, "lambda_rel_diff": abs(lam - info.lambda_max) / lam}
    return {"baseline": base, "parity_ok": ok and base["lambda_rel_diff"] <= 1e-9}


PHASES = ["validate", "lambda_max", "partition_bfs_chunks", "partition_vertex_cover", "partition_minimality",
          "partition_components", "partition_order", "permuted_csr", "block_inverses", "m22_factor",
          "lanczos_on_R", "device_upload"]


def build_phases(info):
    """The index build's wall seconds per phase (katz_index_info_t)."""
    return {k: round(v, 3) for k, v in zip(PHASES, info.build_phase_seconds)}


LEGS = {
    # name: workload, columns per solve, c, rank, precision, oracle tail fraction
    "c3": ("lnsbm4m", 256, 0.5, 32, "fp64", 1e-10),
    "c4": ("cl8m", 512, 0.9, 64, "mixed", 1e-7),
}


def run_leg(leg, args, torch, K, ki, dev, copy_gbs):
    """One batched leg: LRC and CG queries/sec on B columns per solve, the
    dominant kernel's roofline, and (unless --no-cpu) the oracle's series
    and the CPU CG on 8 sampled columns, run on the host cores in a thread
    while the GPU is timed."""
    import threading

    import oracle
    wl, B, c, rank, precision, tail = LEGS[leg]
    t0 = time.time()
    w = ki.workload(wl, scale=args.scale)
    g = w.graph
    log("leg %s: %s n=%d nnz=%d (%.1fs)" % (leg, wl, g.n, g.nnz, time.time() - t0))
    prec = K.KATZ_PREC_MIXED if precision == "mixed" else K.KATZ_PREC_FP64
    tb = time.time()
    idx = K.KatzIndex.from_graph(g, beta_frac=c, rank=rank, max_block=args.max_block, device=0,
                                 labels=g.labels, precision=prec)
    info = idx.info
    log("  index: n1=%d n2=%d blocks=%d build %.1fs, %.1f GB on the device"
        % (info.n1, info.n2, info.nblocks, time.time() - tb, info.device_bytes / 1e9))
    steps, warm = max(2, min(args.steps, 4)), 1
    queries = ki.sample_queries(g, B * (steps + warm), 3003)
    pick = sorted({0, B - 1, *[int(x) for x in np.random.default_rng(7).choice(np.arange(1, B - 1), 6, False)]})
    sample = [int(queries[warm * B + j]) for j in pick]
    tol = 1e-6
    cpu = {}

    def cpu_work():
        try:
            thr = max(1, cpu_threads() - 2)   # two cores stay with the GPU-driving thread
            lam = oracle.lambda_max_mt(g.n, g.row_ptr, g.col, threads=thr)["lambda"]
            cpu["lambda"] = lam
            t = time.perf_counter()
            cpu["series"] = oracle.katz_series_mt(g.n, g.row_ptr, g.col, sample, info.beta, info.beta * lam * (1 + 1e-6),
                                                  tol=tail, threads=thr)
            cpu["series_s"] = time.perf_counter() - t
            t = time.perf_counter()
            r = oracle.cg_mt(g.n, g.row_ptr, g.col, sample, info.beta, tol=tol, threads=thr)
            cpu["cg_s"] = time.perf_counter() - t
            cpu["cg_iters"] = [int(x) for x in r["iters"]]
            cpu["cg_ok"] = bool(r["converged"])
            cpu["threads"] = thr
        except Exception as e:  # reported in the result
            cpu["error"] = repr(e)

    th = None
    if not args.no_cpu:
        th = threading.Thread(target=cpu_work)
        th.start()
    out = torch.empty((B, g.n), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    entry = {"workload": wl, "n": g.n, "nnz": g.nnz, "batch": B, "c": c, "rank": rank, "precision": precision,
             "n1": info.n1, "n2": info.n2, "build_s": round(info.build_seconds, 2), "build_phases": build_phases(info),
             "steps": steps, "warmup": warm}
    picked = None
    for name, method in (("lrc", K.KATZ_METHOD_LRC), ("cg", K.KATZ_METHOD_CG)):
        def step(s):
            q = queries[s * B:(s + 1) * B]
            _, st = idx.query(q, out=out, tol=tol, method=method, stream=stream)
            bad = [x for x in st if x["status"] != 0]
            if bad:
                raise RuntimeError("no convergence: %r" % bad[:2])
            return st
        for s in range(warm):
            step(s)
        torch.cuda.synchronize()
        t = time.perf_counter()
        its, sw, res = [], [], []
        for s in range(steps):
            st = step(warm + s)
            its += [x["iters"] for x in st]
            sw += [x["sweeps"] for x in st]
            res += [x["rel_residual"] for x in st]
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        entry[name] = {"qps": B * steps / el, "ms_per_batch": 1e3 * el / steps,
                       "iters_median": float(np.median(its)), "sweeps_median": float(np.median(sw)),
                       "max_rel_residual": float(np.max(res))}
        log("  %s: %.1f q/s, %.1f ms per batch of %d, iters median %g, sweeps %g"
            % (name, entry[name]["qps"], entry[name]["ms_per_batch"], B, entry[name]["iters_median"],
               entry[name]["sweeps_median"]))
        # sampled columns of the first timed batch (re-solved: the timed steps overwrote the panel)
        step(warm)
        torch.cuda.synchronize()
        cols = np.stack([out[j].cpu().numpy() for j in pick], axis=1)
        if name == "lrc":
            picked = {"lrc": cols}
        else:
            picked["cg"] = cols
        if not args.no_profile_kernels:
            K.katz_profile_reset()
            K.katz_profile_enable(True)
            step(warm)
            torch.cuda.synchronize()
            K.katz_profile_enable(False)
            tab = kernel_rows(K)
            entry[name]["kernels"] = tab
            entry[name]["path_roofline"] = path_roofline(tab, B, entry[name]["qps"])
            if name == "lrc":
                wk = wl if args.scale == 1.0 else "%s_s%g" % (wl, args.scale)
                entry["roofline"] = roofline_of(tab, "%s_b%d_c%g" % (wk, B, c), copy_gbs)
    entry["lrc_over_cg"] = round(entry["lrc"]["qps"] / entry["cg"]["qps"], 3)
    del out
    idx.close()
    torch.cuda.empty_cache()
    if th is not None:
        th.join()
        if "error" in cpu:
            raise RuntimeError("CPU leg failed: %s" % cpu["error"])
        lam = cpu["lambda"]
        c_or = info.beta * lam
        bound = tol * (1 + c_or) / (1 - c_or) + 2 * tail
        errs = {m: [_errs(picked[m][:, t], cpu["series"]["k"][:, t]) for t in range(len(pick))] for m in picked}
        worst = max(e[0] for m in errs for e in errs[m])
        entry["max_rel_err_vs_oracle"] = worst
        entry["err_bound"] = bound
        entry["oracle_sample"] = {"columns": pick, "queries": sample,
                                  "terms": [int(x) for x in cpu["series"]["terms"]],
                                  "lrc_rel_err": [e[0] for e in errs["lrc"]], "cg_rel_err": [e[0] for e in errs["cg"]],
                                  "lrc_max_entry_err": [e[1] for e in errs["lrc"]]}
        entry["lambda_rel_diff"] = abs(lam - info.lambda_max) / lam
        entry["parity_ok"] = bool(all(e[0] <= bound and e[1] <= bound for m in errs for e in errs[m])
                                  and entry["lambda_rel_diff"] <= 1e-9 and cpu["cg_ok"])
        entry["cpu"] = {"oracle": {"value": round(len(sample) / cpu["series_s"], 4), "unit": "queries/s",
                                   "cores": cpu["threads"], "kind": "oracle",
                                   "sample": "%d sampled columns of the first timed batch, one multi-column "
                                             "series to a %g tail bound" % (len(sample), tail)},
                        "cpu_cg": {"value": round(len(sample) / cpu["cg_s"], 4), "unit": "queries/s",
                                   "cores": cpu["threads"], "iters": cpu["cg_iters"],
                                   "kind": "FP64 CG, the %d sampled queries as one multi-RHS block, stop at true "
                                           "residual %g" % (len(sample), tol)},
                        "host": host_info()}
        log("  cpu: oracle %d columns in %.1fs, CPU CG in %.1fs (%d threads); GPU rel err max %.2e (bound %.2e)"
            % (len(sample), cpu["series_s"], cpu["cg_s"], cpu["threads"], worst, bound))
    return entry


if __name__ == "__main__":
    main()
