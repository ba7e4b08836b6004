"""Benchmark of the TripleID-Q query path on one MI355X.

Workload: the medium graph, 50M triples resident in HBM (subjects Zipf(1.0)
over 5M IDs, predicates Zipf(1.2) over 1000, objects Zipf(1.1) over 10M,
seed 2).  One step runs every operator of the path once:
  scan   (?s p ?o) at selectivities near 0.1%, 1% and 10%   3 graph passes
  star   (?s pA oA) . (?s pB ?o1) . (?s pC ?o2), sorted      1 pass + 2 joins
  union  8 subqueries (?s p_r ?o), r = 11..18, DISTINCT      1 pass + sort
  filter (?s ?p ?o) with o in [lo, hi) keeping ~5%           1 pass
value = graph passes x N / step time (triples/s).

Prints one JSON line.  --gpus N with N > 1 is refused: this build measures
one GPU.
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

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E, published


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_hash(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


SCAN_SOURCES = ["paper_1807_01409_amd/csrc/scan.hip", "paper_1807_01409_amd/csrc/compact.hpp",
                "paper_1807_01409_amd/csrc/device_common.hpp"]


def measured_traffic(kernel_hash):
    """HBM bytes per launch of the scan from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "scan_medium_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_hash") != kernel_hash:
        return None
    return d.get("hbm_bytes_per_launch")


def build_workload(g):
    from synth.queries import (predicate_for_selectivity, range_pattern, star_query,
                               union_query)
    from synth import Pattern
    preds = [predicate_for_selectivity(g, s) for s in (1e-3, 1e-2, 1e-1)]
    scans = [Pattern(0, p, 0, 0, -1, 1) for p, _ in preds]
    star, star_info = star_query(g)
    union, union_info = union_query(g)
    rng, rng_info = range_pattern(g)
    return {"preds": preds, "scans": scans, "star": star, "star_info": star_info,
            "union": union, "union_info": union_info, "range": rng, "range_info": rng_info}


def cpu_baseline(g, w):
    """The oracle, as it stands, on this host: one full step of the same
    workload (single-threaded plain C), repeated while under ~20 s."""
    import oracle
    oracle.build(force=False)
    n = g.shape[0]
    reps, t_total = 0, 0.0
    per = {}
    while reps < 3 and t_total < 20.0:
        t0 = time.perf_counter()
        for p in w["scans"]:
            oracle.scan(g, p)
        t1 = time.perf_counter()
        oracle.query(g, w["star"])
        t2 = time.perf_counter()
        oracle.query(g, w["union"])
        t3 = time.perf_counter()
        oracle.scan(g, w["range"])
        t4 = time.perf_counter()
        per = {"scans_s": t1 - t0, "star_s": t2 - t1, "union_s": t3 - t2, "filter_s": t4 - t3}
        t_total += t4 - t0
        reps += 1
    step_s = t_total / reps
    return {"value": 6 * n / step_s, "unit": "triples/s", "cores": 1, "kind": "oracle",
            "sample": f"the full step on the same 50M-triple graph, {reps} rep(s), "
                      f"single-threaded plain C (gcc -O2); last rep: "
                      + ", ".join(f"{k} {v:.2f}" for k, v in per.items())}


def event_time(torch, stream, fn, reps):
    """Average seconds per call of fn, with HIP events on `stream`, calls
    queued back to back.  Each result is released right after its call (in
    stream order), so the allocator reuses one block and no allocation falls
    inside the timed region."""
    fn().free()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(reps):
        fn().free()
    ev1.record(stream)
    ev1.synchronize()
    return ev0.elapsed_time(ev1) / 1e3 / reps


def batched(args):
    """1024 queries (1-6 patterns, star/chain, per-pattern selectivity
    log-uniform in [1e-6, 1e-1]) on the 200M-triple batched graph: one
    tid_query_batch call against 1024 tid_query calls, results compared."""
    import torch
    from paper_1807_01409_amd import Context
    from synth import CONFIGS, make_graph
    from synth.batch import PredIndex, batch_queries

    spec = CONFIGS["batched"] if args.n is None else CONFIGS["batched"].with_n(args.n)
    t0 = time.time()
    g = make_graph(spec)
    log(f"generated {spec.n} triples in {time.time() - t0:.1f}s")
    t0 = time.time()
    idx = PredIndex(g)
    plans, infos = batch_queries(idx, nq=args.queries, seed=spec.seed)
    del idx
    rows = np.array([i["rows"] for i in infos])
    log(f"{len(plans)} queries in {time.time() - t0:.1f}s; rows p50 {np.median(rows):.0f} "
        f"max {rows.max()}; patterns {sum(i['k'] for i in infos)}")
    ctx = Context(0)
    G = ctx.load(g)
    torch.cuda.synchronize()

    def serial():
        return [ctx.query(G, p) for p in plans]

    def batch():
        return ctx.query_batch(G, plans)

    for t in batch():           # warm-up both paths (allocator, code objects)
        t.free()
    for t in serial()[:64]:
        t.free()
    torch.cuda.synchronize()
    res = {}
    for name, fn in (("batched", batch), ("serial", serial)):
        best = None
        for _ in range(args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
            if name == "batched":
                keep_b = out
            else:
                keep_s = out
        res[name] = {"s": best, "qps": len(plans) / best}
        log(f"{name}: {best * 1e3:.1f} ms, {len(plans) / best:.0f} queries/s")
    # identity: each query in the batch equals the same query alone
    mism = 0
    for a, b in zip(keep_b, keep_s):
        if not np.array_equal(a.to_numpy(), b.to_numpy()):
            mism += 1
    out = {
        "metric": "batched vs serial queries/s",
        "value": res["batched"]["qps"], "unit": "queries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": res["batched"]["s"] * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"batched graph {spec.n} triples, {len(plans)} queries, 1-6 "
                               "patterns, star/chain 50/50, selectivity log-U[1e-6,1e-1]",
                   "n_triples": spec.n, "queries": len(plans),
                   "patterns": int(sum(i["k"] for i in infos)),
                   "rows_quantiles": [int(x) for x in np.quantile(rows, [0.5, 0.9, 0.99, 1.0])]},
        "serial_qps": res["serial"]["qps"],
        "speedup_vs_serial": res["batched"]["qps"] / res["serial"]["qps"],
        "batch_equals_alone_mismatches": mism,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def serving(args):
    """Continuous-batching server on the 1B-triple serving graph resident in
    HBM: Poisson arrivals at --qps drawn from a pool of --queries queries of
    the batched mix (1-6 patterns, star/chain, selectivity log-U[1e-6,1e-1]),
    admitted by estimated result bytes against --budget-gb.  Reports p50/p99
    latency and sustained queries/s, and checks that sampled requests return
    the same rows as the same query run alone."""
    from paper_1807_01409_amd.serve import Request, Server
    from synth import CONFIGS, make_graph
    from synth.batch import PredIndex, batch_queries, poisson_arrivals

    spec = CONFIGS["serving"] if args.n is None else CONFIGS["serving"].with_n(args.n)
    t0 = time.time()
    g = make_graph(spec)
    log(f"generated {spec.n} triples in {time.time() - t0:.1f}s")
    t0 = time.time()
    idx = PredIndex(g)
    log(f"index in {time.time() - t0:.1f}s")
    t0 = time.time()
    plans, infos = batch_queries(idx, nq=args.queries, seed=spec.seed)
    del idx
    log(f"{len(plans)} queries in {time.time() - t0:.1f}s")
    n_req = int(args.qps * args.duration)
    arrivals = poisson_arrivals(n_req, args.qps, spec.seed)
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([spec.seed, 0x5E7F])))
    pick = rng.integers(0, len(plans), size=n_req)
    reqs = [Request(i, plans[int(pick[i])], float(arrivals[i])) for i in range(n_req)]
    srv = Server(g, workers=args.serve_workers, budget_bytes=int(args.budget_gb * (1 << 30)),
                 max_batch=args.max_batch)
    log("graph resident; warm-up burst")
    srv.run([Request(-1 - i, plans[i % len(plans)], 0.0) for i in range(2 * args.max_batch)])
    check = set(range(0, n_req, max(1, n_req // 64)))
    st = srv.run(reqs, keep_results=check, warmup_s=args.warmup_s)
    log(f"served {n_req} requests in {st.wall_s:.2f}s: p50 {st.p50_ms:.2f} ms p99 "
        f"{st.p99_ms:.2f} ms, {st.qps:.0f} q/s, mean batch {st.mean_batch:.1f}")
    ctx = srv.ctxs[0]
    mism = 0
    for r in reqs:
        if r.rid in check:
            t = ctx.query(srv.graph, r.plan)
            if not np.array_equal(t.to_numpy(), r.result):
                mism += 1
            t.free()
    rows = np.array([i["rows"] for i in infos])
    out = {
        "metric": "serving p50/p99 latency and sustained queries/s",
        "value": st.qps, "unit": "queries/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": st.wall_s * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "p50_ms": st.p50_ms, "p99_ms": st.p99_ms,
        "config": {"workload": f"serving graph {spec.n} triples resident in HBM; Poisson "
                               f"arrivals at {args.qps:g} q/s for {args.duration:g}s from a pool "
                               f"of {len(plans)} batched-mix queries; result budget "
                               f"{args.budget_gb:g} GiB",
                   "n_triples": spec.n, "requests": n_req, "offered_qps": args.qps,
                   "workers": args.serve_workers, "max_batch": args.max_batch,
                   "warmup_s": args.warmup_s,
                   "pool_rows_quantiles": [int(x) for x in np.quantile(rows, [0.5, 0.9, 0.99, 1.0])]},
        "completed_after_warmup": st.completed, "mean_batch": st.mean_batch,
        "max_queue": st.max_queue, "max_inflight_bytes": st.max_inflight_bytes,
        "mix_equals_alone_checked": len(check), "mix_equals_alone_mismatches": mism,
    }
    print(json.dumps(out), flush=True)
    srv.close()


def scan_profile(args):
    """Short run for rocprofv3 counter collection: each of the benchmark's
    four single-pattern scans `--steps` times, then a plain device copy of a
    graph-sized buffer (the calibration kernel for the byte counters)."""
    import torch
    from paper_1807_01409_amd import Context
    from synth import CONFIGS, make_graph

    spec = CONFIGS["medium"] if args.n is None else CONFIGS["medium"].with_n(args.n)
    g = make_graph(spec)
    w = build_workload(g)
    ctx = Context(0)
    G = ctx.load(g)
    for p in w["scans"] + [w["range"]]:
        for _ in range(args.steps):
            ctx.scan(G, p).free()
    ctx.synchronize()
    src = torch.empty(spec.n * 3, dtype=torch.int32, device="cuda")
    with torch.cuda.stream(ctx.stream):
        for _ in range(args.steps):
            dst = src.clone()
            del dst
    torch.cuda.synchronize()
    log(f"scan-profile done: {len(w['scans']) + 1} scans x {args.steps}, copy of "
        f"{spec.n * 12} bytes x {args.steps}")
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=None, help="override graph size (testing)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=["medium", "batched", "serving", "scan-profile"],
                    default="medium")
    ap.add_argument("--queries", type=int, default=1024)
    ap.add_argument("--qps", type=float, default=2000.0, help="serving: offered load")
    ap.add_argument("--duration", type=float, default=10.0, help="serving: seconds of arrivals")
    ap.add_argument("--warmup-s", type=float, default=1.0, help="serving: arrivals not measured")
    ap.add_argument("--budget-gb", type=float, default=64.0, help="serving: result budget")
    ap.add_argument("--serve-workers", type=int, default=2)
    ap.add_argument("--max-batch", type=int, default=256)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.workload == "batched":
        batched(args)
        return
    if args.workload == "serving":
        serving(args)
        return
    if args.workload == "scan-profile":
        scan_profile(args)
        return

    import torch
    from paper_1807_01409_amd import Context
    from synth import CONFIGS, make_graph

    spec = CONFIGS["medium"] if args.n is None else CONFIGS["medium"].with_n(args.n)
    t0 = time.time()
    g = make_graph(spec)
    log(f"generated {spec.n} triples in {time.time() - t0:.1f}s")
    w = build_workload(g)
    log(f"workload: preds {w['preds']} star {w['star_info']} union {w['union_info']} "
        f"range {w['range_info']}")

    ctx = Context(0)
    G = ctx.load(g)
    torch.cuda.synchronize()
    log("graph resident")

    def step():
        for p in w["scans"]:
            ctx.scan(G, p).free()
        ctx.query(G, w["star"]).free()
        ctx.query(G, w["union"]).free()
        ctx.scan(G, w["range"]).free()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    passes = 6
    ms_per_step = elapsed / args.steps * 1e3
    value = passes * spec.n * args.steps / elapsed
    log(f"{ms_per_step:.3f} ms/step, {value / 1e9:.1f} G triples/s")

    # Dominant kernel: the single-pattern scan.  Average launch duration with
    # HIP events on the context's stream (the stream its kernels run on).
    reps = 20
    alg_bytes = dur_s = 0.0
    per_launch = []
    for p in w["scans"] + [w["range"]]:
        t = ctx.scan(G, p)
        rows, ncols = t.nrows, t.ncols
        t.free()
        d = event_time(torch, ctx.stream, lambda: ctx.scan(G, p), reps)
        b = 12.0 * spec.n + 4.0 * ncols * rows
        alg_bytes += b
        dur_s += d
        per_launch.append({"rows": rows, "cols": ncols, "us": round(d * 1e6, 2),
                           "GBps": round(b / d / 1e9, 1)})
    achieved = alg_bytes / dur_s / 1e9
    khash = source_hash(SCAN_SOURCES)
    breakdown = {
        "star_query_ms": event_time(torch, ctx.stream, lambda: ctx.query(G, w["star"]), 5) * 1e3,
        "union_query_ms": event_time(torch, ctx.stream, lambda: ctx.query(G, w["union"]), 5) * 1e3,
        "star_rows": ctx.query(G, w["star"]).nrows,
        "union_rows": ctx.query(G, w["union"]).nrows,
    }
    log(f"scan launches: {per_launch}; {breakdown}")

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(g, w)
        log(f"cpu baseline {cpu}")

    out = {
        "metric": "scan triples/s (% HBM peak)",
        "value": value,
        "unit": "triples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"medium graph: {spec.n} triples (s Zipf 1.0/5M, p Zipf 1.2/1000, "
                               "o Zipf 1.1/10M); step = 3 scans (0.1/1/10%), 3-star join, "
                               "8-way union DISTINCT, 5% object-range filter",
                   "n_triples": spec.n, "graph_passes_per_step": passes,
                   "scan_predicates": [p for p, _ in w["preds"]],
                   "scan_selectivity": [round(s, 6) for _, s in w["preds"]],
                   "star": w["star_info"], "union": w["union_info"], "range": w["range_info"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(khash),
                     "kernel": "single-pattern scan, ScanSrc<1> 512x8: compact_kernel "
                               "(block-ranged) for sparse outputs, chunk_compact_kernel for "
                               "dense ones",
                     "per_launch": per_launch},
        "breakdown": breakdown,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
