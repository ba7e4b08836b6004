"""Autotuner for the scan kernel's launch shape and the batch engine's choices.

tune_scan sweeps (threads per workgroup, triples per thread, prefetch, LDS
staging words) on the caller's own graph and patterns, times each shape with
HIP events on the context's stream, checks that every shape returns the same
bytes as the first (a race or ordering bug would show up as a difference),
and keeps the fastest.  tune_batch does the same for a batch of plans over
the batch options (when a scan is semi-join filtered, how many patterns make
a wide pass, whether wide passes slice shared predicates, when a semi-join is
an index lookup).  Results are
cached in a JSON file keyed by device name, operation and graph-size bucket;
TID_TUNE_CACHE names the file.
"""
from __future__ import annotations

import json
import math
import os
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

import numpy as np

SHAPES: List[Tuple[int, int]] = [(256, 16), (256, 8), (256, 32), (512, 8), (512, 16),
                                 (1024, 4), (1024, 8), (128, 16), (128, 32)]
STAGE_WORDS = [4096, 8192, 12288, 16384]
KEYS = ("scan_block", "scan_items", "scan_prefetch", "stage_words")
BATCH_GRID = {"semijoin_min": [1 << 12, 1 << 16, 1 << 20], "wide_min": [4, 8, 32],
              "wide_slice": [0, 1], "index_ratio": [1, 4, 16]}
BATCH_KEYS = tuple(BATCH_GRID)


def cache_path() -> str:
    return os.environ.get("TID_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "tripleid_tune.json"))


def _bucket(n: int) -> str:
    return f"2^{max(0, int(math.log2(max(n, 1))))}"


def _device_name() -> str:
    import torch
    return torch.cuda.get_device_name(0)


def load_cache() -> Dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(d: Dict) -> None:
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def apply(ctx, n: int, op: str = "scan") -> Optional[Dict]:
    """Set the cached best options for a graph of n triples, if any."""
    entry = load_cache().get(_device_name(), {}).get(op, {}).get(_bucket(n))
    if entry:
        for k in (BATCH_KEYS if op == "batch" else KEYS):
            if k in entry["options"]:
                ctx.set_option(k, entry["options"][k])
    return entry


def _time(ctx, G, patterns, reps: int) -> float:
    import torch
    keep = []
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(ctx.stream)
    for _ in range(reps):
        for p in patterns:
            keep.append(ctx.scan(G, p))
    e1.record(ctx.stream)
    e1.synchronize()
    for t in keep:
        t.free()
    return e0.elapsed_time(e1) / 1e3 / reps


def tune_scan(ctx, G, patterns: Sequence, reps: int = 10,
              shapes: Iterable[Tuple[int, int]] = SHAPES,
              stage_words: Iterable[int] = STAGE_WORDS,
              prefetch: Iterable[int] = (0, 1), store: bool = True) -> Dict:
    """Sweep launch shapes for these scans; returns {"options", "seconds", "table"}."""
    saved = {k: ctx.get_option(k) for k in KEYS}
    ref = [ctx.scan(G, p).to_numpy() for p in patterns]
    table = []
    try:
        for (b, i) in shapes:
            for pf in prefetch:
                for sw in stage_words:
                    opts = {"scan_block": b, "scan_items": i, "scan_prefetch": pf,
                            "stage_words": sw}
                    for k, v in opts.items():
                        ctx.set_option(k, v)
                    for p, want in zip(patterns, ref):
                        got = ctx.scan(G, p).to_numpy()
                        if not np.array_equal(got, want):
                            raise AssertionError(f"shape {opts} changed a scan result")
                    _time(ctx, G, patterns, 2)
                    table.append((_time(ctx, G, patterns, reps), opts))
    finally:
        for k, v in saved.items():
            ctx.set_option(k, v)
    table.sort(key=lambda x: x[0])
    best_s, best = table[0]
    res = {"options": best, "seconds": best_s,
           "table": [{"seconds": s, **o} for s, o in table]}
    if store:
        d = load_cache()
        d.setdefault(_device_name(), {}).setdefault("scan", {})[_bucket(G.n)] = {
            "options": best, "seconds": best_s}
        save_cache(d)
    return res


def _batch_results(ctx, G, plans, full: bool):
    """Row counts of every result, and the rows themselves where `full` (a
    bool per plan)."""
    tabs = ctx.query_batch(G, plans)
    out = []
    for t, f in zip(tabs, full):
        out.append(t.to_numpy() if f else t.nrows)
        t.free()
    return out


def tune_batch(ctx, G, plans: Sequence, reps: int = 2,
               grid: Optional[Dict[str, Sequence[int]]] = None, store: bool = True,
               full_rows: int = 1 << 26) -> Dict:
    """Sweep the batch options in `grid` (default BATCH_GRID) for this batch of
    plans; returns {"options", "seconds", "table"}.  Every option set must give
    the same results as the first: all of them byte for byte while the first
    set's results hold at most `full_rows` rows in all, else every result's
    row count and every eighth result byte for byte."""
    import itertools
    import time
    grid = dict(BATCH_GRID if grid is None else grid)
    keys = list(grid)
    saved = {k: ctx.get_option(k) for k in keys}
    table = []
    try:
        first = ctx.query_batch(G, plans)
        counts = [t.nrows for t in first]
        for t in first:
            t.free()
        every = sum(counts) <= full_rows
        full = [every or i % 8 == 0 for i in range(len(plans))]
        ref = None
        for values in itertools.product(*(grid[k] for k in keys)):
            opts = dict(zip(keys, values))
            for k, v in opts.items():
                ctx.set_option(k, v)
            got = _batch_results(ctx, G, plans, full)
            if ref is None:
                ref = got
            else:
                for i, (a, b) in enumerate(zip(ref, got)):
                    same = np.array_equal(a, b) if full[i] else a == b
                    if not same:
                        raise AssertionError(f"options {opts} changed the result of plan {i}")
            best = None
            for _ in range(reps):
                ctx.synchronize()
                t0 = time.perf_counter()
                tabs = ctx.query_batch(G, plans)
                ctx.synchronize()
                dt = time.perf_counter() - t0
                for t in tabs:
                    t.free()
                best = dt if best is None else min(best, dt)
            table.append((best, opts))
    finally:
        for k, v in saved.items():
            ctx.set_option(k, v)
    table.sort(key=lambda x: x[0])
    best_s, best = table[0]
    res = {"options": best, "seconds": best_s,
           "table": [{"seconds": s, **o} for s, o in table]}
    if store:
        d = load_cache()
        d.setdefault(_device_name(), {}).setdefault("batch", {})[_bucket(G.n)] = {
            "options": best, "seconds": best_s}
        save_cache(d)
    return res
