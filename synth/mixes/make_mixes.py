"""Draw the query mixes of the batched and serving workloads once and store
them as plain data (JSON), so that a benchmark run loads 1024 plans instead
of drawing them (minutes on the 200M and 1B graphs).

Each file holds the generator's parameters, the graph it was drawn on (name,
triple count, seed), and per query the plan and its draw record (shape,
pattern count, target selectivities, exact row count from the count DP).
The graphs and mixes are functions of their seeds only, so a file drawn on
one machine is the mix any machine draws.

    python -m synth.mixes.make_mixes batched serving
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))

MIXES = {
    # workload: (graph config, queries, selectivity range, max prefix rows, empty redraws)
    "batched": ("batched", 1024, (1e-6, 1e-1), 1 << 22, 16),
    "serving": ("serving", 1024, (1e-6, 1e-1), 1 << 22, 16),
}


def path_of(name: str) -> str:
    return os.path.join(HERE, f"{name}_mix.json")


def make(name: str) -> dict:
    from synth import CONFIGS, make_graph
    from synth.batch import PredIndex, batch_queries
    cfg, nq, sig, max_rows, redraws = MIXES[name]
    spec = CONFIGS[cfg]
    t0 = time.time()
    g = make_graph(spec)
    print(f"[mix] {name}: graph {spec.n} in {time.time() - t0:.0f}s", flush=True)
    idx = PredIndex(g)
    del g
    plans, infos = batch_queries(idx, nq=nq, seed=spec.seed, max_rows=max_rows,
                                 sigma_range=sig, empty_redraws=redraws)
    print(f"[mix] {name}: {nq} queries in {time.time() - t0:.0f}s", flush=True)
    return {"graph": spec.as_dict(), "queries": nq, "sigma_range": list(sig),
            "max_rows": max_rows, "empty_redraws": redraws, "seed": spec.seed,
            "plans": [p.to_dict() for p in plans], "infos": infos}


def load(name: str):
    """(plans, infos, header) of a stored mix."""
    from synth.plan import Plan
    with open(path_of(name)) as f:
        d = json.load(f)
    plans = [Plan.from_dict(p) for p in d["plans"]]
    return plans, d["infos"], {k: v for k, v in d.items() if k not in ("plans", "infos")}


if __name__ == "__main__":
    for name in sys.argv[1:] or list(MIXES):
        d = make(name)
        with open(path_of(name), "w") as f:
            json.dump(d, f, separators=(",", ":"))
        print(f"[mix] wrote {path_of(name)}", flush=True)
