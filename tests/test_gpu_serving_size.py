"""The serving configuration's full size (1B triples, 12 GB resident): a scan
byte for byte against the oracle, and a batch of plans, each of which must
equal the same plan run alone and the oracle's result."""
import sys
import time

import numpy as np
import pytest

import oracle
from oracle_threads import oracle_queries
from synth import Pattern, Plan, pat

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def note(msg):
    print(f"[serving-size] {time.strftime('%H:%M:%S')} {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def serving(ctx, graphs):
    g = graphs("serving")   # drawn before the GPU was initialised (conftest)
    note("loading")
    G = ctx.load(g)
    note("resident")
    yield ctx, g, G
    G.free()


@pytest.mark.timeout(900)
def test_serving_size_scan(serving):
    from synth.queries import predicate_for_selectivity
    ctx, g, G = serving
    p = Pattern(0, predicate_for_selectivity(g, 1e-2)[0], 0, 0, -1, 1)
    note("oracle scan")
    want = oracle.scan(g, p)
    note("device scan")
    assert np.array_equal(ctx.scan(G, p).to_numpy(), want.rows)


@pytest.mark.timeout(900)
def test_serving_size_batch_equals_alone(serving):
    ctx, g, G = serving
    order = np.argsort(-np.bincount(g[:, 1]), kind="stable")
    nsub = int(g[:, 0].max()) + 1
    plans = []
    for r in (5, 50, 300):
        pid = int(order[r - 1])
        note(f"plans for predicate rank {r}")
        rows = g[:, 1] == pid
        # the object closest to 1000 rows of this predicate (subjects are
        # Zipf-distributed: a star join on ?s of the most frequent object with
        # a frequent predicate reaches 1e11 rows at this size)
        oc = np.bincount(g[rows, 2])
        obj = int(np.argmin(np.abs(np.log(np.maximum(oc, 1e-9)) - np.log(1000.0))))
        left = np.bincount(g[rows & (g[:, 2] == obj), 0], minlength=nsub).astype(np.float64)
        # rows of the star join on ?s with each predicate, all in one pass:
        # every triple weighs its subject's left count; the first rarer
        # predicate whose join has 1 .. 2^24 rows is taken
        joined = np.bincount(g[:, 1], weights=left[g[:, 0]])
        q = next(int(q) for q in order[r:] if 0 < joined[q] < 1 << 24)
        note(f"  join with predicate {q}: {int(joined[q])} rows")
        n = {}
        plans.append(Plan().scan(pat(f"?s {pid} ?o", n)))
        n = {}
        plans.append(Plan().scan(pat(f"?s {pid} {obj}", n))
                     .scan(pat(f"?s {q} ?x", n)).join(n["?s"]))
    note("alone")
    alone = [ctx.query(G, q).to_numpy() for q in plans]
    note("batch")
    batch = [t.to_numpy() for t in ctx.query_batch(G, plans)]
    for t, a in zip(batch, alone):
        assert np.array_equal(t, a)
    note("oracle (one host thread per plan)")
    for t, o in zip(batch, oracle_queries(g, plans)):
        assert np.array_equal(t, o.rows)
