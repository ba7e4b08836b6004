"""Batched and served queries: every result inside a batch or a served mix
equals the same query run alone (byte for byte), and the oracle's."""
import numpy as np
import pytest

import oracle
from oracle_threads import oracle_queries
from synth.batch import PredIndex, batch_queries, poisson_arrivals

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mix(graphs):
    g = graphs("medium", 2_000_000)
    plans, infos = batch_queries(PredIndex(g), nq=96, seed=4, max_rows=1 << 16)
    return g, plans, infos


@pytest.fixture(scope="module")
def mix_oracle(mix):
    g, plans, _ = mix
    return [o.rows for o in oracle_queries(g, plans)]


def test_batch_mix_equals_alone_and_oracle(ctx, mix, mix_oracle):
    g, plans, infos = mix
    G = ctx.load(g)
    batch = ctx.query_batch(G, plans)
    for p, t, info in zip(plans, batch, infos):
        alone = ctx.query(G, p).to_numpy()
        got = t.to_numpy()
        assert np.array_equal(got, alone)
        assert got.shape[0] == info["rows"]          # exact count from the generator
    assert sum(1 for i in infos if i["rows"] > 0) >= len(infos) // 2
    for t, o in zip(batch, mix_oracle):
        assert np.array_equal(t.to_numpy(), o)


@pytest.mark.parametrize("semijoin", [1, 0])
def test_batch_mix_partitioned_equals_oracle(ctx, mix, mix_oracle, semijoin):
    """With the predicate-partitioned layout built, the mix's patterns read
    only their slices (whole-slice patterns read nothing, the others go
    through segment passes); every batched and alone result equals the
    oracle's."""
    g, plans, _ = mix
    G = ctx.load(g)
    G.partition(True)
    ctx.set_option("semijoin", semijoin)
    try:
        for t, o in zip(ctx.query_batch(G, plans), mix_oracle):
            assert np.array_equal(t.to_numpy(), o)
        for p, o in zip(plans[:24], mix_oracle[:24]):
            assert np.array_equal(ctx.query(G, p).to_numpy(), o)
    finally:
        ctx.set_option("semijoin", 1)
        G.free()


@pytest.mark.parametrize("budget", [64 << 30, 8 << 20])
def test_served_mix_equals_alone_and_oracle(ctx, mix, mix_oracle, budget):
    from paper_1807_01409_amd.serve import Request, Server
    g, plans, infos = mix
    arrivals = poisson_arrivals(240, qps=4000.0, seed=11)
    reqs = [Request(i, plans[i % len(plans)], float(arrivals[i])) for i in range(240)]
    srv = Server(g, workers=3, budget_bytes=budget, max_batch=48, layout=budget > (1 << 30))
    try:
        stats = srv.run(reqs, keep_results=True)
    finally:
        srv.close()
    assert stats.completed == len(reqs)
    G = ctx.load(g)
    alone = {}
    for r in reqs:
        key = r.rid % len(plans)
        if key not in alone:
            alone[key] = ctx.query(G, r.plan).to_numpy()
        assert np.array_equal(r.result, alone[key]), r.rid
        assert np.array_equal(r.result, mix_oracle[key]), r.rid
    assert stats.p99_ms >= stats.p50_ms > 0


def test_served_group_failure_is_contained(ctx, mix):
    """A group whose batch call fails (forced here from the host: every scan
    output capped at one row with retries off, so scans with more rows fail
    with TID_E_CAPACITY) is retried request by request; requests that still
    fail are reported, the others served, and the server does not abort."""
    from paper_1807_01409_amd.serve import Request, Server
    g, plans, infos = mix
    reqs = [Request(i, plans[i % len(plans)], 0.0) for i in range(40)]
    srv = Server(g, workers=2, budget_bytes=64 << 30, max_batch=16)
    try:
        for c in srv.ctxs:
            c.set_option("capacity_override", 1)
            c.set_option("retry", 0)
        stats = srv.run(reqs, keep_results=True)
    finally:
        srv.close()
    failed = [r for r in reqs if r.error]
    assert stats.failed == len(failed) > 0
    assert all("CAPACITY" in r.error for r in failed)
    for r in reqs:
        if not r.error:
            assert r.result.shape[0] <= 1


@pytest.mark.parametrize("chunks,slots", [(1, 8), (3, 16), (7, 40)])
def test_circular_served_mix_equals_oracle(ctx, mix, mix_oracle, chunks, slots):
    """The circular chunked shared scan (tid_serve_*): queries admitted at
    different chunks of the revolution, results equal the oracle's and
    tid_query's, whatever the chunk and slot counts."""
    from paper_1807_01409_amd.serve import CircularServer, Request
    g, plans, infos = mix
    arrivals = poisson_arrivals(150, qps=3000.0, seed=13)
    reqs = [Request(i, plans[(7 * i) % len(plans)], float(arrivals[i])) for i in range(150)]
    srv = CircularServer(g, chunks=chunks, slots=slots)
    try:
        stats = srv.run(reqs, keep_results=True)
    finally:
        srv.close()
    assert stats.completed == len(reqs) and stats.failed == 0
    for r in reqs:
        assert np.array_equal(r.result, mix_oracle[(7 * r.rid) % len(plans)]), r.rid


def test_circular_tickets_and_errors(ctx, graphs):
    """A ticket's result is taken once; a bad plan is refused at submit; the
    info call tracks waiting and admitted queries."""
    import ctypes
    from paper_1807_01409_amd.serve import CircularServer
    from paper_1807_01409_amd import TidError
    from synth import Plan, pat
    g = graphs("small")
    srv = CircularServer(g, chunks=4, slots=4)
    try:
        n = {}
        plan = Plan().scan(pat("?s 3 ?a", n)).scan(pat("?s 11 ?b", n)).join(n["?s"])
        tickets = [srv._submit(plan) for _ in range(6)]
        w, a, k = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        srv.ctx._lib.tid_serve_info(srv._s, ctypes.byref(w), ctypes.byref(a), ctypes.byref(k))
        assert (w.value, a.value) == (6, 0)
        done = []
        while len(done) < 6:
            done += srv._step()
        assert sorted(done) == sorted(tickets)
        want = oracle.query(g, plan).rows
        for tk in tickets:
            assert np.array_equal(srv._result(tk).to_numpy(), want)
        with pytest.raises(TidError):
            srv._result(tickets[0])
        bad = Plan()
        bad.ops = [99]
        with pytest.raises(TidError):
            srv._submit(bad)
    finally:
        srv.close()


def test_batch_autotuner_keeps_results(ctx, mix, mix_oracle, tmp_path, monkeypatch):
    """The batch autotuner sweeps the batch options, checks every option set
    against the first (byte for byte here), caches the fastest, and the
    cached choice applied to a context still gives the oracle's results."""
    from paper_1807_01409_amd import autotune
    monkeypatch.setenv("TID_TUNE_CACHE", str(tmp_path / "tune.json"))
    g, plans, _ = mix
    grid = {"semijoin_min": [1 << 12, 1 << 16], "wide_min": [4, 32], "wide_slice": [0, 1]}
    G = ctx.load(g)
    G.partition(True)
    defaults = {k: ctx.get_option(k) for k in grid}
    try:
        res = autotune.tune_batch(ctx, G, plans, reps=1, grid=grid)
        assert len(res["table"]) == 8
        assert all(res["options"][k] in v for k, v in grid.items())
        assert {k: ctx.get_option(k) for k in grid} == defaults   # restored
        entry = autotune.apply(ctx, G.n, "batch")
        assert entry["options"] == res["options"]
        assert all(ctx.get_option(k) == v for k, v in res["options"].items())
        for t, o in zip(ctx.query_batch(G, plans), mix_oracle):
            assert np.array_equal(t.to_numpy(), o)
    finally:
        for k, v in defaults.items():
            ctx.set_option(k, v)
        G.free()
