"""The predicate-partitioned layout (the paper's ID assignment for pruning a
search, Sec. 4.3): with the partitioned copy built, scans, multi-pattern
passes and plans whose patterns have constant predicates read only their
predicates' slices, and every result is byte-identical to the oracle's and to
the same call on the TripleID array alone."""
import numpy as np
import pytest

import oracle
from synth import Pattern, Plan, pat

pytestmark = pytest.mark.gpu


def rows(t):
    return t.to_numpy()


PATTERNS = [Pattern(0, 7, 0, 0, -1, 1), Pattern(0, 1, 0, 0, -1, 1), Pattern(0, 50, 0, 0, -1, 1),
            Pattern(0, 51, 0, 0, -1, 1), Pattern(0, 3, 0, 0, -1, 0), Pattern(17, 3, 0, -1, -1, 0),
            Pattern(0, 9, 0, -1, -1, 0, range_pos=2, lo=100, hi=900),
            Pattern(0, 2, 0, 0, -1, -1), Pattern(0, 4, 0, -1, -1, -1)]


@pytest.mark.parametrize("name,n", [("small", 100_000), ("medium", 3_000_001)])
def test_partitioned_scans(ctx, graphs, name, n):
    g = graphs(name, n)
    G = ctx.load(g)
    aos = [rows(ctx.scan(G, p)) for p in PATTERNS]
    G.partition(True)
    for p, a in zip(PATTERNS, aos):
        t = ctx.scan(G, p)
        o = oracle.scan(g, p)
        assert t.vars == o.vars
        assert np.array_equal(rows(t), o.rows), p
        assert np.array_equal(rows(t), a), p
    # multi-pattern passes and plans with constant predicates
    outs = ctx.scan_multi(G, PATTERNS[:4])
    for p, t in zip(PATTERNS[:4], outs):
        assert np.array_equal(rows(t), oracle.scan(g, p).rows)
    n_ = {}
    plan = Plan().scan(pat("?s 3 ?a", n_)).scan(pat("?s 11 ?b", n_)).join(n_["?s"])
    assert np.array_equal(rows(ctx.query(G, plan)), oracle.query(g, plan).rows)
    # a free predicate still reads the array
    p = Pattern(0, 0, 5, 0, 1, -1)
    assert np.array_equal(rows(ctx.scan(G, p)), oracle.scan(g, p).rows)
    ctx.set_option("layout", 0)
    try:
        for p, a in zip(PATTERNS, aos):
            assert np.array_equal(rows(ctx.scan(G, p)), a)
    finally:
        ctx.set_option("layout", 1)
    G.partition(False)
    G.free()


def _slice_patterns(g):
    """Constant-predicate patterns of every kind over the small graph's
    predicates, plus predicates without triples (one of them the largest
    bucketable id) and one id past the bucket table."""
    hot_o = int(np.bincount(g[:, 2]).argmax())
    s0 = int(g[0, 0])
    out = []
    for p in list(range(1, 51)) + [60, 4095, 4096]:
        out += [Pattern(0, p, 0, 0, -1, 1),                 # whole slice (s, o)
                Pattern(0, p, 0, -1, -1, 0),                # whole slice, o only
                Pattern(0, p, 0, -1, -1, -1),               # whole slice, count only
                Pattern(0, p, 0, 0, -1, 0),                 # s == o
                Pattern(0, p, hot_o, 0, -1, -1),            # constant object
                Pattern(s0, p, 0, -1, -1, 0),               # constant subject
                Pattern(0, p, 0, 0, -1, 1, range_pos=2, lo=5, hi=400)]
    return out


@pytest.mark.parametrize("semijoin", [1, 0])
def test_segment_passes_and_whole_slices(ctx, graphs, semijoin):
    """A batch of single-scan plans on a partitioned graph: whole-slice
    patterns become tables over the slices (no pass), the other constant-
    predicate patterns go through one segment pass over their predicates'
    slices, an id past the bucket table through a graph pass.  Every result
    equals the oracle's and the same batch on the TripleID array alone."""
    g = graphs("small", 100_000)
    pats = _slice_patterns(g)
    plans = [Plan().scan(p) for p in pats]
    want = [oracle.query(g, pl).rows for pl in plans]
    G = ctx.load(g)
    ctx.set_option("semijoin", semijoin)
    try:
        aos = [t.to_numpy() for t in ctx.query_batch(G, plans)]
        G.partition(True)
        got = [t.to_numpy() for t in ctx.query_batch(G, plans)]
        for p, a, b, w in zip(pats, aos, got, want):
            assert np.array_equal(a, w), p
            assert np.array_equal(b, w), p
        # joins over whole-slice tables and segment-pass tables
        n_ = {}
        plan = (Plan().scan(pat("?s 3 ?a", n_)).scan(pat("?s 11 ?b", n_)).join(n_["?s"])
                .scan(pat(f"?b 7 {int(g[5, 2])}", n_)).join(n_["?b"]))
        assert np.array_equal(ctx.query(G, plan).to_numpy(), oracle.query(g, plan).rows)
    finally:
        ctx.set_option("semijoin", 1)
        G.free()
