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
