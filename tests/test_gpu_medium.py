"""Full-size parity on the 50M-triple medium graph, in the launch shapes the
benchmark times: every operator of the benchmark step against the oracle,
byte for byte, plus the star's cardinality against an independent count."""
import numpy as np
import pytest

import oracle
from synth import Pattern
from synth.queries import predicate_for_selectivity, range_pattern, star_query, union_query

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def same(gt, ot):
    got = gt.to_numpy()
    assert gt.vars == ot.vars
    assert got.shape == ot.rows.shape, (got.shape, ot.rows.shape)
    assert np.array_equal(got, ot.rows)


@pytest.fixture(scope="module")
def medium(ctx, graphs):
    g = graphs("medium")
    return g, ctx.load(g)


def test_medium_scans(ctx, medium):
    g, G = medium
    for sigma in (1e-3, 1e-2, 1e-1):
        p_id, _ = predicate_for_selectivity(g, sigma)
        p = Pattern(0, p_id, 0, 0, -1, 1)
        same(ctx.scan(G, p), oracle.scan(g, p))


def test_medium_range_filter(ctx, medium):
    g, G = medium
    p, info = range_pattern(g)
    t = ctx.scan(G, p)
    share = t.nrows / g.shape[0]
    assert 0.045 <= share <= 0.055
    same(t, oracle.scan(g, p))


def test_medium_star(ctx, medium):
    g, G = medium
    plan, info = star_query(g)
    t = ctx.query(G, plan)
    assert t.nrows == info["est_rows"]          # sum over s of the product of counts
    assert 1e5 <= t.nrows <= 1e7
    same(t, oracle.query(g, plan))


def test_medium_union(ctx, medium):
    g, G = medium
    plan, info = union_query(g)
    t = ctx.query(G, plan)
    o = oracle.query(g, plan)
    same(t, o)
    # set identity: distinct (s, o) pairs over the eight predicates
    sel = np.isin(g[:, 1], info["predicates"])
    so = g[sel]
    packed = (so[:, 0].astype(np.uint64) << np.uint64(32)) | so[:, 2].astype(np.uint64)
    assert t.nrows == np.unique(packed).size
