"""Outer joins (Sec. 4.2: the Left, Right and Outer kinds besides Inner) and
OPTIONAL in plans, byte for byte against the oracle's nested-loop outer
joins: every kind, both join algorithms, empty sides, hub keys, keys on one
side only; OPTIONAL alone, under a batch, and refused when the two sides share
a second variable."""
import numpy as np
import pytest

import oracle
from synth import Pattern, Plan, pat

pytestmark = pytest.mark.gpu

KINDS = ["inner", "left", "right", "full"]


def same(gt, ot):
    got = gt.to_numpy()
    assert gt.vars == ot.vars, (gt.vars, ot.vars)
    assert got.shape == ot.rows.shape, (got.shape, ot.rows.shape)
    assert np.array_equal(got, ot.rows)


@pytest.mark.parametrize("algo", [1, 2])
@pytest.mark.parametrize("nl,nr,keys", [(0, 50, 10), (50, 0, 10), (1000, 800, 300),
                                        (5000, 3000, 40), (20000, 9000, 20000)])
def test_outer_join_parity(ctx, algo, nl, nr, keys):
    rng = np.random.default_rng(nl * 7 + nr)
    L = np.stack([rng.integers(1, keys + 1, nl), rng.integers(1, 1 << 30, nl)], 1).astype(np.uint32)
    R = np.stack([rng.integers(keys // 2 + 1, keys + keys // 2 + 2, nr),
                  rng.integers(1, 99, nr), rng.integers(1, 5, nr)], 1).astype(np.uint32)
    TL, TR = ctx.table(L, [0, 1]), ctx.table(R, [0, 2, 3])
    OL, OR = oracle.Table(L, [0, 1]), oracle.Table(R, [0, 2, 3])
    for kind in KINDS:
        same(ctx.join_outer(TL, 0, TR, 0, kind, algo), oracle.join_outer(OL, 0, OR, 0, kind))
    # a different column pair (R's third column against L's first)
    for kind in KINDS:
        same(ctx.join_outer(TL, 0, TR, 2, kind, algo), oracle.join_outer(OL, 0, OR, 2, kind))


def test_outer_join_hub_and_sizes(ctx):
    """A hub key on both sides and a key present only on the left: the left
    join's size is the sum over L rows of max(matches, 1)."""
    L = np.array([[1, 10]] * 300 + [[2, 20]] * 5 + [[3, 30]], dtype=np.uint32)
    R = np.array([[1, 7]] * 200 + [[4, 8]] * 3, dtype=np.uint32)
    TL, TR = ctx.table(L, [0, 1]), ctx.table(R, [0, 2])
    for algo in (1, 2):
        t = ctx.join_outer(TL, 0, TR, 0, "left", algo)
        assert t.nrows == 300 * 200 + 5 + 1
        same(t, oracle.join_outer(oracle.Table(L, [0, 1]), 0, oracle.Table(R, [0, 2]), 0, "left"))
        f = ctx.join_outer(TL, 0, TR, 0, "full", algo)
        assert f.nrows == 300 * 200 + 6 + 3


def test_optional_plans(ctx, graphs):
    g = graphs("small")
    G = ctx.load(g)
    plans = []
    for p1, p2 in ((3, 11), (7, 7), (1, 49)):
        n = {}
        plans.append(Plan().scan(pat(f"?s {p1} ?a", n)).scan(pat(f"?s {p2} ?b", n))
                     .optional(n["?s"]))
        n = {}
        plans.append(Plan().scan(pat(f"?s {p1} ?a", n)).scan(pat(f"?a {p2} ?b", n))
                     .optional(n["?a"]).project([n["?s"], n["?b"]]).distinct())
        n = {}   # an inner join first, then OPTIONAL on the result
        plans.append(Plan().scan(pat(f"?s {p1} ?a", n)).scan(pat(f"?s {p2} ?b", n))
                     .join(n["?s"]).scan(pat(f"?b 5 ?c", n)).optional(n["?b"]))
    for plan in plans:
        same(ctx.query(G, plan), oracle.query(g, plan))
    for plan, t in zip(plans, ctx.query_batch(G, plans)):
        same(t, oracle.query(g, plan))
    from paper_1807_01409_amd import TidError
    m = {}
    bad = Plan().scan(pat("?s 1 ?a", m)).scan(pat("?s 2 ?a", m)).optional(m["?s"])
    with pytest.raises(TidError) as ei:
        ctx.query(G, bad)
    assert ei.value.status == -4
