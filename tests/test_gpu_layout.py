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


def _join_rows(a_keys, b_keys):
    va, ca = np.unique(a_keys, return_counts=True)
    vb, cb = np.unique(b_keys, return_counts=True)
    _, ia, ib = np.intersect1d(va, vb, return_indices=True)
    return int((ca[ia].astype(np.int64) * cb[ib]).sum())


def _object_for(g, p, join_keys, lo=100, hi=300_000, first_rank=10):
    """An object O of predicate p such that the pattern (?x p O) joined on its
    subject with `join_keys` (the other pattern's values of the shared
    variable) gives between lo and hi rows: a small semi-join source whose
    plan the oracle runs in seconds."""
    sel = g[:, 1] == p
    objs, cnt = np.unique(g[sel, 2], return_counts=True)
    for ob in objs[np.argsort(-cnt, kind="stable")][first_rank:400]:
        src = g[sel & (g[:, 2] == ob), 0]
        rows = _join_rows(join_keys, src)
        if lo <= rows <= hi:
            return int(ob)
    raise AssertionError(f"no object of predicate {p} gives a join of {lo}..{hi} rows")


def _star3_object(g, pa, pb, pc, hi=200_000):
    """An object O of pb such that the star (?s pa ?x) . (?s pb O) . (?s pc ?z)
    has between 100 and hi rows."""
    s, p, o = g[:, 0], g[:, 1], g[:, 2]

    def counts(mask):
        v, c = np.unique(s[mask], return_counts=True)
        return dict(zip(v.tolist(), c.tolist()))
    A, C = counts(p == pa), counts(p == pc)
    sel = p == pb
    objs, cnt = np.unique(o[sel], return_counts=True)
    for ob in objs[np.argsort(-cnt, kind="stable")][20:600]:
        rows = sum(A.get(k, 0) * b * C.get(k, 0) for k, b in counts(sel & (o == ob)).items())
        if 100 <= rows <= hi:
            return int(ob)
    raise AssertionError("no object gives a small enough star")


@pytest.mark.parametrize("index", [1, 0])
def test_semijoin_by_index(ctx, graphs, index):
    """Scans filtered by a small semi-join source on a partitioned graph look
    the source's values up in the (predicate, subject) or (predicate, object)
    order (index_semijoin = 1; rows then come grouped by value) instead of
    testing every row of the predicate (index_semijoin = 0): stars, a chain
    filtered forward on subjects and one filtered backward on objects,
    sources with repeated values and an empty source.  Every plan equals the
    oracle in both modes, batched and alone."""
    g = graphs("medium", 3_000_001)
    s, p, o = g[:, 0], g[:, 1], g[:, 2]
    o5 = _object_for(g, 5, s[p == 1])
    o30 = _object_for(g, 30, o[p == 1], lo=1, first_rank=0)
    o12 = _star3_object(g, 40, 12, 60)
    plans = []
    n_ = {}
    plans.append(Plan().scan(pat("?s 1 ?a", n_)).scan(pat(f"?s 5 {o5}", n_)).join(n_["?s"]))
    n_ = {}
    plans.append(Plan().scan(pat("?a 40 ?b", n_)).scan(pat("?b 2 ?c", n_)).join(n_["?b"]))
    n_ = {}
    plans.append(Plan().scan(pat("?a 1 ?b", n_)).scan(pat(f"?b 30 {o30}", n_)).join(n_["?b"]))
    n_ = {}
    plans.append(Plan().scan(pat("?s 40 ?x", n_)).scan(pat(f"?s 12 {o12}", n_)).join(n_["?s"])
                 .scan(pat("?s 60 ?z", n_)).join(n_["?s"]))
    n_ = {}
    plans.append(Plan().scan(pat("?s 2 ?x", n_)).scan(pat("?s 2000 ?y", n_)).join(n_["?s"]))
    n_ = {}
    plans.append(Plan().scan(pat("?s 1 ?", n_)).scan(pat(f"?s 5 {o5}", n_)).join(n_["?s"]))
    want = [oracle.query(g, pl).rows for pl in plans]
    assert sum(1 for w in want if w.shape[0] > 0) >= 4
    G = ctx.load(g)
    G.partition(True)
    ctx.set_option("index_semijoin", index)
    try:
        for pl, t, w in zip(plans, ctx.query_batch(G, plans), want):
            assert np.array_equal(t.to_numpy(), w), pl
            assert np.array_equal(ctx.query(G, pl).to_numpy(), w), pl
    finally:
        ctx.set_option("index_semijoin", 1)
        G.free()
