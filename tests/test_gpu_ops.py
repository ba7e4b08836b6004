"""GPU parity of sort / DISTINCT, union, join (hash and sort-merge, all nine
Table 3 relation types) and query plans against the CPU oracle: results must
be byte-identical."""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
from oracle import Table as OTable
from oracle_pins import GOLD, random_plan, tiny_graph
from synth import Pattern, Plan, pat

pytestmark = pytest.mark.gpu


def same(gt, ot):
    got = gt.to_numpy()
    assert gt.vars == ot.vars, (gt.vars, ot.vars)
    assert got.shape == ot.rows.shape, (got.shape, ot.rows.shape)
    assert np.array_equal(got, ot.rows)


def rand_table(rng, n, k, hi):
    rows = rng.integers(0, hi, size=(n, k), dtype=np.int64).astype(np.uint32)
    return rows


@pytest.mark.parametrize("n,k,hi", [(0, 2, 10), (1, 3, 5), (100, 1, 7), (5000, 2, 50),
                                    (70001, 3, 1000), (20000, 3, 2**32 - 1),
                                    (30000, 5, 2**31), (4097, 4, 3), (8192, 3, 2**32 - 1),
                                    (8193, 2, 100), (2, 2, 2**32 - 1), (6000, 5, 2**31)])
def test_sort_and_distinct(ctx, n, k, hi):
    rng = np.random.default_rng(n + k)
    rows = rand_table(rng, n, k, hi)
    t = ctx.table(rows, list(range(k)))
    ot = OTable(rows, list(range(k)))
    same(ctx.sort(t, False), oracle.sort_rows(ot))
    same(ctx.sort(t, True), oracle.distinct(ot))


def test_union(ctx):
    rng = np.random.default_rng(3)
    specs = [([0, 1], 300), ([1, 2], 200), ([0, 1], 0), ([3], 50), ([2, 0, 1], 1000)]
    ts, ots = [], []
    for vs, n in specs:
        rows = rand_table(rng, n, len(vs), 20)
        ts.append(ctx.table(rows, vs))
        ots.append(OTable(rows, vs))
    for r in (1, 2, 3, 5):
        for combo in itertools.combinations(range(len(specs)), r):
            for d in (False, True):
                same(ctx.union([ts[i] for i in combo], d), oracle.union([ots[i] for i in combo], d))


@pytest.mark.parametrize("algo", [1, 2])
@pytest.mark.parametrize("nl,nr,keys", [(0, 10, 5), (10, 0, 5), (1, 1, 1), (500, 700, 40),
                                        (3000, 2000, 3000), (20000, 50, 10),
                                        (50, 20000, 10), (2000, 2000, 1)])
def test_join_parity(ctx, algo, nl, nr, keys):
    rng = np.random.default_rng(nl * 7 + nr)
    L = rand_table(rng, nl, 2, keys)
    R = rand_table(rng, nr, 3, keys)
    gl, gr = ctx.table(L, [0, 1]), ctx.table(R, [2, 3, 4])
    ol, orr = OTable(L, [0, 1]), OTable(R, [2, 3, 4])
    for lc, rc in ((0, 0), (1, 2), (0, 1)):
        want = oracle.join(ol, lc, orr, rc, "sortmerge")
        same(ctx.join(gl, lc, gr, rc, algo), want)


def test_join_hot_key_count_invariant(ctx):
    rng = np.random.default_rng(11)
    L = rand_table(rng, 40000, 2, 2000)
    R = rand_table(rng, 30000, 2, 2000)
    L[rng.random(40000) < 0.1, 0] = 7   # a hub key holding ~10% of each side
    R[rng.random(30000) < 0.1, 0] = 7
    cl = np.bincount(L[:, 0], minlength=2000).astype(np.int64)
    cr = np.bincount(R[:, 0], minlength=2000).astype(np.int64)
    want_n = int((cl * cr).sum())
    for algo in (1, 2):
        j = ctx.join(ctx.table(L, [0, 1]), 0, ctx.table(R, [0, 2]), 0, algo)
        assert j.nrows == want_n
    got = ctx.join(ctx.table(L[:3000], [0, 1]), 0, ctx.table(R[:3000], [0, 2]), 0, 1)
    same(got, oracle.join(OTable(L[:3000], [0, 1]), 0, OTable(R[:3000], [0, 2]), 0, "sortmerge"))


def test_table3_relation_types_queries(ctx):
    with open(os.path.join(GOLD, "table3_reltypes.json")) as f:
        gd = json.load(f)
    g = np.concatenate([tiny_graph(11, 400, 6), tiny_graph(12, 60, 6)])
    G = ctx.load(g)
    for name, (qi, qj) in gd["types"].items():
        consts = [t for t in qi + qj if not t.startswith("?")]
        for vals in itertools.islice(itertools.product(range(1, 7), repeat=len(consts)), 0, 60, 7):
            env = dict(zip(consts, vals))

            def mk(q):
                return Pattern(*[env.get(t, 0) for t in q], *[0 if t == "?V" else -1 for t in q])
            plan = Plan().scan(mk(qi)).scan(mk(qj)).join(0)
            same(ctx.query(G, plan), oracle.query(g, plan))


def test_rule11_query(ctx):
    g = np.array([(76, 84, 56), (31, 84, 77), (56, 84, 78), (56, 84, 77), (44, 83, 2)],
                 dtype=np.uint32)
    G = ctx.load(g)
    n = {}
    plan = (Plan().scan(pat("?x 84 ?y", n)).scan(pat("?y 84 ?z", n)).join(n["?y"])
            .project([n["?x"], n["?z"]]).distinct())
    assert ctx.query(G, plan).to_numpy().tolist() == [[76, 77], [76, 78]]


def test_small_config_queries(ctx, graphs):
    g = graphs("small")
    G = ctx.load(g)
    n = {}
    q1a = Plan().scan(pat("?s 7 ?o", n))
    n = {}
    q1b = Plan().scan(pat("?s 3 ?o1", n)).scan(pat("?s 11 ?o2", n)).join(n["?s"])
    for plan in (q1a, q1b):
        same(ctx.query(G, plan), oracle.query(g, plan))
    # filter after a scan (fused into the search) and after a join (separate)
    n = {}
    p = (Plan().scan(pat("?s 3 ?o1", n)).filter(n["?o1"], 100, 3000)
         .scan(pat("?s 11 ?o2", n)).join(n["?s"]).filter(n["?o2"], 50, 9000))
    same(ctx.query(G, p), oracle.query(g, p))
    # union of 4 subqueries with DISTINCT, projected
    n = {}
    p = Plan()
    for pid in (3, 4, 5, 6):
        p.scan(pat(f"?s {pid} ?o", n))
    p.union(4, True).project([n["?o"]]).distinct()
    same(ctx.query(G, p), oracle.query(g, p))


def test_natural_join_two_shared_vars(ctx):
    g = tiny_graph(31, 3000, 5)
    G = ctx.load(g)
    n = {}
    p = Plan().scan(pat("?a ?b ?c", n)).scan(pat("?c ?b ?a", n)).join(n["?b"])
    same(ctx.query(G, p), oracle.query(g, p))


def _hub_graph(seed):
    """Predicates 1, 2, 4 on a few hub subjects of very different degrees
    (every side of a join on ?s stays within a batched small join, while the
    hub pairs give hundreds of thousands of output rows), predicate 5 and 6
    on many subjects of degree 1-3, and subjects present under one predicate
    only (rows without a match)."""
    rng = np.random.default_rng(seed)
    rows = []
    deg = {1: {101: 700, 102: 37, 103: 5, 104: 1},
           2: {101: 600, 102: 29, 105: 9, 104: 1},
           4: {101: 333, 103: 64, 102: 1},
           7: {101: 2, 102: 3}}
    for p, subj in deg.items():
        for s, d in subj.items():
            for o in rng.choice(100000, size=d, replace=False) + 1:
                rows.append((s, p, o))
    for s in range(1000, 2500):
        for p in (5, 6):
            for o in rng.choice(50, size=int(rng.integers(1, 4)), replace=False) + 1:
                rows.append((s, p, o))
    g = np.array(rows, dtype=np.uint32)
    return g[rng.permutation(len(g))]


def test_small_join_large_output(ctx):
    """Joins whose sides are small but whose output is large (hub keys) are
    expanded output-row-parallel; alone and in one batch with small-output
    joins, every result equals the oracle's."""
    g = _hub_graph(5)
    G = ctx.load(g)
    plans = []
    for a, b in ((1, 2), (1, 4), (2, 4), (5, 6), (4, 1)):
        n = {}
        plans.append(Plan().scan(pat(f"?s {a} ?x", n)).scan(pat(f"?s {b} ?y", n)).join(n["?s"]))
    n = {}  # a 3-way star: the second join's left side is the first's output
    plans.append(Plan().scan(pat("?s 1 ?x", n)).scan(pat("?s 7 ?y", n)).join(n["?s"])
                 .scan(pat("?s 2 ?z", n)).join(n["?s"]))
    want = [oracle.query(g, p) for p in plans]
    assert want[0].rows.shape[0] == 700 * 600 + 37 * 29 + 1
    for p, w in zip(plans, want):
        same(ctx.query(G, p), w)
    for t, w in zip(ctx.query_batch(G, plans), want):
        same(t, w)


def test_small_join_key_at_id_maximum(ctx):
    """The batched small join's LDS table marks empty slots with 2^32 - 1, also
    a valid ID: join keys equal to it (a hub and a single row), next to keys
    hashing anywhere, with and without a second shared variable, alone and
    batched, equal the oracle's results."""
    top = 2**32 - 1

    def fmix32(x):  # the published MurmurHash3 finaliser, which places keys in the table
        x ^= x >> 16
        x = (x * 0x85EBCA6B) & 0xFFFFFFFF
        x ^= x >> 13
        x = (x * 0xC2B2AE35) & 0xFFFFFFFF
        return x ^ (x >> 16)
    # subjects whose home slot is that of 2^32 - 1 in tables of 64-256 slots
    near = [s for s in range(20, 200000) if fmix32(s) & 255 == fmix32(top) & 255][:4]
    assert len(near) == 4
    rows = []
    for p, subj in {1: {top: 40, top - 1: 3, 5: 7, 9: 1, **{s: 2 for s in near}},
                    2: {top: 30, top - 1: 2, 9: 4, 11: 2, **{s: 1 for s in near[:3]}},
                    3: {top: 1, 5: 2}}.items():
        for s, d in subj.items():
            for o in range(d):
                rows.append((s, p, top - o if s == top else o + 1))
    g = np.array(rows, dtype=np.uint32)
    G = ctx.load(g)
    plans = []
    for a, b in ((1, 2), (2, 1), (1, 3)):
        n = {}
        plans.append(Plan().scan(pat(f"?s {a} ?x", n)).scan(pat(f"?s {b} ?y", n)).join(n["?s"]))
    n = {}  # a second shared variable: the object
    plans.append(Plan().scan(pat("?s 1 ?o", n)).scan(pat("?s 2 ?o", n)).join(n["?s"]))
    want = [oracle.query(g, p) for p in plans]
    assert want[0].rows.shape[0] == 40 * 30 + 3 * 2 + 1 * 4 + 3 * 2
    assert want[3].rows.shape[0] > 0
    for p, w in zip(plans, want):
        same(ctx.query(G, p), w)
    for t, w in zip(ctx.query_batch(G, plans), want):
        same(t, w)


def test_random_plans(ctx):
    rng = np.random.default_rng(2024)
    for i in range(150):
        g = tiny_graph(500 + i, int(rng.integers(1, 40)), 4)
        plan = random_plan(rng)
        G = ctx.load(g)
        same(ctx.query(G, plan), oracle.query(g, plan))
        G.free()


def test_query_errors(ctx, graphs):
    from paper_1807_01409_amd import TidError
    G = ctx.load(graphs("small", 1000))
    with pytest.raises(TidError) as e:
        ctx.query(G, Plan().scan(pat("?s 7 ?o")).join(5))        # one table for a JOIN
    assert e.value.status == -1
    n = {}
    with pytest.raises(TidError) as e:
        ctx.query(G, Plan().scan(pat("?a 7 ?b", n)).scan(pat("?c 8 ?d", n)).join(n["?a"]))
    assert e.value.status == -5


def test_query_batch_equals_alone(ctx, graphs):
    """Every plan inside a batch returns exactly what it returns alone, and
    what the oracle returns (small graph, mixed star/chain/union plans)."""
    g = graphs("small")
    G = ctx.load(g)
    rng = np.random.default_rng(77)
    plans = []
    for i in range(40):
        n = {}
        k = int(rng.integers(1, 5))
        preds = rng.integers(1, 51, size=k)
        p = Plan()
        if i % 3 == 0:      # star on ?s
            for j, pid in enumerate(preds):
                p.scan(pat(f"?s {pid} ?o{j}", n))
                if j:
                    p.join(n["?s"])
        elif i % 3 == 1:    # chain
            for j, pid in enumerate(preds):
                p.scan(pat(f"?x{j} {pid} ?x{j + 1}", n))
                if j:
                    p.join(n[f"?x{j}"])
        else:               # union of single patterns, DISTINCT
            for pid in preds:
                p.scan(pat(f"?s {pid} ?o", n))
            p.union(k, True)
        plans.append(p)
    batch = ctx.query_batch(G, plans)
    for p, t in zip(plans, batch):
        alone = ctx.query(G, p)
        assert np.array_equal(t.to_numpy(), alone.to_numpy())
        same(t, oracle.query(g, p))
    assert ctx.query_batch(G, []) == []


def test_union_of_scans(ctx, graphs):
    """UNIONs of scans, fusable into one scan (distinct constants in one
    position) and not (repeated constants, different variable layouts, more
    constants than a set holds, different ranges), with and without
    DISTINCT, alone and under a join: all equal the oracle."""
    g = graphs("small")
    G = ctx.load(g)
    hub = int(np.bincount(g[:, 2]).argmax())

    def union_plan(patterns, dedupe, tail=None):
        n = {}
        p = Plan()
        for text in patterns:
            p.scan(text if isinstance(text, Pattern) else pat(text, n))
        p.union(len(patterns), dedupe)
        if tail:
            tail(p, n)
        return p

    cases = [
        (["?s 3 ?o", "?s 4 ?o", "?s 5 ?o", "?s 6 ?o"], False),
        (["?s 3 ?o", "?s 4 ?o", "?s 5 ?o", "?s 6 ?o"], True),
        (["?s 3 ?o", "?s 3 ?o", "?s 5 ?o"], False),           # repeated constant: bag
        ([f"?s {q} {hub}" for q in range(1, 12)], False),       # set on the predicate, one variable
        (["?s 3 ?o", "?o 4 ?s", "?s 5 ?o"], False),           # variables move
        ([f"?s {q} ?o" for q in range(1, 19)], True),           # more than a set holds
        ([Pattern(0, 3, 0, 0, -1, 1, range_pos=2, lo=1, hi=4000),
          Pattern(0, 4, 0, 0, -1, 1, range_pos=2, lo=1, hi=4000)], False),
        ([Pattern(0, 3, 0, 0, -1, 1, range_pos=2, lo=1, hi=4000),
          Pattern(0, 4, 0, 0, -1, 1, range_pos=2, lo=1, hi=9000)], False),
    ]
    for patterns, dedupe in cases:
        plan = union_plan(patterns, dedupe)
        same(ctx.query(G, plan), oracle.query(g, plan))
    # a fused union joined with another scan on ?s
    plan = union_plan(["?s 3 ?o", "?s 4 ?o", "?s 5 ?o"], False,
                      lambda p, n: p.scan(pat("?s 7 ?x", n)).join(n["?s"]))
    same(ctx.query(G, plan), oracle.query(g, plan))
    # the same unions inside one batch
    plans = [union_plan(pp, d) for pp, d in cases[:4]]
    for t, plan in zip(ctx.query_batch(G, plans), plans):
        same(t, oracle.query(g, plan))


@pytest.mark.parametrize("semijoin_min", [0, 1 << 16])
def test_semijoin_reduced_plans(ctx, graphs, semijoin_min):
    """Star and chain plans of the batched mix with semi-join rounds (forced on
    every scan by a zero threshold, and at the default threshold) equal the
    oracle, alone and in a batch."""
    from synth.batch import PredIndex, batch_queries
    g = graphs("small")
    G = ctx.load(g)
    plans, _ = batch_queries(PredIndex(g), nq=64, seed=7, max_rows=1 << 16, workers=1)
    ctx.set_option("semijoin_min", semijoin_min)
    try:
        for p in plans:
            same(ctx.query(G, p), oracle.query(g, p))
        for t, p in zip(ctx.query_batch(G, plans), plans):
            same(t, oracle.query(g, p))
    finally:
        ctx.set_option("semijoin_min", 1 << 16)


def test_semijoin_random_plans(ctx):
    """Random plans (joins, unions, filters, projections, DISTINCT) with the
    reduction forced wherever a plan is conjunctive, and switched off: both
    equal the oracle."""
    rng = np.random.default_rng(77)
    try:
        for i in range(120):
            g = tiny_graph(900 + i, int(rng.integers(1, 40)), 4)
            plan = random_plan(rng)
            G = ctx.load(g)
            want = oracle.query(g, plan)
            ctx.set_option("semijoin_min", 0)
            same(ctx.query(G, plan), want)
            ctx.set_option("semijoin", 0)
            same(ctx.query(G, plan), want)
            ctx.set_option("semijoin", 1)
            G.free()
    finally:
        ctx.set_option("semijoin", 1)
        ctx.set_option("semijoin_min", 1 << 16)


@pytest.mark.parametrize("slice_rows", [1, 0])
def test_wide_slices(ctx, graphs, slice_rows):
    """Single-scan plans sharing predicates, run as one batch through the wide
    pass, with every shared predicate sliced (slice_rows 1) and at the default
    threshold (no predicate of this graph reaches it), and with slicing off:
    every table equals the oracle's.  The shapes cover bound subjects and
    objects, a repeated variable, ranges on each position and projections."""
    g = graphs("small")
    G = ctx.load(g)
    rng = np.random.default_rng(31)
    preds = np.argsort(-np.bincount(g[:, 1]), kind="stable")[:3]
    plans = []
    for i in range(60):
        p = int(preds[i % 3])
        rows = g[g[:, 1] == p]
        r = rows[int(rng.integers(rows.shape[0]))]
        shape = i % 6
        if shape == 0:
            q = Pattern(0, p, 0, 0, -1, 1)
        elif shape == 1:
            q = Pattern(int(r[0]), p, 0, -1, -1, 0)
        elif shape == 2:
            q = Pattern(0, p, int(r[2]), 0, -1, -1)
        elif shape == 3:
            q = Pattern(0, p, 0, 0, -1, 0)
        elif shape == 4:
            lo = int(rng.integers(1, 5000))
            q = Pattern(0, p, 0, 0, -1, 1, range_pos=int(rng.choice([0, 2])), lo=lo,
                        hi=lo + int(rng.integers(1, 8000)))
        else:
            q = Pattern(0, p, 0, -1, -1, 0, range_pos=1, lo=p, hi=p + 1 + i % 2)
        plans.append(Plan().scan(q))
    try:
        ctx.set_option("wide_min", 1)
        for mode in ((1, slice_rows), (0, 0)):
            ctx.set_option("wide_slice", mode[0])
            ctx.set_option("slice_rows", mode[1])
            for t, p in zip(ctx.query_batch(G, plans), plans):
                same(t, oracle.query(g, p))
    finally:
        ctx.set_option("wide_min", 0)
        ctx.set_option("wide_slice", 1)
        ctx.set_option("slice_rows", 0)


def test_wide_slices_semijoin_batch(ctx, graphs):
    """The batched star/chain mix with semi-join rounds forced on every scan,
    the wide pass forced on every round and every shared predicate sliced:
    equal to the oracle."""
    from synth.batch import PredIndex, batch_queries
    g = graphs("small")
    G = ctx.load(g)
    plans, _ = batch_queries(PredIndex(g), nq=96, seed=11, max_rows=1 << 16, workers=1)
    try:
        ctx.set_option("semijoin_min", 0)
        ctx.set_option("wide_min", 1)
        ctx.set_option("slice_rows", 1)
        for t, p in zip(ctx.query_batch(G, plans), plans):
            same(t, oracle.query(g, p))
    finally:
        ctx.set_option("semijoin_min", 1 << 16)
        ctx.set_option("wide_min", 0)
        ctx.set_option("slice_rows", 0)
