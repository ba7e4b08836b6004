"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each check raises AssertionError on failure.  They are collected as tests in
test_oracle_pins.py and re-run against deliberately broken copies of the
oracle in test_oracle_mutants.py, to show that a plausible slip anywhere in
the oracle (a dropped term, a wrong index, a flipped comparison, a transposed
operand) trips at least one of them.
"""
from __future__ import annotations

import itertools
import json
import os

import numpy as np

from bruteforce import bf_filter, bf_join, bf_query, bf_scan, bf_union
from synth import Pattern, Plan, pat

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _rows(t):
    return [tuple(int(x) for x in r) for r in t.rows]


def tiny_graph(seed: int, n: int = 12, ids: int = 4) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.integers(1, ids + 1, size=(n, 3)).astype(np.uint32)


# ---------------------------------------------------------------------------
# values the paper prints
# ---------------------------------------------------------------------------

def check_rule11(O):
    """Sec. 5.7, Rule 11 worked example: both positionArrays, both hash
    tables, and the combined (x, z) result."""
    gd = _gold("rule11_example.json")
    g = np.array(gd["data"], dtype=np.uint32)
    k1 = gd["step1_key"]
    f1 = O.scan_flags(g, Pattern(k1[0], k1[1], k1[2]))
    assert f1.tolist() == gd["step1_positionArray"], f1
    # hashTable1: object -> subjects of the step-1 matches
    t1 = O.scan(g, pat("?x 84 ?y"))
    ht1 = {}
    for x, y in _rows(t1):
        ht1.setdefault(str(y), []).append(x)
    assert {k: sorted(v) for k, v in ht1.items()} == \
        {k: sorted(v) for k, v in gd["step1_hashTable1_object_to_subjects"].items()}
    # step 2 searches the distinct step-1 objects as keys (keysArray)
    keys = sorted({y for _, y in _rows(t1)})
    assert [[k, 84, 0] for k in keys] == gd["step2_keysArray"]
    member = O.scan_multi(g, [Pattern(k, 84, 0) for k in keys])
    f2 = (member != 0).astype(int).tolist()
    assert f2 == gd["step2_positionArray"], f2
    ht2 = {}
    for i in np.nonzero(member)[0]:
        ht2.setdefault(str(int(g[i, 0])), []).append(int(g[i, 2]))
    assert {k: sorted(v) for k, v in ht2.items()} == \
        {k: sorted(v) for k, v in gd["step2_hashTable2_subject_to_objects"].items()}
    want = sorted(tuple(r) for r in gd["result_x_z"])
    n = {}
    plan = (Plan().scan(pat("?x 84 ?y", n)).scan(pat("?y 84 ?z", n)).join(n["?y"])
            .project([n["?x"], n["?z"]]).distinct())
    res = O.query(g, plan)
    assert _rows(res) == want, _rows(res)
    # the same result through the raw join (OS relation: object of q0 with subject of q1)
    for method in ("nested", "sortmerge"):
        j = O.join(O.scan(g, pat("?x 84 ?y")), 1, O.scan(g, pat("?y 84 ?z")), 0, method)
        assert sorted({(r[0], r[2]) for r in _rows(j)}) == want


def check_toy_sec3(O):
    """Sec. 3 walk-through: 'ABCPress publishes ?' becomes key (1,2,?) and
    finds TripleID (1,2,1)."""
    gd = _gold("toy_sec3.json")
    g, dicts = O.encode_graph(gd["triples"], shared=False)
    key = [dicts[i][t] if t != "?" else 0 for i, t in enumerate(gd["query_terms"])]
    assert key == gd["key"]
    flags = O.scan_flags(g, Pattern(*key))
    found = g[flags.astype(bool)].tolist()
    assert found == gd["found"], found
    t = O.scan(g, Pattern(key[0], key[1], key[2], vo=0))
    assert _rows(t) == [(1,)]


# ---------------------------------------------------------------------------
# brute force on tiny inputs
# ---------------------------------------------------------------------------

VAR_LAYOUTS = [(0, 1, 2), (-1, -1, -1), (0, 0, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1),
               (2, 1, 0), (-1, 0, -1), (0, -1, 1)]


def _layout_pattern(consts, layout, rng_spec=None):
    vs = [layout[x] if consts[x] == 0 else -1 for x in range(3)]
    kw = {}
    if rng_spec:
        kw = dict(range_pos=rng_spec[0], lo=rng_spec[1], hi=rng_spec[2])
    return Pattern(consts[0], consts[1], consts[2], vs[0], vs[1], vs[2], **kw)


def check_exhaustive_scan(O, seeds=(0, 1, 2), ids=4):
    """All 125 constant patterns over IDs 0..4, under several variable
    layouts and a few ranges, against brute force, on graphs with duplicates."""
    for seed in seeds:
        g = tiny_graph(seed, 12, ids)
        g = np.concatenate([g, g[:3]])          # guaranteed duplicate triples
        for consts in itertools.product(range(ids + 1), repeat=3):
            for layout in VAR_LAYOUTS:
                for rs in (None, (2, 2, 4), (0, 3, 3), (1, 1, 5)):
                    p = _layout_pattern(consts, layout, rs)
                    rows, vs = bf_scan(g, p)
                    t = O.scan(g, p)
                    assert t.vars == vs, (p, t.vars, vs)
                    assert _rows(t) == rows, (p, _rows(t), rows)
                    f = O.scan_flags(g, p)
                    assert int(f.sum()) == len(rows)


def check_exhaustive_join(O, ids=4):
    """Joins on every column pair of a set of tiny tables, both oracle join
    methods, against brute force; includes empty tables."""
    g = tiny_graph(7, 14, ids)
    pats = [pat("?a ? ?b"), pat("?a 1 ?b"), pat("?a ?b 2"), pat("3 ?a ?b"), pat("?a ?b ?c"),
            pat("?a 4 ?a"), pat("4 4 ?a")]
    tabs = [O.scan(g, p) for p in pats]
    for L, R in itertools.product(tabs, repeat=2):
        for lc in range(L.ncols):
            for rc in range(R.ncols):
                want = bf_join(_rows(L), lc, _rows(R), rc)
                for method in ("nested", "sortmerge"):
                    j = O.join(L, lc, R, rc, method)
                    assert _rows(j) == want, (method, lc, rc)
                    assert j.vars == L.vars + [v for i, v in enumerate(R.vars) if i != rc]


def check_table3_matrix(O, ids=3):
    """The nine relation types of Table 3, each with every choice of its four
    constants from 1..ids, as scan-scan-join plans against brute force."""
    gd = _gold("table3_reltypes.json")
    g = np.concatenate([tiny_graph(11, 20, ids), tiny_graph(12, 6, ids)])
    nonempty = {}
    for name, (qi, qj) in gd["types"].items():
        const_names = [t for t in qi + qj if not t.startswith("?")]
        for vals in itertools.product(range(1, ids + 1), repeat=len(const_names)):
            env = dict(zip(const_names, vals))
            def mk(q):
                return Pattern(*[env.get(t, 0) for t in q],
                               *[0 if t == "?V" else -1 for t in q])
            plan = Plan().scan(mk(qi)).scan(mk(qj)).join(0)
            want, wv = bf_query(g, plan)
            got = O.query(g, plan)
            assert _rows(got) == want and got.vars == wv, (name, env)
            nonempty[name] = nonempty.get(name, 0) + (len(want) > 0)
    assert all(v > 0 for v in nonempty.values()), nonempty


def check_union_listing4(O):
    """Sec. 4.1: one triple can answer two subqueries (Listing 4 shape
    '{C ?v0 ?v1} UNION {?v2 P ?v3}').  Without DISTINCT it appears under both
    subqueries; the outer-union schema fills unbound variables with 0."""
    C, P = 5, 9
    g = np.array([[C, P, 1], [C, 2, 3], [4, P, 6], [7, 8, 9], [C, P, 1]], dtype=np.uint32)
    a = O.scan(g, Pattern(C, 0, 0, -1, 0, 1))
    b = O.scan(g, Pattern(0, P, 0, 2, -1, 3))
    u = O.union([a, b], False)
    assert u.vars == [0, 1, 2, 3]
    assert _rows(u) == [(P, 1, 0, 0), (2, 3, 0, 0), (P, 1, 0, 0),
                        (0, 0, C, 1), (0, 0, 4, 6), (0, 0, C, 1)]
    # same schema: the triple (C,P,1) answers '?s P ?o' and '?s ? ?o' with o in
    # [1,2); without DISTINCT it appears under both, with DISTINCT once
    a2 = O.scan(g, Pattern(0, P, 0, 0, -1, 1))
    b2 = O.scan(g, Pattern(0, 0, 0, 0, -1, 1, range_pos=2, lo=1, hi=2))
    assert _rows(O.union([a2, b2], False)) == [(C, 1), (4, 6), (C, 1), (C, 1), (C, 1)]
    assert _rows(O.union([a2, b2], True)) == [(4, 6), (C, 1)]
    # a narrower schema is padded with 0 before rows are compared
    b3 = O.scan(g, Pattern(0, 0, 1, 0, -1, -1))
    u3 = O.union([a2, b3], True)
    want, _ = bf_union([(_rows(a2), a2.vars), (_rows(b3), b3.vars)], True)
    assert _rows(u3) == want
    assert _rows(u3) == sorted({(C, 1), (4, 6), (C, 0)})


def check_scan_multi_bruteforce(O):
    """Sec. 4.1: the membership of triple i lists exactly the subqueries it
    answers (bit j set iff triple i matches pattern j)."""
    from bruteforce import bf_match
    g = tiny_graph(21, 25, 3)
    pats = [Pattern(*c) for c in itertools.product(range(4), repeat=3)][:40]
    member = O.scan_multi(g, pats)
    for i, t in enumerate(g):
        want = 0
        for j, p in enumerate(pats):
            if bf_match(t, p):
                want |= 1 << j
        assert int(member[i]) == want, (i, hex(int(member[i])), hex(want))


def check_union_bruteforce(O):
    g = tiny_graph(3, 16, 4)
    pats = [pat("?a 1 ?b"), pat("?b 2 ?a"), pat("?a ?c 3"), pat("?c ? ?c"), pat("? ? ?")]
    tabs = [O.scan(g, p) for p in pats]
    for k in (1, 2, 3, 5):
        for combo in itertools.combinations(range(len(tabs)), k):
            ins = [tabs[i] for i in combo]
            for d in (False, True):
                want, wv = bf_union([(_rows(t), t.vars) for t in ins], d)
                got = O.union(ins, d)
                assert got.vars == wv
                assert _rows(got) == want, (combo, d)


def check_filter_bruteforce(O):
    g = tiny_graph(5, 30, 6)
    t = O.scan(g, pat("?a ?b ?c"))
    for col in range(3):
        for lo in range(0, 8):
            for hi in range(0, 8):
                want = bf_filter(_rows(t), col, lo, hi)
                assert _rows(O.filter(t, col, lo, hi)) == want, (col, lo, hi)


def random_plan(rng, ids=4):
    """A random postfix plan of 1..3 patterns over variables 0..2."""
    def rpat():
        while True:
            consts = [int(rng.integers(0, ids + 1)) if rng.random() < 0.4 else 0
                      for _ in range(3)]
            vs = [int(rng.integers(0, 3)) if c == 0 else -1 for c in consts]
            if any(v >= 0 for v in vs):
                return Pattern(*consts, *vs)
    plan = Plan()
    p = rpat()
    plan.scan(p)
    schema = set(p.out_vars())
    for _ in range(int(rng.integers(0, 3))):
        q = rpat()
        shared = schema & set(q.out_vars())
        if shared and rng.random() < 0.6:
            plan.scan(q).join(sorted(shared)[0])
            schema |= set(q.out_vars())
        else:
            plan.scan(q).union(2, bool(rng.integers(0, 2)))
            schema |= set(q.out_vars())
    if rng.random() < 0.4:
        v = sorted(schema)[0]
        plan.filter(v, int(rng.integers(0, 3)), int(rng.integers(2, 6)))
    if rng.random() < 0.4:
        keep = sorted(schema)[: int(rng.integers(1, len(schema) + 1))]
        plan.project(keep)
    if rng.random() < 0.4:
        plan.distinct()
    return plan


def check_random_plans(O, n=300, seed=99):
    rng = np.random.default_rng(seed)
    for i in range(n):
        g = tiny_graph(1000 + i, int(rng.integers(0, 16)), 4)
        plan = random_plan(rng)
        want, wv = bf_query(g, plan)
        got = O.query(g, plan)
        assert got.vars == wv and _rows(got) == want, (i, plan)


def check_random_plans_sortmerge(O, n=300, seed=77):
    """The same plans with every plan join forced onto the sort-merge path."""
    O.set_nested_join_limit(0.0)
    try:
        check_random_plans(O, n, seed)
    finally:
        O.set_nested_join_limit(1e8)


# ---------------------------------------------------------------------------
# invariants at size (independent numpy arithmetic)
# ---------------------------------------------------------------------------

def check_invariants_small_config(O, g):
    N = g.shape[0]
    # sum over predicates of |scan(?, p, ?)| = N, and per-p counts = histogram
    hist = np.bincount(g[:, 1])
    total = 0
    for p in np.nonzero(hist)[0]:
        t = O.scan(g, Pattern(0, int(p), 0, 0, -1, 1))
        assert t.nrows == hist[p]
        total += t.nrows
    assert total == N
    # scan result = the matching rows of the input, in position order
    t = O.scan(g, pat("?s 7 ?o"))
    sel = g[g[:, 1] == 7]
    assert np.array_equal(t.rows, sel[:, [0, 2]])
    # |L join R| = sum_k cL(k) cR(k)
    L = O.scan(g, pat("?s 3 ?o1"))
    R = O.scan(g, pat("?s 11 ?o2"))
    cl = np.bincount(L.rows[:, 0], minlength=10_001).astype(np.int64)
    cr = np.bincount(R.rows[:, 0], minlength=10_001).astype(np.int64)
    j1 = O.join(L, 0, R, 0, "nested")
    j2 = O.join(L, 0, R, 0, "sortmerge")
    assert j1.nrows == int((cl * cr).sum())
    assert np.array_equal(j1.rows, j2.rows)
    # output rows are in strict lexicographic order up to duplicates
    r = j1.rows.astype(np.int64)
    key = (r[:, 0] << 40) | (r[:, 1] << 20) | r[:, 2]
    assert np.all(np.diff(key) >= 0)
    # union with DISTINCT = set union
    a = O.scan(g, pat("?s 7 ?o"))
    b = O.scan(g, pat("?s 8 ?o"))
    u = O.union([a, b], True)
    want = sorted(set(map(tuple, a.rows.tolist())) | set(map(tuple, b.rows.tolist())))
    assert _rows(u) == want
    # filter: idempotent, monotone, empty when lo >= hi
    f = O.filter(a, 1, 100, 5000)
    assert np.array_equal(O.filter(f, 1, 100, 5000).rows, f.rows)
    wide = O.filter(a, 1, 50, 9000)
    assert set(map(tuple, f.rows.tolist())) <= set(map(tuple, wide.rows.tolist()))
    assert O.filter(a, 1, 5000, 100).nrows == 0
    # fused range in the scan = scan then filter
    fs = O.scan(g, Pattern(0, 7, 0, 0, -1, 1, range_pos=2, lo=100, hi=5000))
    assert np.array_equal(fs.rows, f.rows)
    # star on ?s: |result| = sum_s prod_i c_i(s)
    n = {}
    plan = (Plan().scan(pat("?s 3 ?a", n)).scan(pat("?s 11 ?b", n)).join(n["?s"])
            .scan(pat("?s 20 ?c", n)).join(n["?s"]))
    q = O.query(g, plan)
    c3 = np.bincount(O.scan(g, pat("?s 20 ?c")).rows[:, 0], minlength=10_001).astype(np.int64)
    assert q.nrows == int((cl * cr * c3).sum())


def check_invariants_tiny_config(O):
    from synth import CONFIGS, make_graph
    check_invariants_small_config(O, make_graph(CONFIGS["small"].with_n(20_000)))


ALL_CHECKS = [check_rule11, check_toy_sec3, check_exhaustive_scan, check_exhaustive_join,
              check_table3_matrix, check_union_listing4, check_scan_multi_bruteforce,
              check_union_bruteforce, check_filter_bruteforce, check_random_plans,
              check_random_plans_sortmerge, check_invariants_tiny_config]


# ---------------------------------------------------------------------------
# dictionary encoder (Sec. 3: terms -> IDs from 1, first appearance, s p o)
# ---------------------------------------------------------------------------

SUBCLASS_TRIPLES = [["Cat", "subClassOf", "Mammal"], ["Mammal", "subClassOf", "Animal"],
                    ["Dog", "subClassOf", "Mammal"], ["Animal", "subClassOf", "Thing"],
                    ["Cat", "label", "cat"], ["Fish", "subClassOf", "Animal"],
                    ["Mammal", "subClassOf", "Vertebrate"], ["Cat", "subClassOf", "Mammal"]]


def _first_appearance_ids(triples):
    """IDs by first appearance over the flattened s, p, o stream, computed
    with numpy's unique (an independent construction of the same order)."""
    flat = np.array([x for t in triples for x in t], dtype=object)
    uniq, first = np.unique(flat.astype(str), return_index=True)
    order = np.argsort(first, kind="stable")
    return {str(uniq[j]): i + 1 for i, j in enumerate(order)}


def check_encoder(O):
    """Shared and per-position dictionaries: IDs from 1 in order of first
    appearance; decode inverts encode; and with one shared dictionary a join
    that pairs an object with a subject (Table 3's OS type) gives, decoded,
    exactly the join computed on the strings themselves."""
    gd = _gold("toy_sec3.json")
    for triples in (gd["triples"], SUBCLASS_TRIPLES):
        g, dicts = O.encode_graph(triples, shared=True)
        assert dicts[0] is dicts[1] is dicts[2]
        want = _first_appearance_ids(triples)
        assert dicts[0] == want, (dicts[0], want)
        assert g.min() >= 1 and g.max() == len(want)
        for row, t in zip(g.tolist(), triples):
            assert O.decode_row(row, dicts, (0, 1, 2)) == tuple(t)
        gs, ds = O.encode_graph(triples, shared=False)
        for pos in range(3):
            col = [t[pos] for t in triples]
            assert ds[pos] == _first_appearance_ids([[x] for x in col])
        for row, t in zip(gs.tolist(), triples):
            assert O.decode_row(row, ds, (0, 1, 2)) == tuple(t)
    # the Sec. 3 walk-through under one shared dictionary: 'publishes' is
    # the 4th distinct term, so the key of "ABCPress publishes ?" is (1,4,?)
    g, dicts = O.encode_graph(gd["triples"], shared=True)
    key = [dicts[0][t] if t != "?" else 0 for t in gd["query_terms"]]
    assert key == [1, 4, 0]
    assert O.decode_row(g[O.scan_flags(g, Pattern(*key)).astype(bool)][0], dicts,
                        (0, 1, 2)) == ("ABCPress", "publishes", "JournalA")
    # OS join on strings, by nested loops over the string triples
    want = sorted({(a[0], b[2]) for a in SUBCLASS_TRIPLES for b in SUBCLASS_TRIPLES
                   if a[1] == b[1] == "subClassOf" and a[2] == b[0]})
    g, dicts = O.encode_graph(SUBCLASS_TRIPLES, shared=True)
    sc = dicts[0]["subClassOf"]
    n = {}
    plan = (Plan().scan(pat(f"?x {sc} ?y", n)).scan(pat(f"?y {sc} ?z", n)).join(n["?y"])
            .project([n["?x"], n["?z"]]).distinct())
    got = sorted(O.decode_row(r, dicts, (0, 2)) for r in O.query(g, plan).rows.tolist())
    assert got == want, (got, want)
    assert len(want) == 6   # Cat, Dog (x2 each), Mammal and Fish two steps up


# ---------------------------------------------------------------------------
# outer joins (Sec. 4.2: Left, Right and Outer kinds besides Inner)
# ---------------------------------------------------------------------------

def _pandas_outer(L, lc, R, rc, how):
    """The same join by pandas' merge (an independent library routine), with
    missing cells filled by 0 and the right key column dropped (its value
    moved into the left key column where the left side is missing)."""
    import pandas as pd
    lnames = [f"l{i}" for i in range(L.shape[1])]
    rnames = [f"r{i}" for i in range(R.shape[1])]
    dl = pd.DataFrame(L.astype(np.int64), columns=lnames)
    dr = pd.DataFrame(R.astype(np.int64), columns=rnames)
    m = dl.merge(dr, left_on=f"l{lc}", right_on=f"r{rc}", how=how)
    m[f"l{lc}"] = m[f"l{lc}"].fillna(m[f"r{rc}"])
    m = m.fillna(0)
    cols = lnames + [c for i, c in enumerate(rnames) if i != rc]
    out = m[cols].to_numpy().astype(np.uint32) if len(m) else np.zeros((0, len(cols)), np.uint32)
    return sorted(tuple(int(x) for x in r) for r in out)


def check_outer_joins(O):
    """or_join_outer against pandas' merge on every column pair of small
    random tables (with repeated keys, keys on one side only, empty sides),
    plus the identities inner = join, |left| = sum over L rows of
    max(matches, 1), and right(L, R) = left(R, L) with columns reordered."""
    rng = np.random.default_rng(31)
    shapes = [(9, 2, 7, 2), (6, 3, 0, 2), (0, 2, 5, 1), (12, 1, 12, 3), (5, 2, 8, 2)]
    for nl, kl, nr, kr in shapes:
        L = rng.integers(1, 6, size=(nl, kl)).astype(np.uint32)
        R = rng.integers(3, 9, size=(nr, kr)).astype(np.uint32)
        TL = O.Table(L, list(range(kl)))
        TR = O.Table(R, list(range(10, 10 + kr)))
        for lc in range(kl):
            for rc in range(kr):
                inner = O.join_outer(TL, lc, TR, rc, "inner")
                assert _rows(inner) == bf_join([tuple(r) for r in L.tolist()], lc,
                                               [tuple(r) for r in R.tolist()], rc)
                for kind, how in (("left", "left"), ("right", "right"), ("full", "outer")):
                    got = O.join_outer(TL, lc, TR, rc, kind)
                    assert got.vars == inner.vars
                    assert _rows(got) == _pandas_outer(L, lc, R, rc, how), (kind, lc, rc)
                left = O.join_outer(TL, lc, TR, rc, "left")
                cnt = np.array([np.sum(R[:, rc] == x) for x in L[:, lc]], dtype=np.int64) \
                    if nr else np.zeros(nl, np.int64)
                assert left.nrows == int(np.maximum(cnt, 1).sum())
                # right(L, R) is left(R, L) with the columns put back in order
                right = O.join_outer(TL, lc, TR, rc, "right")
                swapped = O.join_outer(TR, rc, TL, lc, "left")
                perm = []
                for v in right.vars:
                    perm.append(swapped.vars.index(v) if v in swapped.vars
                                else swapped.vars.index(TR.vars[rc]))
                back = sorted(tuple(int(r[j]) for j in perm) for r in swapped.rows.tolist())
                assert _rows(right) == back


def check_optional_plans(O):
    """OPTIONAL in a plan: (?s p1 ?a) OPTIONAL (?s p2 ?b) equals the left join
    of the two scans by brute force; a plan whose sides share a second
    variable is refused."""
    g = tiny_graph(41, 40, 5)
    n = {}
    plan = Plan().scan(pat("?s 1 ?a", n)).scan(pat("?s 2 ?b", n)).optional(n["?s"])
    res = O.query(g, plan)
    A, av = bf_scan(g, pat("?s 1 ?a", dict(n)))
    B, bv = bf_scan(g, pat("?s 2 ?b", dict(n)))
    want = []
    for a in A:
        hit = [b for b in B if b[0] == a[0]]
        want += [tuple(a) + (b[1],) for b in hit] or [tuple(a) + (0,)]
    assert _rows(res) == sorted(want)
    m = {}
    bad = (Plan().scan(pat("?s 1 ?a", m)).scan(pat("?s 2 ?a", m)).optional(m["?s"]))
    try:
        O.query(g, bad)
    except Exception as e:  # noqa: BLE001
        assert getattr(e, "status", None) == -4
    else:
        raise AssertionError("OPTIONAL with two shared variables was not refused")


ALL_CHECKS += [check_outer_joins, check_optional_plans]


# ---------------------------------------------------------------------------
# multi-key search and RDFS entailment (Sec. 4.1 keysArray; Sec. 5.7)
# ---------------------------------------------------------------------------

def bf_entail(g, rule, voc):
    """The rule table by brute force: every pair of triples (t1, t2) meeting
    the rule's two conditions gives one derived triple (a set)."""
    T, SC, SPO, DOM, RNG = voc
    rows = [tuple(int(x) for x in r) for r in g.tolist()]
    out = set()
    for a in rows:
        for b in rows:
            if rule == 2 and b[1] == DOM and a[1] == b[0]:
                out.add((a[0], T, b[2]))
            elif rule == 3 and b[1] == RNG and a[1] == b[0]:
                out.add((a[2], T, b[2]))
            elif rule == 5 and a[1] == SPO and b[1] == SPO and a[2] == b[0]:
                out.add((a[0], SPO, b[2]))
            elif rule == 7 and b[1] == SPO and a[1] == b[0]:
                out.add((a[0], b[2], a[2]))
            elif rule == 9 and a[1] == T and b[1] == SC and a[2] == b[0]:
                out.add((a[0], T, b[2]))
            elif rule == 11 and a[1] == SC and b[1] == SC and a[2] == b[0]:
                out.add((a[0], SC, b[2]))
    return sorted(out)


def check_entailment(O):
    """Rule 11's worked example (Sec. 5.7): step-1 keys {56, 77, 78}, step-2
    positionArray {0,0,1,1,0}, derived {(76,78), (76,77)}; every rule against
    brute force over pairs of triples on small RDFS graphs; the keyed scan
    against brute-force membership."""
    gd = _gold("rule11_example.json")
    g = np.array(gd["data"], dtype=np.uint32)
    voc = [1, 84, 3, 4, 5]
    keys = [k[0] for k in gd["step2_keysArray"]]
    t2 = O.scan_keyed(g, Pattern(0, 84, 0, 0, -1, 1), 0, keys)
    flags = [int(any((r == list(x)) for x in t2.rows.tolist())) for r in
             [[int(v[0]), int(v[2])] for v in g.tolist()]]
    assert flags == gd["step2_positionArray"], flags
    res = O.entail(g, 11, voc)
    assert sorted((r[0], r[2]) for r in _rows(res)) == sorted(tuple(x) for x in gd["result_x_z"])
    assert all(r[1] == 84 for r in _rows(res))
    from synth.rdfs import VOCAB, RdfsSpec, make_rdfs_graph
    for seed in (1, 2):
        g = make_rdfs_graph(RdfsSpec(n_data=120, n_classes=14, n_props=9, n_resources=25,
                                     seed=seed))
        for rule in (2, 3, 5, 7, 9, 11):
            got = O.entail(g, rule, VOCAB)
            assert got.vars == [0, 1, 2]
            assert _rows(got) == bf_entail(g, rule, VOCAB), (seed, rule)
    rng = np.random.default_rng(3)
    g = tiny_graph(5, 60, 6)
    for pos in range(3):
        for keys in ([], [2], [1, 3, 3, 5], list(range(1, 7))):
            q = _layout_pattern([0, 0, 0], (0, 1, 2))
            got = O.scan_keyed(g, q, pos, keys)
            want = [tuple(int(x) for x in r) for r in g.tolist() if r[pos] in keys]
            assert _rows(got) == want, (pos, keys)
        q = Pattern(0, 2, 0, 0, -1, 1)
        got = O.scan_keyed(g, q, 0, [1, 4])
        assert _rows(got) == [(int(r[0]), int(r[2])) for r in g.tolist()
                              if r[1] == 2 and r[0] in (1, 4)]


ALL_CHECKS += [check_entailment]
