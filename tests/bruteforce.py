"""Pure-Python brute force over tiny inputs, written independently of the C
oracle, used to pin it.  Tables are (rows: list of tuples, vars: list)."""
from __future__ import annotations

from typing import List, Sequence, Tuple

from synth.plan import (OP_DISTINCT, OP_FILTER, OP_JOIN, OP_PROJECT, OP_SCAN,
                        OP_UNION)

Rows = List[Tuple[int, ...]]


def bf_match(t, p) -> bool:
    vals = (int(t[0]), int(t[1]), int(t[2]))
    consts, vars_ = p.consts, p.vars
    for x in range(3):
        if consts[x] and vals[x] != consts[x]:
            return False
    seen = {}
    for x in range(3):
        v = vars_[x]
        if v >= 0:
            if v in seen and seen[v] != vals[x]:
                return False
            seen[v] = vals[x]
    if p.range_pos >= 0 and not (p.lo <= vals[p.range_pos] < p.hi):
        return False
    return True


def bf_scan(g, p) -> Tuple[Rows, list]:
    schema, src = [], []
    for x, v in enumerate(p.vars):
        if v >= 0 and v not in schema:
            schema.append(v)
            src.append(x)
    rows = [tuple(int(t[x]) for x in src) for t in g if bf_match(t, p)]
    return rows, schema


def bf_join(L: Rows, lc: int, R: Rows, rc: int) -> Rows:
    out = []
    for l in L:
        for r in R:
            if l[lc] == r[rc]:
                out.append(tuple(l) + tuple(v for i, v in enumerate(r) if i != rc))
    return sorted(out)


def bf_filter(T: Rows, col: int, lo: int, hi: int) -> Rows:
    return [r for r in T if lo <= r[col] < hi]


def bf_union(tables: Sequence[Tuple[Rows, list]], dedupe: bool) -> Tuple[Rows, list]:
    schema = []
    for _, vs in tables:
        for v in vs:
            if v not in schema:
                schema.append(v)
    out = []
    for rows, vs in tables:
        for r in rows:
            d = dict(zip(vs, r))
            out.append(tuple(d.get(v, 0) for v in schema))
    if dedupe:
        out = sorted(set(out))
    return out, schema


def bf_query(g, plan) -> Tuple[Rows, list]:
    st: list = []
    ops = list(plan.ops)
    i = 0
    while i < len(ops):
        op = ops[i]
        i += 1
        if op == OP_SCAN:
            st.append(bf_scan(g, plan.patterns[ops[i]]))
            i += 1
        elif op == OP_JOIN:
            v = ops[i]
            i += 1
            (R, rv), (L, lv) = st.pop(), st.pop()
            shared = [w for w in rv if w in lv]
            keep = [j for j, w in enumerate(rv) if w not in lv]
            rows = []
            for l in L:
                dl = dict(zip(lv, l))
                for r in R:
                    dr = dict(zip(rv, r))
                    if dl[v] == dr[v] and all(dl[w] == dr[w] for w in shared):
                        rows.append(tuple(l) + tuple(r[j] for j in keep))
            st.append((rows, lv + [rv[j] for j in keep]))
        elif op == OP_UNION:
            k, d = ops[i], ops[i + 1]
            i += 2
            ins = st[-k:]
            del st[-k:]
            st.append(bf_union(ins, bool(d)))
        elif op == OP_FILTER:
            v, lo, hi = ops[i], ops[i + 1], ops[i + 2]
            i += 3
            rows, vs = st.pop()
            c = vs.index(v)
            st.append((bf_filter(rows, c, lo, hi), vs))
        elif op == OP_PROJECT:
            n = ops[i]
            want = ops[i + 1:i + 1 + n]
            i += 1 + n
            rows, vs = st.pop()
            idx = [vs.index(w) for w in want]
            st.append(([tuple(r[j] for j in idx) for r in rows], list(want)))
        elif op == OP_DISTINCT:
            rows, vs = st.pop()
            st.append((sorted(set(rows)), vs))
        else:
            raise ValueError(op)
    assert len(st) == 1
    rows, vs = st[0]
    return sorted(rows), vs
