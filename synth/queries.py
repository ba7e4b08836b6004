"""Seeded query choices for the synthetic workloads.

These functions only choose constants (predicates, objects, ID ranges) from
histograms of the generated graph so that each query lands in the size band
its workload asks for.  Star sizes are estimated as sum over subjects of the
product of per-pattern subject counts (a count, not a result).
"""
from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np

from .plan import Pattern, Plan, pat


def predicate_for_selectivity(g: np.ndarray, sigma: float) -> Tuple[int, float]:
    """The predicate whose share of triples is closest to sigma in log scale."""
    hist = np.bincount(g[:, 1])
    n = g.shape[0]
    share = np.maximum(hist, 1) / n
    p = int(np.argmin(np.abs(np.log(share) - np.log(sigma))))
    return p, float(hist[p]) / n


def star_query(g: np.ndarray, lo: float = 1e5, hi: float = 1e7, target: float = 1e6,
               a_ranks=(50, 100, 200, 400, 700), bc_ranks=range(20, 1001, 20)
               ) -> Tuple[Plan, Dict]:
    """3-pattern star on ?s:  (?s pA oA) . (?s pB ?o1) . (?s pC ?o2).

    pA runs over a few predicate frequency ranks, oA is the most frequent
    object of pA, and (pB, pC) are chosen among predicate ranks so that the
    star's size is in [lo, hi], closest to `target` in log scale.  Hub
    subjects make stars on frequent predicates explode, so the candidates are
    the rarer predicates."""
    s, p, o = g[:, 0], g[:, 1], g[:, 2]
    hist_p = np.bincount(p)
    order = np.argsort(-hist_p, kind="stable")  # predicate IDs by frequency rank
    best = None
    subj_by_p: Dict[int, np.ndarray] = {}

    def subjects_of(pid):
        if pid not in subj_by_p:
            subj_by_p[pid] = s[p == pid]
        return subj_by_p[pid]

    nranks = int((hist_p > 0).sum())
    for ra in a_ranks:
        if ra > nranks:
            continue
        pA = int(order[ra - 1])
        objs = o[p == pA]
        oA = int(np.bincount(objs).argmax())
        sa = s[(p == pA) & (o == oA)]
        supp, ca = np.unique(sa, return_counts=True)
        if supp.size == 0:
            continue
        counts = {}
        for rb in bc_ranks:
            if rb > nranks:
                continue
            pid = int(order[rb - 1])
            if pid == pA:
                continue
            sb = subjects_of(pid)
            idx = np.searchsorted(supp, sb)
            idx = np.clip(idx, 0, supp.size - 1)
            hit = supp[idx] == sb
            counts[pid] = np.bincount(idx[hit], minlength=supp.size).astype(np.float64)
        pids = sorted(counts)
        for i, pB in enumerate(pids):
            for pC in pids[i + 1:]:
                size = float((ca * counts[pB] * counts[pC]).sum())
                if lo <= size <= hi:
                    score = abs(np.log(size) - np.log(target))
                    if best is None or score < best[0]:
                        best = (score, pA, oA, pB, pC, size)
    if best is None:
        raise ValueError("no star in the requested size band")
    _, pA, oA, pB, pC, size = best
    n: Dict[str, int] = {}
    plan = (Plan().scan(pat(f"?s {pA} {oA}", n)).scan(pat(f"?s {pB} ?o1", n))
            .join(n["?s"]).scan(pat(f"?s {pC} ?o2", n)).join(n["?s"]))
    return plan, {"pA": pA, "oA": oA, "pB": pB, "pC": pC, "est_rows": int(round(size))}


def union_query(g: np.ndarray, ranks=range(11, 19)) -> Tuple[Plan, Dict]:
    """Union of (?s p_r ?o) for the given predicate frequency ranks, DISTINCT."""
    hist_p = np.bincount(g[:, 1])
    order = np.argsort(-hist_p, kind="stable")
    pids = [int(order[r - 1]) for r in ranks]
    n: Dict[str, int] = {}
    plan = Plan()
    for pid in pids:
        plan.scan(pat(f"?s {pid} ?o", n))
    plan.union(len(pids), True)
    return plan, {"predicates": pids, "rows_in": int(sum(hist_p[q] for q in pids))}


def object_range(g: np.ndarray, keep: float = 0.05, start: float = 0.3,
                 tol: float = 0.1) -> Tuple[int, int]:
    """[lo, hi) over object IDs holding keep*(1 +- tol) of the triples; the
    window starts at the `start` quantile of the object CDF in ID order and
    moves up in 1% steps until its share is in the band (a hub object can
    make one window too heavy)."""
    hist = np.bincount(g[:, 2])
    cdf = np.concatenate([[0], np.cumsum(hist)])  # cdf[i] = #triples with o < i
    n = g.shape[0]
    for k in range(60):
        st = start + 0.01 * k
        lo = max(1, int(np.searchsorted(cdf, st * n, side="left")))
        hi = max(lo + 1, int(np.searchsorted(cdf, (st + keep) * n, side="left")))
        share = (cdf[min(hi, len(cdf) - 1)] - cdf[min(lo, len(cdf) - 1)]) / n
        if abs(share - keep) <= tol * keep:
            return lo, hi
    raise ValueError("no object range with the requested share")


def range_pattern(g: np.ndarray, keep: float = 0.05) -> Tuple[Pattern, Dict]:
    lo, hi = object_range(g, keep)
    p = Pattern(0, 0, 0, 0, 1, 2, range_pos=2, lo=lo, hi=hi)
    return p, {"lo": lo, "hi": hi}


def chain_count(g: np.ndarray, pids, rows_of=None) -> int:
    """Exact row count of the chain (?x0 p1 ?x1) . (?x1 p2 ?x2) . ... by
    propagating per-value path counts hop by hop (a count, not a result):
    w(v) = number of paths ending in value v; one hop over predicate q maps
    w to w'(o) = sum over triples (s, q, o) of w(s).  rows_of(q), if given,
    returns the (s, o) columns of predicate q's triples."""
    if rows_of is None:
        def rows_of(q):
            sel = g[:, 1] == q
            return g[sel, 0], g[sel, 2]
    size = int(max(g[:, 0].max(), g[:, 2].max())) + 1 if g.shape[0] else 1
    s, o = rows_of(pids[0])
    w = np.bincount(o, minlength=size).astype(np.float64)
    for q in pids[1:]:
        s, o = rows_of(q)
        w = np.bincount(o, weights=w[s], minlength=size)
    return int(round(w.sum()))


def chain_query(g: np.ndarray, start_rank: int = 2, lo: float = 1e6, hi: float = 1e8,
                length: int = 4) -> Tuple[Plan, Dict]:
    """4-pattern chain (?a p1 ?b) . (?b p2 ?c) . (?c p3 ?d) . (?d p4 ?e) over
    predicates given by frequency rank.  Candidates start from every hop at
    rank `start_rank`; while the exact count is below `lo`, hops move one at
    a time, left to right, to the next more frequent rank (2,2,2,2 ->
    1,2,2,2 -> 1,1,2,2 -> ...); while it is above `hi`, to the next rarer
    one (2,2,2,2 -> 3,2,2,2 -> ...).  The first candidate in [lo, hi] is
    taken."""
    hist_p = np.bincount(g[:, 1])
    order = np.argsort(-hist_p, kind="stable")
    nranks = int((hist_p > 0).sum())
    ranks = [start_rank] * length
    tried = {}
    cols = {}

    def rows_of(q):
        if q not in cols:
            sel = g[:, 1] == q
            cols[q] = (g[sel, 0], g[sel, 2])
        return cols[q]

    while all(1 <= r <= nranks for r in ranks) and tuple(ranks) not in tried:
        pids = [int(order[r - 1]) for r in ranks]
        c = tried[tuple(ranks)] = chain_count(g, pids, rows_of)
        if lo <= c <= hi:
            break
        step = -1 if c < lo else 1
        # the leftmost hop still at the current rank level moves one rank
        level = max(ranks) if step < 0 else min(ranks)
        i = ranks.index(level)
        ranks[i] += step
    else:
        raise ValueError(f"no chain in the requested size band: {tried}")
    pids = [int(order[r - 1]) for r in ranks]
    names = ["?a", "?b", "?c", "?d", "?e", "?f", "?g"][:length + 1]
    n: Dict[str, int] = {}
    plan = Plan()
    for i in range(length):
        plan.scan(pat(f"{names[i]} {pids[i]} {names[i + 1]}", n))
        if i:
            plan.join(n[names[i]])
    return plan, {"ranks": list(ranks), "predicates": pids, "rows": tried[tuple(ranks)],
                  "pattern_rows": [int(hist_p[q]) for q in pids]}
