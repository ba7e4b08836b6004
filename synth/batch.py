"""Seeded query mixes for the batched and serving workloads.

Each query has 1..6 patterns, is a star on ?s or a chain, half and half, and
draws a target selectivity per pattern log-uniformly in [1e-6, 1e-1].  A
target is met with a predicate whose share of the graph is closest (in log
scale) or, below the rarest predicate's share, with a (predicate, object)
pair of about the target count; in a chain only the last pattern may bind an
object.  The pattern count and shape of a query are drawn once; its
selectivities are drawn again while its join prefix (in plan order, left to
right) would exceed `max_rows` rows, and while its result is empty, up to
`empty_redraws` times (then an empty result is kept).  Sizes are counted from a
(predicate, subject)-ordered copy of the graph: counts only, no bindings.
"""
from __future__ import annotations

import os
from dataclasses import dataclass
from typing import Dict, List, Tuple

import numpy as np

from .graph import _gpu_initialised
from .plan import Pattern, Plan


class PredIndex:
    """Triples ordered by (predicate, subject); per predicate the slice bounds."""

    def __init__(self, g: np.ndarray):
        # Bucket by predicate (a radix argsort when IDs fit 16 bits), then
        # sort each bucket's packed (subject, object) words in place: within
        # a predicate the order is (s, o), which is a (p, s) order.
        self.n = g.shape[0]
        pcol = g[:, 1]
        hist = np.bincount(pcol)
        self.start = np.concatenate([[0], np.cumsum(hist)]).astype(np.int64)
        key = pcol.astype(np.uint16) if hist.size <= 1 << 16 else pcol
        order = np.argsort(key, kind="stable")
        del key
        packed = g[order, 0].astype(np.uint64) << np.uint64(32)
        packed |= g[order, 2]
        del order
        # numpy's sort releases the interpreter lock: predicates in parallel
        from concurrent.futures import ThreadPoolExecutor
        preds = [int(p) for p in np.nonzero(hist > 1)[0]]
        with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
            list(ex.map(lambda p: packed[self.start[p]:self.start[p + 1]].sort(), preds))
        self.s = (packed >> np.uint64(32)).astype(np.uint32)
        self.o = packed.astype(np.uint32)
        del packed
        self.share = hist / self.n
        self.preds = np.nonzero(hist)[0]
        self._obj_counts: Dict[int, Tuple[np.ndarray, np.ndarray]] = {}
        self._subj_counts: Dict[int, Tuple[np.ndarray, np.ndarray]] = {}

    def subjects(self, p: int) -> np.ndarray:
        return self.s[self.start[p]:self.start[p + 1]]

    def objects(self, p: int) -> np.ndarray:
        return self.o[self.start[p]:self.start[p + 1]]

    def subject_counts(self, p: int) -> Tuple[np.ndarray, np.ndarray]:
        """Distinct subjects of predicate p (sorted) and their triple counts."""
        if p not in self._subj_counts:
            s = self.subjects(p)  # already sorted
            if s.size == 0:
                self._subj_counts[p] = (s, s.astype(np.float64))
            else:
                edge = np.concatenate([[True], s[1:] != s[:-1]])
                ids = s[edge]
                idx = np.nonzero(edge)[0]
                cnt = np.diff(np.concatenate([idx, [s.size]])).astype(np.float64)
                self._subj_counts[p] = (ids, cnt)
        return self._subj_counts[p]

    def object_counts(self, p: int) -> Tuple[np.ndarray, np.ndarray]:
        if p not in self._obj_counts:
            ids, cnt = np.unique(self.objects(p), return_counts=True)
            self._obj_counts[p] = (ids, cnt.astype(np.float64))
        return self._obj_counts[p]


def _lookup(ids: np.ndarray, cnt: np.ndarray, keys: np.ndarray) -> np.ndarray:
    """cnt of each key in (ids, cnt), 0 where absent."""
    if ids.size == 0:
        return np.zeros(keys.size)
    i = np.clip(np.searchsorted(ids, keys), 0, ids.size - 1)
    return np.where(ids[i] == keys, cnt[i], 0.0)


@dataclass
class Term:
    p: int
    o: int = 0   # 0: free object


def _realise(idx: PredIndex, sigma: float, rng, allow_object: bool) -> Term:
    shares = idx.share[idx.preds]
    smin = shares.min()
    if sigma >= smin or not allow_object:
        j = int(np.argmin(np.abs(np.log(shares) - np.log(max(sigma, smin)))))
        return Term(int(idx.preds[j]))
    target = sigma * idx.n
    # rare predicates first: their objects give the small counts
    order = idx.preds[np.argsort(shares)]
    best = None
    for p in order[:60]:
        ids, cnt = idx.object_counts(int(p))
        j = int(np.argmin(np.abs(np.log(cnt) - np.log(target))))
        score = abs(np.log(cnt[j]) - np.log(target))
        if best is None or score < best[0]:
            best = (score, int(p), int(ids[j]))
    return Term(best[1], best[2])


def _star_prefix_counts(idx: PredIndex, terms: List[Term]) -> List[float]:
    """Rows after each join of a star on ?s, in plan order."""
    out = []
    supp, w = None, None
    for t in terms:
        if t.o:
            s = idx.subjects(t.p)[idx.objects(t.p) == t.o]
            ids, cnt = np.unique(s, return_counts=True)
            cnt = cnt.astype(np.float64)
        else:
            ids, cnt = idx.subject_counts(t.p)
        if supp is None:
            supp, w = ids, cnt
        else:
            c = _lookup(ids, cnt, supp)
            keep = c > 0
            supp, w = supp[keep], w[keep] * c[keep]
        out.append(float(w.sum()))
    return out


def _chain_prefix_counts(idx: PredIndex, terms: List[Term], cap: float) -> List[float]:
    """Rows after each join of a chain ?x0 p1 ?x1 . ?x1 p2 ?x2 . ..., in plan
    order; stops early (returns inf) once a prefix exceeds `cap`."""
    out = []
    # weights on the chain's current end variable
    t0 = terms[0]
    s0, o0 = idx.subjects(t0.p), idx.objects(t0.p)
    if t0.o:
        o0 = o0[o0 == t0.o]
    ends, w = np.unique(o0, return_counts=True)
    w = w.astype(np.float64)
    out.append(float(w.sum()))
    for t in terms[1:]:
        if out[-1] > cap:
            return out + [np.inf] * (len(terms) - len(out))
        sp = idx.subjects(t.p)
        lo = np.searchsorted(sp, ends, side="left")
        hi = np.searchsorted(sp, ends, side="right")
        reps = hi - lo
        total_paths = float((reps * w).sum()) if reps.size else 0.0
        if not t.o and total_paths > cap:
            return out + [np.inf] * (len(terms) - len(out))
        base = idx.start[t.p]
        tot = int(reps.sum())
        if tot > 4 * cap:
            return out + [np.inf] * (len(terms) - len(out))
        sel = np.repeat(np.arange(ends.size), reps)
        # positions lo[j] + 0 .. reps[j]-1 for every end j, vectorised
        first = np.concatenate([[0], np.cumsum(reps)[:-1]]) if reps.size else reps
        pos = base + np.repeat(lo - first, reps) + np.arange(tot)
        objs = idx.o[pos]
        ww = w[sel]
        if t.o:
            keep = objs == t.o
            objs, ww = objs[keep], ww[keep]
        ends, inv = np.unique(objs, return_inverse=True)
        w = np.bincount(inv, weights=ww, minlength=ends.size) if ends.size else np.zeros(0)
        out.append(float(w.sum()))
    return out


def _plan(shape: str, terms: List[Term]) -> Plan:
    plan = Plan()
    if shape == "star":
        for i, t in enumerate(terms):
            if t.o:
                plan.scan(Pattern(0, t.p, t.o, 0, -1, -1))
            else:
                plan.scan(Pattern(0, t.p, 0, 0, -1, 1 + i))
            if i:
                plan.join(0)
    else:
        for i, t in enumerate(terms):
            plan.scan(Pattern(0, t.p, t.o, i, -1, -1 if t.o else i + 1))
            if i:
                plan.join(i)
    return plan


def _one_query(idx: PredIndex, q: int, seed: int, lo: float, hi: float, max_rows: int,
               max_patterns: int, empty_redraws: int = 0) -> Tuple[Plan, Dict]:
    """Query q of the mix, drawn from its own seeded stream (so queries can be
    drawn in any order or process and come out the same)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 0xBA7C, q])))
    # The pattern count and shape are drawn first and kept, so their laws are
    # the configured ones; the selectivities are drawn again while the join
    # prefix exceeds max_rows, and while the result is empty, up to
    # `empty_redraws` bounded draws (then the last bounded draw is kept, empty
    # or not).  A count and shape with no bounded draw in 200 tries (a rare
    # case) are drawn again.
    bounded = None
    empties = 0
    k = int(rng.integers(1, max_patterns + 1))
    shape = "star" if rng.random() < 0.5 else "chain"
    for attempt in range(100000):
        if bounded is None and attempt and attempt % 200 == 0:
            k = int(rng.integers(1, max_patterns + 1))
            shape = "star" if rng.random() < 0.5 else "chain"
        sig = 10.0 ** rng.uniform(lo, hi, size=k)
        terms = [_realise(idx, float(s), rng, shape == "star" or i == k - 1)
                 for i, s in enumerate(sig)]
        if shape == "star":
            pref = _star_prefix_counts(idx, terms)
        else:
            pref = _chain_prefix_counts(idx, terms, max_rows)
        pat_rows = [float(idx.start[t.p + 1] - idx.start[t.p]) for t in terms]
        if max(pref) <= max_rows:
            bounded = (k, shape, sig, terms, pref, pat_rows)
            if pref[-1] >= 1 or empties >= empty_redraws:
                break
            empties += 1
    k, shape, sig, terms, pref, pat_rows = bounded
    info = {"shape": shape, "k": k, "sigma": [float(s) for s in sig],
            "rows": int(pref[-1]), "prefix_rows": [int(x) for x in pref],
            "pattern_rows_max": int(max(pat_rows)), "attempts": attempt + 1}
    return _plan(shape, terms), info


_POOL_IDX = None   # the index forked workers read (copy-on-write)


def _pool_query(args):
    return _one_query(_POOL_IDX, *args)


def batch_queries(idx: PredIndex, nq: int = 1024, seed: int = 4, max_rows: int = 1 << 22,
                  sigma_range=(1e-6, 1e-1), max_patterns: int = 6,
                  workers: int | None = None, empty_redraws: int = 16
                  ) -> Tuple[List[Plan], List[Dict]]:
    """nq queries of the mix.  Large mixes are drawn by forked workers unless
    this process has initialised a GPU (then serially); the result does not
    depend on the number of workers."""
    global _POOL_IDX
    lo, hi = np.log10(sigma_range[0]), np.log10(sigma_range[1])
    jobs = [(q, seed, lo, hi, max_rows, max_patterns, empty_redraws) for q in range(nq)]
    if workers is None:
        workers = min(16, os.cpu_count() or 1)
    if workers <= 1 or nq < 64 or _gpu_initialised():
        res = [_one_query(idx, *j) for j in jobs]
    else:
        from concurrent.futures import ProcessPoolExecutor
        from multiprocessing import get_context
        _POOL_IDX = idx
        try:
            with ProcessPoolExecutor(max_workers=workers, mp_context=get_context("fork")) as ex:
                res = list(ex.map(_pool_query, jobs, chunksize=4))
        finally:
            _POOL_IDX = None
    return [r[0] for r in res], [r[1] for r in res]


def poisson_arrivals(n: int, qps: float, seed: int) -> np.ndarray:
    """Arrival times (seconds) of an open-loop Poisson process at rate qps
    (seeded exponential gaps)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 0x5E7E])))
    return np.cumsum(rng.exponential(1.0 / qps, size=n))
