"""CPU oracle for the TripleID-Q query path -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark import this package.  It wraps the plain C oracle in oracle.c
(built with gcc into liboracle.so) and a tiny dictionary encoder; it shares
no code with the GPU library and never loads it.

Parity status: every function here is pinned by tests against values the
paper prints, brute force on tiny inputs, or invariants (see the oracle pin
tests).  None is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import List, Sequence

import numpy as np

from .encode import decode_row, encode_graph

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
MAXCOLS = 32


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain -O2)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
             "-o", tmp, os.path.join(_HERE, "oracle.c")])
        os.replace(tmp, _SO)
    return _SO


class _Pat(ctypes.Structure):
    _fields_ = [("c", ctypes.c_uint32 * 3), ("v", ctypes.c_int32 * 3),
                ("range_pos", ctypes.c_int32), ("lo", ctypes.c_uint32),
                ("hi", ctypes.c_uint32)]


class _Tab(ctypes.Structure):
    _fields_ = [("rows", ctypes.POINTER(ctypes.c_uint32)), ("nrows", ctypes.c_uint64),
                ("ncols", ctypes.c_int32), ("vars", ctypes.c_int32 * MAXCOLS)]


_lib = None


def _setup(lib):
    """Declare the C signatures on a loaded liboracle."""
    P = ctypes.POINTER
    u32p = P(ctypes.c_uint32)
    lib.or_scan_flags.argtypes = [u32p, ctypes.c_uint64, P(_Pat), P(ctypes.c_uint8)]
    lib.or_scan_multi.argtypes = [u32p, ctypes.c_uint64, P(_Pat), ctypes.c_int32,
                                  P(ctypes.c_uint64)]
    lib.or_scan.argtypes = [u32p, ctypes.c_uint64, P(_Pat), P(_Tab)]
    lib.or_filter.argtypes = [P(_Tab), ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint32,
                              P(_Tab)]
    lib.or_join_nested.argtypes = [P(_Tab), ctypes.c_int32, P(_Tab), ctypes.c_int32, P(_Tab)]
    lib.or_join_sortmerge.argtypes = [P(_Tab), ctypes.c_int32, P(_Tab), ctypes.c_int32,
                                      P(_Tab)]
    lib.or_join_outer.argtypes = [P(_Tab), ctypes.c_int32, P(_Tab), ctypes.c_int32,
                                  ctypes.c_int32, P(_Tab)]
    lib.or_scan_keyed.argtypes = [u32p, ctypes.c_uint64, P(_Pat), ctypes.c_int32, u32p,
                                  ctypes.c_uint64, P(_Tab)]
    lib.or_entail.argtypes = [u32p, ctypes.c_uint64, ctypes.c_int32, u32p, P(_Tab)]
    lib.or_union.argtypes = [P(P(_Tab)), ctypes.c_int32, ctypes.c_int32, P(_Tab)]
    lib.or_sort_rows.argtypes = [P(_Tab)]
    lib.or_distinct.argtypes = [P(_Tab)]
    lib.or_query.argtypes = [u32p, ctypes.c_uint64, P(_Pat), ctypes.c_int32, u32p,
                             ctypes.c_int32, P(_Tab)]
    lib.or_table_free.argtypes = [P(_Tab)]
    lib.or_table_free.restype = None
    lib.or_set_nested_join_limit.argtypes = [ctypes.c_double]
    lib.or_set_nested_join_limit.restype = None
    return lib


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        _lib = _setup(ctypes.CDLL(_SO))
    return _lib


class OracleError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"oracle {what} failed with status {status}")
        self.status = status


@dataclass
class Table:
    """A result table: rows (nrows, ncols) uint32 and one variable id per column."""
    rows: np.ndarray
    vars: List[int] = field(default_factory=list)

    @property
    def nrows(self) -> int:
        return int(self.rows.shape[0])

    @property
    def ncols(self) -> int:
        return int(self.rows.shape[1])


def _graph(g) -> np.ndarray:
    g = np.ascontiguousarray(g, dtype=np.uint32)
    if g.ndim != 2 or g.shape[1] != 3:
        raise ValueError("graph must be an (N, 3) uint32 array")
    return g


def _u32p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def _pat(p) -> _Pat:
    q = _Pat()
    q.c[0], q.c[1], q.c[2] = int(p.s), int(p.p), int(p.o)
    q.v[0], q.v[1], q.v[2] = int(p.vs), int(p.vp), int(p.vo)
    q.range_pos, q.lo, q.hi = int(p.range_pos), int(p.lo), int(p.hi)
    return q


def _to_c(t: Table, keep: list) -> _Tab:
    rows = np.ascontiguousarray(t.rows, dtype=np.uint32)
    if rows.ndim != 2:
        raise ValueError("table rows must be 2-D")
    keep.append(rows)
    c = _Tab()
    c.rows = _u32p(rows) if rows.size else ctypes.POINTER(ctypes.c_uint32)()
    c.nrows = rows.shape[0]
    c.ncols = rows.shape[1]
    for i, v in enumerate(t.vars):
        c.vars[i] = v
    return c


def _from_c(c: _Tab) -> Table:
    n, k = int(c.nrows), int(c.ncols)
    if n and k:
        rows = np.ctypeslib.as_array(c.rows, shape=(n * k,)).copy().reshape(n, k)
    else:
        rows = np.zeros((n, k), dtype=np.uint32)
    t = Table(rows, [int(c.vars[i]) for i in range(k)])
    _L().or_table_free(ctypes.byref(c))
    return t


def _check(st: int, what: str):
    if st != 0:
        raise OracleError(st, what)


def scan_flags(g, p) -> np.ndarray:
    g = _graph(g)
    out = np.zeros(g.shape[0], dtype=np.uint8)
    q = _pat(p)
    _check(_L().or_scan_flags(_u32p(g), g.shape[0], ctypes.byref(q),
                              out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))), "scan_flags")
    return out


def scan_multi(g, pats: Sequence) -> np.ndarray:
    g = _graph(g)
    arr = (_Pat * max(1, len(pats)))(*[_pat(p) for p in pats])
    out = np.zeros(g.shape[0], dtype=np.uint64)
    _check(_L().or_scan_multi(_u32p(g), g.shape[0], arr, len(pats),
                              out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))), "scan_multi")
    return out


def scan(g, p) -> Table:
    g = _graph(g)
    q = _pat(p)
    res = _Tab()
    _check(_L().or_scan(_u32p(g), g.shape[0], ctypes.byref(q), ctypes.byref(res)), "scan")
    return _from_c(res)


def filter(t: Table, col: int, lo: int, hi: int) -> Table:  # noqa: A001 - paper's name
    keep: list = []
    a = _to_c(t, keep)
    res = _Tab()
    _check(_L().or_filter(ctypes.byref(a), col, lo, hi, ctypes.byref(res)), "filter")
    return _from_c(res)


def join(l: Table, lc: int, r: Table, rc: int, method: str = "nested") -> Table:
    keep: list = []
    a, b = _to_c(l, keep), _to_c(r, keep)
    res = _Tab()
    fn = _L().or_join_nested if method == "nested" else _L().or_join_sortmerge
    _check(fn(ctypes.byref(a), lc, ctypes.byref(b), rc, ctypes.byref(res)), "join")
    return _from_c(res)


def scan_keyed(g, p, pos: int, keys) -> Table:
    """Bindings of the triples matching p whose value at `pos` is in keys."""
    g = _graph(g)
    k = np.ascontiguousarray(np.asarray(keys, dtype=np.uint32).ravel())
    q = _pat(p)
    res = _Tab()
    _check(_L().or_scan_keyed(_u32p(g), g.shape[0], ctypes.byref(q), int(pos),
                              _u32p(k) if k.size else ctypes.POINTER(ctypes.c_uint32)(),
                              k.size, ctypes.byref(res)), "scan_keyed")
    return _from_c(res)


RDFS_VOCAB = ("type", "subClassOf", "subPropertyOf", "domain", "range")


def entail(g, rule: int, vocab) -> Table:
    """Triples derived by RDFS rule 2, 3, 5, 7, 9 or 11; vocab = IDs of
    rdf:type, rdfs:subClassOf, rdfs:subPropertyOf, rdfs:domain, rdfs:range."""
    g = _graph(g)
    v = np.ascontiguousarray(np.asarray(vocab, dtype=np.uint32))
    assert v.size == 5
    res = _Tab()
    _check(_L().or_entail(_u32p(g), g.shape[0], int(rule), _u32p(v), ctypes.byref(res)),
           "entail")
    return _from_c(res)


JOIN_KINDS = {"inner": 0, "left": 1, "right": 2, "full": 3}


def join_outer(l: Table, lc: int, r: Table, rc: int, kind: str = "left") -> Table:
    """Inner/left/right/full join by nested loops (or_join_outer)."""
    keep: list = []
    a, b = _to_c(l, keep), _to_c(r, keep)
    res = _Tab()
    _check(_L().or_join_outer(ctypes.byref(a), lc, ctypes.byref(b), rc, JOIN_KINDS[kind],
                              ctypes.byref(res)), "join_outer")
    return _from_c(res)


def union(ts: Sequence[Table], dedupe: bool) -> Table:
    keep: list = []
    cs = [_to_c(t, keep) for t in ts]
    ptrs = (ctypes.POINTER(_Tab) * len(cs))(*[ctypes.pointer(c) for c in cs])
    res = _Tab()
    _check(_L().or_union(ptrs, len(cs), int(bool(dedupe)), ctypes.byref(res)), "union")
    return _from_c(res)


def sort_rows(t: Table) -> Table:
    keep: list = []
    a = _to_c(Table(t.rows.copy(), list(t.vars)), keep)
    _check(_L().or_sort_rows(ctypes.byref(a)), "sort_rows")
    return Table(keep[0], list(t.vars))


def distinct(t: Table) -> Table:
    keep: list = []
    a = _to_c(Table(t.rows.copy(), list(t.vars)), keep)
    _check(_L().or_distinct(ctypes.byref(a)), "distinct")
    return Table(keep[0][: int(a.nrows)].copy(), list(t.vars))


def set_nested_join_limit(pairs: float) -> None:
    """Plan joins above this many row pairs use sort-merge (default 1e8)."""
    _L().or_set_nested_join_limit(float(pairs))


def query(g, plan) -> Table:
    g = _graph(g)
    pats = (_Pat * max(1, len(plan.patterns)))(*[_pat(p) for p in plan.patterns])
    ops = np.ascontiguousarray(np.asarray(plan.ops, dtype=np.int64).astype(np.uint32))
    res = _Tab()
    _check(_L().or_query(_u32p(g), g.shape[0], pats, len(plan.patterns), _u32p(ops),
                         len(ops), ctypes.byref(res)), "query")
    return _from_c(res)


__all__ = ["build", "Table", "OracleError", "scan_flags", "scan_multi", "scan",
           "filter", "join", "union", "sort_rows", "distinct", "query", "encode_graph",
           "decode_row", "join_outer", "JOIN_KINDS", "scan_keyed", "entail", "RDFS_VOCAB"]
