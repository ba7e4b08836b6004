"""Python binding of libtid: argument marshalling over the C ABI only.

Every function named tid_* here calls the C entry point of the same name;
every step of the query path runs in the library's HIP kernels.  PyTorch
supplies the stream, and optionally the device memory (its caching
allocator, through the allocation callbacks); by default the library's own
native pool allocates.
"""
from __future__ import annotations

import atexit
import ctypes
import weakref
from typing import List, Optional, Sequence

import numpy as np

from . import _lib as L


class TidError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{L.STATUS.get(status, status)}: {msg}")
        self.status = status


def _check(ctx_ptr, st: int):
    if st != 0:
        lib = L.load_library()
        msg = lib.tid_last_error(ctx_ptr).decode() if ctx_ptr else ""
        raise TidError(st, msg)


def _pattern(p) -> L.tid_pattern:
    return L.tid_pattern(int(p.s), int(p.p), int(p.o), int(p.vs), int(p.vp), int(p.vo),
                         int(p.range_pos), int(p.lo), int(p.hi))


_LIVE: "weakref.WeakSet" = weakref.WeakSet()


@atexit.register
def _close_all():
    """Close contexts before the interpreter tears torch down (their free
    callbacks call into torch)."""
    for c in list(_LIVE):
        try:
            c.close()
        except Exception:  # noqa: BLE001
            pass


class Context:
    """A tid_ctx bound to one device and stream.

    The context enqueues on `stream` (a torch.cuda.Stream); by default it makes
    a stream of its own, so that its work never rides on the legacy default
    stream.  allocator="pool" (default) uses the library's own native pool;
    allocator="torch" routes device memory through torch's caching allocator
    on that stream (one Python callback per allocation), for callers that
    share memory accounting with torch."""

    def __init__(self, device: int = 0, stream=None, allocator: str = "pool"):
        import torch
        lib = L.load_library()
        self._torch = torch
        self.device = int(device)
        torch.cuda.set_device(self.device)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        if int(self.stream.cuda_stream) == 0:
            raise ValueError("pass a non-default stream (the legacy default stream has handle 0)")
        sptr = ctypes.c_void_p(int(self.stream.cuda_stream))
        if allocator == "torch":
            dev = self.device

            def _alloc(user, nbytes, stream):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), dev, int(stream or 0))
                except Exception:  # noqa: BLE001 - reported to the library as NULL (OOM)
                    return None

            def _free(user, ptr, nbytes, stream):
                if torch.cuda is not None:
                    torch.cuda.caching_allocator_delete(int(ptr))

            self._cb = (L.ALLOC_FN(_alloc), L.FREE_FN(_free))
        elif allocator == "pool":
            self._cb = (L.ALLOC_FN(), L.FREE_FN())
        else:
            raise ValueError("allocator must be 'torch' or 'pool'")
        out = ctypes.c_void_p()
        st = lib.tid_ctx_create(self.device, sptr, self._cb[0], self._cb[1], None,
                                ctypes.byref(out))
        if st != 0:
            raise TidError(st, "tid_ctx_create failed")
        self._p = out
        self._lib = lib
        _LIVE.add(self)

    # -- lifetime ---------------------------------------------------------
    def close(self):
        if getattr(self, "_p", None):
            self._lib.tid_ctx_synchronize(self._p)
            self._lib.tid_ctx_destroy(self._p)
            self._p = None

    def __del__(self):  # pragma: no cover - interpreter shutdown order
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def ptr(self):
        return self._p

    # -- options ------------------------------------------------------------
    def set_option(self, key: str, value: int):
        _check(self._p, self._lib.tid_ctx_set_option(self._p, key.encode(), int(value)))

    def get_option(self, key: str) -> int:
        v = ctypes.c_int64()
        _check(self._p, self._lib.tid_ctx_get_option(self._p, key.encode(), ctypes.byref(v)))
        return int(v.value)

    def synchronize(self):
        _check(self._p, self._lib.tid_ctx_synchronize(self._p))

    # -- graph --------------------------------------------------------------
    def load(self, triples) -> "Graph":
        return tid_load(self, triples)

    # -- operators -------------------------------------------------------------
    def scan(self, g: "Graph", pattern) -> "Table":
        return tid_scan(self, g, pattern)

    def scan_multi(self, g: "Graph", patterns) -> List["Table"]:
        return tid_scan_multi(self, g, patterns)

    def filter(self, t: "Table", col: int, lo: int, hi: int) -> "Table":
        return tid_filter(self, t, col, lo, hi)

    def join(self, l: "Table", lcol: int, r: "Table", rcol: int, algo: int = 0) -> "Table":
        return tid_join(self, l, lcol, r, rcol, algo)

    def join_outer(self, l: "Table", lcol: int, r: "Table", rcol: int, kind: str = "left",
                   algo: int = 0) -> "Table":
        return tid_join_outer(self, l, lcol, r, rcol, kind, algo)

    def union(self, ts: Sequence["Table"], dedupe: bool) -> "Table":
        return tid_union(self, ts, dedupe)

    def sort(self, t: "Table", distinct: bool = False) -> "Table":
        return tid_sort(self, t, distinct)

    def query(self, g: "Graph", plan) -> "Table":
        return tid_query(self, g, plan)

    def query_batch(self, g: "Graph", plans) -> List["Table"]:
        return tid_query_batch(self, g, plans)

    def plan_estimate(self, g: "Graph", plan) -> int:
        return tid_plan_estimate(self, g, plan)

    def scan_keyed(self, g: "Graph", pattern, pos: int, keys: "Table", col: int = 0) -> "Table":
        return tid_scan_keyed(self, g, pattern, pos, keys, col)

    def entail(self, g: "Graph", rule: int, vocab) -> "Table":
        return tid_entail(self, g, rule, vocab)

    def encode(self, triples):
        return tid_encode(self, triples)

    def read_probe(self, device_ptr: int, nbytes: int, mode: int = 0):
        tid_read_probe(self, device_ptr, nbytes, mode)

    def table(self, rows: np.ndarray, vars_: Sequence[int]) -> "Table":
        return tid_table_from_columns(self, rows, vars_)


class Graph:
    def __init__(self, ctx: Context, ptr):
        self.ctx = ctx
        self._p = ptr
        n = ctypes.c_uint64()
        d = ctypes.c_void_p()
        _check(ctx.ptr, ctx._lib.tid_graph_info(ptr, ctypes.byref(n), ctypes.byref(d)))
        self.n = int(n.value)
        self.device_ptr = int(d.value or 0)

    def partition(self, enable: bool = True):
        _check(self.ctx.ptr, self.ctx._lib.tid_graph_partition(self.ctx.ptr, self._p,
                                                               int(bool(enable))))

    def count(self, pos: int, lo: int, hi: int) -> int:
        return tid_graph_count(self, pos, lo, hi)

    def free(self):
        if self._p:
            self.ctx._lib.tid_graph_free(self._p)
            self._p = None

    def __del__(self):  # pragma: no cover
        try:
            if self._p and self.ctx._p:
                self.free()
        except Exception:  # noqa: BLE001
            pass


class Table:
    def __init__(self, ctx: Context, ptr):
        self.ctx = ctx
        self._p = ptr

    def info(self):
        n = ctypes.c_uint64()
        k = ctypes.c_int32()
        vs = (ctypes.c_int32 * L.TID_MAX_COLS)()
        _check(self.ctx.ptr, self.ctx._lib.tid_table_info(self.ctx.ptr, self._p, ctypes.byref(n),
                                                          ctypes.byref(k), vs))
        return int(n.value), int(k.value), [int(vs[i]) for i in range(k.value)]

    @property
    def nrows(self) -> int:
        return self.info()[0]

    @property
    def ncols(self) -> int:
        return self.info()[1]

    @property
    def vars(self) -> List[int]:
        return self.info()[2]

    def column_ptr(self, c: int) -> int:
        d = ctypes.c_void_p()
        _check(self.ctx.ptr, self.ctx._lib.tid_table_column(self._p, c, ctypes.byref(d)))
        return int(d.value or 0)

    def to_numpy(self) -> np.ndarray:
        n, k, _ = self.info()
        out = np.zeros((n, k), dtype=np.uint32)
        if n and k:
            _check(self.ctx.ptr, self.ctx._lib.tid_table_to_host(
                self.ctx.ptr, self._p, out.ctypes.data_as(ctypes.c_void_p), n))
        return out

    def free(self):
        if self._p:
            self.ctx._lib.tid_table_free(self._p)
            self._p = None

    def __del__(self):  # pragma: no cover
        try:
            if self._p and self.ctx._p:
                self.free()
        except Exception:  # noqa: BLE001
            pass


# ---------------------------------------------------------------------------
# entry points, same names as the C ABI
# ---------------------------------------------------------------------------

def tid_load(ctx: Context, triples) -> Graph:
    out = ctypes.c_void_p()
    torch = ctx._torch
    if isinstance(triples, torch.Tensor):
        if triples.dtype not in (torch.int32, torch.uint32) or triples.dim() != 2 \
                or triples.shape[1] != 3:
            raise ValueError("triples must be an (N, 3) 32-bit tensor")
        t = triples.contiguous()
        on_dev = 1 if t.is_cuda else 0
        _check(ctx.ptr, ctx._lib.tid_load(ctx.ptr, ctypes.c_void_p(t.data_ptr()), t.shape[0],
                                          on_dev, ctypes.byref(out)))
    else:
        a = np.ascontiguousarray(triples, dtype=np.uint32)
        if a.ndim != 2 or a.shape[1] != 3:
            raise ValueError("triples must be an (N, 3) uint32 array")
        _check(ctx.ptr, ctx._lib.tid_load(ctx.ptr, a.ctypes.data_as(ctypes.c_void_p),
                                          a.shape[0], 0, ctypes.byref(out)))
    return Graph(ctx, out)


def tid_load_file(ctx: Context, path: str) -> Graph:
    out = ctypes.c_void_p()
    _check(ctx.ptr, ctx._lib.tid_load_file(ctx.ptr, path.encode(), ctypes.byref(out)))
    return Graph(ctx, out)


def tid_read_probe(ctx: Context, device_ptr: int, nbytes: int, mode: int = 0) -> None:
    _check(ctx.ptr, ctx._lib.tid_read_probe(ctx.ptr, ctypes.c_void_p(int(device_ptr)),
                                            int(nbytes), int(mode)))


def tid_graph_count(g: Graph, pos: int, lo: int, hi: int) -> int:
    v = ctypes.c_uint64()
    _check(g.ctx.ptr, g.ctx._lib.tid_graph_count(g._p, int(pos), int(lo), int(hi),
                                                 ctypes.byref(v)))
    return int(v.value)


def tid_scan(ctx: Context, g: Graph, pattern) -> Table:
    out = ctypes.c_void_p()
    q = _pattern(pattern)
    _check(ctx.ptr, ctx._lib.tid_scan(ctx.ptr, g._p, ctypes.byref(q), ctypes.byref(out)))
    return Table(ctx, out)


def tid_scan_multi(ctx: Context, g: Graph, patterns) -> List[Table]:
    k = len(patterns)
    arr = (L.tid_pattern * k)(*[_pattern(p) for p in patterns])
    outs = (ctypes.c_void_p * k)()
    _check(ctx.ptr, ctx._lib.tid_scan_multi(ctx.ptr, g._p, arr, k, outs))
    return [Table(ctx, ctypes.c_void_p(outs[j])) for j in range(k)]


def tid_scan_keyed(ctx: Context, g: Graph, pattern, pos: int, keys: Table, col: int = 0) -> Table:
    out = ctypes.c_void_p()
    q = _pattern(pattern)
    _check(ctx.ptr, ctx._lib.tid_scan_keyed(ctx.ptr, g._p, ctypes.byref(q), int(pos), keys._p,
                                            int(col), ctypes.byref(out)))
    return Table(ctx, out)


def tid_entail(ctx: Context, g: Graph, rule: int, vocab) -> Table:
    v = (ctypes.c_uint32 * 5)(*[int(x) for x in vocab])
    out = ctypes.c_void_p()
    _check(ctx.ptr, ctx._lib.tid_entail(ctx.ptr, g._p, int(rule), v, ctypes.byref(out)))
    return Table(ctx, out)


class Dict:
    """A term dictionary on the device (tid_encode's output)."""

    def __init__(self, ctx: Context, ptr):
        self.ctx = ctx
        self._p = ptr

    def info(self):
        n, b = ctypes.c_uint64(), ctypes.c_uint64()
        _check(self.ctx.ptr, self.ctx._lib.tid_dict_info(self._p, ctypes.byref(n), ctypes.byref(b)))
        return int(n.value), int(b.value)

    def decode(self, ids) -> List[str]:
        return tid_decode(self.ctx, self, ids)

    def free(self):
        if self._p:
            self.ctx._lib.tid_dict_free(self._p)
            self._p = None

    def __del__(self):  # pragma: no cover
        try:
            if self._p and self.ctx._p:
                self.free()
        except Exception:  # noqa: BLE001
            pass


def tid_encode(ctx: Context, triples):
    """Encode string triples on the GPU; returns ((n, 3) uint32 rows, Dict).
    Marshalling only: the terms are UTF-8 encoded and laid out as bytes and
    3n + 1 offsets."""
    torch = ctx._torch
    terms = [str(x).encode("utf-8") for t in triples for x in t]
    if len(terms) % 3:
        raise ValueError("triples must have three terms each")
    n = len(terms) // 3
    blob = b"".join(terms)
    off = np.zeros(len(terms) + 1, dtype=np.uint64)
    if terms:
        off[1:] = np.cumsum([len(x) for x in terms], dtype=np.uint64)
    buf = np.frombuffer(blob, dtype=np.uint8) if blob else np.zeros(1, np.uint8)
    rows = torch.empty(max(1, 3 * n), dtype=torch.int32, device=f"cuda:{ctx.device}")
    out = ctypes.c_void_p()
    _check(ctx.ptr, ctx._lib.tid_encode(ctx.ptr, buf.ctypes.data_as(ctypes.c_void_p), len(blob),
                                        off.ctypes.data_as(ctypes.c_void_p), n, 0,
                                        ctypes.c_void_p(rows.data_ptr()), ctypes.byref(out)))
    ctx.synchronize()
    r = rows[:3 * n].cpu().numpy().view(np.uint32).reshape(n, 3)
    return r, Dict(ctx, out)


def tid_decode(ctx: Context, d: Dict, ids) -> List[str]:
    a = np.ascontiguousarray(np.asarray(ids, dtype=np.uint32).ravel())
    n = a.size
    off = np.zeros(n + 1, dtype=np.uint64)
    st = ctx._lib.tid_decode(ctx.ptr, d._p, a.ctypes.data_as(ctypes.c_void_p), n, 0,
                             off.ctypes.data_as(ctypes.c_void_p), None, 0)
    total = int(off[n]) if st in (0, -3) else 0
    if st not in (0, -3):
        _check(ctx.ptr, st)
    buf = np.zeros(max(1, total), dtype=np.uint8)
    if total:
        _check(ctx.ptr, ctx._lib.tid_decode(ctx.ptr, d._p, a.ctypes.data_as(ctypes.c_void_p), n,
                                            0, off.ctypes.data_as(ctypes.c_void_p),
                                            buf.ctypes.data_as(ctypes.c_void_p), total))
    raw = buf.tobytes()
    return [raw[int(off[i]):int(off[i + 1])].decode("utf-8") for i in range(n)]


def tid_filter(ctx: Context, t: Table, col: int, lo: int, hi: int) -> Table:
    out = ctypes.c_void_p()
    _check(ctx.ptr, ctx._lib.tid_filter(ctx.ptr, t._p, int(col), int(lo), int(hi),
                                        ctypes.byref(out)))
    return Table(ctx, out)


def tid_join(ctx: Context, l: Table, lcol: int, r: Table, rcol: int, algo: int = 0) -> Table:
    out = ctypes.c_void_p()
    _check(ctx.ptr, ctx._lib.tid_join(ctx.ptr, l._p, int(lcol), r._p, int(rcol), int(algo),
                                      ctypes.byref(out)))
    return Table(ctx, out)


JOIN_KINDS = {"inner": 0, "left": 1, "right": 2, "full": 3}


def tid_join_outer(ctx: Context, l: Table, lcol: int, r: Table, rcol: int, kind="left",
                   algo: int = 0) -> Table:
    out = ctypes.c_void_p()
    k = JOIN_KINDS[kind] if isinstance(kind, str) else int(kind)
    _check(ctx.ptr, ctx._lib.tid_join_outer(ctx.ptr, l._p, int(lcol), r._p, int(rcol), k,
                                            int(algo), ctypes.byref(out)))
    return Table(ctx, out)


def tid_union(ctx: Context, ts: Sequence[Table], dedupe: bool) -> Table:
    k = len(ts)
    arr = (ctypes.c_void_p * k)(*[t._p.value if isinstance(t._p, ctypes.c_void_p) else t._p
                                  for t in ts])
    out = ctypes.c_void_p()
    _check(ctx.ptr, ctx._lib.tid_union(ctx.ptr, arr, k, int(bool(dedupe)), ctypes.byref(out)))
    return Table(ctx, out)


def tid_sort(ctx: Context, t: Table, distinct: bool = False) -> Table:
    out = ctypes.c_void_p()
    _check(ctx.ptr, ctx._lib.tid_sort(ctx.ptr, t._p, int(bool(distinct)), ctypes.byref(out)))
    return Table(ctx, out)


def _plan(plan, keep: list) -> L.tid_plan:
    pats = (L.tid_pattern * max(1, len(plan.patterns)))(*[_pattern(p) for p in plan.patterns])
    ops = np.ascontiguousarray(np.asarray(plan.ops, dtype=np.int64).astype(np.uint32))
    keep.extend([pats, ops])
    return L.tid_plan(len(plan.patterns), pats, len(ops),
                      ops.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))


def tid_query_batch(ctx: Context, g: Graph, plans) -> List[Table]:
    keep: list = []
    cps = [_plan(p, keep) for p in plans]
    arr = (ctypes.POINTER(L.tid_plan) * max(1, len(cps)))(*[ctypes.pointer(c) for c in cps])
    outs = (ctypes.c_void_p * max(1, len(cps)))()
    _check(ctx.ptr, ctx._lib.tid_query_batch(ctx.ptr, g._p, arr, len(cps), outs))
    return [Table(ctx, ctypes.c_void_p(outs[i])) for i in range(len(cps))]


def tid_plan_estimate(ctx: Context, g: Graph, plan) -> int:
    keep: list = []
    cp = _plan(plan, keep)
    v = ctypes.c_uint64()
    _check(ctx.ptr, ctx._lib.tid_plan_estimate(ctx.ptr, g._p, ctypes.byref(cp), ctypes.byref(v)))
    return int(v.value)


def tid_query(ctx: Context, g: Graph, plan) -> Table:
    keep: list = []
    cp = _plan(plan, keep)
    out = ctypes.c_void_p()
    _check(ctx.ptr, ctx._lib.tid_query(ctx.ptr, g._p, ctypes.byref(cp), ctypes.byref(out)))
    return Table(ctx, out)


def tid_table_from_columns(ctx: Context, rows: np.ndarray, vars_: Sequence[int]) -> Table:
    a = np.asarray(rows, dtype=np.uint32)
    if a.ndim != 2:
        raise ValueError("rows must be 2-D")
    k = a.shape[1]
    cols = [np.ascontiguousarray(a[:, c]) for c in range(k)]
    ptrs = (ctypes.c_void_p * max(1, k))(*[c.ctypes.data for c in cols])
    vs = (ctypes.c_int32 * max(1, k))(*[int(v) for v in vars_])
    out = ctypes.c_void_p()
    _check(ctx.ptr, ctx._lib.tid_table_from_columns(ctx.ptr, ptrs, k, vs, a.shape[0], 0,
                                                    ctypes.byref(out)))
    return Table(ctx, out)
