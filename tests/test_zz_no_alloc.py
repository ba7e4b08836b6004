"""tid_scan_noalloc, the allocation-free scan (for callers that cannot
allocate device memory): through the C ABI, with output columns and the
count word allocated by the caller, its rows equal tid_scan's byte for byte,
on two calls in a row, the second on a smaller graph; plus the count-only
form, a result larger than the caller's capacity, and the empty graph."""
import ctypes

import numpy as np
import pytest

from synth import Pattern

pytestmark = pytest.mark.gpu


def scan_noalloc(ctx, G, p, cap):
    """Call tid_scan_noalloc with torch-allocated outputs; returns (rows, count)."""
    import torch
    from paper_1807_01409_amd import _lib as L
    from paper_1807_01409_amd.tid import _check, _pattern
    ncols = len(p.out_vars())
    cols = [torch.full((max(cap, 1),), 0xABCD, dtype=torch.int32, device="cuda")
            for _ in range(ncols)]
    count = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    ptrs = (ctypes.c_void_p * max(1, ncols))(*[c.data_ptr() for c in cols])
    q = _pattern(p)
    _check(ctx.ptr, ctx._lib.tid_scan_noalloc(ctx.ptr, G._p, ctypes.byref(q),
                                              ptrs if ncols else None, ncols, cap,
                                              ctypes.c_void_p(count.data_ptr())))
    ctx.synchronize()
    n = int(count.item())
    k = min(n, cap)
    rows = np.stack([c[:k].cpu().numpy().view(np.uint32) for c in cols], axis=1) if ncols \
        else np.zeros((k, 0), dtype=np.uint32)
    return rows, n


PATTERNS = [Pattern(0, 7, 0, 0, -1, 1), Pattern(0, 2, 0, 0, -1, 1),
            Pattern(0, 0, 0, 0, 1, 2, range_pos=2, lo=100, hi=5000),
            Pattern(0, 3, 0, 0, -1, 0), Pattern(5, 0, 0, -1, 0, 1)]


def test_noalloc_equals_scan_two_calls(ctx, graphs):
    big = graphs("medium", 3_000_000)
    small = graphs("small", 70001)
    for g in (big, small):                       # the second call has a smaller input
        G = ctx.load(g)
        for p in PATTERNS:
            want = ctx.scan(G, p).to_numpy()
            cap = G.count(1, p.p, p.p + 1) if p.p else g.shape[0]
            got, n = scan_noalloc(ctx, G, p, cap)
            assert n == want.shape[0]
            assert np.array_equal(got, want), (g.shape[0], p)
        G.free()


def test_noalloc_count_only_capacity_and_empty(ctx, graphs):
    g = graphs("small", 70001)
    G = ctx.load(g)
    p = Pattern(0, 7, 0, -1, -1, -1)              # no named variable: count only
    got, n = scan_noalloc(ctx, G, p, 0)
    assert got.shape == (0, 0) and n == int((g[:, 1] == 7).sum())
    p = Pattern(0, 7, 0, 0, -1, 1)
    want = ctx.scan(G, p).to_numpy()
    got, n = scan_noalloc(ctx, G, p, 100)         # fewer rows than the result
    assert n == want.shape[0] > 100
    assert np.array_equal(got, want[:100])
    G.free()
    E = ctx.load(np.zeros((0, 3), dtype=np.uint32))
    got, n = scan_noalloc(ctx, E, p, 10)
    assert n == 0 and got.shape == (0, 2)
    E.free()


def test_noalloc_scans_replayed_from_a_hip_graph(ctx, graphs):
    """The allocation-free scan is the fixed-shape part of the path a caller
    can record in a HIP graph: three scans into caller buffers are captured
    once and replayed five times, with other scans (eager, other patterns) run
    between the replays; every replay equals tid_scan's rows."""
    import torch
    from paper_1807_01409_amd.tid import _check, _pattern
    g = graphs("medium", 3_000_000)
    G = ctx.load(g)
    pats = [Pattern(0, 2, 0, 0, -1, 1), Pattern(0, 14, 0, 0, -1, 1),
            Pattern(0, 0, 0, 0, 1, 2, range_pos=2, lo=1000, hi=90000)]
    want = [ctx.scan(G, p).to_numpy() for p in pats]
    bufs = []
    for p, w in zip(pats, want):
        cap = w.shape[0] + 16
        cols = [torch.zeros(cap, dtype=torch.int32, device="cuda") for _ in range(w.shape[1])]
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        bufs.append((p, cols, cnt, cap))
    keep = []

    def enqueue():
        for p, cols, cnt, cap in bufs:
            ptrs = (ctypes.c_void_p * len(cols))(*[c.data_ptr() for c in cols])
            q = _pattern(p)
            keep.append((ptrs, q))
            _check(ctx.ptr, ctx._lib.tid_scan_noalloc(ctx.ptr, G._p, ctypes.byref(q), ptrs,
                                                      len(cols), cap,
                                                      ctypes.c_void_p(cnt.data_ptr())))

    enqueue()                     # warm-up outside the capture
    ctx.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=ctx.stream, capture_error_mode="relaxed"):
        enqueue()
    other = Pattern(0, 7, 0, 0, -1, 1)
    for rep in range(5):
        for _, cols, cnt, _ in bufs:
            for c in cols:
                c.fill_(-1)
            cnt.fill_(-1)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for (p, cols, cnt, cap), w in zip(bufs, want):
            n = int(cnt.item())
            assert n == w.shape[0], (rep, p)
            got = np.stack([c[:n].cpu().numpy().view(np.uint32) for c in cols], axis=1)
            assert np.array_equal(got, w), (rep, p)
        ctx.scan(G, other).free()                   # eager work between replays
        scan_noalloc(ctx, G, other, G.count(1, 7, 8))
        ctx.synchronize()
    G.free()
