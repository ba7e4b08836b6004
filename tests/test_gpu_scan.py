"""GPU parity of the scan (Sec. 3, GPUSearch), the multi-pattern pass
(Sec. 4.1) and the range filter (Sec. 4.3) against the CPU oracle: results
must be byte-identical, rows in ascending triple position."""
import itertools

import numpy as np
import pytest

import oracle
from oracle_pins import VAR_LAYOUTS, _layout_pattern, tiny_graph
from synth import Pattern, pat

pytestmark = pytest.mark.gpu


def same(gpu_table, ora):
    got = gpu_table.to_numpy()
    assert gpu_table.vars == ora.vars
    assert got.shape == ora.rows.shape, (got.shape, ora.rows.shape)
    assert np.array_equal(got, ora.rows)


def test_scan_small_config(ctx, graphs):
    g = graphs("small")
    G = ctx.load(g)
    for p in (pat("?s 7 ?o"), pat("?s 3 ?o"), pat("?s ?p ?o"), pat("? 11 ?o"),
              Pattern(0, 0, 0, 0, 1, 2, range_pos=2, lo=1, hi=500)):
        same(ctx.scan(G, p), oracle.scan(g, p))


def test_scan_exhaustive_tiny(ctx):
    for seed in (0, 1):
        g = tiny_graph(seed, 15, 4)
        g = np.concatenate([g, g[:4]])
        G = ctx.load(g)
        for consts in itertools.product(range(5), repeat=3):
            for layout in VAR_LAYOUTS[:6]:
                for rs in (None, (2, 2, 4)):
                    p = _layout_pattern(consts, layout, rs)
                    t = ctx.scan(G, p)
                    o = oracle.scan(g, p)
                    assert t.nrows == o.nrows, (p,)
                    same(t, o)


@pytest.mark.parametrize("n", [1, 63, 64, 65, 255, 4095, 4096, 4097, 3 * 4096 + 17, 70001])
def test_scan_ragged_sizes(ctx, graphs, n):
    g = graphs("small", n)
    G = ctx.load(g)
    assert G.n == n
    fully = Pattern(int(g[n // 2, 0]), int(g[n // 2, 1]), int(g[n // 2, 2]))
    for p in (pat("?s ?p ?o"), pat("?s 7 ?o"), fully, pat("?s 999 ?o"),
              Pattern(0, 0, 0, 0, -1, 1, range_pos=0, lo=1, hi=0xFFFFFFFF),
              Pattern(0, 5, 0)):
        same(ctx.scan(G, p), oracle.scan(g, p))


def test_scan_empty_graph(ctx):
    g = np.zeros((0, 3), dtype=np.uint32)
    G = ctx.load(g)
    t = ctx.scan(G, pat("?s ?p ?o"))
    assert t.nrows == 0 and t.vars == [0, 1, 2]


def test_scan_hot_key(ctx):
    rng = np.random.default_rng(5)
    n = 200_000
    g = rng.integers(1, 5000, size=(n, 3)).astype(np.uint32)
    g[rng.random(n) < 0.10, 1] = 1          # one predicate holds ~10% of the rows
    G = ctx.load(g)
    for p in (pat("?s 1 ?o"), pat("?s ?p 17"), pat("?x 1 ?x")):
        same(ctx.scan(G, p), oracle.scan(g, p))


def test_scan_medium_selectivities(ctx, graphs):
    g = graphs("medium", 5_000_000)
    G = ctx.load(g)
    hist = np.bincount(g[:, 1])
    n = g.shape[0]
    for sigma in (1e-3, 1e-2, 1e-1):
        p_id = int(np.argmin(np.abs(np.log(np.maximum(hist, 1) / n) - np.log(sigma))))
        p = Pattern(0, p_id, 0, 0, -1, 1)
        t = ctx.scan(G, p)
        assert t.nrows == hist[p_id]
        same(t, oracle.scan(g, p))


def test_scan_shapes_and_repeats_identical(ctx, graphs):
    g = graphs("medium", 1_000_000)
    G = ctx.load(g)
    p = pat("?s 2 ?o")
    want = oracle.scan(g, p).rows
    shapes = [(256, 16), (256, 8), (256, 32), (512, 8), (512, 16), (1024, 4), (1024, 8),
              (128, 16), (128, 32)]
    try:
        for b, i in shapes:
            ctx.set_option("scan_block", b)
            ctx.set_option("scan_items", i)
            for _ in range(2):
                assert np.array_equal(ctx.scan(G, p).to_numpy(), want), (b, i)
    finally:
        ctx.set_option("scan_block", 0)
        ctx.set_option("scan_items", 0)


@pytest.mark.parametrize("k", [1, 2, 4, 5, 16])
def test_scan_multi(ctx, graphs, k):
    g = graphs("small")
    G = ctx.load(g)
    pats = [pat(f"?s {p} ?o") for p in range(1, k + 1)]
    pats[-1] = Pattern(0, 0, 0, 0, 1, 2, range_pos=2, lo=10, hi=90)
    outs = ctx.scan_multi(G, pats)
    for p, t in zip(pats, outs):
        same(t, oracle.scan(g, p))


def test_scan_multi_rule11_membership(ctx):
    # Sec. 5.7 Rule 11: the second search with keysArray {56,84,0, 77,84,0, 78,84,0}
    g = np.array([(76, 84, 56), (31, 84, 77), (56, 84, 78), (56, 84, 77), (44, 83, 2)],
                 dtype=np.uint32)
    G = ctx.load(g)
    outs = ctx.scan_multi(G, [Pattern(k, 84, 0, -1, -1, 0) for k in (56, 77, 78)])
    assert [t.to_numpy().ravel().tolist() for t in outs] == [[78, 77], [], []]


def test_capacity_override_retry(ctx, graphs):
    g = graphs("small")
    G = ctx.load(g)
    p = pat("?s 7 ?o")
    want = oracle.scan(g, p).rows
    try:
        ctx.set_option("capacity_override", 10)
        assert np.array_equal(ctx.scan(G, p).to_numpy(), want)
        f = ctx.filter(ctx.scan(G, p), 1, 0, 10**9)
        assert np.array_equal(f.to_numpy(), want)
        ctx.set_option("retry", 0)
        from paper_1807_01409_amd import TidError
        with pytest.raises(TidError) as ei:
            ctx.scan(G, p)
        assert ei.value.status == -3
    finally:
        ctx.set_option("capacity_override", 0)
        ctx.set_option("retry", 1)


def test_load_rejects_reserved_zero(ctx):
    from paper_1807_01409_amd import TidError
    g = np.array([[1, 2, 3], [4, 0, 6]], dtype=np.uint32)
    with pytest.raises(TidError) as ei:
        ctx.load(g)
    assert ei.value.status == -1


@pytest.mark.parametrize("name,n", [("small", 70001), ("medium", 3_000_000)])
def test_load_histograms(ctx, graphs, name, n):
    """The per-position counts built at load (one LDS-aggregated pass) equal
    numpy's bincount of each column, on uniform and on Zipf-skewed columns
    (hub subjects and objects), for single IDs and ranges."""
    g = graphs(name, n)
    G = ctx.load(g)
    rng = np.random.default_rng(5)
    for pos in range(3):
        want = np.bincount(g[:, pos])
        cdf = np.concatenate([[0], np.cumsum(want)])
        top = np.argsort(-want, kind="stable")[:50]
        ids = np.concatenate([top, rng.integers(1, want.size, 50), [want.size, want.size + 7]])
        for v in ids:
            v = int(v)
            assert G.count(pos, v, v + 1) == (int(want[v]) if v < want.size else 0), (pos, v)
        for _ in range(30):
            lo, hi = sorted(int(x) for x in rng.integers(0, want.size + 3, 2))
            w = int(cdf[min(hi, want.size)] - cdf[min(lo, want.size)])
            assert G.count(pos, lo, hi) == w, (pos, lo, hi)
        assert G.count(pos, 0, (1 << 32) - 1) == g.shape[0]
        assert G.count(pos, 9, 9) == 0
    G.free()


def test_load_file(ctx, graphs, tmp_path):
    """tid_load_file on a raw TripleID file (N x 12 bytes, little-endian)
    equals tid_load of the same rows; malformed files are refused."""
    from paper_1807_01409_amd import TidError
    from paper_1807_01409_amd.tid import tid_load_file
    from synth import save_tid
    g = graphs("small", 70001)
    path = str(tmp_path / "g.tid")
    save_tid(path, g)
    G = tid_load_file(ctx, path)
    assert G.n == g.shape[0]
    for p in (Pattern(0, 7, 0, 0, -1, 1), Pattern(0, 0, 0, 0, 1, 2)):
        assert np.array_equal(ctx.scan(G, p).to_numpy(), oracle.scan(g, p).rows)
    G.free()
    empty = str(tmp_path / "empty.tid")
    open(empty, "wb").close()
    E = tid_load_file(ctx, empty)
    assert E.n == 0
    E.free()
    bad = str(tmp_path / "bad.tid")
    with open(bad, "wb") as f:
        f.write(g[:5].tobytes() + b"\x01\x00")
    zero = str(tmp_path / "zero.tid")
    z = g[:5].copy()
    z[3, 2] = 0
    z.astype("<u4").tofile(zero)
    for path in (bad, zero, str(tmp_path / "missing.tid")):
        with pytest.raises(TidError) as ei:
            tid_load_file(ctx, path)
        assert ei.value.status == -1


def test_invalid_pattern_rejected(ctx, graphs):
    from paper_1807_01409_amd import TidError
    from paper_1807_01409_amd import _lib as L
    import ctypes
    G = ctx.load(graphs("small", 1000))
    q = L.tid_pattern(3, 0, 0, 1, -1, -1, -1, 0, 0)  # bound position naming a variable
    out = ctypes.c_void_p()
    assert ctx._lib.tid_scan(ctx.ptr, G._p, ctypes.byref(q), ctypes.byref(out)) == -1


def test_filter_parity(ctx, graphs):
    g = graphs("small")
    G = ctx.load(g)
    p = pat("?s ?p ?o")
    t = ctx.scan(G, p)
    o = oracle.scan(g, p)
    for col, lo, hi in ((2, 100, 5000), (0, 1, 2), (1, 7, 8), (2, 5000, 100), (0, 0, 2**32 - 1)):
        same(ctx.filter(t, col, lo, hi), oracle.filter(o, col, lo, hi))


def test_torch_allocator_matches(ctx, graphs):
    from paper_1807_01409_amd import Context
    g = graphs("small")
    with Context(0, allocator="torch") as c2:
        G = c2.load(g)
        p = pat("?s 9 ?o")
        assert np.array_equal(c2.scan(G, p).to_numpy(), oracle.scan(g, p).rows)


@pytest.mark.slow
def test_scan_full_medium(ctx, graphs):
    """The 50M-triple medium graph in the launch shape the benchmark times."""
    g = graphs("medium")
    G = ctx.load(g)
    hist = np.bincount(g[:, 1])
    n = g.shape[0]
    for sigma in (1e-3, 1e-2, 1e-1):
        p_id = int(np.argmin(np.abs(np.log(np.maximum(hist, 1) / n) - np.log(sigma))))
        p = Pattern(0, p_id, 0, 0, -1, 1)
        same(ctx.scan(G, p), oracle.scan(g, p))


def test_autotune_shapes_agree(ctx, graphs, tmp_path, monkeypatch):
    """The autotuner's sweep checks every shape against the first: results
    are byte-identical across launch shapes, prefetch and staging sizes."""
    from paper_1807_01409_amd import autotune
    monkeypatch.setenv("TID_TUNE_CACHE", str(tmp_path / "tune.json"))
    g = graphs("medium", 300_000)
    G = ctx.load(g)
    res = autotune.tune_scan(ctx, G, [pat("?s 2 ?o"), pat("?s 14 ?o")], reps=2,
                             shapes=[(256, 16), (512, 8), (1024, 4)], stage_words=[4096, 16384])
    assert len(res["table"]) == 12
    entry = autotune.apply(ctx, G.n)
    assert entry is not None and entry["options"] == res["options"]
    for k in autotune.KEYS:
        ctx.set_option(k, -1 if k == "scan_prefetch" else 0)


def _clustered(g):
    """The same triples ordered by predicate: a predicate's matches are then
    contiguous, so whole chunks match and staging areas overflow."""
    return g[np.argsort(g[:, 1], kind="stable")]


@pytest.mark.parametrize("kernel", [0, 1, 2])
def test_compact_kernels_big_chunks(ctx, graphs, kernel):
    """Both compaction kernels on 6M triples (big chunks, a single-tile tail,
    many workgroups), at sparse and dense selectivities, on the graph in
    generation order and ordered by predicate."""
    from synth.queries import predicate_for_selectivity
    g0 = graphs("medium", 6_000_000)
    ctx.set_option("compact_kernel", kernel)
    try:
        for g in (g0, _clustered(g0)):
            G = ctx.load(g)
            pats = [Pattern(0, predicate_for_selectivity(g, s)[0], 0, 0, -1, 1)
                    for s in (1e-4, 1e-2, 0.1, 0.3)]
            pats.append(Pattern(0, 0, 0, 0, 1, 2, range_pos=1, lo=1, hi=40))
            for p in pats:
                same(ctx.scan(G, p), oracle.scan(g, p))
            G.free()
    finally:
        ctx.set_option("compact_kernel", 0)


def test_chunk_epoch_wrap(ctx, graphs):
    """Launch stamps past the largest epoch restart at 1 after the slots are
    cleared; results stay exact on both sides of the wrap."""
    g = graphs("medium", 6_000_000)
    G = ctx.load(g)
    p = pat("?s 3 ?o")
    want = oracle.scan(g, p)
    top = (1 << 23) - 1
    ctx.set_option("compact_kernel", 2)
    try:
        ctx.set_option("chunk_epoch", top - 2)
        for _ in range(5):
            same(ctx.scan(G, p), want)
        assert 1 <= ctx.get_option("chunk_epoch") <= 3
    finally:
        ctx.set_option("compact_kernel", 0)
