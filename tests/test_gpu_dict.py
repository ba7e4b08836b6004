"""Dictionary encoding on the GPU (Sec. 3: terms to TripleID rows) against
the oracle's encoder: the same IDs (one shared dictionary, first appearance,
s p o order), decoding back to the same strings, the Sec. 3 walk-through, a
graph of synthetic IRIs with heavy repetition, empty and one-triple inputs,
multi-byte UTF-8 terms, and refused IDs."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def synthetic_terms(n, seed, n_subj=5000, n_pred=40, n_obj=20000):
    rng = np.random.default_rng(seed)
    s = rng.zipf(1.3, n) % n_subj
    p = rng.integers(0, n_pred, n)
    o = rng.zipf(1.2, n) % n_obj
    lit = rng.random(n) < 0.2
    out = []
    for i in range(n):
        obj = f'"literal {o[i]} é中"' if lit[i] else f"<http://example.org/r/{o[i]}>"
        out.append((f"<http://example.org/r/{s[i]}>", f"<http://example.org/p#{p[i]}>", obj))
    return out


@pytest.mark.parametrize("triples", [
    [("ABCPress", "owns", "JournalA"), ("ABCPress", "publishes", "JournalA"),
     ("XPress", "publishes", "JournalB"), ("XPress", "owns", "JournalA")],
    [("a", "b", "c")], [("x", "x", "x")], [],
    synthetic_terms(20_000, 1), synthetic_terms(300_000, 2)])
def test_encode_matches_oracle(ctx, triples):
    rows, d = ctx.encode(triples)
    want, dicts = oracle.encode_graph(triples, shared=True)
    assert rows.shape == (len(triples), 3)
    assert np.array_equal(rows, want.reshape(-1, 3))
    n_terms, _ = d.info()
    assert n_terms == len(dicts[0])
    ids = rows.ravel()
    back = d.decode(ids)
    assert back == [x for t in triples for x in t]
    assert d.decode(np.arange(1, n_terms + 1)) == sorted(dicts[0], key=dicts[0].get)
    d.free()


def test_decode_refuses_bad_ids(ctx):
    from paper_1807_01409_amd import TidError
    rows, d = ctx.encode([("a", "b", "c")])
    for bad in ([0], [4], [1, 2, 99]):
        with pytest.raises(TidError) as ei:
            d.decode(bad)
        assert ei.value.status == -1
    d.free()
