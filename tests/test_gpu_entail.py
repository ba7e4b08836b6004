"""Multi-key search and RDFS entailment (Sec. 4.1 keysArray; Sec. 5.7) on
the GPU, byte for byte against the oracle: the Rule-11 worked example, each
of rules 2, 3, 5, 7, 9 and 11 on synthetic RDFS graphs of two sizes, and the
keyed scan at every position with empty, repeated and out-of-range keys."""
import numpy as np
import pytest

import oracle
from synth import Pattern
from synth.rdfs import VOCAB, RdfsSpec, make_rdfs_graph

pytestmark = pytest.mark.gpu


def same(gt, ot):
    got = gt.to_numpy()
    assert gt.vars == ot.vars, (gt.vars, ot.vars)
    assert got.shape == ot.rows.shape, (got.shape, ot.rows.shape)
    assert np.array_equal(got, ot.rows)


def test_rule11_worked_example(ctx):
    g = np.array([[76, 84, 56], [31, 84, 77], [56, 84, 78], [56, 84, 77], [44, 83, 2]],
                 dtype=np.uint32)
    G = ctx.load(g)
    t = ctx.entail(G, 11, [1, 84, 3, 4, 5]).to_numpy()
    assert t.tolist() == [[76, 84, 77], [76, 84, 78]]     # x subClassOf z (Sec. 5.7)


@pytest.mark.parametrize("spec", [RdfsSpec(), RdfsSpec(n_data=2_000_000, n_classes=20_000,
                                                        n_props=3_000, n_resources=1_000_000,
                                                        seed=9)])
def test_rules_against_oracle(ctx, spec):
    g = make_rdfs_graph(spec)
    G = ctx.load(g)
    for rule in (2, 3, 5, 7, 9, 11):
        t = ctx.entail(G, rule, VOCAB)
        same(t, oracle.entail(g, rule, VOCAB))
        assert t.nrows > 0, rule


def test_keyed_scan(ctx):
    g = make_rdfs_graph(RdfsSpec(seed=4))
    G = ctx.load(g)
    rng = np.random.default_rng(2)
    for pos in range(3):
        col = g[:, pos]
        for keys in (np.zeros(0, np.uint32), rng.choice(col, 50).astype(np.uint32),
                     np.repeat(rng.choice(col, 7), 5).astype(np.uint32),
                     np.array([0, int(col.max()) + 5, 1 << 31], np.uint32),
                     np.unique(col)):
            K = ctx.table(keys.reshape(-1, 1), [9])
            p = Pattern(0, 0, 0, 0, 1, 2)
            same(ctx.scan_keyed(G, p, pos, K, 0), oracle.scan_keyed(g, p, pos, keys))
        q = Pattern(0, VOCAB[1], 0, 0, -1, 1)      # a constant elsewhere in the pattern
        keys = rng.choice(g[:, 0], 300).astype(np.uint32)
        K = ctx.table(keys.reshape(-1, 1), [9])
        same(ctx.scan_keyed(G, q, 0, K, 0), oracle.scan_keyed(g, q, 0, keys))
