"""The CPU oracle pinned against the paper's worked examples, brute force on
tiny inputs and invariants (no GPU)."""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle_pins as P
from bruteforce import bf_query, bf_scan
from synth import CONFIGS, Pattern, make_graph


def test_rule11_worked_example(oracle_lib):
    P.check_rule11(oracle_lib)


def test_sec3_toy(oracle_lib):
    P.check_toy_sec3(oracle_lib)


def test_exhaustive_tiny_scan(oracle_lib):
    P.check_exhaustive_scan(oracle_lib)


def test_exhaustive_tiny_join(oracle_lib):
    P.check_exhaustive_join(oracle_lib)


def test_table3_relation_matrix(oracle_lib):
    P.check_table3_matrix(oracle_lib)


def test_union_listing4(oracle_lib):
    P.check_union_listing4(oracle_lib)


def test_union_bruteforce(oracle_lib):
    P.check_union_bruteforce(oracle_lib)


def test_filter_bruteforce(oracle_lib):
    P.check_filter_bruteforce(oracle_lib)


def test_random_plans(oracle_lib):
    P.check_random_plans(oracle_lib)


def test_invariants_small_config(oracle_lib):
    g = make_graph(CONFIGS["small"].with_n(20_000))
    P.check_invariants_small_config(oracle_lib, g)


def test_empty_graph(oracle_lib):
    g = np.zeros((0, 3), dtype=np.uint32)
    t = oracle_lib.scan(g, Pattern(0, 0, 0, 0, 1, 2))
    assert t.nrows == 0 and t.vars == [0, 1, 2]
    j = oracle_lib.join(t, 0, t, 0)
    assert j.nrows == 0 and j.ncols == 5


def test_zero_width_scan_counts(oracle_lib):
    g = P.tiny_graph(4, 10, 3)
    t = oracle_lib.scan(g, Pattern(0, 2, 0))
    assert t.ncols == 0 and t.nrows == int((g[:, 1] == 2).sum())


def test_invalid_pattern_rejected(oracle_lib):
    g = P.tiny_graph(4, 10, 3)
    from oracle import OracleError, _Pat, _L, _u32p, _Tab
    import ctypes
    q = _Pat()
    q.c[0] = 3
    q.v[0] = 1          # a bound position cannot name a variable
    q.v[1] = q.v[2] = -1
    q.range_pos = -1
    res = _Tab()
    assert _L().or_scan(_u32p(np.ascontiguousarray(g)), g.shape[0], ctypes.byref(q),
                        ctypes.byref(res)) == -1


@settings(max_examples=150, deadline=None)
@given(st.lists(st.tuples(st.integers(1, 5), st.integers(1, 5), st.integers(1, 5)),
                max_size=20),
       st.tuples(st.integers(0, 5), st.integers(0, 5), st.integers(0, 5)),
       st.sampled_from(P.VAR_LAYOUTS))
def test_hypothesis_scan(oracle_lib, triples, consts, layout):
    g = np.array(triples, dtype=np.uint32).reshape(-1, 3)
    p = P._layout_pattern(consts, layout)
    rows, vs = bf_scan(g, p)
    t = oracle_lib.scan(g, p)
    assert t.vars == vs and P._rows(t) == rows


@settings(max_examples=100, deadline=None)
@given(st.integers(0, 2**31))
def test_hypothesis_plans(oracle_lib, seed):
    rng = np.random.default_rng(seed)
    g = P.tiny_graph(seed % 1000, int(rng.integers(0, 14)), 4)
    plan = P.random_plan(rng)
    want, wv = bf_query(g, plan)
    got = oracle_lib.query(g, plan)
    assert got.vars == wv and P._rows(got) == want


def test_scan_multi_bruteforce(oracle_lib):
    P.check_scan_multi_bruteforce(oracle_lib)


def test_random_plans_sortmerge_joins(oracle_lib):
    P.check_random_plans_sortmerge(oracle_lib)


def test_dictionary_encoder(oracle_lib):
    P.check_encoder(oracle_lib)


def test_outer_joins(oracle_lib):
    P.check_outer_joins(oracle_lib)


def test_optional_plans(oracle_lib):
    P.check_optional_plans(oracle_lib)


def test_entailment(oracle_lib):
    P.check_entailment(oracle_lib)
