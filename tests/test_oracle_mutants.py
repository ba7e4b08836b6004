"""Plant plausible mistakes in copies of the C oracle (on the CPU only) and
check that the pins catch every one of them.  Each mutant keeps its memory
accesses in bounds, so a broken copy gives wrong answers but never crashes."""
import ctypes
import os
import subprocess

import pytest

import oracle
import oracle_pins as P

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

# (name, text in oracle.c, replacement); every occurrence is replaced
MUTANTS = [
    ("filter_inclusive_hi", " < hi)", " <= hi)"),
    ("match_ignores_object",
     "for (int x = 0; x < 3; ++x)\n        if (q->c[x] != 0 && t[x] != q->c[x]) return 0;",
     "for (int x = 0; x < 2; ++x)\n        if (q->c[x] != 0 && t[x] != q->c[x]) return 0;"),
    ("repeated_var_unchecked",
     "if (q->v[x] >= 0 && q->v[x] == q->v[y] && t[x] != t[y]) return 0;", ";"),
    ("range_exclusive_lo", "q->lo <= val && val < q->hi", "q->lo < val && val < q->hi"),
    ("bind_positions_transposed", "src[k] = x;", "src[k] = 2 - x;"),
    ("sort_descending", "if (ra[c] < rb[c]) return -1;", "if (ra[c] < rb[c]) return 1;"),
    ("join_drops_wrong_column", "if (x != rc) dst[c++] = rr[x];", "if (x != 0) dst[c++] = rr[x];"),
    ("merge_skips_equal_keys", "if (kl[a].key < kr[b].key) { ++a; continue; }",
     "if (kl[a].key <= kr[b].key) { ++a; continue; }"),
    ("union_unbound_not_zero", "uint32_t val = 0;", "uint32_t val = 1;"),
    ("union_dedupe_inverted", "if (dedupe) return or_distinct(out);",
     "if (!dedupe) return or_distinct(out);"),
    ("natural_join_ignores_shared", "if (lr[eq_l[e]] != rr[eq_r[e]]) ok = 0;", ";"),
    ("distinct_without_sort", "    or_sort_rows(t);\n    uint64_t w = 1;", "    uint64_t w = 1;"),
    ("membership_bit_shifted", "m |= (uint64_t)1 << j;", "m |= (uint64_t)1 << (j + 1) % 64;"),
    ("project_ignores_order", "src[j] = col_of(t, (int32_t)vlist[j]);",
     "src[j] = col_of(t, (int32_t)vlist[j]) >= 0 ? j : -1;"),
    ("keyed_scan_ignores_keys", "if (!bsearch(&t[pos], sorted,", "if (0 && !bsearch(&t[pos], sorted,"),
    ("rule9_keys_on_subject", "r->shared = 0; r->key_pos = 2; r->out_s = 2; r->out_p = type;",
     "r->shared = 0; r->key_pos = 0; r->out_s = 2; r->out_p = type;"),
    ("rule3_derives_subject", "r->a = mkpat(0, rng, 0, 0, -1, 1); r->b = mkpat(0, 0, 0, -1, 0, 2);",
     "r->a = mkpat(0, rng, 0, 0, -1, 1); r->b = mkpat(0, 0, 0, 2, 0, -1);"),
    ("outer_left_drops_unmatched", "if (!matched && keep_l) {", "if (0) {"),
    ("outer_right_key_not_moved", "dst[c++] = x == lc ? rr[rc] : 0u;", "dst[c++] = 0u;"),
    ("outer_pads_with_left_value", "dst[x] = x < l->ncols ? l->rows[i * l->ncols + x] : 0u;",
     "dst[x] = x < l->ncols ? l->rows[i * l->ncols + x] : l->rows[i * l->ncols];"),
]


def _build_mutant(tmp_path, name, old, new):
    src = open(SRC).read()
    assert old in src, f"mutation {name}: text not found"
    mut = src.replace(old, new)
    c = tmp_path / f"{name}.c"
    c.write_text(mut)
    (tmp_path / "oracle.h").write_text(open(SRC[:-1] + "h").read())
    so = tmp_path / f"{name}.so"
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-w",
                           "-o", str(so), str(c)])
    return oracle._setup(ctypes.CDLL(str(so)))


def _first_failure():
    for chk in P.ALL_CHECKS:
        try:
            chk(oracle)
        except Exception as e:  # noqa: BLE001 - any failure counts as caught
            return f"{chk.__name__}: {type(e).__name__}"
    return None


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(tmp_path, monkeypatch, oracle_lib, name, old, new):
    lib = _build_mutant(tmp_path, name, old, new)
    monkeypatch.setattr(oracle, "_lib", lib)
    caught = _first_failure()
    assert caught is not None, f"mutant {name} passed every pin"


def test_pristine_oracle_passes_all_pins(oracle_lib):
    assert _first_failure() is None
