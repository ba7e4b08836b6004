/*
 * oracle.c -- plain, slow, single-threaded CPU oracle for the TripleID-Q
 * query path.  TEST INFRASTRUCTURE ONLY (see oracle.h for what may use it and
 * for the paper passages each function follows).
 *
 * Every function here is written for a reader checking it against the paper:
 * plain loops, the C library's qsort as the only sorting step, no blocking,
 * no fusion.  Counts are 64-bit; IDs are 32-bit.
 */
#define _GNU_SOURCE
#include "oracle.h"

#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* helpers                                                             */
/* ------------------------------------------------------------------ */

static int32_t col_of(const or_table *t, int32_t var);

static int table_alloc(or_table *t, uint64_t nrows, int32_t ncols)
{
    t->nrows = nrows;
    t->ncols = ncols;
    t->rows = NULL;
    if (nrows && ncols) {
        t->rows = (uint32_t *)malloc((size_t)nrows * (size_t)ncols * sizeof(uint32_t));
        if (!t->rows) return OR_E_OOM;
    }
    return OR_OK;
}

void or_table_free(or_table *t)
{
    if (!t) return;
    free(t->rows);
    t->rows = NULL;
    t->nrows = 0;
}

static int pattern_ok(const or_pattern *q)
{
    for (int x = 0; x < 3; ++x) {
        if (q->c[x] != 0 && q->v[x] != -1) return 0;  /* bound positions name no variable */
        if (q->v[x] < -1) return 0;
    }
    return q->range_pos >= -1 && q->range_pos <= 2;
}

/* The match predicate of GPUSearch (Sec. 3): every bound key position equals
   the triple's value, 0 in the key is the free variable.  Free positions that
   name the same variable must hold equal values; an optional ID range applies
   to one position. */
static int triple_matches(const uint32_t *t, const or_pattern *q)
{
    for (int x = 0; x < 3; ++x)
        if (q->c[x] != 0 && t[x] != q->c[x]) return 0;
    for (int x = 0; x < 3; ++x)
        for (int y = x + 1; y < 3; ++y)
            if (q->v[x] >= 0 && q->v[x] == q->v[y] && t[x] != t[y]) return 0;
    if (q->range_pos >= 0) {
        uint32_t val = t[q->range_pos];
        if (!(q->lo <= val && val < q->hi)) return 0;
    }
    return 1;
}

/* output schema of a pattern: distinct named variables in s, p, o order;
   src[c] is the triple position feeding column c */
static int32_t pattern_schema(const or_pattern *q, int32_t *vars, int32_t *src)
{
    int32_t k = 0;
    for (int x = 0; x < 3; ++x) {
        if (q->v[x] < 0) continue;
        int seen = 0;
        for (int j = 0; j < k; ++j)
            if (vars[j] == q->v[x]) seen = 1;
        if (!seen) {
            vars[k] = q->v[x];
            src[k] = x;
            ++k;
        }
    }
    return k;
}

/* lexicographic comparison of two rows of `ncols` columns */
static int row_cmp(const void *a, const void *b, void *arg)
{
    const uint32_t *ra = (const uint32_t *)a, *rb = (const uint32_t *)b;
    int32_t ncols = *(const int32_t *)arg;
    for (int32_t c = 0; c < ncols; ++c) {
        if (ra[c] < rb[c]) return -1;
        if (ra[c] > rb[c]) return 1;
    }
    return 0;
}

int or_sort_rows(or_table *t)
{
    if (t->nrows > 1 && t->ncols > 0)
        qsort_r(t->rows, (size_t)t->nrows, (size_t)t->ncols * sizeof(uint32_t), row_cmp,
                &t->ncols);
    return OR_OK;
}

int or_distinct(or_table *t)
{
    if (t->nrows == 0) return OR_OK;
    if (t->ncols == 0) {            /* every zero-width row is the same row */
        t->nrows = 1;
        return OR_OK;
    }
    or_sort_rows(t);
    uint64_t w = 1;
    for (uint64_t i = 1; i < t->nrows; ++i) {
        const uint32_t *prev = t->rows + (w - 1) * t->ncols;
        const uint32_t *cur = t->rows + i * t->ncols;
        if (row_cmp(prev, cur, &t->ncols) != 0) {
            if (w != i) memmove(t->rows + w * t->ncols, cur, t->ncols * sizeof(uint32_t));
            ++w;
        }
    }
    t->nrows = w;
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* scan (Sec. 3, Algorithm 1) and multi-subquery marking (Sec. 4.1)    */
/* ------------------------------------------------------------------ */

int or_scan_flags(const uint32_t *g, uint64_t n, const or_pattern *q, uint8_t *flags)
{
    if (!pattern_ok(q)) return OR_E_INVALID;
    for (uint64_t i = 0; i < n; ++i)
        flags[i] = (uint8_t)triple_matches(g + 3 * i, q);
    return OR_OK;
}

int or_scan_multi(const uint32_t *g, uint64_t n, const or_pattern *qs, int32_t k,
                  uint64_t *member)
{
    if (k < 0 || k > 64) return OR_E_INVALID;
    for (int32_t j = 0; j < k; ++j)
        if (!pattern_ok(&qs[j])) return OR_E_INVALID;
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t m = 0;
        for (int32_t j = 0; j < k; ++j)
            if (triple_matches(g + 3 * i, &qs[j])) m |= (uint64_t)1 << j;
        member[i] = m;
    }
    return OR_OK;
}

int or_scan(const uint32_t *g, uint64_t n, const or_pattern *q, or_table *out)
{
    if (!pattern_ok(q)) return OR_E_INVALID;
    int32_t vars[3], src[3];
    int32_t k = pattern_schema(q, vars, src);
    uint64_t cnt = 0;
    for (uint64_t i = 0; i < n; ++i)
        cnt += (uint64_t)triple_matches(g + 3 * i, q);
    int st = table_alloc(out, cnt, k);
    if (st) return st;
    for (int32_t c = 0; c < k; ++c) out->vars[c] = vars[c];
    uint64_t r = 0;
    for (uint64_t i = 0; i < n; ++i) {
        const uint32_t *t = g + 3 * i;
        if (!triple_matches(t, q)) continue;
        for (int32_t c = 0; c < k; ++c) out->rows[r * k + c] = t[src[c]];
        ++r;
    }
    return OR_OK;
}

static int u32_cmp(const void *a, const void *b)
{
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return x < y ? -1 : (x > y);
}

int or_scan_keyed(const uint32_t *g, uint64_t n, const or_pattern *q, int32_t pos,
                  const uint32_t *keys, uint64_t nkeys, or_table *out)
{
    if (!pattern_ok(q) || pos < 0 || pos > 2 || q->c[pos] != 0) return OR_E_INVALID;
    uint32_t *sorted = (uint32_t *)malloc((nkeys ? nkeys : 1) * sizeof(uint32_t));
    if (!sorted) return OR_E_OOM;
    if (nkeys) memcpy(sorted, keys, nkeys * sizeof(uint32_t));
    qsort(sorted, (size_t)nkeys, sizeof(uint32_t), u32_cmp);
    int32_t vars[3], src[3];
    int32_t k = pattern_schema(q, vars, src);
    uint64_t cnt = 0;
    for (int pass = 0; pass < 2; ++pass) {
        uint64_t r = 0;
        for (uint64_t i = 0; i < n; ++i) {
            const uint32_t *t = g + 3 * i;
            if (!triple_matches(t, q)) continue;
            if (!bsearch(&t[pos], sorted, (size_t)nkeys, sizeof(uint32_t), u32_cmp)) continue;
            if (pass)
                for (int32_t c = 0; c < k; ++c) out->rows[r * k + c] = t[src[c]];
            ++r;
        }
        if (!pass) {
            cnt = r;
            int st = table_alloc(out, cnt, k);
            if (st) { free(sorted); return st; }
            for (int32_t c = 0; c < k; ++c) out->vars[c] = vars[c];
        }
    }
    free(sorted);
    return OR_OK;
}

/* The rules of the entailment table as two patterns: A, the rule's schema
   triple, searched first; B, the data triple, searched with the distinct
   values A bound to the shared variable as keys at position key_pos.  Variable
   ids: 0..3 name the rule's letters in the order given below; the derived
   triple takes (subject var or constant, predicate, object var). */
typedef struct {
    or_pattern a, b;
    int32_t shared, key_pos;        /* shared variable; its position in B */
    int32_t out_s, out_o;           /* variables of the derived subject / object */
    uint32_t out_p;                 /* constant predicate, or 0: variable out_pv */
    int32_t out_pv;
} rule_plan;

static or_pattern mkpat(uint32_t s, uint32_t p, uint32_t o, int32_t vs, int32_t vp, int32_t vo)
{
    or_pattern q;
    memset(&q, 0, sizeof q);
    q.c[0] = s; q.c[1] = p; q.c[2] = o;
    q.v[0] = vs; q.v[1] = vp; q.v[2] = vo;
    q.range_pos = -1;
    return q;
}

static int rule_of(int32_t rule, const uint32_t *voc, rule_plan *r)
{
    const uint32_t type = voc[0], sc = voc[1], spo = voc[2], dom = voc[3], rng = voc[4];
    memset(r, 0, sizeof *r);
    r->out_pv = -1;
    switch (rule) {
    case 2:   /* s p o && p domain D  =>  s type D      vars: p 0, D 1, s 2 */
        r->a = mkpat(0, dom, 0, 0, -1, 1); r->b = mkpat(0, 0, 0, 2, 0, -1);
        r->shared = 0; r->key_pos = 1; r->out_s = 2; r->out_p = type; r->out_o = 1; break;
    case 3:   /* s p o && p range R  =>  o type R       vars: p 0, R 1, o 2 */
        r->a = mkpat(0, rng, 0, 0, -1, 1); r->b = mkpat(0, 0, 0, -1, 0, 2);
        r->shared = 0; r->key_pos = 1; r->out_s = 2; r->out_p = type; r->out_o = 1; break;
    case 5:   /* p spo q && q spo r  =>  p spo r        vars: p 0, q 1, r 2 */
        r->a = mkpat(0, spo, 0, 0, -1, 1); r->b = mkpat(0, spo, 0, 1, -1, 2);
        r->shared = 1; r->key_pos = 0; r->out_s = 0; r->out_p = spo; r->out_o = 2; break;
    case 7:   /* s p o && p spo q  =>  s q o            vars: p 0, q 1, s 2, o 3 */
        r->a = mkpat(0, spo, 0, 0, -1, 1); r->b = mkpat(0, 0, 0, 2, 0, 3);
        r->shared = 0; r->key_pos = 1; r->out_s = 2; r->out_p = 0; r->out_pv = 1;
        r->out_o = 3; break;
    case 9:   /* s type x && x sc y  =>  s type y       vars: x 0, y 1, s 2 */
        r->a = mkpat(0, sc, 0, 0, -1, 1); r->b = mkpat(0, type, 0, 2, -1, 0);
        r->shared = 0; r->key_pos = 2; r->out_s = 2; r->out_p = type; r->out_o = 1; break;
    case 11:  /* x sc y && y sc z  =>  x sc z           vars: x 0, y 1, z 2 */
        r->a = mkpat(0, sc, 0, 0, -1, 1); r->b = mkpat(0, sc, 0, 1, -1, 2);
        r->shared = 1; r->key_pos = 0; r->out_s = 0; r->out_p = sc; r->out_o = 2; break;
    default:
        return OR_E_INVALID;
    }
    return OR_OK;
}

int or_entail(const uint32_t *g, uint64_t n, int32_t rule, const uint32_t *vocab, or_table *out)
{
    rule_plan r;
    int st = rule_of(rule, vocab, &r);
    if (st) return st;
    or_table ta, tb, tj;
    st = or_scan(g, n, &r.a, &ta);
    if (st) return st;
    /* keysArray: the values the first search bound to the shared variable */
    int32_t ka = col_of(&ta, r.shared);
    uint32_t *keys = (uint32_t *)malloc((ta.nrows ? ta.nrows : 1) * sizeof(uint32_t));
    if (!keys) { or_table_free(&ta); return OR_E_OOM; }
    for (uint64_t i = 0; i < ta.nrows; ++i) keys[i] = ta.rows[i * ta.ncols + ka];
    st = or_scan_keyed(g, n, &r.b, r.key_pos, keys, ta.nrows, &tb);
    free(keys);
    if (st) { or_table_free(&ta); return st; }
    st = or_join_sortmerge(&ta, ka, &tb, col_of(&tb, r.shared), &tj);
    or_table_free(&ta);
    or_table_free(&tb);
    if (st) return st;
    st = table_alloc(out, tj.nrows, 3);
    if (st) { or_table_free(&tj); return st; }
    out->vars[0] = 0; out->vars[1] = 1; out->vars[2] = 2;
    int32_t cs = col_of(&tj, r.out_s), co = col_of(&tj, r.out_o);
    int32_t cp = r.out_p ? -1 : col_of(&tj, r.out_pv);
    for (uint64_t i = 0; i < tj.nrows; ++i) {
        const uint32_t *row = tj.rows + i * tj.ncols;
        out->rows[3 * i] = row[cs];
        out->rows[3 * i + 1] = r.out_p ? r.out_p : row[cp];
        out->rows[3 * i + 2] = row[co];
    }
    or_table_free(&tj);
    return or_distinct(out);
}

/* ------------------------------------------------------------------ */
/* filter by ID range (Sec. 4.3, range form)                           */
/* ------------------------------------------------------------------ */

int or_filter(const or_table *t, int32_t col, uint32_t lo, uint32_t hi, or_table *out)
{
    if (col < 0 || col >= t->ncols) return OR_E_INVALID;
    uint64_t cnt = 0;
    for (uint64_t i = 0; i < t->nrows; ++i) {
        uint32_t x = t->rows[i * t->ncols + col];
        if (lo <= x && x < hi) ++cnt;
    }
    int st = table_alloc(out, cnt, t->ncols);
    if (st) return st;
    memcpy(out->vars, t->vars, sizeof(out->vars));
    uint64_t r = 0;
    for (uint64_t i = 0; i < t->nrows; ++i) {
        const uint32_t *row = t->rows + i * t->ncols;
        if (lo <= row[col] && row[col] < hi) {
            memcpy(out->rows + r * t->ncols, row, t->ncols * sizeof(uint32_t));
            ++r;
        }
    }
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* join (Sec. 4.2)                                                     */
/* ------------------------------------------------------------------ */

static int join_schema(const or_table *l, int32_t lc, const or_table *r, int32_t rc,
                       or_table *out, uint64_t nrows)
{
    if (lc < 0 || lc >= l->ncols || rc < 0 || rc >= r->ncols) return OR_E_INVALID;
    int32_t nc = l->ncols + r->ncols - 1;
    if (nc > OR_MAXCOLS) return OR_E_SCHEMA;
    int st = table_alloc(out, nrows, nc);
    if (st) return st;
    int32_t c = 0;
    for (int32_t j = 0; j < l->ncols; ++j) out->vars[c++] = l->vars[j];
    for (int32_t j = 0; j < r->ncols; ++j)
        if (j != rc) out->vars[c++] = r->vars[j];
    return OR_OK;
}

/* output row = L row ++ (R row without its key column) */
static void emit_pair(const or_table *l, uint64_t i, const or_table *r, uint64_t j,
                      int32_t rc, uint32_t *dst)
{
    const uint32_t *lr = l->rows + i * l->ncols;
    const uint32_t *rr = r->rows + j * r->ncols;
    int32_t c = 0;
    for (int32_t x = 0; x < l->ncols; ++x) dst[c++] = lr[x];
    for (int32_t x = 0; x < r->ncols; ++x)
        if (x != rc) dst[c++] = rr[x];
}

int or_join_nested(const or_table *l, int32_t lc, const or_table *r, int32_t rc, or_table *out)
{
    if (lc < 0 || lc >= l->ncols || rc < 0 || rc >= r->ncols) return OR_E_INVALID;
    uint64_t cnt = 0;
    for (uint64_t i = 0; i < l->nrows; ++i)
        for (uint64_t j = 0; j < r->nrows; ++j)
            if (l->rows[i * l->ncols + lc] == r->rows[j * r->ncols + rc]) ++cnt;
    int st = join_schema(l, lc, r, rc, out, cnt);
    if (st) return st;
    uint64_t w = 0;
    for (uint64_t i = 0; i < l->nrows; ++i)
        for (uint64_t j = 0; j < r->nrows; ++j)
            if (l->rows[i * l->ncols + lc] == r->rows[j * r->ncols + rc]) {
                emit_pair(l, i, r, j, rc, out->rows + w * out->ncols);
                ++w;
            }
    return or_sort_rows(out);
}

/* Outer joins by the nested-loop definition: the inner pairs in (L, R)
   order, then the L rows without a partner (left, full), then the R rows
   without a partner (right, full); the result is sorted like every join. */
int or_join_outer(const or_table *l, int32_t lc, const or_table *r, int32_t rc, int32_t kind,
                  or_table *out)
{
    if (lc < 0 || lc >= l->ncols || rc < 0 || rc >= r->ncols) return OR_E_INVALID;
    if (kind < OR_JOIN_INNER || kind > OR_JOIN_FULL) return OR_E_INVALID;
    int keep_l = kind == OR_JOIN_LEFT || kind == OR_JOIN_FULL;
    int keep_r = kind == OR_JOIN_RIGHT || kind == OR_JOIN_FULL;
    uint64_t cnt = 0;
    for (int pass = 0; pass < 2; ++pass) {
        uint64_t w = 0;
        for (uint64_t i = 0; i < l->nrows; ++i) {
            int matched = 0;
            for (uint64_t j = 0; j < r->nrows; ++j)
                if (l->rows[i * l->ncols + lc] == r->rows[j * r->ncols + rc]) {
                    if (pass) emit_pair(l, i, r, j, rc, out->rows + w * out->ncols);
                    ++w;
                    matched = 1;
                }
            if (!matched && keep_l) {
                if (pass) {
                    uint32_t *dst = out->rows + w * out->ncols;
                    for (int32_t x = 0; x < out->ncols; ++x)
                        dst[x] = x < l->ncols ? l->rows[i * l->ncols + x] : 0u;
                }
                ++w;
            }
        }
        if (keep_r)
            for (uint64_t j = 0; j < r->nrows; ++j) {
                int matched = 0;
                for (uint64_t i = 0; i < l->nrows && !matched; ++i)
                    if (l->rows[i * l->ncols + lc] == r->rows[j * r->ncols + rc]) matched = 1;
                if (matched) continue;
                if (pass) {
                    uint32_t *dst = out->rows + w * out->ncols;
                    const uint32_t *rr = r->rows + j * r->ncols;
                    int32_t c = 0;
                    for (int32_t x = 0; x < l->ncols; ++x) dst[c++] = x == lc ? rr[rc] : 0u;
                    for (int32_t x = 0; x < r->ncols; ++x)
                        if (x != rc) dst[c++] = rr[x];
                }
                ++w;
            }
        if (pass == 0) {
            cnt = w;
            int st = join_schema(l, lc, r, rc, out, cnt);
            if (st) return st;
        }
    }
    return or_sort_rows(out);
}

typedef struct { uint32_t key; uint64_t idx; } key_idx;

static int key_idx_cmp(const void *a, const void *b)
{
    const key_idx *x = (const key_idx *)a, *y = (const key_idx *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->idx < y->idx ? -1 : (x->idx > y->idx);
}

/* Sec. 4.2 steps 2-3: copy the key column of each side into a key vector,
   sort the key vectors, merge them into pairs of positions whose keys are
   equal, then gather the value parts of both sides through those pairs. */
int or_join_sortmerge(const or_table *l, int32_t lc, const or_table *r, int32_t rc, or_table *out)
{
    if (lc < 0 || lc >= l->ncols || rc < 0 || rc >= r->ncols) return OR_E_INVALID;
    key_idx *kl = (key_idx *)malloc((l->nrows ? l->nrows : 1) * sizeof(key_idx));
    key_idx *kr = (key_idx *)malloc((r->nrows ? r->nrows : 1) * sizeof(key_idx));
    if (!kl || !kr) { free(kl); free(kr); return OR_E_OOM; }
    for (uint64_t i = 0; i < l->nrows; ++i) { kl[i].key = l->rows[i * l->ncols + lc]; kl[i].idx = i; }
    for (uint64_t j = 0; j < r->nrows; ++j) { kr[j].key = r->rows[j * r->ncols + rc]; kr[j].idx = j; }
    qsort(kl, (size_t)l->nrows, sizeof(key_idx), key_idx_cmp);
    qsort(kr, (size_t)r->nrows, sizeof(key_idx), key_idx_cmp);

    /* merge: count first, so the output is allocated once */
    uint64_t cnt = 0;
    for (int pass = 0; pass < 2; ++pass) {
        uint64_t a = 0, b = 0, w = 0;
        while (a < l->nrows && b < r->nrows) {
            if (kl[a].key < kr[b].key) { ++a; continue; }
            if (kl[a].key > kr[b].key) { ++b; continue; }
            uint64_t a2 = a, b2 = b;
            while (a2 < l->nrows && kl[a2].key == kl[a].key) ++a2;
            while (b2 < r->nrows && kr[b2].key == kr[b].key) ++b2;
            if (pass == 0) {
                cnt += (a2 - a) * (b2 - b);
            } else {
                for (uint64_t x = a; x < a2; ++x)
                    for (uint64_t y = b; y < b2; ++y) {
                        emit_pair(l, kl[x].idx, r, kr[y].idx, rc, out->rows + w * out->ncols);
                        ++w;
                    }
            }
            a = a2;
            b = b2;
        }
        if (pass == 0) {
            int st = join_schema(l, lc, r, rc, out, cnt);
            if (st) { free(kl); free(kr); return st; }
        }
    }
    free(kl);
    free(kr);
    return or_sort_rows(out);
}

/* ------------------------------------------------------------------ */
/* union (Sec. 4.1) with optional DISTINCT (Sec. 4.3)                  */
/* ------------------------------------------------------------------ */

int or_union(const or_table *const *ts, int32_t k, int32_t dedupe, or_table *out)
{
    if (k < 1) return OR_E_INVALID;
    int32_t vars[OR_MAXCOLS];
    int32_t nc = 0;
    uint64_t total = 0;
    for (int32_t t = 0; t < k; ++t) {
        for (int32_t c = 0; c < ts[t]->ncols; ++c) {
            int seen = 0;
            for (int32_t j = 0; j < nc; ++j)
                if (vars[j] == ts[t]->vars[c]) seen = 1;
            if (!seen) {
                if (nc == OR_MAXCOLS) return OR_E_SCHEMA;
                vars[nc++] = ts[t]->vars[c];
            }
        }
        total += ts[t]->nrows;
    }
    int st = table_alloc(out, total, nc);
    if (st) return st;
    for (int32_t j = 0; j < nc; ++j) out->vars[j] = vars[j];
    uint64_t w = 0;
    for (int32_t t = 0; t < k; ++t) {
        const or_table *in = ts[t];
        for (uint64_t i = 0; i < in->nrows; ++i, ++w) {
            for (int32_t j = 0; j < nc; ++j) {
                uint32_t val = 0;             /* unbound */
                for (int32_t c = 0; c < in->ncols; ++c)
                    if (in->vars[c] == vars[j]) val = in->rows[i * in->ncols + c];
                if (nc) out->rows[w * nc + j] = val;
            }
        }
    }
    if (dedupe) return or_distinct(out);
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* query plan (Sec. 4.3, Fig. 6)                                       */
/* ------------------------------------------------------------------ */

#define OP_SCAN 1
#define OP_JOIN 2
#define OP_UNION 3
#define OP_FILTER 4
#define OP_PROJECT 5
#define OP_DISTINCT 6
#define OP_OPTIONAL 7
#define OR_STACK 64

static int32_t col_of(const or_table *t, int32_t var)
{
    for (int32_t c = 0; c < t->ncols; ++c)
        if (t->vars[c] == var) return c;
    return -1;
}

/* Plan joins switch from nested loops to Sec. 4.2's sort-merge when the
   number of row pairs exceeds this; both give the same multiset. */
static double g_nested_limit = 1e8;

void or_set_nested_join_limit(double pairs) { g_nested_limit = pairs; }

/* Join of two subquery results on variable `var`: the inner join on that
   column pair (Sec. 4.2); any other variable the two sides share must also
   agree, and appears once in the output. */
static int natural_join(const or_table *l, const or_table *r, int32_t var, or_table *out)
{
    int32_t lc = col_of(l, var), rc = col_of(r, var);
    if (lc < 0 || rc < 0) return OR_E_SCHEMA;
    /* columns of R kept in the output, and R/L column pairs that must agree */
    int32_t keep[OR_MAXCOLS], nkeep = 0, eq_l[OR_MAXCOLS], eq_r[OR_MAXCOLS], neq = 0;
    for (int32_t c = 0; c < r->ncols; ++c) {
        if (c == rc) continue;
        int32_t lcol = col_of(l, r->vars[c]);
        if (lcol >= 0) { eq_l[neq] = lcol; eq_r[neq] = c; ++neq; }
        else keep[nkeep++] = c;
    }
    int32_t nc = l->ncols + nkeep;
    if (nc > OR_MAXCOLS) return OR_E_SCHEMA;

    /* candidate pairs (i, j) with equal keys: all pairs for nested loops, or
       the equal-key runs of the two sorted key vectors for sort-merge */
    int sortmerge = (double)l->nrows * (double)r->nrows > g_nested_limit;
    key_idx *kl = NULL, *kr = NULL;
    if (sortmerge) {
        kl = (key_idx *)malloc((l->nrows ? l->nrows : 1) * sizeof(key_idx));
        kr = (key_idx *)malloc((r->nrows ? r->nrows : 1) * sizeof(key_idx));
        if (!kl || !kr) { free(kl); free(kr); return OR_E_OOM; }
        for (uint64_t i = 0; i < l->nrows; ++i) { kl[i].key = l->rows[i * l->ncols + lc]; kl[i].idx = i; }
        for (uint64_t j = 0; j < r->nrows; ++j) { kr[j].key = r->rows[j * r->ncols + rc]; kr[j].idx = j; }
        qsort(kl, (size_t)l->nrows, sizeof(key_idx), key_idx_cmp);
        qsort(kr, (size_t)r->nrows, sizeof(key_idx), key_idx_cmp);
    }
    uint64_t cnt = 0;
    for (int pass = 0; pass < 2; ++pass) {
        uint64_t w = 0;
        uint64_t a = 0, b = 0;
        /* iterate candidate pairs */
        for (;;) {
            uint64_t i0, i1, j0, j1;
            if (sortmerge) {
                while (a < l->nrows && b < r->nrows && kl[a].key != kr[b].key) {
                    if (kl[a].key < kr[b].key) ++a; else ++b;
                }
                if (a >= l->nrows || b >= r->nrows) break;
                uint64_t a2 = a, b2 = b;
                while (a2 < l->nrows && kl[a2].key == kl[a].key) ++a2;
                while (b2 < r->nrows && kr[b2].key == kr[b].key) ++b2;
                i0 = a; i1 = a2; j0 = b; j1 = b2;
                a = a2; b = b2;
            } else {
                if (a > 0) break;
                i0 = 0; i1 = l->nrows; j0 = 0; j1 = r->nrows;
                a = 1;
            }
            for (uint64_t x = i0; x < i1; ++x) {
                uint64_t i = sortmerge ? kl[x].idx : x;
                const uint32_t *lr = l->rows + i * l->ncols;
                for (uint64_t y = j0; y < j1; ++y) {
                    uint64_t j = sortmerge ? kr[y].idx : y;
                    const uint32_t *rr = r->rows + j * r->ncols;
                    if (lr[lc] != rr[rc]) continue;
                    int ok = 1;
                    for (int32_t e = 0; e < neq; ++e)
                        if (lr[eq_l[e]] != rr[eq_r[e]]) ok = 0;
                    if (!ok) continue;
                    if (pass == 1) {
                        uint32_t *dst = out->rows + w * nc;
                        for (int32_t c = 0; c < l->ncols; ++c) dst[c] = lr[c];
                        for (int32_t c = 0; c < nkeep; ++c) dst[l->ncols + c] = rr[keep[c]];
                    }
                    ++w;
                }
            }
        }
        if (pass == 0) {
            cnt = w;
            int st = table_alloc(out, cnt, nc);
            if (st) { free(kl); free(kr); return st; }
            for (int32_t c = 0; c < l->ncols; ++c) out->vars[c] = l->vars[c];
            for (int32_t c = 0; c < nkeep; ++c) out->vars[l->ncols + c] = r->vars[keep[c]];
        }
    }
    free(kl);
    free(kr);
    return OR_OK;
}

static int project(const or_table *t, const uint32_t *vlist, int32_t n, or_table *out)
{
    if (n < 0 || n > OR_MAXCOLS) return OR_E_SCHEMA;
    int32_t src[OR_MAXCOLS];
    for (int32_t j = 0; j < n; ++j) {
        src[j] = col_of(t, (int32_t)vlist[j]);
        if (src[j] < 0) return OR_E_SCHEMA;
        for (int32_t i = 0; i < j; ++i)
            if (vlist[i] == vlist[j]) return OR_E_SCHEMA;
    }
    int st = table_alloc(out, t->nrows, n);
    if (st) return st;
    for (int32_t j = 0; j < n; ++j) out->vars[j] = (int32_t)vlist[j];
    for (uint64_t i = 0; i < t->nrows; ++i)
        for (int32_t j = 0; j < n; ++j)
            out->rows[i * n + j] = t->rows[i * t->ncols + src[j]];
    return OR_OK;
}

int or_query(const uint32_t *g, uint64_t n, const or_pattern *pats, int32_t npats,
             const uint32_t *ops, int32_t nops, or_table *out)
{
    or_table stack[OR_STACK];
    int32_t sp = 0;
    int st = OR_OK;
    int32_t pc = 0;
#define NEED(words) do { if (pc + (words) > nops) { st = OR_E_INVALID; goto fail; } } while (0)
    while (pc < nops) {
        uint32_t op = ops[pc++];
        if (op == OP_SCAN) {
            NEED(1);
            uint32_t i = ops[pc++];
            if (i >= (uint32_t)npats || sp == OR_STACK) { st = OR_E_INVALID; goto fail; }
            st = or_scan(g, n, &pats[i], &stack[sp]);
            if (st) goto fail;
            ++sp;
        } else if (op == OP_JOIN) {
            NEED(1);
            int32_t var = (int32_t)ops[pc++];
            if (sp < 2) { st = OR_E_INVALID; goto fail; }
            or_table res;
            st = natural_join(&stack[sp - 2], &stack[sp - 1], var, &res);
            if (st) goto fail;
            or_table_free(&stack[sp - 1]);
            or_table_free(&stack[sp - 2]);
            sp -= 2;
            stack[sp++] = res;
        } else if (op == OP_OPTIONAL) {
            /* SPARQL OPTIONAL on one shared variable: the left outer join;
               the two sides may share no other variable */
            NEED(1);
            int32_t var = (int32_t)ops[pc++];
            if (sp < 2) { st = OR_E_INVALID; goto fail; }
            const or_table *l = &stack[sp - 2], *r = &stack[sp - 1];
            int32_t lc = col_of(l, var), rc = col_of(r, var);
            if (lc < 0 || rc < 0) { st = OR_E_SCHEMA; goto fail; }
            for (int32_t c = 0; c < r->ncols; ++c)
                if (c != rc && col_of(l, r->vars[c]) >= 0) { st = OR_E_UNSUPPORTED; goto fail; }
            or_table res;
            st = or_join_outer(l, lc, r, rc, OR_JOIN_LEFT, &res);
            if (st) goto fail;
            or_table_free(&stack[sp - 1]);
            or_table_free(&stack[sp - 2]);
            sp -= 2;
            stack[sp++] = res;
        } else if (op == OP_UNION) {
            NEED(2);
            int32_t k = (int32_t)ops[pc++];
            int32_t d = (int32_t)ops[pc++];
            if (k < 1 || k > sp) { st = OR_E_INVALID; goto fail; }
            const or_table *ins[OR_STACK];
            for (int32_t j = 0; j < k; ++j) ins[j] = &stack[sp - k + j];
            or_table res;
            st = or_union(ins, k, d, &res);
            if (st) goto fail;
            for (int32_t j = 0; j < k; ++j) or_table_free(&stack[sp - 1 - j]);
            sp -= k;
            stack[sp++] = res;
        } else if (op == OP_FILTER) {
            NEED(3);
            int32_t var = (int32_t)ops[pc++];
            uint32_t lo = ops[pc++], hi = ops[pc++];
            if (sp < 1) { st = OR_E_INVALID; goto fail; }
            int32_t c = col_of(&stack[sp - 1], var);
            if (c < 0) { st = OR_E_SCHEMA; goto fail; }
            or_table res;
            st = or_filter(&stack[sp - 1], c, lo, hi, &res);
            if (st) goto fail;
            or_table_free(&stack[sp - 1]);
            stack[sp - 1] = res;
        } else if (op == OP_PROJECT) {
            NEED(1);
            int32_t cnt = (int32_t)ops[pc++];
            NEED(cnt);
            if (sp < 1) { st = OR_E_INVALID; goto fail; }
            or_table res;
            st = project(&stack[sp - 1], ops + pc, cnt, &res);
            if (st) goto fail;
            pc += cnt;
            or_table_free(&stack[sp - 1]);
            stack[sp - 1] = res;
        } else if (op == OP_DISTINCT) {
            if (sp < 1) { st = OR_E_INVALID; goto fail; }
            or_distinct(&stack[sp - 1]);
        } else {
            st = OR_E_INVALID;
            goto fail;
        }
    }
    if (sp != 1) { st = OR_E_INVALID; goto fail; }
    *out = stack[0];
    return or_sort_rows(out);
fail:
    for (int32_t j = 0; j < sp; ++j) or_table_free(&stack[j]);
    return st;
#undef NEED
}
