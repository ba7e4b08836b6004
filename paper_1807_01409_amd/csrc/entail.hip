// entail.hip -- the multi-key search and RDFS entailment (Sec. 5.7).
//
// Multi-key search: a pattern whose value at one free position must be one
// of a set of keys -- the keysArray the paper builds from the distinct
// results of an earlier search (Sec. 4.1, Sec. 5.7).  The keys become an
// exact bitmap over the position's ID range (one bit per ID, set with one
// atomic OR per key row, duplicates included, so no separate DISTINCT step
// is needed); the scan kernel tests it only on triples that pass the
// pattern's constants.
//
// Entailment: each rule of the paper's rule table (2, 3, 5, 7, 9, 11) is two
// searches -- the rule's schema pattern, then the data pattern keyed by the
// values the first search bound to the shared variable -- and the join of
// the two results on that variable; the derived triples are returned as
// distinct (s, p, o) rows in lexicographic order.
#include "compact.hpp"

#include <algorithm>

namespace tid {

void fill(tid_ctx *ctx, uint32_t *p, uint64_t n, uint32_t v);
std::unique_ptr<tid_table> sort_rows(tid_ctx *ctx, const tid_table *t, uint64_t n, int distinct);
std::unique_ptr<tid_table> join_unsorted(tid_ctx *ctx, const tid_table *L, uint64_t nl, int lc,
                                         const tid_table *R, uint64_t nr, int rc, int algo,
                                         const JoinPlan &jp, int kind);

__global__ void bitmap_set(const uint32_t *__restrict__ vals, uint64_t n, uint32_t maxv,
                           uint32_t *bits) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t x = vals[i];
        if (x <= maxv) atomicOr(&bits[x >> 5], 1u << (x & 31u));
    }
}

// A scan of `p` keeping only triples whose value at `pos` is in keys[0..nkeys)
// (a device column).  The bitmap covers IDs up to the graph's largest ID at
// that position: keys above it cannot match.
std::unique_ptr<tid_table> scan_keyed(tid_ctx *ctx, const tid_graph *g, const tid_pattern &p,
                                      int pos, const uint32_t *keys, uint64_t nkeys) {
    TID_REQUIRE(pos >= 0 && pos <= 2, TID_E_INVALID_ARG, "keyed scan: position must be 0, 1 or 2");
    const uint32_t c[3] = {p.s, p.p, p.o};
    TID_REQUIRE(c[pos] == 0, TID_E_INVALID_ARG, "keyed scan: the keyed position must be free");
    const uint32_t maxv = g->n ? g->max_id[pos] : 0;
    const uint64_t words = (uint64_t)maxv / 32 + 1;
    DevBuf bits(ctx, words * 4);
    TID_HIP(hipMemsetAsync(bits.get(), 0, words * 4, ctx->stream));
    if (nkeys) {
        const unsigned grid = (unsigned)std::min<uint64_t>((nkeys + 255) / 256, 8192);
        hipLaunchKernelGGL(bitmap_set, dim3(grid), dim3(256), 0, ctx->stream, keys, nkeys, maxv,
                           bits.get<uint32_t>());
        TID_HIP(hipGetLastError());
    }
    ScanFilter f;
    f.bits = bits.get<const uint32_t>();
    f.mask = maxv;
    f.pos = pos;
    f.exact = 1;
    std::unique_ptr<tid_table> out;
    scan_multi(ctx, g, &p, 1, &out, nullptr, &f);
    return out;  // `bits` goes back to the pool in stream order, after the scan
}

namespace {

// A rule as two patterns (variable ids 0..3 name the rule's letters): A, the
// schema triple, searched first; B, the data triple, keyed at key_pos by the
// values A bound to `shared`.  The derived triple is (out_s, out_p or the
// variable out_pv, out_o).
struct Rule {
    tid_pattern a, b;
    int32_t shared, key_pos, out_s, out_o, out_pv;
    uint32_t out_p;
};

tid_pattern pattern(uint32_t s, uint32_t p, uint32_t o, int32_t vs, int32_t vp, int32_t vo) {
    tid_pattern q{};
    q.s = s;
    q.p = p;
    q.o = o;
    q.vs = vs;
    q.vp = vp;
    q.vo = vo;
    q.range_pos = -1;
    return q;
}

Rule rule_of(int rule, const uint32_t *voc) {
    const uint32_t type = voc[0], sc = voc[1], spo = voc[2], dom = voc[3], rng = voc[4];
    Rule r{};
    r.out_pv = -1;
    switch (rule) {
        case 2:  // s p o, p domain D => s type D   (p 0, D 1, s 2)
            r.a = pattern(0, dom, 0, 0, -1, 1);
            r.b = pattern(0, 0, 0, 2, 0, -1);
            r.shared = 0, r.key_pos = 1, r.out_s = 2, r.out_p = type, r.out_o = 1;
            break;
        case 3:  // s p o, p range R => o type R    (p 0, R 1, o 2)
            r.a = pattern(0, rng, 0, 0, -1, 1);
            r.b = pattern(0, 0, 0, -1, 0, 2);
            r.shared = 0, r.key_pos = 1, r.out_s = 2, r.out_p = type, r.out_o = 1;
            break;
        case 5:  // p spo q, q spo r => p spo r     (p 0, q 1, r 2)
            r.a = pattern(0, spo, 0, 0, -1, 1);
            r.b = pattern(0, spo, 0, 1, -1, 2);
            r.shared = 1, r.key_pos = 0, r.out_s = 0, r.out_p = spo, r.out_o = 2;
            break;
        case 7:  // s p o, p spo q => s q o         (p 0, q 1, s 2, o 3)
            r.a = pattern(0, spo, 0, 0, -1, 1);
            r.b = pattern(0, 0, 0, 2, 0, 3);
            r.shared = 0, r.key_pos = 1, r.out_s = 2, r.out_p = 0, r.out_pv = 1, r.out_o = 3;
            break;
        case 9:  // s type x, x sc y => s type y    (x 0, y 1, s 2)
            r.a = pattern(0, sc, 0, 0, -1, 1);
            r.b = pattern(0, type, 0, 2, -1, 0);
            r.shared = 0, r.key_pos = 2, r.out_s = 2, r.out_p = type, r.out_o = 1;
            break;
        case 11:  // x sc y, y sc z => x sc z       (x 0, y 1, z 2)
            r.a = pattern(0, sc, 0, 0, -1, 1);
            r.b = pattern(0, sc, 0, 1, -1, 2);
            r.shared = 1, r.key_pos = 0, r.out_s = 0, r.out_p = sc, r.out_o = 2;
            break;
        default:
            throw Error(TID_E_INVALID_ARG, "entail: rule must be 2, 3, 5, 7, 9 or 11");
    }
    return r;
}

int col_in(const tid_table *t, int32_t var) {
    for (int c = 0; c < t->ncols; ++c)
        if (t->vars[c] == var) return c;
    throw Error(TID_E_INTERNAL, "entail: variable missing from a result");
}

}  // namespace

std::unique_ptr<tid_table> entail(tid_ctx *ctx, const tid_graph *g, int rule,
                                  const uint32_t *vocab) {
    TID_REQUIRE(vocab, TID_E_INVALID_ARG, "entail: null vocabulary");
    for (int i = 0; i < 5; ++i)
        TID_REQUIRE(vocab[i] != 0, TID_E_INVALID_ARG, "entail: vocabulary IDs must be >= 1");
    const Rule r = rule_of(rule, vocab);
    // first search: the schema pattern; its values of the shared variable
    // are the keys of the second search
    std::unique_ptr<tid_table> ta;
    scan_multi(ctx, g, &r.a, 1, &ta);
    tid_table *tap = ta.get();
    resolve_counts(ctx, &tap, 1);
    const int ka = col_in(ta.get(), r.shared);
    auto tb = scan_keyed(ctx, g, r.b, r.key_pos, ta->col[ka], ta->nrows);
    tid_table *tbp = tb.get();
    resolve_counts(ctx, &tbp, 1);
    const int kb = col_in(tb.get(), r.shared);
    JoinPlan jp;
    for (int c = 0; c < ta->ncols; ++c) jp.lkeep.push_back(c);
    for (int c = 0; c < tb->ncols; ++c)
        if (c != kb) jp.rkeep.push_back(c);
    auto tj = join_unsorted(ctx, ta.get(), ta->nrows, ka, tb.get(), tb->nrows, kb, 0, jp,
                            kJoinInner);
    tid_table *tjp = tj.get();
    resolve_counts(ctx, &tjp, 1);
    const uint64_t n = tj->nrows;
    // derived triples (s, p, o), then distinct rows in lexicographic order
    const int32_t vars[3] = {0, 1, 2};
    auto tri = make_table(ctx, 3, vars, n);
    const int cs = col_in(tj.get(), r.out_s), co = col_in(tj.get(), r.out_o);
    if (n) {
        TID_HIP(hipMemcpyAsync(tri->col[0], tj->col[cs], n * 4, hipMemcpyDeviceToDevice,
                               ctx->stream));
        TID_HIP(hipMemcpyAsync(tri->col[2], tj->col[co], n * 4, hipMemcpyDeviceToDevice,
                               ctx->stream));
        if (r.out_p)
            fill(ctx, tri->col[1], n, r.out_p);
        else
            TID_HIP(hipMemcpyAsync(tri->col[1], tj->col[col_in(tj.get(), r.out_pv)], n * 4,
                                   hipMemcpyDeviceToDevice, ctx->stream));
    }
    set_count(ctx, tri.get(), n);
    tri->maxv_known = true;
    tri->maxv[0] = std::max({g->max_id[0], g->max_id[1], g->max_id[2]});
    tri->maxv[1] = tri->maxv[0];
    tri->maxv[2] = tri->maxv[0];
    return sort_rows(ctx, tri.get(), n, 1);
}

}  // namespace tid
