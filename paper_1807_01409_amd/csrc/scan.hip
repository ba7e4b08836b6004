// scan.hip -- the triple-pattern scan (Sec. 3, GPUSearch of Algorithm 1) with
// order-preserving stream compaction of the matches into binding columns,
// the multi-pattern single pass (Sec. 4.1, keysArray / positionArray[i].query),
// and the ID-range filter on tables (Sec. 4.3, FILTER in range form).
//
// Layout and mapping.  The graph is the TripleID array: n rows of (s,p,o)
// uint32, 12 bytes per triple, in HBM.  A workgroup of BLOCK threads takes
// tiles of BLOCK*IPT consecutive triples; item `it` of thread `tid` is triple
// tile_base + it*BLOCK + tid, so each load instruction of a wave reads 64
// consecutive triples (768 contiguous bytes) with one 12-byte load per lane.
// Match bits become wave ballots; per (item, wave) match counts go to LDS and
// one wave turns them into exclusive offsets in triple order.  The range
// compaction of compact.hpp places the rows, so the graph is read once and
// the output keeps ascending triple position.
#include "compact.hpp"

#include <algorithm>

namespace tid {

struct __attribute__((packed, aligned(4))) Tri {
    uint32_t v[3];
};

// A pattern compiled for the device: constant test by xor+mask, equalities
// between free positions named by one variable, optional range on one
// position as (x - lo) < span (unsigned), output column sources.
struct DevPattern {
    uint32_t key[3];
    uint32_t msk[3];
    uint32_t eq;      // bit0: s==p, bit1: s==o, bit2: p==o
    int32_t rpos;     // -1: no range
    uint32_t lo, span;
    int32_t ncols;
    int32_t src[3];
};

template <int MAXK>
struct ScanSrc {
    const uint32_t *g;
    uint64_t n;
    DevPattern pat[MAXK];
    using Item = Tri;
    __device__ __forceinline__ Item load(uint64_t i) const {
        return *reinterpret_cast<const Tri *>(g + 3 * i);
    }
    __device__ __forceinline__ bool match(int j, const Item &t) const;
    __device__ __forceinline__ uint32_t value(int j, int c, const Item &t, uint64_t) const;
};

__device__ __forceinline__ uint32_t pick(const Tri &t, int pos) {
    return pos == 0 ? t.v[0] : (pos == 1 ? t.v[1] : t.v[2]);
}

__device__ __forceinline__ bool match_pattern(const DevPattern &q, const Tri &t) {
    uint32_t diff = ((t.v[0] ^ q.key[0]) & q.msk[0]) | ((t.v[1] ^ q.key[1]) & q.msk[1]) |
                    ((t.v[2] ^ q.key[2]) & q.msk[2]);
    bool ok = diff == 0;
    ok &= !(q.eq & 1u) || t.v[0] == t.v[1];
    ok &= !(q.eq & 2u) || t.v[0] == t.v[2];
    ok &= !(q.eq & 4u) || t.v[1] == t.v[2];
    if (q.rpos >= 0) ok &= (pick(t, q.rpos) - q.lo) < q.span;
    return ok;
}

template <int MAXK>
__device__ __forceinline__ bool ScanSrc<MAXK>::match(int j, const Item &t) const {
    return match_pattern(pat[j], t);
}

template <int MAXK>
__device__ __forceinline__ uint32_t ScanSrc<MAXK>::value(int j, int c, const Item &t,
                                                         uint64_t) const {
    return pick(t, pat[j].src[c]);
}

// Rows of a table whose column `key` lies in [lo, lo + span).
struct FilterSrc {
    const uint32_t *in[TID_MAX_COLS];
    const uint32_t *key;
    uint64_t n;
    uint32_t lo, span;
    using Item = uint32_t;
    __device__ __forceinline__ Item load(uint64_t i) const { return key[i]; }
    __device__ __forceinline__ bool match(int, Item x) const { return (x - lo) < span; }
    __device__ __forceinline__ uint32_t value(int, int c, Item, uint64_t i) const {
        return in[c][i];
    }
};

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

int pattern_schema(const tid_pattern &p, int32_t *vars, int32_t *src) {
    const uint32_t c[3] = {p.s, p.p, p.o};
    const int32_t v[3] = {p.vs, p.vp, p.vo};
    for (int x = 0; x < 3; ++x) {
        TID_REQUIRE(v[x] >= -1, TID_E_INVALID_ARG, "pattern: variable ids must be >= -1");
        TID_REQUIRE(c[x] == 0 || v[x] == -1, TID_E_INVALID_ARG,
                    "pattern: a bound position cannot name a variable");
    }
    TID_REQUIRE(p.range_pos >= -1 && p.range_pos <= 2, TID_E_INVALID_ARG,
                "pattern: range_pos must be -1, 0, 1 or 2");
    int k = 0;
    for (int x = 0; x < 3; ++x) {
        if (v[x] < 0) continue;
        bool seen = false;
        for (int j = 0; j < k; ++j) seen |= vars[j] == v[x];
        if (!seen) {
            vars[k] = v[x];
            src[k] = x;
            ++k;
        }
    }
    return k;
}

static DevPattern compile_pattern(const tid_pattern &p) {
    DevPattern d{};
    int32_t vars[3], src[3];
    d.ncols = pattern_schema(p, vars, src);
    const uint32_t c[3] = {p.s, p.p, p.o};
    const int32_t v[3] = {p.vs, p.vp, p.vo};
    for (int x = 0; x < 3; ++x) {
        d.key[x] = c[x];
        d.msk[x] = c[x] ? 0xFFFFFFFFu : 0u;
    }
    if (v[0] >= 0 && v[0] == v[1]) d.eq |= 1u;
    if (v[0] >= 0 && v[0] == v[2]) d.eq |= 2u;
    if (v[1] >= 0 && v[1] == v[2]) d.eq |= 4u;
    d.rpos = p.range_pos;
    d.lo = p.lo;
    d.span = p.hi > p.lo ? p.hi - p.lo : 0u;
    for (int j = 0; j < d.ncols; ++j) d.src[j] = src[j];
    return d;
}

// Upper bound on the rows a pattern can produce, from the load-time
// histograms: the count of its rarest constant, and of its range.
static uint64_t pattern_bound(const tid_graph *g, const tid_pattern &p) {
    uint64_t b = g->n;
    const uint32_t c[3] = {p.s, p.p, p.o};
    for (int x = 0; x < 3; ++x)
        if (c[x] != 0) b = std::min(b, g->count_in(x, c[x], (uint64_t)c[x] + 1));
    if (p.range_pos >= 0) b = std::min(b, g->count_in(p.range_pos, p.lo, p.hi));
    return b;
}

struct Shape {
    int block, ipt;
};

static Shape scan_shape(tid_ctx *ctx) {
    Shape s{512, 16};
    if (ctx->opt.scan_block) s.block = (int)ctx->opt.scan_block;
    if (ctx->opt.scan_items) s.ipt = (int)ctx->opt.scan_items;
    return s;
}

static uint32_t stage_words(tid_ctx *ctx) {
    return ctx->opt.stage_words > 0 ? (uint32_t)ctx->opt.stage_words : 16384u;
}

// One pass over the graph for k patterns into the given tables.
template <int MAXK>
static void run_scan(tid_ctx *ctx, const tid_graph *g, const tid_pattern *pats, int k,
                     tid_table *const *outs) {
    ScanSrc<MAXK> src{};
    src.g = g->data.get<const uint32_t>();
    src.n = g->n;
    CompactArgs<MAXK, 3> a{};
    for (int j = 0; j < k; ++j) {
        src.pat[j] = compile_pattern(pats[j]);
        for (int c = 0; c < outs[j]->ncols; ++c) a.out[j].col[c] = outs[j]->col[c];
        a.out[j].cap = outs[j]->cap;
        a.out[j].count = outs[j]->d_count;
        a.out[j].ncols = outs[j]->ncols;
    }
    const Shape sh = scan_shape(ctx);
    const uint32_t sw = stage_words(ctx);
#define TID_SCAN_CASE(B, I)                                                         \
    if (sh.block == B && sh.ipt == I) {                                             \
        launch_compact<ScanSrc<MAXK>, B, I, MAXK, 3>(ctx, src, a, k, sw);          \
        return;                                                                     \
    }
    TID_SCAN_CASE(256, 16)
    TID_SCAN_CASE(256, 8)
    TID_SCAN_CASE(256, 32)
    TID_SCAN_CASE(512, 8)
    TID_SCAN_CASE(512, 16)
    TID_SCAN_CASE(1024, 4)
    TID_SCAN_CASE(1024, 8)
    TID_SCAN_CASE(128, 16)
    TID_SCAN_CASE(128, 32)
#undef TID_SCAN_CASE
    throw Error(TID_E_INVALID_ARG, "scan: unsupported (block, items) shape");
}

static void run_scan_any(tid_ctx *ctx, const tid_graph *g, const tid_pattern *pats, int k,
                         tid_table *const *outs) {
    if (k == 1)
        run_scan<1>(ctx, g, pats, k, outs);
    else if (k <= 4)
        run_scan<4>(ctx, g, pats, k, outs);
    else
        run_scan<TID_MAX_MULTI>(ctx, g, pats, k, outs);
}

void scan_multi(tid_ctx *ctx, const tid_graph *g, const tid_pattern *pats, int k,
                std::unique_ptr<tid_table> *outs) {
    TID_REQUIRE(k >= 1 && k <= TID_MAX_MULTI, TID_E_INVALID_ARG, "scan: 1..16 patterns per pass");
    std::vector<uint64_t> bound(k);
    for (int j = 0; j < k; ++j) {
        int32_t vars[3], src[3];
        const int nc = pattern_schema(pats[j], vars, src);
        bound[j] = pattern_bound(g, pats[j]);
        uint64_t cap = ctx->opt.capacity_override > 0 ? (uint64_t)ctx->opt.capacity_override
                                                      : bound[j];
        outs[j] = make_table(ctx, nc, vars, cap);
    }
    if (g->n == 0) {
        for (int j = 0; j < k; ++j) set_count(ctx, outs[j].get(), 0);
        return;
    }
    std::vector<tid_table *> raw(k);
    for (int j = 0; j < k; ++j) raw[j] = outs[j].get();
    run_scan_any(ctx, g, pats, k, raw.data());

    // Outputs sized by the histogram bound cannot overflow.  A smaller
    // capacity (forced for tests) is checked and, if allowed, run again at
    // the exact size the first pass counted.
    bool may_overflow = false;
    for (int j = 0; j < k; ++j) may_overflow |= outs[j]->cap < bound[j];
    if (!may_overflow) return;
    resolve_counts(ctx, raw.data(), k);
    std::vector<int> redo;
    for (int j = 0; j < k; ++j)
        if (outs[j]->nrows > outs[j]->cap) redo.push_back(j);
    if (redo.empty()) return;
    TID_REQUIRE(ctx->opt.retry, TID_E_CAPACITY, "scan: result exceeds the output capacity");
    std::vector<tid_pattern> rp;
    std::vector<tid_table *> rt;
    for (int j : redo) {
        const uint64_t need = outs[j]->nrows;
        outs[j] = make_table(ctx, outs[j]->ncols, outs[j]->vars, need);
        rp.push_back(pats[j]);
        rt.push_back(outs[j].get());
    }
    run_scan_any(ctx, g, rp.data(), (int)rp.size(), rt.data());
}

// ---------------------------------------------------------------------------
// ID-range filter over a table (stable compaction of rows)
// ---------------------------------------------------------------------------

static void run_filter(tid_ctx *ctx, const tid_table *t, uint64_t in_rows, int col, uint32_t lo,
                       uint32_t hi, tid_table *dst) {
    FilterSrc src{};
    for (int c = 0; c < t->ncols; ++c) src.in[c] = t->col[c];
    src.key = t->col[col];
    src.n = in_rows;
    src.lo = lo;
    src.span = hi > lo ? hi - lo : 0u;
    CompactArgs<1, TID_MAX_COLS> a{};
    for (int c = 0; c < t->ncols; ++c) a.out[0].col[c] = dst->col[c];
    a.out[0].cap = dst->cap;
    a.out[0].count = dst->d_count;
    a.out[0].ncols = t->ncols;
    launch_compact<FilterSrc, 256, 16, 1, TID_MAX_COLS>(ctx, src, a, 1, stage_words(ctx));
}

std::unique_ptr<tid_table> filter_range(tid_ctx *ctx, const tid_table *t, int col, uint32_t lo,
                                        uint32_t hi) {
    TID_REQUIRE(col >= 0 && col < t->ncols, TID_E_INVALID_ARG, "filter: column out of range");
    // The input row count bounds the output; it may still be on the device.
    const uint64_t in_rows = const_cast<tid_table *>(t)->rows();
    uint64_t cap = in_rows;
    if (ctx->opt.capacity_override > 0) cap = (uint64_t)ctx->opt.capacity_override;
    auto out = make_table(ctx, t->ncols, t->vars, cap);
    if (in_rows == 0) {
        set_count(ctx, out.get(), 0);
        return out;
    }
    run_filter(ctx, t, in_rows, col, lo, hi, out.get());
    if (out->cap >= in_rows) return out;
    tid_table *o = out.get();
    resolve_counts(ctx, &o, 1);
    if (out->nrows <= out->cap) return out;
    TID_REQUIRE(ctx->opt.retry, TID_E_CAPACITY, "filter: result exceeds the output capacity");
    auto again = make_table(ctx, t->ncols, t->vars, out->nrows);
    run_filter(ctx, t, in_rows, col, lo, hi, again.get());
    return again;
}

}  // namespace tid
