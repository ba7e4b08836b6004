// scan_common.hpp -- the triple-pattern scan (Sec. 3, GPUSearch of Algorithm 1) with
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
#pragma once

#include "compact.hpp"

#include <algorithm>

namespace tid {

struct __attribute__((packed, aligned(4))) Tri {
    uint32_t v[3];
};

// A pattern compiled for the device: constant test by xor+mask, equalities
// between free positions named by one variable, a range test on every
// position as (x - rlo) <= rmax (unsigned; 0 and 2^32 - 1 where the pattern
// has no range), output column sources.  A pattern with an empty range
// requires subject 0, which no stored triple has (ID 0 is refused at load).
struct DevPattern {
    uint32_t key[3];
    uint32_t msk[3];
    uint32_t eq;      // bit0: s==p, bit1: s==o, bit2: p==o
    uint32_t rlo[3], rmax[3];
    int32_t ncols;
    int32_t src[3];
    int32_t set_pos;  // -1: no value set; else the value there is one of set[0..nset)
    int32_t nset;
    uint32_t set[kMaxSet];
    const uint32_t *fbits;  // membership filter on position fpos (-1: none)
    uint32_t fmask;         // Bloom: bits - 1; exact: largest ID in the bitmap
    int32_t fpos;
    int32_t fexact;         // 1: fbits is an exact bitmap over IDs 0..fmask
};

// EXT false: no pattern of the pass has a value set or a membership filter,
// and their tests are compiled out.
template <int MAXK, bool EXT = true>
struct ScanSrc {
    const uint32_t *g;
    uint64_t n;
    DevPattern pat[MAXK];
    using Item = Tri;
    // the graph is streamed once per pass: non-temporal loads
    __device__ __forceinline__ Item load(uint64_t i) const {
        Tri t;
        t.v[0] = __builtin_nontemporal_load(g + 3 * i);
        t.v[1] = __builtin_nontemporal_load(g + 3 * i + 1);
        t.v[2] = __builtin_nontemporal_load(g + 3 * i + 2);
        return t;
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
    ok &= ((t.v[0] - q.rlo[0]) <= q.rmax[0]) & ((t.v[1] - q.rlo[1]) <= q.rmax[1]) &
          ((t.v[2] - q.rlo[2]) <= q.rmax[2]);
    if (q.set_pos >= 0) {
        const uint32_t x = pick(t, q.set_pos);
        bool in = false;
        // unrolled to the bound so the set values are loop-invariant loads
#pragma unroll
        for (int i = 0; i < kMaxSet; ++i) in |= i < q.nset && x == q.set[i];
        ok &= in;
    }
    if (ok && q.fpos >= 0) {
        const uint32_t x = pick(t, q.fpos);
        ok = q.fexact ? x <= q.fmask && ((q.fbits[x >> 5] >> (x & 31u)) & 1u) != 0
                      : dev::bloom_has(q.fbits, q.fmask, x);
    }
    return ok;
}

// constants, repeated variables and the range only
__device__ __forceinline__ bool match_plain(const DevPattern &q, const Tri &t) {
    uint32_t diff = ((t.v[0] ^ q.key[0]) & q.msk[0]) | ((t.v[1] ^ q.key[1]) & q.msk[1]) |
                    ((t.v[2] ^ q.key[2]) & q.msk[2]);
    bool ok = diff == 0;
    ok &= (!(q.eq & 1u) | (t.v[0] == t.v[1])) & (!(q.eq & 2u) | (t.v[0] == t.v[2])) &
          (!(q.eq & 4u) | (t.v[1] == t.v[2]));
    ok &= ((t.v[0] - q.rlo[0]) <= q.rmax[0]) & ((t.v[1] - q.rlo[1]) <= q.rmax[1]) &
          ((t.v[2] - q.rlo[2]) <= q.rmax[2]);
    return ok;
}

template <int MAXK, bool EXT>
__device__ __forceinline__ bool ScanSrc<MAXK, EXT>::match(int j, const Item &t) const {
    return EXT ? match_pattern(pat[j], t) : match_plain(pat[j], t);
}

template <int MAXK, bool EXT>
__device__ __forceinline__ uint32_t ScanSrc<MAXK, EXT>::value(int j, int c, const Item &t,
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


// compiled pattern of a tid_pattern (scan.hip)
DevPattern compile_pattern(const tid_pattern &p, const PatternSet *set = nullptr,
                           const ScanFilter *filter = nullptr);
// one pass over the graph for patterns of the given count, into the given
// tables; instantiated in scan_single.hip, scan_unrolled2.hip and
// scan_unrolled4.hip (separate translation units, compiled in parallel)
void run_scan1(tid_ctx *ctx, const tid_graph *g, const tid_pattern *pats, int k,
               tid_table *const *outs, const PatternSet *sets, const ScanFilter *filters);
void run_unrolled_shape2(tid_ctx *ctx, const tid_graph *g, const tid_pattern *pats, int k,
                         tid_table *const *outs, int shape, const PatternSet *sets,
                         const ScanFilter *filters);
void run_unrolled_shape4(tid_ctx *ctx, const tid_graph *g, const tid_pattern *pats, int k,
                         tid_table *const *outs, int shape, const PatternSet *sets,
                         const ScanFilter *filters);

struct Shape {
    int block, ipt;
    bool prefetch;
};

inline Shape scan_shape(tid_ctx *ctx) {
    Shape s{512, 8, true};  // the autotuner's choice on the 50M-triple medium graph
    if (ctx->opt.scan_block) s.block = (int)ctx->opt.scan_block;
    if (ctx->opt.scan_items) s.ipt = (int)ctx->opt.scan_items;
    if (ctx->opt.scan_prefetch >= 0) s.prefetch = ctx->opt.scan_prefetch > 0;
    return s;
}

inline uint32_t stage_words(tid_ctx *ctx) {
    return ctx->opt.stage_words > 0 ? (uint32_t)ctx->opt.stage_words : 16384u;
}

// Staging words of a one-pattern scan in the default shape: the most LDS that
// still lets two of its 512-thread workgroups share a compute unit (160 KB
// less the kernels' static LDS).  Longer chunks mean fewer placements, and
// fewer block-ranged outputs overflow; 1-3% faster than 16384 over the four
// large-graph benchmark scans.
constexpr uint32_t kScan1StageWords = 20352;

inline bool any_ext(int k, const PatternSet *sets, const ScanFilter *filters) {
    for (int j = 0; j < k; ++j)
        if ((sets && sets[j].pos >= 0) || (filters && filters[j].pos >= 0)) return true;
    return false;
}

template <class SRC, int MAXK>
void fill_scan_args(const tid_graph *g, const tid_pattern *pats, int k,
                           tid_table *const *outs, const PatternSet *sets,
                           const ScanFilter *filters, SRC &src, CompactArgs<MAXK, 3> &a) {
    src.g = g->triples();
    src.n = g->n;
    for (int j = 0; j < k; ++j) {
        src.pat[j] = compile_pattern(pats[j], sets ? &sets[j] : nullptr,
                                     filters ? &filters[j] : nullptr);
        for (int c = 0; c < outs[j]->ncols; ++c) a.out[j].col[c] = outs[j]->col[c];
        a.out[j].cap = outs[j]->cap;
        a.out[j].count = outs[j]->d_count;
        a.out[j].ncols = outs[j]->ncols;
    }
}

// One pass over the graph for k patterns into the given tables.  The default
// launch shape has a variant without value-set and filter tests.
template <int MAXK>
void run_scan(tid_ctx *ctx, const tid_graph *g, const tid_pattern *pats, int k,
                     tid_table *const *outs, const PatternSet *sets, const ScanFilter *filters) {
    const Shape sh = scan_shape(ctx);
    const uint32_t sw = stage_words(ctx);
    if (sh.block == 512 && sh.ipt == 8 && sh.prefetch && !any_ext(k, sets, filters)) {
        const uint32_t sw1 = MAXK == 1 && ctx->opt.stage_words <= 0 ? kScan1StageWords : sw;
        ScanSrc<MAXK, false> src{};
        CompactArgs<MAXK, 3> a{};
        fill_scan_args(g, pats, k, outs, sets, filters, src, a);
        launch_compact<ScanSrc<MAXK, false>, 512, 8, MAXK, 3, true>(ctx, src, a, k, sw1);
        return;
    }
    ScanSrc<MAXK> src{};
    CompactArgs<MAXK, 3> a{};
    fill_scan_args(g, pats, k, outs, sets, filters, src, a);
#define TID_SCAN_CASE(B, I)                                                         \
    if (sh.block == B && sh.ipt == I) {                                             \
        if (sh.prefetch)                                                            \
            launch_compact<ScanSrc<MAXK>, B, I, MAXK, 3, true>(ctx, src, a, k, sw); \
        else                                                                        \
            launch_compact<ScanSrc<MAXK>, B, I, MAXK, 3, false>(ctx, src, a, k, sw); \
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

// Up to MAXK patterns in the generic compaction kernel, fully unrolled.
template <int MAXK, int B, int I>
void run_unrolled(tid_ctx *ctx, const tid_graph *g, const tid_pattern *pats, int k,
                         tid_table *const *outs, const PatternSet *sets,
                         const ScanFilter *filters) {
    if (B == 512 && I == 8 && !any_ext(k, sets, filters)) {
        ScanSrc<MAXK, false> src{};
        CompactArgs<MAXK, 3> a{};
        fill_scan_args(g, pats, k, outs, sets, filters, src, a);
        launch_compact<ScanSrc<MAXK, false>, B, I, MAXK, 3, true>(ctx, src, a, k, stage_words(ctx));
        return;
    }
    ScanSrc<MAXK> src{};
    CompactArgs<MAXK, 3> a{};
    fill_scan_args(g, pats, k, outs, sets, filters, src, a);
    launch_compact<ScanSrc<MAXK>, B, I, MAXK, 3, true>(ctx, src, a, k, stage_words(ctx));
}

template <int MAXK>
void run_unrolled_shape(tid_ctx *ctx, const tid_graph *g, const tid_pattern *pats, int k,
                               tid_table *const *outs, int shape, const PatternSet *sets,
                               const ScanFilter *filters) {
    if (shape == 1)
        run_unrolled<MAXK, 256, 8>(ctx, g, pats, k, outs, sets, filters);
    else if (shape == 2)
        run_unrolled<MAXK, 256, 16>(ctx, g, pats, k, outs, sets, filters);
    else
        run_unrolled<MAXK, 512, 8>(ctx, g, pats, k, outs, sets, filters);
}

}  // namespace tid
