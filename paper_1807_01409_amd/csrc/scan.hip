// scan.hip -- the multi-pattern scan of Sec. 4.1 (keysArray /
// positionArray[i].query) in one kernel with LDS-resident patterns, the
// host side of every scan (patterns compiled for the device, output bounds
// from the load-time histograms, passes over the graph), and the ID-range
// filter on tables (Sec. 4.3, FILTER in range form).  The scan kernels and
// their data types are in scan_common.hpp.
#include "scan_common.hpp"

#include <algorithm>

namespace tid {

// ---------------------------------------------------------------------------
// Multi-pattern pass (Sec. 4.1): up to 16 patterns tested against every triple
// of one read of the graph.  The patterns and output descriptors live in LDS
// and are walked by a runtime loop, so the register footprint does not grow
// with the number of patterns.  Compaction and placement follow the range
// scheme of compact.hpp, with one staging area per pattern.
// ---------------------------------------------------------------------------

struct MultiOut {
    uint32_t *col[3];
    uint64_t cap;
    uint64_t *count;
    int32_t ncols;
    uint32_t stage_off, stage_cap;
};

struct MultiArgs {
    DevPattern pat[TID_MAX_MULTI];
    MultiOut out[TID_MAX_MULTI];
    int32_t k;
    uint32_t P;
    uint64_t range;
    uint32_t epoch;  // stamp of this launch's count words
};

template <int BLOCK, int IPT>
__device__ __forceinline__ uint32_t multi_bits(const DevPattern &q, const Tri *t, uint64_t t0,
                                               uint64_t r1) {
    uint32_t mb = 0;
#pragma unroll
    for (int it = 0; it < IPT; ++it)
        if (t0 + (uint64_t)it * BLOCK + threadIdx.x < r1 && match_pattern(q, t[it]))
            mb |= 1u << it;
    return mb;
}

template <int BLOCK, int IPT>
__global__ __launch_bounds__(BLOCK) void scan_multi_kernel(const uint32_t *__restrict__ g,
                                                            uint64_t n, MultiArgs a,
                                                            uint64_t *sync, uint32_t *counters,
                                                            uint32_t *flags) {
    constexpr int NW = BLOCK / dev::kWave;
    constexpr int NV = IPT * NW;
    constexpr uint64_t TILE = (uint64_t)BLOCK * IPT;
    extern __shared__ uint32_t stage[];
    __shared__ DevPattern s_pat[TID_MAX_MULTI];
    __shared__ MultiOut s_out[TID_MAX_MULTI];
    __shared__ uint32_t s_off[TID_MAX_MULTI][NV];
    __shared__ uint32_t s_tot[TID_MAX_MULTI];
    __shared__ uint64_t s_cnt[TID_MAX_MULTI], s_staged[TID_MAX_MULTI], s_ovf[TID_MAX_MULTI];
    __shared__ uint64_t s_pre[TID_MAX_MULTI], s_run[TID_MAX_MULTI];
    __shared__ uint64_t s_red[TID_MAX_MULTI][NW];
    __shared__ uint32_t s_wg;

    const int tid = threadIdx.x, wave = tid / dev::kWave, lane = tid % dev::kWave;
    const int k = a.k;
    const uint32_t P = a.P;
    const uint64_t stamp = (uint64_t)a.epoch << kEpochShift;
    // thread j copies descriptor j (static indices into the kernel arguments)
#pragma unroll
    for (int j = 0; j < TID_MAX_MULTI; ++j)
        if (tid == j && j < k) {
            s_pat[j] = a.pat[j];
            s_out[j] = a.out[j];
            s_cnt[j] = 0;
            s_staged[j] = 0;
            s_ovf[j] = kNoTile;
        }
    if (tid == 0) s_wg = atomicAdd(&counters[0], 1u);
    __syncthreads();
    const uint32_t wg = s_wg;
    const uint64_t r0 = (uint64_t)wg * a.range;
    const uint64_t r1 = min(n, r0 + a.range);
    Tri t[IPT];

    auto load_tile = [&](uint64_t t0) {
#pragma unroll
        for (int it = 0; it < IPT; ++it) {
            const uint64_t i = t0 + (uint64_t)it * BLOCK + tid;
            if (i < r1) {  // streamed once: non-temporal loads
                t[it].v[0] = __builtin_nontemporal_load(g + 3 * i);
                t[it].v[1] = __builtin_nontemporal_load(g + 3 * i + 1);
                t[it].v[2] = __builtin_nontemporal_load(g + 3 * i + 2);
            } else {
                t[it].v[0] = t[it].v[1] = t[it].v[2] = 0;
            }
        }
    };
    auto count_tile = [&](uint64_t t0) {
        for (int j = 0; j < k; ++j) {
            const uint32_t mb = multi_bits<BLOCK, IPT>(s_pat[j], t, t0, r1);
#pragma unroll
            for (int it = 0; it < IPT; ++it) {
                const uint64_t b = dev::ballot((mb >> it) & 1u);
                if (lane == 0) s_off[j][it * NW + wave] = (uint32_t)__popcll(b);
            }
        }
        __syncthreads();
        for (int j = wave; j < k; j += NW) {
            const uint32_t tot = dev::offsets_in_place<NV>(s_off[j]);
            if (lane == 0) s_tot[j] = tot;
        }
        __syncthreads();
    };

    // ---- phase 1 ------------------------------------------------------------
    for (uint64_t t0 = r0; t0 < r1; t0 += TILE) {
        load_tile(t0);
        count_tile(t0);
        for (int j = 0; j < k; ++j) {
            const MultiOut &o = s_out[j];
            const uint64_t cnt = s_cnt[j];
            if (o.ncols == 0 || s_ovf[j] != kNoTile || cnt + s_tot[j] > o.stage_cap) continue;
            const DevPattern &q = s_pat[j];
            const uint32_t mb = multi_bits<BLOCK, IPT>(q, t, t0, r1);
#pragma unroll
            for (int it = 0; it < IPT; ++it) {
                const bool bit = (mb >> it) & 1u;
                const uint64_t b = dev::ballot(bit);
                if (bit) {
                    const uint32_t r =
                        (uint32_t)cnt + s_off[j][it * NW + wave] + dev::rank_in_mask(b);
                    TID_FOR_COLS(3, c, o.ncols)
                        stage[o.stage_off + (uint32_t)c * o.stage_cap + r] = pick(t[it], q.src[c]);
                }
            }
        }
        __syncthreads();
        if (tid < k) {
            if (s_ovf[tid] == kNoTile && s_cnt[tid] + s_tot[tid] > s_out[tid].stage_cap) {
                s_ovf[tid] = t0;
                s_staged[tid] = s_cnt[tid];
            }
            s_cnt[tid] += s_tot[tid];
        }
    }
    __syncthreads();

    // ---- prefix over earlier ranges ----------------------------------------
    if (tid < k) {
        if (s_ovf[tid] == kNoTile) s_staged[tid] = s_cnt[tid];
        dev::publish(&sync[(size_t)tid * P + wg], stamp | s_cnt[tid]);
    }
    for (int j = 0; j < k; ++j) {
        uint64_t w[kPrefixPer];
#pragma unroll
        for (int u = 0; u < kPrefixPer; ++u) {
            const uint32_t i = tid + u * BLOCK;
            w[u] = i < wg ? dev::peek(&sync[(size_t)j * P + i]) : stamp;
        }
        uint64_t part = 0;
#pragma unroll
        for (int u = 0; u < kPrefixPer; ++u) {
            const uint32_t i = tid + u * BLOCK;
            uint32_t spins = 0;
            while ((w[u] >> kEpochShift) != a.epoch) {
                if (++spins > kSpinLimit) {
                    atomicOr(&flags[0], 1u);
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
                w[u] = dev::peek(&sync[(size_t)j * P + i]);
            }
            part += w[u] & kRowsMask;
        }
        part = dev::wave_sum(part);
        if (lane == 0) s_red[j][wave] = part;
    }
    __syncthreads();
    if (tid < k) {
        uint64_t sum = 0;
        for (int w = 0; w < NW; ++w) sum += s_red[tid][w];
        s_pre[tid] = sum;
        s_run[tid] = s_staged[tid];
    }
    __syncthreads();

    // ---- phase 2 ------------------------------------------------------------
    for (int j = 0; j < k; ++j) {
        const MultiOut &o = s_out[j];
        if (o.ncols == 0) continue;
        const uint64_t pre = s_pre[j];
        const uint32_t st = (uint32_t)s_staged[j];
        for (uint32_t r = tid; r < st; r += BLOCK) {
            const uint64_t dst = pre + r;
            if (dst < o.cap) {
                TID_FOR_COLS(3, c, o.ncols)
                    o.col[c][dst] = stage[o.stage_off + (uint32_t)c * o.stage_cap + r];
            } else {
                atomicOr(&flags[1], 1u);
            }
        }
    }
    uint64_t first = kNoTile;
    for (int j = 0; j < k; ++j) first = min(first, s_ovf[j]);
    for (uint64_t t0 = first; t0 < r1; t0 += TILE) {
        load_tile(t0);
        count_tile(t0);
        for (int j = 0; j < k; ++j) {
            if (s_ovf[j] > t0) continue;
            const MultiOut &o = s_out[j];
            const DevPattern &q = s_pat[j];
            const uint64_t base = s_pre[j] + s_run[j];
            const uint32_t mb = multi_bits<BLOCK, IPT>(q, t, t0, r1);
#pragma unroll
            for (int it = 0; it < IPT; ++it) {
                const bool bit = (mb >> it) & 1u;
                const uint64_t b = dev::ballot(bit);
                if (bit) {
                    const uint64_t dst = base + s_off[j][it * NW + wave] + dev::rank_in_mask(b);
                    if (dst < o.cap) {
                        TID_FOR_COLS(3, c, o.ncols) o.col[c][dst] = pick(t[it], q.src[c]);
                    } else {
                        atomicOr(&flags[1], 1u);
                    }
                }
            }
        }
        __syncthreads();
        if (tid < k && s_ovf[tid] <= t0) s_run[tid] += s_tot[tid];
    }
    if (wg == P - 1 && tid < k) *s_out[tid].count = s_pre[tid] + s_cnt[tid];
    __syncthreads();
    if (tid == 0) {
        const uint32_t d = __hip_atomic_fetch_add(&counters[1], 1u, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
        if (d == P - 1) {
            __hip_atomic_store(&counters[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&counters[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

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

DevPattern compile_pattern(const tid_pattern &p, const PatternSet *set,
                           const ScanFilter *filter) {
    DevPattern d{};
    d.set_pos = -1;
    d.fpos = -1;
    if (filter && filter->pos >= 0) {
        TID_REQUIRE(filter->pos <= 2 && filter->bits, TID_E_INTERNAL, "scan filter: bad position");
        d.fbits = filter->bits;
        d.fmask = filter->mask;
        d.fpos = filter->pos;
        d.fexact = filter->exact;
    }
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
    for (int x = 0; x < 3; ++x) {
        d.rlo[x] = 0;
        d.rmax[x] = 0xFFFFFFFFu;
    }
    if (p.range_pos >= 0 && p.hi > p.lo) {
        d.rlo[p.range_pos] = p.lo;
        d.rmax[p.range_pos] = p.hi - p.lo - 1;
    }
    for (int j = 0; j < d.ncols; ++j) d.src[j] = src[j];
    if (set && set->pos >= 0) {
        TID_REQUIRE(set->pos <= 2 && set->n >= 1 && set->n <= kMaxSet, TID_E_INTERNAL,
                    "pattern set: bad position or size");
        d.key[set->pos] = 0;
        d.msk[set->pos] = 0;
        d.set_pos = set->pos;
        d.nset = set->n;
        for (int i = 0; i < set->n; ++i) d.set[i] = set->v[i];
    }
    if (p.range_pos >= 0 && p.hi <= p.lo) {
        // an empty range: require ID 0 at a position without a value set,
        // which no stored triple has (tid_load refuses ID 0)
        const int x = d.set_pos == 0 ? 1 : 0;
        d.key[x] = 0;
        d.msk[x] = 0xFFFFFFFFu;
    }
    return d;
}

// Upper bound on the rows a pattern can produce, from the load-time
// histograms: the count of its rarest constant, and of its range; with a
// value set, the sum of that bound over the set's values.
static uint64_t pattern_bound(const tid_graph *g, const tid_pattern &p,
                              const PatternSet *set = nullptr) {
    if (set && set->pos >= 0) {
        uint64_t sum = 0;
        for (int i = 0; i < set->n; ++i) {
            tid_pattern q = p;
            (set->pos == 0 ? q.s : set->pos == 1 ? q.p : q.o) = set->v[i];
            sum += pattern_bound(g, q);
        }
        return std::min<uint64_t>(sum, g->n);
    }
    uint64_t b = g->n;
    const uint32_t c[3] = {p.s, p.p, p.o};
    for (int x = 0; x < 3; ++x)
        if (c[x] != 0) b = std::min(b, g->count_in(x, c[x], (uint64_t)c[x] + 1));
    if (p.range_pos >= 0) b = std::min(b, g->count_in(p.range_pos, p.lo, p.hi));
    return b;
}

uint64_t pattern_output_bound(const tid_graph *g, const tid_pattern &p, const PatternSet *set) {
    return pattern_bound(g, p, set);
}

template <int BLOCK, int IPT>
static void launch_multi(tid_ctx *ctx, const tid_graph *g, MultiArgs &a, int k, uint32_t sw) {
    constexpr uint64_t TILE = (uint64_t)BLOCK * IPT;
    auto kern = scan_multi_kernel<BLOCK, IPT>;
    const size_t lds = (size_t)sw * sizeof(uint32_t);
    const int blocks_per_cu = resident_blocks((const void *)kern, BLOCK, lds);
    uint64_t cols_total = 0;
    for (int j = 0; j < k; ++j) cols_total += (uint64_t)a.out[j].ncols;
    const uint32_t rows_per = (uint32_t)(sw / std::max<uint64_t>(cols_total, 1));
    uint32_t off = 0;
    for (int j = 0; j < k; ++j) {
        a.out[j].stage_off = off;
        a.out[j].stage_cap = a.out[j].ncols ? rows_per : 0xFFFFFFFFu;
        off += rows_per * (uint32_t)a.out[j].ncols;
    }
    const uint64_t n = g->n;
    const uint64_t tiles = (n + TILE - 1) / TILE;
    const uint64_t resident = (uint64_t)blocks_per_cu * (uint64_t)device_cus(ctx);
    uint64_t P = std::max<uint64_t>(1, std::min({tiles, resident, (uint64_t)BLOCK * kPrefixPer}));
    const uint64_t range = (tiles + P - 1) / P * TILE;
    P = (n + range - 1) / range;
    a.k = k;
    a.P = (uint32_t)P;
    a.range = range;
    uint64_t *state = nullptr;
    a.epoch = ctx->next_epoch(((size_t)k * P + 1) * sizeof(uint64_t), &state);
    uint64_t *sync = state + 1;
    uint32_t *counters = reinterpret_cast<uint32_t *>(state);
    hipLaunchKernelGGL(kern, dim3((uint32_t)P), dim3(BLOCK), lds, ctx->stream,
                       g->triples(), n, a, sync, counters, ctx->d_flags);
    TID_HIP(hipGetLastError());
}

// multi_kernel option: 0 (default) the unrolled kernel for up to 4 patterns,
// and more patterns as several passes of at most 4 (balanced); 1 the LDS
// pattern-loop kernel (one pass for up to 16).  Per pattern, the loop kernel
// stages a sixteenth of the LDS and falls back to re-reading the graph once
// the outputs are dense; four-pattern passes keep the automatic choice
// between block-ranged and chunked placement, and measure 2.5x faster for
// eight patterns of ~1% selectivity.  multi_shape 0 is 512 threads x 8
// triples for both.
void scan_slice(tid_ctx *ctx, const tid_graph *g, const tid_pattern &p, tid_table *out,
                const ScanFilter *filter);

// With the predicate-partitioned layout built, patterns that all have a
// constant predicate (and no value set) read only their predicates' slices,
// one pass per pattern, when those slices (8 B per triple) add up to less
// than one read of the TripleID array (12 B per triple).
static bool use_slices(tid_ctx *ctx, const tid_graph *g, const tid_pattern *pats, int k,
                       const PatternSet *sets) {
    if (!g->partitioned || ctx->opt.layout == 0) return false;
    uint64_t rows = 0;
    for (int j = 0; j < k; ++j) {
        if (pats[j].p == 0 || (sets && sets[j].pos >= 0)) return false;
        rows += g->count_in(1, pats[j].p, (uint64_t)pats[j].p + 1);
    }
    return 8 * rows < 12 * g->n;
}

static void run_scan_any(tid_ctx *ctx, const tid_graph *g, const tid_pattern *pats, int k,
                         tid_table *const *outs, const PatternSet *sets,
                         const ScanFilter *filters) {
    if (use_slices(ctx, g, pats, k, sets)) {
        for (int j = 0; j < k; ++j) scan_slice(ctx, g, pats[j], outs[j], filters ? &filters[j] : nullptr);
        return;
    }
    if (k == 1) {
        run_scan1(ctx, g, pats, k, outs, sets, filters);
        return;
    }
    const int shape = (int)ctx->opt.multi_shape;
    if (ctx->opt.multi_kernel == 0) {
        const int passes = (k + 3) / 4;
        for (int p0 = 0, p = 0; p < passes; ++p) {
            const int m = (k - p0) / (passes - p);
            const PatternSet *ps = sets ? sets + p0 : nullptr;
            const ScanFilter *pf = filters ? filters + p0 : nullptr;
            if (m == 1)
                run_scan1(ctx, g, pats + p0, 1, outs + p0, ps, pf);
            else if (m == 2)
                run_unrolled_shape2(ctx, g, pats + p0, m, outs + p0, shape, ps, pf);
            else
                run_unrolled_shape4(ctx, g, pats + p0, m, outs + p0, shape, ps, pf);
            p0 += m;
        }
        return;
    }
    MultiArgs a{};
    for (int j = 0; j < k; ++j) {
        a.pat[j] = compile_pattern(pats[j], sets ? &sets[j] : nullptr,
                                   filters ? &filters[j] : nullptr);
        for (int c = 0; c < outs[j]->ncols; ++c) a.out[j].col[c] = outs[j]->col[c];
        a.out[j].cap = outs[j]->cap;
        a.out[j].count = outs[j]->d_count;
        a.out[j].ncols = outs[j]->ncols;
    }
    const uint32_t sw = stage_words(ctx);
    if (shape == 1)
        launch_multi<512, 16>(ctx, g, a, k, sw);
    else if (shape == 2)
        launch_multi<256, 16>(ctx, g, a, k, sw);
    else if (shape == 3)
        launch_multi<1024, 8>(ctx, g, a, k, sw);
    else
        launch_multi<512, 8>(ctx, g, a, k, sw);
}

bool wide_eligible(const tid_pattern &p);
void run_wide(tid_ctx *ctx, const tid_graph *g, const tid_pattern *pats, int k,
              tid_table *const *outs, const ScanFilter *filters);
void run_wide_parts(tid_ctx *ctx, const tid_graph *g, const tid_pattern *pats, int k,
                    tid_table *const *outs, const ScanFilter *filters);
void index_semijoin(tid_ctx *ctx, const tid_graph *g, const tid_pattern *pats,
                    const ScanFilter *filters, int J, std::unique_ptr<tid_table> *outs);

// A pattern whose rows are exactly its predicate's slice of the partitioned
// layout: a constant predicate, subject and object free (and not one
// variable), no range, no filter and no value set.
static bool whole_slice(const tid_pattern &p, const PatternSet *set, const ScanFilter *f) {
    return p.p != 0 && p.s == 0 && p.o == 0 && p.range_pos < 0 && !(p.vs >= 0 && p.vs == p.vo) &&
           (!set || set->pos < 0) && (!f || f->pos < 0);
}

// The rows of a whole-slice pattern without a pass: the table's columns point
// into the partitioned layout (read only, valid while the graph's layout is).
static std::unique_ptr<tid_table> slice_table(tid_ctx *ctx, const tid_graph *g,
                                              const tid_pattern &p) {
    int32_t vars[3], src[3];
    const int nc = pattern_schema(p, vars, src);
    const auto &cdf = g->cdf[1];
    const uint64_t last = cdf.size() - 1;
    const uint64_t a = cdf[std::min<uint64_t>(p.p, last)];
    const uint64_t b = cdf[std::min<uint64_t>((uint64_t)p.p + 1, last)];
    auto t = make_table(ctx, nc, vars, 0);  // the count word only
    for (int c = 0; c < nc; ++c) {
        t->col[c] = const_cast<uint32_t *>(
            (src[c] == 0 ? g->part_s : g->part_o).get<const uint32_t>() + a);
        t->maxv[c] = g->max_id[src[c]];
    }
    t->maxv_known = true;
    t->cap = b - a;
    set_count_later(ctx, t.get(), b - a);  // written when scan_many returns
    return t;
}

// Any number of patterns: those with a constant (bucketable) predicate go
// through wide passes of up to 1024 patterns when there are at least
// `wide_min` of them; the rest through passes of up to 16.  With the graph's
// partitioned layout built, a constant predicate's patterns read only its
// slice: a whole-slice pattern reads nothing (its table is the slice), the
// others go through segment passes over the slices they need.  Tables that
// point into the layout are for plan evaluation only: every plan result is a
// table of its own.
void scan_many(tid_ctx *ctx, const tid_graph *g, const tid_pattern *pats, int k,
               std::unique_ptr<tid_table> *outs, const PatternSet *sets,
               const ScanFilter *filters) {
    PendingCountsGuard counts_guard(ctx);
    const int64_t wide_min = ctx->opt.wide_min > 0 ? ctx->opt.wide_min : 8;
    const bool parts = g->partitioned && ctx->opt.layout != 0 && g->n > 0 &&
                       ctx->opt.capacity_override <= 0 && !g->cdf[1].empty();
    // semi-joins by index: every such pattern of the call in one batch
    std::vector<int> idx;
    for (int j = 0; j < k && filters; ++j)
        if (filters[j].index) idx.push_back(j);
    if (!idx.empty()) {
        std::vector<tid_pattern> ip;
        std::vector<ScanFilter> ifl;
        for (int j : idx) {
            ip.push_back(pats[j]);
            ifl.push_back(filters[j]);
        }
        std::vector<std::unique_ptr<tid_table>> io(idx.size());
        index_semijoin(ctx, g, ip.data(), ifl.data(), (int)idx.size(), io.data());
        for (size_t x = 0; x < idx.size(); ++x) outs[idx[x]] = std::move(io[x]);
    }
    std::vector<int> wide, rest;
    for (int j = 0; j < k; ++j) {
        const PatternSet *set = sets ? &sets[j] : nullptr;
        const ScanFilter *f = filters ? &filters[j] : nullptr;
        if (f && f->index) continue;
        if (parts && whole_slice(pats[j], set, f)) {
            outs[j] = slice_table(ctx, g, pats[j]);
            continue;
        }
        const bool ok = (!set || set->pos < 0) && !(f && f->pos >= 0 && f->exact) &&
                        wide_eligible(pats[j]);
        (ok ? wide : rest).push_back(j);
    }
    if (parts && wide.size() >= 2) {
        // segment passes, however few the patterns: one read of their slices
        // to count and one to write, against a graph read per 4 patterns
        for (size_t w0 = 0; w0 < wide.size(); w0 += 1024) {
            const int m = (int)std::min<size_t>(1024, wide.size() - w0);
            std::vector<tid_pattern> wp(m);
            std::vector<ScanFilter> wf(m);
            std::vector<tid_table *> wt(m);
            for (int j = 0; j < m; ++j) {
                const tid_pattern &p = pats[wide[w0 + j]];
                int32_t vars[3], src[3];
                const int nc = pattern_schema(p, vars, src);
                auto t = make_table(ctx, nc, vars, pattern_bound(g, p));
                for (int c = 0; c < nc; ++c) t->maxv[c] = g->max_id[src[c]];
                t->maxv_known = true;
                wp[j] = p;
                if (filters) wf[j] = filters[wide[w0 + j]];
                wt[j] = t.get();
                outs[wide[w0 + j]] = std::move(t);
            }
            run_wide_parts(ctx, g, wp.data(), m, wt.data(), wf.data());
        }
        wide.clear();
    }
    if ((int64_t)wide.size() < wide_min || ctx->opt.capacity_override > 0 || g->n == 0) {
        rest.insert(rest.end(), wide.begin(), wide.end());
        wide.clear();
    }
    // wide passes: tables sized by the histogram bounds, which cannot overflow
    for (size_t w0 = 0; w0 < wide.size(); w0 += 1024) {
        const int m = (int)std::min<size_t>(1024, wide.size() - w0);
        std::vector<tid_pattern> wp(m);
        std::vector<ScanFilter> wf(m);
        std::vector<tid_table *> wt(m);
        for (int j = 0; j < m; ++j) {
            const tid_pattern &p = pats[wide[w0 + j]];
            int32_t vars[3], src[3];
            const int nc = pattern_schema(p, vars, src);
            auto t = make_table(ctx, nc, vars, pattern_bound(g, p));
            for (int c = 0; c < nc; ++c) t->maxv[c] = g->max_id[src[c]];
            t->maxv_known = true;
            wp[j] = p;
            if (filters) wf[j] = filters[wide[w0 + j]];
            wt[j] = t.get();
            outs[wide[w0 + j]] = std::move(t);
        }
        run_wide(ctx, g, wp.data(), m, wt.data(), wf.data());
    }
    for (size_t r0 = 0; r0 < rest.size(); r0 += TID_MAX_MULTI) {
        const int m = (int)std::min<size_t>(TID_MAX_MULTI, rest.size() - r0);
        std::vector<tid_pattern> rp(m);
        std::vector<PatternSet> rs(m);
        std::vector<ScanFilter> rf(m);
        std::unique_ptr<tid_table> rt[TID_MAX_MULTI];
        for (int j = 0; j < m; ++j) {
            rp[j] = pats[rest[r0 + j]];
            if (sets) rs[j] = sets[rest[r0 + j]];
            if (filters) rf[j] = filters[rest[r0 + j]];
        }
        scan_multi(ctx, g, rp.data(), m, rt, rs.data(), rf.data());
        for (int j = 0; j < m; ++j) outs[rest[r0 + j]] = std::move(rt[j]);
    }
    flush_counts(ctx);  // the whole-slice tables' count words
}

void scan_multi(tid_ctx *ctx, const tid_graph *g, const tid_pattern *pats, int k,
                std::unique_ptr<tid_table> *outs, const PatternSet *sets,
                const ScanFilter *filters) {
    TID_REQUIRE(k >= 1 && k <= TID_MAX_MULTI, TID_E_INVALID_ARG, "scan: 1..16 patterns per pass");
    std::vector<uint64_t> bound(k);
    for (int j = 0; j < k; ++j) {
        int32_t vars[3], src[3];
        const int nc = pattern_schema(pats[j], vars, src);
        bound[j] = pattern_bound(g, pats[j], sets ? &sets[j] : nullptr);
        uint64_t cap = ctx->opt.capacity_override > 0 ? (uint64_t)ctx->opt.capacity_override
                                                      : bound[j];
        outs[j] = make_table(ctx, nc, vars, cap);
        for (int c = 0; c < nc; ++c) outs[j]->maxv[c] = g->max_id[src[c]];
        outs[j]->maxv_known = true;
    }
    if (g->n == 0) {
        for (int j = 0; j < k; ++j) set_count(ctx, outs[j].get(), 0);
        return;
    }
    std::vector<tid_table *> raw(k);
    for (int j = 0; j < k; ++j) raw[j] = outs[j].get();
    run_scan_any(ctx, g, pats, k, raw.data(), sets, filters);

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
    std::vector<PatternSet> rs;
    std::vector<ScanFilter> rf;
    std::vector<tid_table *> rt;
    for (int j : redo) {
        const uint64_t need = outs[j]->nrows;
        auto bigger = make_table(ctx, outs[j]->ncols, outs[j]->vars, need);
        copy_bounds(bigger.get(), outs[j].get(), nullptr, outs[j]->ncols);
        bigger->maxv_known = outs[j]->maxv_known;
        outs[j] = std::move(bigger);
        rp.push_back(pats[j]);
        rs.push_back(sets ? sets[j] : PatternSet{});
        rf.push_back(filters ? filters[j] : ScanFilter{});
        rt.push_back(outs[j].get());
    }
    run_scan_any(ctx, g, rp.data(), (int)rp.size(), rt.data(), rs.data(), rf.data());
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
    out->maxv_known = t->maxv_known;
    copy_bounds(out.get(), t, nullptr, t->ncols);
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
    again->maxv_known = t->maxv_known;
    copy_bounds(again.get(), t, nullptr, t->ncols);
    run_filter(ctx, t, in_rows, col, lo, hi, again.get());
    return again;
}

}  // namespace tid
