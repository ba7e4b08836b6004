// wide.hip -- one pass over the graph for many patterns at once (Sec. 4.1's
// keysArray at batch scale: a triple may answer several subqueries, and each
// subquery gets its own result).  For up to kWideMax patterns with a constant
// predicate:
//   - the patterns sit in LDS, bucketed by predicate ID, so a triple is tested
//     only against the patterns of its own predicate;
//   - every wave owns one contiguous sub-range of the graph, so the per-pattern
//     counts and ranks of a sub-range need no workgroup barrier: lanes that
//     match the same pattern in the same step are grouped with ballots and
//     their leader advances the wave's LDS counter for that pattern;
//   - count pass -> column-wise exclusive scan of the (sub-range x pattern)
//     count matrix -> write pass, which places every match at its pattern's
//     offset for the sub-range plus its rank: ascending triple position per
//     pattern, as a single-pattern scan gives;
//   - a pass reads the TripleID array, or segments of (subject, object)
//     columns, each segment the rows of one predicate in triple order (a
//     slice of the predicate-partitioned layout, or of a temporary slice).
// The graph is read twice per pass; the work per triple is the size of its
// predicate's bucket, and a wave steps through the longest bucket among its
// lanes.  A predicate that many patterns of one pass share is therefore
// sliced: the graph pass writes that predicate's (s, o) rows once, in triple
// order, in place of its patterns, and a second pass over the slice alone
// tests them, every lane on the same predicate.
#include "compact.hpp"

#include <algorithm>
#include <cmath>
#include <mutex>

namespace tid {

constexpr int kWideMax = 1024;       // patterns per pass (10-bit ids)
constexpr int kWideIdBits = 10;
constexpr uint32_t kWidePreds = 4096;  // predicate IDs 1..4095 can be bucketed
constexpr int kWideBlock = 256;
constexpr int kWideNW = kWideBlock / dev::kWave;
constexpr int kWideIPT = 8;

// A pattern with a constant predicate, compacted for LDS.
struct WidePat {
    const uint32_t *fbits;  // membership filter (Bloom bits), if flagged
    uint32_t s, o;          // constants (0 = free)
    uint32_t lo, span;      // range test (x - lo) < span on position rpos
    uint32_t flags;         // bit0 s bound, bit1 o bound, bit2 s==o, bits 3-4 range pos+1,
                            // bits 5-6 ncols, bits 8-9/10-11/12-13 source position of
                            // col 0/1/2, bit 14 filtered, bits 15-16 filter position
    uint32_t fmask;         // filter bits - 1
};
constexpr uint32_t kWideFiltered = 1u << 14;

struct WideOut {
    uint32_t *col[3];
    uint64_t cap;
};

// One predicate's rows in a segment pass: `len` rows of the subject and object
// columns from `pbase` on, all with predicate p, at virtual position vbase
// (each segment starts on a walk unit, so a unit never spans two segments).
struct WideSeg {
    uint64_t vbase, pbase;
    uint32_t len, p;
};

struct WideArgs {
    const uint32_t *g;          // AoS triples (graph pass)
    const uint32_t *ss, *so;    // segment pass: subject and object columns
    const WideSeg *segs;        // segment pass: nseg segments by ascending vbase
    uint32_t nseg;
    uint64_t n;                 // triples (graph pass) or virtual positions (segment pass)
    const WidePat *pats;      // k
    const uint32_t *bucket;   // kWidePreds words: start << 12 | len
    const uint16_t *ids;      // k pattern ids grouped by predicate
    const WideOut *outs;      // k
    uint64_t **counts_out;    // k device row-count words
    int k;
    uint64_t sub;             // triples per wave sub-range (graph pass)
    const uint64_t *wbound;   // segment pass: W + 1 sub-range bounds (virtual positions)
    uint32_t W;               // sub-ranges
    uint32_t *cnt;            // W x k counts, then offsets in place
    uint64_t *tot;            // k totals
};

struct __attribute__((packed, aligned(4))) WTri {
    uint32_t v[3];
};

__device__ __forceinline__ bool wide_match(const WidePat &q, const WTri &t) {
    bool ok = true;
    if (q.flags & 1u) ok &= t.v[0] == q.s;
    if (q.flags & 2u) ok &= t.v[2] == q.o;
    if (q.flags & 4u) ok &= t.v[0] == t.v[2];
    const uint32_t rp = (q.flags >> 3) & 3u;
    if (rp) ok &= (t.v[rp - 1] - q.lo) < q.span;
    return ok;
}

// Lanes that match the same pattern id as the calling lane (0 if it matches
// none).  No ballots beyond the first when nothing matched, and one more when
// every matching lane tests the same pattern (always so in a slice pass).
__device__ __forceinline__ uint64_t match_pid(uint32_t pid, bool m) {
    uint64_t peers = dev::ballot(m);
    if (peers == 0) return 0;
    const uint32_t lead = __builtin_amdgcn_readlane(pid, __builtin_ctzll(peers));
    if (dev::ballot(m && pid != lead) == 0) return m ? peers : 0;
#pragma unroll
    for (int b = 0; b < kWideIdBits; ++b) {
        const bool bit = (pid >> b) & 1u;
        const uint64_t mb = dev::ballot(bit);
        peers &= bit ? mb : ~mb;
    }
    return m ? peers : 0ull;
}

// load the pattern table and predicate buckets into LDS
__device__ __forceinline__ void wide_setup(const WideArgs &a, WidePat *s_pat, uint32_t *s_bucket,
                                           uint16_t *s_ids) {
    for (int i = threadIdx.x; i < a.k; i += blockDim.x) {
        s_pat[i] = a.pats[i];
        s_ids[i] = a.ids[i];
    }
    for (uint32_t p = threadIdx.x; p < kWidePreds; p += blockDim.x) s_bucket[p] = a.bucket[p];
}

// Walk the calling wave's sub-range in triple order.  For every match the
// wave's running count of that pattern (s_run) advances by the number of
// lanes matching it in the same step; the write pass (WRITE) also stores the
// binding at that running count plus the lane's rank among them.
constexpr uint64_t kWideUnit = (uint64_t)dev::kWave * kWideIPT;  // triples a wave loads per step

// the last segment whose virtual base is at most v
__device__ __forceinline__ uint32_t wide_seg_of(const WideArgs &a, uint64_t v) {
    uint32_t lo = 0, hi = a.nseg;  // answer in [lo, hi)
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) / 2;
        if (a.segs[mid].vbase <= v) lo = mid;
        else hi = mid;
    }
    return lo;
}

template <bool WRITE, bool SLICE>
__device__ __forceinline__ void wide_walk(const WideArgs &a, const WidePat *s_pat,
                                          const uint32_t *s_bucket, const uint16_t *s_ids,
                                          uint32_t *s_run, uint64_t r0, uint64_t r1,
                                          uint32_t *flags) {
    const int lane = dev::lane_id();
    const uint64_t lt = (1ull << lane) - 1ull;
    // segment pass: the segment holding the current step (steps only move forward)
    uint32_t sg = SLICE && r0 < r1 ? wide_seg_of(a, r0) : 0u;
    for (uint64_t t0 = r0; t0 < r1; t0 += kWideUnit) {
        WTri t[kWideIPT];
        if (SLICE) {
            while (sg + 1 < a.nseg && a.segs[sg + 1].vbase <= t0) ++sg;
            const WideSeg sgm = a.segs[sg];
            const uint64_t off = t0 - sgm.vbase;
#pragma unroll
            for (int it = 0; it < kWideIPT; ++it) {
                const uint64_t l = off + (uint64_t)it * dev::kWave + lane;
                if (l < sgm.len) {
                    t[it].v[0] = __builtin_nontemporal_load(a.ss + sgm.pbase + l);
                    t[it].v[1] = sgm.p;
                    t[it].v[2] = __builtin_nontemporal_load(a.so + sgm.pbase + l);
                } else {
                    t[it].v[0] = t[it].v[1] = t[it].v[2] = 0;
                }
            }
        } else {
            // the graph is streamed once per pass: non-temporal loads
#pragma unroll
            for (int it = 0; it < kWideIPT; ++it) {
                const uint64_t i = t0 + (uint64_t)it * dev::kWave + lane;
                if (i < r1) {
                    t[it].v[0] = __builtin_nontemporal_load(a.g + 3 * i);
                    t[it].v[1] = __builtin_nontemporal_load(a.g + 3 * i + 1);
                    t[it].v[2] = __builtin_nontemporal_load(a.g + 3 * i + 2);
                } else {
                    t[it].v[0] = t[it].v[1] = t[it].v[2] = 0;
                }
            }
        }
#pragma unroll
        for (int it = 0; it < kWideIPT; ++it) {
            const uint32_t p = t[it].v[1];
            const uint32_t b = (p > 0 && p < kWidePreds) ? s_bucket[p] : 0u;
            const uint32_t start = b >> 12, len = b & 0xFFFu;
            for (uint32_t c = 0; dev::ballot(c < len); ++c) {
                const bool has = c < len;
                const uint32_t pid = has ? s_ids[start + c] : 0u;
                bool m = has && wide_match(s_pat[pid], t[it]);
                if (m && (s_pat[pid].flags & kWideFiltered)) {
                    const WidePat &q = s_pat[pid];
                    const uint32_t fp = (q.flags >> 15) & 3u;
                    const uint32_t x = fp == 0 ? t[it].v[0] : (fp == 1 ? t[it].v[1] : t[it].v[2]);
                    m = dev::bloom_has(q.fbits, q.fmask, x);
                }
                const uint64_t peers = match_pid(pid, m);
                if (!m) continue;
                const uint32_t before = s_run[pid];
                if (WRITE) {
                    const uint64_t pos = (uint64_t)before + (uint32_t)__popcll(peers & lt);
                    const WidePat &q = s_pat[pid];
                    const WideOut &o = a.outs[pid];
                    const int nc = (q.flags >> 5) & 3u;
                    if (pos < o.cap) {
                        TID_FOR_COLS(3, cc, nc) {
                            const uint32_t src = (q.flags >> (8 + 2 * cc)) & 3u;
                            o.col[cc][pos] = t[it].v[src];
                        }
                    } else {
                        atomicOr(&flags[1], 1u);
                    }
                }
                if (lane == __builtin_ctzll(peers)) s_run[pid] = before + (uint32_t)__popcll(peers);
            }
        }
    }
}

// LDS layout: patterns (k), predicate buckets, pattern ids (k, padded to
// words), then one running counter per (wave, pattern)
struct WideLds {
    WidePat *pat;
    uint32_t *bucket;
    uint16_t *ids;
    uint32_t *run;
};

__device__ __forceinline__ WideLds wide_lds(uint32_t *lds, int k) {
    WideLds l;
    l.pat = reinterpret_cast<WidePat *>(lds);
    l.bucket = reinterpret_cast<uint32_t *>(l.pat + k);
    l.ids = reinterpret_cast<uint16_t *>(l.bucket + kWidePreds);
    l.run = reinterpret_cast<uint32_t *>(l.ids + ((k + 1) & ~1));
    return l;
}

template <bool SLICE>
__global__ __launch_bounds__(kWideBlock) void wide_count(WideArgs a, uint32_t *flags) {
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    const WideLds l = wide_lds(lds, a.k);
    WidePat *s_pat = l.pat;
    uint32_t *s_bucket = l.bucket;
    uint16_t *s_ids = l.ids;
    uint32_t *s_cnt = l.run;  // [NW][k]
    wide_setup(a, s_pat, s_bucket, s_ids);
    const int wave = threadIdx.x / dev::kWave, lane = dev::lane_id();
    uint32_t *run = s_cnt + (size_t)wave * a.k;
    for (int j = lane; j < a.k; j += dev::kWave) run[j] = 0;
    __syncthreads();
    const uint32_t gw = blockIdx.x * kWideNW + wave;
    if (gw < a.W) {
        const uint64_t r0 = a.wbound ? a.wbound[gw] : (uint64_t)gw * a.sub;
        const uint64_t r1 = a.wbound ? a.wbound[gw + 1] : min(a.n, r0 + a.sub);
        wide_walk<false, SLICE>(a, s_pat, s_bucket, s_ids, run, r0, r1, flags);
        for (int j = lane; j < a.k; j += dev::kWave) a.cnt[(size_t)gw * a.k + j] = run[j];
    }
}

// Column-wise exclusive scan of the W x k count matrix, in place; totals to
// tot[] and to every pattern's table count.  One workgroup per 64 patterns:
// lane = pattern, wave = a slice of the sub-ranges.
constexpr int kColBlock = 1024;
__global__ __launch_bounds__(kColBlock) void wide_offsets(WideArgs a) {
    constexpr int kParts = kColBlock / dev::kWave;
    __shared__ uint32_t s_part[kParts][dev::kWave];
    const int lane = dev::lane_id(), part = threadIdx.x / dev::kWave;
    const int j = blockIdx.x * dev::kWave + lane;
    const uint32_t per = (a.W + kParts - 1) / kParts;
    const uint32_t w0 = min(a.W, part * per), w1 = min(a.W, w0 + per);
    uint32_t sum = 0;
    if (j < a.k)
        for (uint32_t w = w0; w < w1; ++w) sum += a.cnt[(size_t)w * a.k + j];
    s_part[part][lane] = sum;
    __syncthreads();
    uint32_t run = 0;
    for (int x = 0; x < part; ++x) run += s_part[x][lane];
    if (j < a.k) {
        for (uint32_t w = w0; w < w1; ++w) {
            const uint32_t c = a.cnt[(size_t)w * a.k + j];
            a.cnt[(size_t)w * a.k + j] = run;
            run += c;
        }
        if (part == kParts - 1) {
            a.tot[j] = run;
            *a.counts_out[j] = run;
        }
    }
}

template <bool SLICE>
__global__ __launch_bounds__(kWideBlock) void wide_write(WideArgs a, uint32_t *flags) {
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    const WideLds l = wide_lds(lds, a.k);
    WidePat *s_pat = l.pat;
    uint32_t *s_bucket = l.bucket;
    uint16_t *s_ids = l.ids;
    uint32_t *s_run = l.run;
    wide_setup(a, s_pat, s_bucket, s_ids);
    const int wave = threadIdx.x / dev::kWave, lane = dev::lane_id();
    uint32_t *run = s_run + (size_t)wave * a.k;
    const uint32_t gw = blockIdx.x * kWideNW + wave;
    if (gw < a.W)
        for (int j = lane; j < a.k; j += dev::kWave) run[j] = a.cnt[(size_t)gw * a.k + j];
    __syncthreads();
    if (gw < a.W) {
        const uint64_t r0 = a.wbound ? a.wbound[gw] : (uint64_t)gw * a.sub;
        const uint64_t r1 = a.wbound ? a.wbound[gw + 1] : min(a.n, r0 + a.sub);
        wide_walk<true, SLICE>(a, s_pat, s_bucket, s_ids, run, r0, r1, flags);
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

int pattern_schema(const tid_pattern &p, int32_t *vars, int32_t *src);

// Can the pattern go through the wide pass?  Needs a constant predicate
// that fits the bucket table and no variable repeated on the predicate.
bool wide_eligible(const tid_pattern &p) {
    return p.p != 0 && p.p < kWidePreds;
}

static WidePat compile_wide(const tid_pattern &p) {
    int32_t vars[3], src[3];
    const int nc = pattern_schema(p, vars, src);
    WidePat w{};
    w.s = p.s;
    w.o = p.o;
    if (p.s) w.flags |= 1u;
    if (p.o) w.flags |= 2u;
    if (p.vs >= 0 && p.vs == p.vo) w.flags |= 4u;
    if (p.range_pos >= 0) {
        w.flags |= (uint32_t)(p.range_pos + 1) << 3;
        w.lo = p.lo;
        w.span = p.hi > p.lo ? p.hi - p.lo : 0u;
    }
    w.flags |= (uint32_t)nc << 5;
    for (int c = 0; c < nc; ++c) w.flags |= (uint32_t)src[c] << (8 + 2 * c);
    return w;
}

static size_t wide_lds_bytes(int k) {
    return sizeof(WidePat) * (size_t)k + 4 * kWidePreds + 2 * (size_t)((k + 1) & ~1) +
           4 * (size_t)kWideNW * (size_t)k;
}

// What one pass reads: the graph, or segments of (s, o) columns, each the
// rows of one predicate in triple order (segs: vbase is filled in here).
struct WideSource {
    const uint32_t *g = nullptr;
    const uint32_t *s = nullptr, *o = nullptr;
    std::vector<WideSeg> segs;
    uint64_t n = 0;  // graph pass: triples
};

// Allow up to 160 KB of dynamic LDS per workgroup: once per process, also
// when several host threads (each with its own context) arrive together.
template <bool SLICE>
static void set_wide_lds_limit() {
    static std::once_flag once;
    std::call_once(once, [] {
        TID_HIP(hipFuncSetAttribute((const void *)wide_count<SLICE>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
        TID_HIP(hipFuncSetAttribute((const void *)wide_write<SLICE>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
    });
}

// One pass for k <= kWideMax eligible patterns into preallocated tables.  In
// a segment pass every pattern's predicate is one of the segments'.
static void wide_pass(tid_ctx *ctx, WideSource src, const tid_pattern *pats, int k,
                      tid_table *const *outs, const ScanFilter *filters) {
    TID_REQUIRE(k >= 1 && k <= kWideMax, TID_E_INTERNAL, "wide pass: bad pattern count");
    const bool slice = src.g == nullptr;
    if (slice) {
        // virtual positions: every segment starts on a walk unit
        std::vector<char> seg_pred(kWidePreds, 0);
        uint64_t v = 0;
        for (WideSeg &sg : src.segs) {
            TID_REQUIRE(sg.p > 0 && sg.p < kWidePreds && sg.len > 0, TID_E_INTERNAL,
                        "wide pass: bad segment");
            seg_pred[sg.p] = 1;
            sg.vbase = v;
            v += (sg.len + kWideUnit - 1) / kWideUnit * kWideUnit;
        }
        src.n = v;
        for (int j = 0; j < k; ++j)
            TID_REQUIRE(wide_eligible(pats[j]) && seg_pred[pats[j].p], TID_E_INTERNAL,
                        "wide pass: pattern without segment");
        if (v == 0) {
            for (int j = 0; j < k; ++j) set_count(ctx, outs[j], 0);
            return;
        }
    }
    std::vector<WidePat> wp(k);
    std::vector<WideOut> wo(k);
    std::vector<uint64_t *> wc(k);
    std::vector<std::vector<uint16_t>> by_pred(kWidePreds);
    for (int j = 0; j < k; ++j) {
        TID_REQUIRE(wide_eligible(pats[j]), TID_E_INTERNAL, "wide pass: pattern not eligible");
        wp[j] = compile_wide(pats[j]);
        if (filters && filters[j].pos >= 0) {
            wp[j].flags |= kWideFiltered | ((uint32_t)filters[j].pos << 15);
            TID_REQUIRE(!filters[j].exact, TID_E_INTERNAL, "wide pass: exact filters go to scans");
            wp[j].fbits = filters[j].bits;
            wp[j].fmask = filters[j].mask;
        }
        for (int c = 0; c < 3; ++c) wo[j].col[c] = c < outs[j]->ncols ? outs[j]->col[c] : nullptr;
        wo[j].cap = outs[j]->cap;
        wc[j] = outs[j]->d_count;
        by_pred[pats[j].p].push_back((uint16_t)j);
    }
    std::vector<uint32_t> bucket(kWidePreds, 0);
    std::vector<uint16_t> ids;
    for (uint32_t p = 0; p < kWidePreds; ++p) {
        if (by_pred[p].empty()) continue;
        bucket[p] = ((uint32_t)ids.size() << 12) | (uint32_t)by_pred[p].size();
        ids.insert(ids.end(), by_pred[p].begin(), by_pred[p].end());
    }
    // the grid: one sub-range per resident wave
    const size_t lds = wide_lds_bytes(k);
    const void *count_fn = slice ? (const void *)wide_count<true> : (const void *)wide_count<false>;
    const void *write_fn = slice ? (const void *)wide_write<true> : (const void *)wide_write<false>;
    if (slice) set_wide_lds_limit<true>();
    else set_wide_lds_limit<false>();
    const int per_cu = resident_blocks(write_fn, kWideBlock, lds);
    const uint64_t waves = (uint64_t)per_cu * device_cus(ctx) * kWideNW;
    const uint64_t unit = kWideUnit;
    const uint64_t units = (src.n + unit - 1) / unit;
    uint64_t W = std::max<uint64_t>(1, std::min(units, waves));
    const uint64_t sub = (units + W - 1) / W * unit;
    std::vector<uint64_t> wb;  // segment pass: W + 1 sub-range bounds
    if (slice) {
        // A row costs its load plus one test per pattern of its predicate, so
        // equal rows per wave would leave the waves on a predicate with many
        // patterns far behind: bounds are placed (on walk units) at equal
        // shares of the summed cost instead.
        double total = 0;
        std::vector<double> unit_cost(src.segs.size());
        for (size_t x = 0; x < src.segs.size(); ++x) {
            unit_cost[x] = (double)unit * (1.0 + (double)by_pred[src.segs[x].p].size());
            total += unit_cost[x] * (double)((src.segs[x].len + unit - 1) / unit);
        }
        wb.assign(W + 1, src.n);
        wb[0] = 0;
        uint64_t w = 1;
        double acc = 0;
        for (size_t x = 0; x < src.segs.size() && w < W; ++x) {
            const uint64_t su = (src.segs[x].len + unit - 1) / unit;
            const double seg_cost = unit_cost[x] * (double)su;
            while (w < W && acc + seg_cost >= total * (double)w / (double)W) {
                const double need = total * (double)w / (double)W - acc;
                const uint64_t u = std::min<uint64_t>(su, (uint64_t)std::ceil(need / unit_cost[x]));
                wb[w] = std::max(wb[w - 1], src.segs[x].vbase + u * unit);
                ++w;
            }
            acc += seg_cost;
        }
    } else {
        W = std::max<uint64_t>(1, (src.n + sub - 1) / sub);
    }
    DevBuf cnt(ctx, (size_t)W * k * 4);

    // tables of constants, in one device block
    const size_t nseg = src.segs.size();
    const size_t b_pats = align_up(sizeof(WidePat) * k), b_bucket = align_up(4 * kWidePreds),
                 b_ids = align_up(2 * (size_t)k), b_outs = align_up(sizeof(WideOut) * k),
                 b_cnts = align_up(8 * (size_t)k), b_tot = align_up(8 * (size_t)k),
                 b_segs = align_up(sizeof(WideSeg) * std::max<size_t>(nseg, 1)),
                 b_wb = align_up(8 * std::max<size_t>(wb.size(), 1));
    const size_t consts = b_pats + b_bucket + b_ids + b_outs + b_cnts + b_tot + b_segs + b_wb;
    std::vector<char> host(consts, 0);
    char *h = host.data();
    std::memcpy(h, wp.data(), sizeof(WidePat) * k);
    std::memcpy(h + b_pats, bucket.data(), 4 * kWidePreds);
    std::memcpy(h + b_pats + b_bucket, ids.data(), 2 * (size_t)k);
    std::memcpy(h + b_pats + b_bucket + b_ids, wo.data(), sizeof(WideOut) * k);
    std::memcpy(h + b_pats + b_bucket + b_ids + b_outs, wc.data(), 8 * (size_t)k);
    const size_t at_segs = b_pats + b_bucket + b_ids + b_outs + b_cnts + b_tot;
    if (nseg) std::memcpy(h + at_segs, src.segs.data(), sizeof(WideSeg) * nseg);
    const size_t at_wb = at_segs + b_segs;
    if (!wb.empty()) std::memcpy(h + at_wb, wb.data(), 8 * wb.size());
    DevBuf dconst(ctx, consts);
    TID_HIP(hipMemcpyAsync(dconst.get(), host.data(), consts, hipMemcpyHostToDevice, ctx->stream));
    char *d = dconst.get<char>();

    WideArgs a{};
    a.g = src.g;
    a.ss = src.s;
    a.so = src.o;
    a.segs = reinterpret_cast<const WideSeg *>(d + at_segs);
    a.nseg = (uint32_t)nseg;
    a.wbound = wb.empty() ? nullptr : reinterpret_cast<const uint64_t *>(d + at_wb);
    a.n = src.n;
    a.pats = reinterpret_cast<const WidePat *>(d);
    a.bucket = reinterpret_cast<const uint32_t *>(d + b_pats);
    a.ids = reinterpret_cast<const uint16_t *>(d + b_pats + b_bucket);
    a.outs = reinterpret_cast<const WideOut *>(d + b_pats + b_bucket + b_ids);
    a.counts_out = reinterpret_cast<uint64_t **>(d + b_pats + b_bucket + b_ids + b_outs);
    a.tot = reinterpret_cast<uint64_t *>(d + b_pats + b_bucket + b_ids + b_outs + b_cnts);
    a.k = k;
    a.sub = sub;
    a.W = (uint32_t)W;
    a.cnt = cnt.get<uint32_t>();
    const unsigned blocks = (unsigned)((W + kWideNW - 1) / kWideNW);
    void *args[] = {&a, &ctx->d_flags};
    TID_HIP(hipLaunchKernel(count_fn, dim3(blocks), dim3(kWideBlock), args, lds, ctx->stream));
    TID_HIP(hipGetLastError());
    hipLaunchKernelGGL(wide_offsets, dim3((unsigned)((k + dev::kWave - 1) / dev::kWave)),
                       dim3(kColBlock), 0, ctx->stream, a);
    TID_HIP(hipGetLastError());
    TID_HIP(hipLaunchKernel(write_fn, dim3(blocks), dim3(kWideBlock), args, lds, ctx->stream));
}

// One wide pass over the graph for k <= kWideMax eligible patterns.  Each
// predicate with at least two of the patterns and, by the histograms, at
// least the slice threshold's rows is sliced: the graph pass carries one
// (?s p ?o) pattern for it instead, into a temporary two-column table, and a
// slice pass over that table then fills the predicate's own patterns.  Both
// keep triple order, so every table comes out as the graph pass alone would
// write it.
void run_wide(tid_ctx *ctx, const tid_graph *g, const tid_pattern *pats, int k,
              tid_table *const *outs, const ScanFilter *filters) {
    WideSource whole;
    whole.g = g->triples();
    whole.n = g->n;
    std::vector<std::vector<int>> by_pred(kWidePreds);
    for (int j = 0; j < k; ++j)
        if (wide_eligible(pats[j])) by_pred[pats[j].p].push_back(j);
    const uint64_t min_rows = ctx->opt.slice_rows > 0
                                  ? (uint64_t)ctx->opt.slice_rows
                                  : std::max<uint64_t>(uint64_t(1) << 16, g->n >> 12);
    std::vector<uint32_t> sliced;
    if (ctx->opt.wide_slice && !g->cdf[1].empty())
        for (uint32_t p = 1; p < kWidePreds; ++p)
            if (by_pred[p].size() >= 2 && g->count_in(1, p, p + 1) >= min_rows) sliced.push_back(p);
    if (sliced.empty()) {
        wide_pass(ctx, whole, pats, k, outs, filters);
        return;
    }
    std::vector<char> is_sliced(kWidePreds, 0);
    for (uint32_t p : sliced) is_sliced[p] = 1;
    std::vector<tid_pattern> gp;
    std::vector<tid_table *> gt;
    std::vector<ScanFilter> gf;
    for (int j = 0; j < k; ++j) {
        if (wide_eligible(pats[j]) && is_sliced[pats[j].p]) continue;
        gp.push_back(pats[j]);
        gt.push_back(outs[j]);
        gf.push_back(filters ? filters[j] : ScanFilter{});
    }
    std::vector<std::unique_ptr<tid_table>> slices;
    for (uint32_t p : sliced) {
        tid_pattern v{};  // (?a p ?b): two projected columns, s then o
        v.p = p;
        v.vs = 0;
        v.vp = -1;
        v.vo = 1;
        v.range_pos = -1;
        const int32_t vars[2] = {0, 1};
        slices.push_back(make_table(ctx, 2, vars, g->count_in(1, p, p + 1)));
        gp.push_back(v);
        gt.push_back(slices.back().get());
        gf.push_back(ScanFilter{});
    }
    wide_pass(ctx, whole, gp.data(), (int)gp.size(), gt.data(), gf.data());
    for (size_t i = 0; i < sliced.size(); ++i) {
        const uint32_t p = sliced[i];
        WideSource part;
        part.s = slices[i]->col[0];
        part.o = slices[i]->col[1];
        part.segs.push_back(WideSeg{0, 0, (uint32_t)slices[i]->cap, p});  // the count is exact
        std::vector<tid_pattern> sp;
        std::vector<tid_table *> st;
        std::vector<ScanFilter> sf;
        for (int j : by_pred[p]) {
            sp.push_back(pats[j]);
            st.push_back(outs[j]);
            sf.push_back(filters ? filters[j] : ScanFilter{});
        }
        wide_pass(ctx, part, sp.data(), (int)sp.size(), st.data(), sf.data());
    }
}

// One segment pass over the predicate-partitioned layout for k <= kWideMax
// eligible patterns: only the slices of the patterns' predicates are read (8 B
// per row, once to count and once to write) instead of the whole TripleID
// array.  A slice keeps triple order, so every table comes out as the graph
// pass would write it.
void run_wide_parts(tid_ctx *ctx, const tid_graph *g, const tid_pattern *pats, int k,
                    tid_table *const *outs, const ScanFilter *filters) {
    TID_REQUIRE(g->partitioned && !g->cdf[1].empty(), TID_E_INTERNAL,
                "segment pass: the graph has no partitioned layout");
    const auto &cdf = g->cdf[1];
    const uint64_t last = cdf.size() - 1;
    auto slice_of = [&](uint32_t p, uint64_t &a, uint64_t &b) {
        a = cdf[std::min<uint64_t>(p, last)];
        b = cdf[std::min<uint64_t>((uint64_t)p + 1, last)];
    };
    std::vector<char> used(kWidePreds, 0);
    std::vector<tid_pattern> sp;
    std::vector<tid_table *> st;
    std::vector<ScanFilter> sf;
    for (int j = 0; j < k; ++j) {
        TID_REQUIRE(wide_eligible(pats[j]), TID_E_INTERNAL, "segment pass: pattern not eligible");
        uint64_t a, b;
        slice_of(pats[j].p, a, b);
        if (b == a) {  // no triple has the predicate
            set_count(ctx, outs[j], 0);
            continue;
        }
        used[pats[j].p] = 1;
        sp.push_back(pats[j]);
        st.push_back(outs[j]);
        sf.push_back(filters ? filters[j] : ScanFilter{});
    }
    if (sp.empty()) return;
    WideSource src;
    src.s = g->part_s.get<const uint32_t>();
    src.o = g->part_o.get<const uint32_t>();
    for (uint32_t p = 1; p < kWidePreds; ++p) {
        if (!used[p]) continue;
        uint64_t a, b;
        slice_of(p, a, b);
        src.segs.push_back(WideSeg{0, a, (uint32_t)(b - a), p});
    }
    wide_pass(ctx, std::move(src), sp.data(), (int)sp.size(), st.data(), sf.data());
}

}  // namespace tid
