// layout.hip -- a predicate-partitioned layout of the TripleID array: the
// paper suggests assigning IDs so that a search can be pruned (Sec. 4.3); here
// the triples are kept sorted by predicate, stably, as two columns (subject,
// object) next to the array of Sec. 3.  A scan whose pattern has a constant
// predicate p reads only p's slice, 8 B per triple of p instead of 12 B per
// triple of the graph, and finds the same rows in the same order (ascending
// triple position, since the sort is stable).  Patterns with a free
// predicate still read the TripleID array.  The same rows are also kept in
// (predicate, subject) and (predicate, object) order, where a semi-join looks
// its source's values up (index_semijoin, at the end of this file).
#include "batch.hpp"
#include "scan_common.hpp"

#include <algorithm>

namespace tid {

bool radix_sort_pairs(tid_ctx *ctx, uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1,
                      uint64_t n, int bits);

namespace {

// key[i] = predicate of triple i, then (when vbits > 0) its value at
// position vpos in the low vbits bits; pos[i] = i
__global__ void predicate_keys(const uint32_t *__restrict__ g, uint64_t n, int vpos, int vbits,
                               uint64_t *key, uint32_t *pos) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint64_t p = g[3 * i + 1];
        key[i] = vbits ? (p << vbits) | g[3 * i + vpos] : p;
        pos[i] = (uint32_t)i;
    }
}

__global__ void gather_so(const uint32_t *__restrict__ g, const uint32_t *__restrict__ perm,
                          uint64_t n, uint32_t *s, uint32_t *o) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint64_t t = perm[i];
        s[i] = g[3 * t];
        o[i] = g[3 * t + 2];
    }
}

unsigned grid_of(uint64_t n) {
    return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((n + 255) / 256, 16384));
}

// The triples of one predicate's slice: (s[i], p, o[i]).
struct SliceSrc {
    const uint32_t *s, *o;
    uint32_t p;
    uint64_t n;
    DevPattern pat[1];
    using Item = Tri;
    __device__ __forceinline__ Item load(uint64_t i) const {
        Tri t;
        t.v[0] = __builtin_nontemporal_load(s + i);
        t.v[1] = p;
        t.v[2] = __builtin_nontemporal_load(o + i);
        return t;
    }
    __device__ __forceinline__ bool match(int, const Item &t) const {
        return match_pattern(pat[0], t);
    }
    __device__ __forceinline__ uint32_t value(int, int c, const Item &t, uint64_t) const {
        return pick(t, pat[0].src[c]);
    }
};

}  // namespace

static int bits_of(uint32_t v) { return 32 - __builtin_clz(std::max<uint32_t>(v, 1)); }

void partition_graph(tid_ctx *ctx, tid_graph *g, bool enable) {
    if (!enable) {
        g->part_s.reset();
        g->part_o.reset();
        g->ps_s.reset();
        g->ps_o.reset();
        g->po_s.reset();
        g->po_o.reset();
        g->partitioned = false;
        return;
    }
    if (g->partitioned) return;
    TID_REQUIRE(!g->cdf[1].empty(), TID_E_UNSUPPORTED,
                "partition: the graph has no predicate histogram");
    TID_REQUIRE(g->n < (1ull << 32), TID_E_UNSUPPORTED, "partition: 2^32 triples or more");
    const uint64_t n = g->n;
    const size_t col = std::max<uint64_t>(n, 1) * 4;
    DevBuf cols[6] = {DevBuf(ctx, col), DevBuf(ctx, col), DevBuf(ctx, col),
                      DevBuf(ctx, col), DevBuf(ctx, col), DevBuf(ctx, col)};
    if (n) {
        DevBuf k0(ctx, n * 8), k1(ctx, n * 8), v0(ctx, n * 4), v1(ctx, n * 4);
        const int pbits = bits_of(g->max_id[1]);
        // predicate order, then (predicate, subject), then (predicate, object);
        // every sort is stable, so ties stay in triple order
        const int vpos[3] = {0, 0, 2};
        for (int x = 0; x < 3; ++x) {
            const int vbits = x == 0 ? 0 : bits_of(g->max_id[vpos[x]]);
            hipLaunchKernelGGL(predicate_keys, dim3(grid_of(n)), dim3(256), 0, ctx->stream,
                               g->triples(), n, vpos[x], vbits, k0.get<uint64_t>(),
                               v0.get<uint32_t>());
            TID_HIP(hipGetLastError());
            const bool moved = radix_sort_pairs(ctx, k0.get<uint64_t>(), v0.get<uint32_t>(),
                                                k1.get<uint64_t>(), v1.get<uint32_t>(), n,
                                                pbits + vbits);
            const uint32_t *perm = moved ? v1.get<const uint32_t>() : v0.get<const uint32_t>();
            hipLaunchKernelGGL(gather_so, dim3(grid_of(n)), dim3(256), 0, ctx->stream,
                               g->triples(), perm, n, cols[2 * x].get<uint32_t>(),
                               cols[2 * x + 1].get<uint32_t>());
            TID_HIP(hipGetLastError());
        }
        TID_HIP(hipStreamSynchronize(ctx->stream));  // the sort buffers go back to the pool
    }
    g->part_s = std::move(cols[0]);
    g->part_o = std::move(cols[1]);
    g->ps_s = std::move(cols[2]);
    g->ps_o = std::move(cols[3]);
    g->po_s = std::move(cols[4]);
    g->po_o = std::move(cols[5]);
    g->partitioned = true;
}

// A single pattern with a constant predicate over its slice of the
// partitioned layout; `out` is sized by the caller.  Filters and value sets
// are not routed here (the caller checks).
void scan_slice(tid_ctx *ctx, const tid_graph *g, const tid_pattern &p, tid_table *out,
                const ScanFilter *filter) {
    TID_REQUIRE(g->partitioned && p.p != 0, TID_E_INTERNAL, "slice scan: no slice");
    const auto &cdf = g->cdf[1];
    const uint64_t last = cdf.size() - 1;
    const uint64_t a = cdf[std::min<uint64_t>(p.p, last)];
    const uint64_t b = cdf[std::min<uint64_t>((uint64_t)p.p + 1, last)];
    if (b == a) {
        set_count(ctx, out, 0);
        return;
    }
    SliceSrc src{};
    src.s = g->part_s.get<const uint32_t>() + a;
    src.o = g->part_o.get<const uint32_t>() + a;
    src.p = p.p;
    src.n = b - a;
    src.pat[0] = compile_pattern(p, nullptr, filter);
    CompactArgs<1, 3> args{};
    for (int c = 0; c < out->ncols; ++c) args.out[0].col[c] = out->col[c];
    args.out[0].cap = out->cap;
    args.out[0].count = out->d_count;
    args.out[0].ncols = out->ncols;
    launch_compact<SliceSrc, 512, 8, 1, 3, true>(ctx, src, args, 1, 16384u);
}

// ---------------------------------------------------------------------------
// Semi-join by index.  A pattern (?x p ?y) filtered on x (or y) by the values
// of a small source table needs the rows of p whose subject (object) is one
// of those values.  Instead of testing every row of p against a filter, each
// distinct value is looked up in p's rows in (predicate, subject) or
// (predicate, object) order: two binary searches give its run of rows.  All
// jobs of a round go together: the values are sorted (the batched row sort),
// one launch finds every value's run (repeats of a value get an empty run),
// an exclusive scan places the runs, and after one read of the totals one
// launch writes every output row.  A job's rows come grouped by value, in
// ascending value order, each run in triple order.
// ---------------------------------------------------------------------------

void exclusive_scan_async(tid_ctx *ctx, const uint32_t *in, uint64_t n, uint64_t *out);
void read_words(tid_ctx *ctx, const std::vector<const uint64_t *> &src, uint64_t *dst);

namespace {

struct IdxJob {
    const uint32_t *keys;     // sorted values of the job (nkeys)
    const uint32_t *col;      // the searched column of the predicate's run
    const uint32_t *vs, *vo;  // subject and object columns of the same rows
    uint64_t nkeys, nrun;     // values; rows of the predicate
    uint64_t pbase;           // first (job, value) pair of the job
    uint64_t obase;           // first output row of the job (all jobs' rows concatenated)
    uint32_t *out[3];
    int32_t src[3];           // output column c is the subject (0) or object (2)
    int32_t ncols;
};

__device__ __forceinline__ int idx_job_of(const IdxJob *jobs, int J, uint64_t q) {
    int lo = 0, hi = J;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (jobs[mid].pbase <= q) lo = mid;
        else hi = mid;
    }
    return lo;
}

// first index in col[0, n) whose value is >= key (upper: > key)
__device__ __forceinline__ uint64_t bound_of(const uint32_t *col, uint64_t n, uint32_t key,
                                             bool upper) {
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        const uint32_t v = col[mid];
        if (v < key || (upper && v == key)) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// per (job, value) pair: the first row of the value's run and the run length
// (0 for a repeat of the previous value)
__global__ void idx_count(const IdxJob *jobs, int J, uint64_t P, uint32_t *cnt, uint32_t *first) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < P; q += stride) {
        const IdxJob &j = jobs[idx_job_of(jobs, J, q)];
        const uint64_t i = q - j.pbase;
        const uint32_t key = j.keys[i];
        uint32_t c = 0, f = 0;
        if (i == 0 || j.keys[i - 1] != key) {
            const uint64_t lo = bound_of(j.col, j.nrun, key, false);
            const uint64_t hi = bound_of(j.col + lo, j.nrun - lo, key, true) + lo;
            c = (uint32_t)(hi - lo);
            f = (uint32_t)lo;
        }
        cnt[q] = c;
        first[q] = f;
    }
}

// The same, one pair per wave, for launches with few pairs: each round the 64
// lanes probe evenly spaced rows of the bound's interval and a ballot keeps
// the part between the last probe before the bound and the first at or past
// it, so a run of n rows takes about log64(n) dependent loads, not log2(n).
__device__ uint64_t wave_bound(const uint32_t *col, uint64_t n, uint32_t key, bool upper) {
    const uint64_t lane = (uint64_t)dev::lane_id();
    uint64_t lo = 0, hi = n;  // the bound is in [lo, hi]
    while (hi > lo) {         // wave-uniform
        const uint64_t step = (hi - lo + dev::kWave - 1) / dev::kWave;
        const uint64_t p = lo + lane * step;
        bool before = false;  // the bound is past row p
        if (p < hi) {
            const uint32_t v = col[p];
            before = v < key || (upper && v == key);
        }
        const uint64_t t = (uint64_t)__popcll(dev::ballot(before));  // a prefix of the lanes
        const uint64_t nlo = t == 0 ? lo : lo + (t - 1) * step + 1;
        hi = std::min<uint64_t>(hi, lo + t * step);
        lo = nlo;
    }
    return lo;
}

__global__ __launch_bounds__(256) void idx_count_wave(const IdxJob *jobs, int J, uint64_t P,
                                                      uint32_t *cnt, uint32_t *first) {
    constexpr uint64_t kWaves = 256 / dev::kWave;
    const uint64_t stride = (uint64_t)gridDim.x * kWaves;
    for (uint64_t q = (uint64_t)blockIdx.x * kWaves + threadIdx.x / dev::kWave; q < P;
         q += stride) {  // q is the same for every lane of a wave
        const IdxJob &j = jobs[idx_job_of(jobs, J, q)];
        const uint64_t i = q - j.pbase;
        const uint32_t key = j.keys[i];
        uint32_t c = 0, f = 0;
        if (i == 0 || j.keys[i - 1] != key) {
            const uint64_t lo = wave_bound(j.col, j.nrun, key, false);
            const uint64_t hi = wave_bound(j.col + lo, j.nrun - lo, key, true) + lo;
            c = (uint32_t)(hi - lo);
            f = (uint32_t)lo;
        }
        if (dev::lane_id() == 0) {
            cnt[q] = c;
            first[q] = f;
        }
    }
}

// output row r (over all jobs) -> its pair (offs: exclusive sums of the run
// lengths, P + 1 entries) -> the row of the predicate's run it copies
__global__ void idx_expand(const IdxJob *jobs, int J, const uint64_t *offs, uint64_t P,
                           const uint32_t *first, uint64_t R) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < R; r += stride) {
        uint64_t lo = 0, hi = P;  // the last pair q with offs[q] <= r
        while (hi - lo > 1) {
            const uint64_t mid = (lo + hi) >> 1;
            if (offs[mid] <= r) lo = mid;
            else hi = mid;
        }
        const uint64_t q = lo;
        const IdxJob &j = jobs[idx_job_of(jobs, J, q)];
        const uint64_t row = (uint64_t)first[q] + (r - offs[q]);
        const uint64_t at = r - j.obase;
        for (int c = 0; c < j.ncols; ++c) j.out[c][at] = j.src[c] == 0 ? j.vs[row] : j.vo[row];
    }
}

// launches with at most this many (job, value) pairs search a pair per wave
constexpr uint64_t kWavePairs = 16384;

unsigned grid_for_rows(uint64_t n) {
    return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((n + 255) / 256, 16384));
}

}  // namespace

// The patterns' rows (one output table each, allocated here): pattern j has a
// constant predicate, a free subject and object, and filters[j].index set,
// with its values at filters[j].keys.  Synchronises once.
void index_semijoin(tid_ctx *ctx, const tid_graph *g, const tid_pattern *pats,
                    const ScanFilter *filters, int J, std::unique_ptr<tid_table> *outs) {
    TID_REQUIRE(g->partitioned && !g->cdf[1].empty(), TID_E_INTERNAL,
                "index semi-join: no partitioned layout");
    if (J == 0) return;
    const auto &cdf = g->cdf[1];
    const uint64_t last = cdf.size() - 1;
    std::vector<DevBuf> keep;
    std::vector<std::vector<char>> host_keep;
    // 1. every job's values, sorted (tables of one column)
    std::vector<tid_table> in(J);
    std::vector<std::unique_ptr<tid_table>> sorted(J);
    std::vector<RowSortJob> sorts;
    for (int j = 0; j < J; ++j) {
        const ScanFilter &f = filters[j];
        TID_REQUIRE(f.index && (f.pos == 0 || f.pos == 2) && pats[j].p != 0, TID_E_INTERNAL,
                    "index semi-join: bad job");
        const int32_t var = 0;
        sorted[j] = make_table(ctx, 1, &var, std::max<uint64_t>(f.nkeys, 1));
        if (f.nkeys > 1) {
            in[j].ctx = ctx;
            in[j].ncols = 1;
            in[j].col[0] = const_cast<uint32_t *>(f.keys);
            in[j].maxv[0] = f.key_max;
            in[j].maxv_known = true;
            in[j].nrows = f.nkeys;
            in[j].count_known = true;
            sorts.push_back(RowSortJob{&in[j], sorted[j].get(), f.nkeys});
        } else if (f.nkeys == 1) {
            TID_HIP(hipMemcpyAsync(sorted[j]->col[0], f.keys, 4, hipMemcpyDeviceToDevice,
                                   ctx->stream));
        }
    }
    sort_rows_batched(ctx, sorts, keep, host_keep);
    // 2. runs of every (job, value)
    std::vector<IdxJob> jobs(J);
    uint64_t P = 0;
    for (int j = 0; j < J; ++j) {
        const ScanFilter &f = filters[j];
        const uint64_t a = cdf[std::min<uint64_t>(pats[j].p, last)];
        const uint64_t b = cdf[std::min<uint64_t>((uint64_t)pats[j].p + 1, last)];
        const bool by_s = f.pos == 0;
        IdxJob &x = jobs[j];
        x = IdxJob{};
        x.keys = sorted[j]->col[0];
        x.vs = (by_s ? g->ps_s : g->po_s).get<const uint32_t>() + a;
        x.vo = (by_s ? g->ps_o : g->po_o).get<const uint32_t>() + a;
        x.col = by_s ? x.vs : x.vo;
        x.nkeys = f.nkeys;
        x.nrun = b - a;
        x.pbase = P;
        P += f.nkeys;
    }
    DevBuf cnt(ctx, std::max<uint64_t>(P, 1) * 4), first(ctx, std::max<uint64_t>(P, 1) * 4),
        offs(ctx, (P + 1) * 8), djobs(ctx, sizeof(IdxJob) * J);
    TID_HIP(hipMemcpyAsync(djobs.get(), jobs.data(), sizeof(IdxJob) * J, hipMemcpyHostToDevice,
                           ctx->stream));
    if (P > kWavePairs) {
        hipLaunchKernelGGL(idx_count, dim3(grid_for_rows(P)), dim3(256), 0, ctx->stream,
                           djobs.get<const IdxJob>(), J, P, cnt.get<uint32_t>(),
                           first.get<uint32_t>());
        TID_HIP(hipGetLastError());
    } else if (P) {  // few pairs: a wave each, for latency
        hipLaunchKernelGGL(idx_count_wave, dim3((unsigned)((P + 3) / 4)), dim3(256), 0,
                           ctx->stream, djobs.get<const IdxJob>(), J, P, cnt.get<uint32_t>(),
                           first.get<uint32_t>());
        TID_HIP(hipGetLastError());
    }
    exclusive_scan_async(ctx, cnt.get<const uint32_t>(), P, offs.get<uint64_t>());
    // 3. every job's row count: one read
    std::vector<const uint64_t *> src(J + 1);
    for (int j = 0; j < J; ++j) src[j] = offs.get<const uint64_t>() + jobs[j].pbase;
    src[J] = offs.get<const uint64_t>() + P;
    std::vector<uint64_t> at(J + 1);
    read_words(ctx, src, at.data());
    // 4. the tables, then every row in one launch
    for (int j = 0; j < J; ++j) {
        int32_t vars[3], srcpos[3];
        const int nc = pattern_schema(pats[j], vars, srcpos);
        const uint64_t rows = at[j + 1] - at[j];
        outs[j] = make_table(ctx, nc, vars, rows);
        for (int c = 0; c < nc; ++c) {
            outs[j]->maxv[c] = g->max_id[srcpos[c]];
            jobs[j].out[c] = outs[j]->col[c];
            jobs[j].src[c] = srcpos[c];
        }
        outs[j]->maxv_known = true;
        jobs[j].ncols = nc;
        jobs[j].obase = at[j];
        set_count_later(ctx, outs[j].get(), rows);
    }
    flush_counts(ctx);
    const uint64_t R = at[J];
    if (R) {
        DevBuf djobs2(ctx, sizeof(IdxJob) * J);
        TID_HIP(hipMemcpyAsync(djobs2.get(), jobs.data(), sizeof(IdxJob) * J,
                               hipMemcpyHostToDevice, ctx->stream));
        hipLaunchKernelGGL(idx_expand, dim3(grid_for_rows(R)), dim3(256), 0, ctx->stream,
                           djobs2.get<const IdxJob>(), J, offs.get<const uint64_t>(), P,
                           first.get<const uint32_t>(), R);
        TID_HIP(hipGetLastError());
        TID_HIP(hipStreamSynchronize(ctx->stream));  // the job tables are read by now
    }
}

}  // namespace tid
