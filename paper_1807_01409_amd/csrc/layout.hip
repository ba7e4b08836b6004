// layout.hip -- a predicate-partitioned layout of the TripleID array: the
// paper suggests assigning IDs so that a search can be pruned (Sec. 4.3); here
// the triples are kept sorted by predicate, stably, as two columns (subject,
// object) next to the array of Sec. 3.  A scan whose pattern has a constant
// predicate p reads only p's slice, 8 B per triple of p instead of 12 B per
// triple of the graph, and finds the same rows in the same order (ascending
// triple position, since the sort is stable).  Patterns with a free
// predicate still read the TripleID array.
#include "scan_common.hpp"

#include <algorithm>

namespace tid {

bool radix_sort_pairs(tid_ctx *ctx, uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1,
                      uint64_t n, int bits);

namespace {

__global__ void predicate_keys(const uint32_t *__restrict__ g, uint64_t n, uint64_t *key,
                               uint32_t *pos) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        key[i] = g[3 * i + 1];
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

void partition_graph(tid_ctx *ctx, tid_graph *g, bool enable) {
    if (!enable) {
        g->part_s.reset();
        g->part_o.reset();
        g->partitioned = false;
        return;
    }
    if (g->partitioned) return;
    TID_REQUIRE(!g->cdf[1].empty(), TID_E_UNSUPPORTED,
                "partition: the graph has no predicate histogram");
    TID_REQUIRE(g->n < (1ull << 32), TID_E_UNSUPPORTED, "partition: 2^32 triples or more");
    const uint64_t n = g->n;
    DevBuf s(ctx, std::max<uint64_t>(n, 1) * 4), o(ctx, std::max<uint64_t>(n, 1) * 4);
    if (n) {
        DevBuf k0(ctx, n * 8), k1(ctx, n * 8), v0(ctx, n * 4), v1(ctx, n * 4);
        hipLaunchKernelGGL(predicate_keys, dim3(grid_of(n)), dim3(256), 0, ctx->stream,
                           g->triples(), n, k0.get<uint64_t>(),
                           v0.get<uint32_t>());
        TID_HIP(hipGetLastError());
        const int bits = 32 - __builtin_clz(std::max<uint32_t>(g->max_id[1], 1));
        const bool moved = radix_sort_pairs(ctx, k0.get<uint64_t>(), v0.get<uint32_t>(),
                                            k1.get<uint64_t>(), v1.get<uint32_t>(), n, bits);
        const uint32_t *perm = moved ? v1.get<const uint32_t>() : v0.get<const uint32_t>();
        hipLaunchKernelGGL(gather_so, dim3(grid_of(n)), dim3(256), 0, ctx->stream,
                           g->triples(), perm, n, s.get<uint32_t>(),
                           o.get<uint32_t>());
        TID_HIP(hipGetLastError());
        TID_HIP(hipStreamSynchronize(ctx->stream));  // the sort buffers go back to the pool
    }
    g->part_s = std::move(s);
    g->part_o = std::move(o);
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

}  // namespace tid
