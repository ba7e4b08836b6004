// runtime.hip -- context, device memory, tables, graph load and load-time
// statistics of libtid.
#include "device_common.hpp"
#include "internal.hpp"

#include <algorithm>
#include <cstdio>

namespace tid {

// ---------------------------------------------------------------------------
// caching pool
// ---------------------------------------------------------------------------

size_t Pool::size_class(size_t bytes) {
    if (bytes <= 4096) return 4096;
    size_t p = 1;
    while (p < bytes) p <<= 1;
    // Up to 256 MiB a block is the next power of two, so that blocks of the
    // many intermediate tables of varying size are reused rather than
    // allocated again; above, 1/8 of the next power of two (at most 12.5%
    // slack) keeps large tables and graphs tight.
    if (p <= (size_t(256) << 20)) return p;
    const size_t step = p / 8;
    return (bytes + step - 1) / step * step;
}

void *Pool::alloc(size_t bytes) {
    const size_t sz = size_class(bytes);
    auto it = free_.lower_bound(sz);
    if (it != free_.end() && it->first <= sz + sz / 4) {
        void *p = it->second;
        live_[p] = it->first;
        free_.erase(it);
        return p;
    }
    void *p = nullptr;
    if (hipMalloc(&p, sz) != hipSuccess) {
        (void)hipGetLastError();
        release_all();  // give cached blocks back and try once more
        if (hipMalloc(&p, sz) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
    }
    live_[p] = sz;
    return p;
}

void Pool::free(void *p, size_t) {
    auto it = live_.find(p);
    if (it == live_.end()) return;
    free_.emplace(it->second, p);
    live_.erase(it);
}

void Pool::release_all() {
    for (auto &kv : free_) (void)hipFree(kv.second);
    free_.clear();
}

Pool::~Pool() {
    release_all();
    for (auto &kv : live_) (void)hipFree(kv.first);
    live_.clear();
}

// ---------------------------------------------------------------------------
// tables
// ---------------------------------------------------------------------------

__global__ void set_u64(uint64_t *p, uint64_t v) { *p = v; }

std::unique_ptr<tid_table> make_table(tid_ctx *ctx, int32_t ncols, const int32_t *vars,
                                      uint64_t cap) {
    TID_REQUIRE(ncols >= 0 && ncols <= TID_MAX_COLS, TID_E_SCHEMA, "table: too many columns");
    auto t = std::make_unique<tid_table>();
    t->ctx = ctx;
    t->ncols = ncols;
    for (int c = 0; c < ncols; ++c) t->vars[c] = vars[c];
    t->cap = cap;
    const size_t stride = align_up(std::max<uint64_t>(cap, 1) * sizeof(uint32_t));
    const size_t bytes = stride * (size_t)ncols + kAlign;
    t->block = std::make_shared<DevBuf>(ctx, bytes);
    char *base = t->block->get<char>();
    for (int c = 0; c < ncols; ++c) t->col[c] = reinterpret_cast<uint32_t *>(base + stride * c);
    t->d_count = reinterpret_cast<uint64_t *>(base + stride * (size_t)ncols);
    return t;
}

void copy_bounds(tid_table *dst, const tid_table *src, const int *map, int n, int dst_off) {
    if (!src->maxv_known) {
        dst->maxv_known = false;
        return;
    }
    for (int c = 0; c < n; ++c) dst->maxv[dst_off + c] = src->maxv[map ? map[c] : c];
}

void set_count(tid_ctx *ctx, tid_table *t, uint64_t n) {
    hipLaunchKernelGGL(set_u64, dim3(1), dim3(1), 0, ctx->stream, t->d_count, n);
    TID_HIP(hipGetLastError());
    t->nrows = n;
    t->count_known = true;
}

constexpr int kCountSets = 128;
struct CountSets {
    uint64_t *p[kCountSets];
    uint64_t v[kCountSets];
    int n;
};

__global__ void set_u64_many(CountSets s) {
    if ((int)threadIdx.x < s.n) *s.p[threadIdx.x] = s.v[threadIdx.x];
}

void set_count_later(tid_ctx *ctx, tid_table *t, uint64_t n) {
    ctx->pending_counts.emplace_back(t->d_count, n);
    t->nrows = n;
    t->count_known = true;
}

void flush_counts(tid_ctx *ctx) {
    auto &pc = ctx->pending_counts;
    for (size_t i = 0; i < pc.size(); i += kCountSets) {
        CountSets s{};
        s.n = (int)std::min<size_t>(kCountSets, pc.size() - i);
        for (int j = 0; j < s.n; ++j) {
            s.p[j] = pc[i + j].first;
            s.v[j] = pc[i + j].second;
        }
        hipLaunchKernelGGL(set_u64_many, dim3(1), dim3(kCountSets), 0, ctx->stream, s);
        TID_HIP(hipGetLastError());
    }
    pc.clear();
}

__global__ void gather_words(const uint64_t *const *src, uint64_t *dst, int n,
                             const uint32_t *flags) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += gridDim.x * blockDim.x)
        dst[i] = i < n ? *src[i] : (uint64_t)flags[0];
}

void read_words(tid_ctx *ctx, const std::vector<const uint64_t *> &src, uint64_t *dst) {
    const size_t n = src.size();
    if (n == 0) return;
    if (ctx->rw_cap < n + 1) {
        if (ctx->rw_host_ptrs) (void)hipHostFree(ctx->rw_host_ptrs);
        if (ctx->rw_host_vals) (void)hipHostFree(ctx->rw_host_vals);
        if (ctx->rw_dev) ctx->free(ctx->rw_dev, ctx->rw_cap * 16);
        ctx->rw_host_ptrs = nullptr;
        ctx->rw_host_vals = nullptr;
        ctx->rw_dev = nullptr;
        const size_t cap = std::max<size_t>(n + 1, 2 * ctx->rw_cap);
        TID_HIP(hipHostMalloc((void **)&ctx->rw_host_ptrs, cap * 8, hipHostMallocDefault));
        TID_HIP(hipHostMalloc((void **)&ctx->rw_host_vals, cap * 8, hipHostMallocDefault));
        ctx->rw_dev = ctx->alloc(cap * 16);
        ctx->rw_cap = cap;
    }
    for (size_t i = 0; i < n; ++i) ctx->rw_host_ptrs[i] = src[i];
    const uint64_t **dptrs = static_cast<const uint64_t **>(ctx->rw_dev);
    uint64_t *dvals = reinterpret_cast<uint64_t *>(static_cast<char *>(ctx->rw_dev) + ctx->rw_cap * 8);
    TID_HIP(hipMemcpyAsync(dptrs, ctx->rw_host_ptrs, n * 8, hipMemcpyHostToDevice, ctx->stream));
    hipLaunchKernelGGL(gather_words, dim3((unsigned)std::min<size_t>((n + 256) / 256, 1024)),
                       dim3(256), 0, ctx->stream, dptrs, dvals, (int)n, ctx->d_flags);
    TID_HIP(hipGetLastError());
    TID_HIP(hipMemcpyAsync(ctx->rw_host_vals, dvals, (n + 1) * 8, hipMemcpyDeviceToHost,
                           ctx->stream));
    TID_HIP(hipStreamSynchronize(ctx->stream));
    TID_REQUIRE(ctx->rw_host_vals[n] == 0, TID_E_INTERNAL,
                "a cross-workgroup wait exceeded its spin bound (device state inconsistent)");
    for (size_t i = 0; i < n; ++i) dst[i] = ctx->rw_host_vals[i];
}

void resolve_counts(tid_ctx *ctx, tid_table *const *ts, int k) {
    std::vector<const uint64_t *> src;
    std::vector<tid_table *> who;
    for (int j = 0; j < k; ++j)
        if (!ts[j]->count_known) {
            src.push_back(ts[j]->d_count);
            who.push_back(ts[j]);
        }
    if (src.empty()) return;
    std::vector<uint64_t> v(src.size());
    read_words(ctx, src, v.data());
    for (size_t i = 0; i < who.size(); ++i) {
        who[i]->nrows = v[i];
        who[i]->count_known = true;
    }
}

std::unique_ptr<tid_table> copy_columns(tid_ctx *ctx, const uint32_t *const *cols, int32_t ncols,
                                        const int32_t *vars, uint64_t nrows, int on_device) {
    auto t = make_table(ctx, ncols, vars, nrows);
    for (int c = 0; c < ncols; ++c) {
        TID_REQUIRE(nrows == 0 || cols[c], TID_E_INVALID_ARG, "null column");
        if (nrows)
            TID_HIP(hipMemcpyAsync(t->col[c], cols[c], nrows * sizeof(uint32_t),
                                   on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                                   ctx->stream));
    }
    set_count(ctx, t.get(), nrows);
    return t;
}

// ---------------------------------------------------------------------------
// load-time checks and statistics
// ---------------------------------------------------------------------------

// per position minimum and maximum ID (mm[0..2] = min, mm[3..5] = max)
__global__ void minmax_kernel(const uint32_t *__restrict__ g, uint64_t n, uint32_t *mm) {
    uint32_t lo[3] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu}, hi[3] = {0, 0, 0};
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
#pragma unroll
        for (int x = 0; x < 3; ++x) {
            uint32_t v = g[3 * i + x];
            lo[x] = min(lo[x], v);
            hi[x] = max(hi[x], v);
        }
    }
#pragma unroll
    for (int x = 0; x < 3; ++x) {
        for (int d = 32; d >= 1; d >>= 1) {
            lo[x] = min(lo[x], (uint32_t)__shfl_xor((int)lo[x], d, 64));
            hi[x] = max(hi[x], (uint32_t)__shfl_xor((int)hi[x], d, 64));
        }
    }
    if (dev::lane_id() == 0) {
#pragma unroll
        for (int x = 0; x < 3; ++x) {
            atomicMin(&mm[x], lo[x]);
            atomicMax(&mm[3 + x], hi[x]);
        }
    }
}

__global__ void init_minmax(uint32_t *mm) {
    if (threadIdx.x < 3) mm[threadIdx.x] = 0xFFFFFFFFu;
    else if (threadIdx.x < 6) mm[threadIdx.x] = 0u;
}

// Per-position ID histograms in one pass over the graph.  Each workgroup
// counts in LDS first and adds its counts to the global bins at the end:
//  - a position whose IDs fit kDirectBins bins (the predicates) is counted
//    in LDS bins directly;
//  - any other position goes through a small open-addressing LDS table of
//    kHashEntries (ID, count) entries, so the hubs of a skewed position
//    (Zipf subjects and objects) cost one global atomic per workgroup
//    instead of one per triple; an ID that finds no free entry within
//    kHashProbes steps is added to its global bin directly.
// IDs are >= 1 here (checked before), so key 0 marks an empty entry.
int device_cus(tid_ctx *ctx);

constexpr uint32_t kDirectBins = 8192;
constexpr uint32_t kHashEntries = 2048;
constexpr int kHashProbes = 16;
constexpr int kHistBlock = 1024;

struct HistArgs {
    uint32_t *hist[3];   // global bins per position (null: not counted)
    uint32_t nbins[3];
};

__global__ __launch_bounds__(kHistBlock) void hist3_kernel(const uint32_t *__restrict__ g,
                                                           uint64_t n, HistArgs a) {
    // per position a region of kDirectBins words: direct bins, or hash keys
    // (first kHashEntries words) and their counts (next kHashEntries words)
    __shared__ uint32_t s[3][kDirectBins];
    for (int x = 0; x < 3; ++x)
        for (uint32_t b = threadIdx.x; b < kDirectBins; b += kHistBlock) s[x][b] = 0;
    __syncthreads();
    bool direct[3];
#pragma unroll
    for (int x = 0; x < 3; ++x) direct[x] = a.nbins[x] <= kDirectBins;
    const uint64_t stride = (uint64_t)gridDim.x * kHistBlock;
    for (uint64_t i = (uint64_t)blockIdx.x * kHistBlock + threadIdx.x; i < n; i += stride) {
        uint32_t v[3];
        v[0] = __builtin_nontemporal_load(g + 3 * i);
        v[1] = __builtin_nontemporal_load(g + 3 * i + 1);
        v[2] = __builtin_nontemporal_load(g + 3 * i + 2);
#pragma unroll
        for (int x = 0; x < 3; ++x) {
            if (!a.hist[x]) continue;
            if (direct[x]) {
                atomicAdd(&s[x][v[x]], 1u);
                continue;
            }
            uint32_t h = dev::hash32(v[x]) & (kHashEntries - 1);
            bool done = false;
            for (int probe = 0; probe < kHashProbes && !done; ++probe) {
                uint32_t k = s[x][h];
                if (k == 0) k = atomicCAS(&s[x][h], 0u, v[x]);
                if (k == 0 || k == v[x]) {
                    atomicAdd(&s[x][kHashEntries + h], 1u);
                    done = true;
                }
                h = (h + 1) & (kHashEntries - 1);
            }
            if (!done) atomicAdd(&a.hist[x][v[x]], 1u);
        }
    }
    __syncthreads();
    for (int x = 0; x < 3; ++x) {
        if (!a.hist[x]) continue;
        if (direct[x]) {
            for (uint32_t b = threadIdx.x; b < a.nbins[x]; b += kHistBlock)
                if (s[x][b]) atomicAdd(&a.hist[x][b], s[x][b]);
        } else {
            for (uint32_t e = threadIdx.x; e < kHashEntries; e += kHistBlock) {
                const uint32_t k = s[x][e], c = s[x][kHashEntries + e];
                if (k && c) atomicAdd(&a.hist[x][k], c);
            }
        }
    }
}

constexpr uint32_t kMaxHistIds = 1u << 28;  // 1 GiB of uint32 counts per position

void build_stats(tid_ctx *ctx, tid_graph *g) {
    if (g->n == 0) return;
    DevBuf mm(ctx, 6 * sizeof(uint32_t));
    hipLaunchKernelGGL(init_minmax, dim3(1), dim3(64), 0, ctx->stream, mm.get<uint32_t>());
    const int blocks = (int)std::min<uint64_t>((g->n + 255) / 256, 4096);
    hipLaunchKernelGGL(minmax_kernel, dim3(blocks), dim3(256), 0, ctx->stream,
                       g->data.get<const uint32_t>(), g->n, mm.get<uint32_t>());
    TID_HIP(hipGetLastError());
    uint32_t h[6];
    TID_HIP(hipMemcpyAsync(h, mm.get(), sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    TID_HIP(hipStreamSynchronize(ctx->stream));
    for (int x = 0; x < 3; ++x) {
        TID_REQUIRE(h[x] != 0, TID_E_INVALID_ARG,
                    "load: ID 0 is reserved for the free variable and may not appear in a triple");
        g->max_id[x] = h[3 + x];
    }
    if (g->n >= (1ull << 32)) return;  // counts would not fit the uint32 bins
    // bins of the counted positions, one allocation, one clear
    HistArgs a{};
    size_t off[3] = {0, 0, 0}, total = 0;
    for (int x = 0; x < 3; ++x) {
        if (h[3 + x] >= kMaxHistIds) continue;
        a.nbins[x] = h[3 + x] + 1;
        off[x] = total;
        total += align_up((size_t)a.nbins[x] * sizeof(uint32_t));
    }
    if (total == 0) return;
    DevBuf hist(ctx, total);
    TID_HIP(hipMemsetAsync(hist.get(), 0, total, ctx->stream));
    for (int x = 0; x < 3; ++x)
        if (a.nbins[x]) a.hist[x] = reinterpret_cast<uint32_t *>(hist.get<char>() + off[x]);
    const int hb = (int)std::min<uint64_t>((g->n + kHistBlock - 1) / kHistBlock,
                                           2ull * (uint64_t)device_cus(ctx));
    hipLaunchKernelGGL(hist3_kernel, dim3(hb), dim3(kHistBlock), 0, ctx->stream,
                       g->data.get<const uint32_t>(), g->n, a);
    TID_HIP(hipGetLastError());
    std::vector<uint32_t> hh(total / sizeof(uint32_t));
    TID_HIP(hipMemcpyAsync(hh.data(), hist.get(), total, hipMemcpyDeviceToHost, ctx->stream));
    TID_HIP(hipStreamSynchronize(ctx->stream));
    for (int x = 0; x < 3; ++x) {
        if (!a.nbins[x]) continue;
        const uint32_t *b = hh.data() + off[x] / sizeof(uint32_t);
        auto &c = g->cdf[x];
        c.resize((size_t)a.nbins[x] + 1);
        c[0] = 0;
        for (uint32_t i = 0; i < a.nbins[x]; ++i) c[i + 1] = c[i] + b[i];
    }
}

}  // namespace tid

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------

void *tid_ctx::alloc(size_t bytes) {
    void *p = alloc_fn ? alloc_fn(user, bytes, (void *)stream) : pool.alloc(bytes);
    if (!p) throw tid::Error(TID_E_OOM, "device allocation of " + std::to_string(bytes) +
                                            " bytes failed");
    return p;
}

void tid_ctx::free(void *p, size_t bytes) {
    if (!p) return;
    if (free_fn)
        free_fn(user, p, bytes, (void *)stream);
    else
        pool.free(p, bytes);
}

// Look-back state shared by the context's kernels (one stream, so launches
// never overlap).  Kernels leave it all zero when they finish; a new buffer is
// cleared here once.
uint32_t tid_ctx::next_epoch(size_t bytes, uint64_t **state) {
    bool zero = false;
    if (ep_bytes < bytes) {
        const size_t want = tid::align_up(std::max(bytes, ep_bytes + ep_bytes / 2), 1 << 16);
        if (ep_state) free(ep_state, ep_bytes);
        ep_state = nullptr;
        ep_bytes = 0;
        ep_state = alloc(want);
        ep_bytes = want;
        zero = true;
    }
    if (++epoch > tid::kEpochMax) {
        epoch = 1;
        zero = true;
    }
    if (zero) TID_HIP(hipMemsetAsync(ep_state, 0, ep_bytes, stream));
    *state = static_cast<uint64_t *>(ep_state);
    return epoch;
}

void tid_ctx::sync() { TID_HIP(hipStreamSynchronize(stream)); }

namespace tid {

// The predicate histogram of a chunk view (its other positions take their
// bounds from the whole graph's histograms).
void chunk_stats(tid_ctx *ctx, tid_graph *v) {
    if (v->n == 0 || v->max_id[1] >= kMaxHistIds) return;
    HistArgs a{};
    a.nbins[1] = v->max_id[1] + 1;
    DevBuf hist(ctx, (size_t)a.nbins[1] * sizeof(uint32_t));
    TID_HIP(hipMemsetAsync(hist.get(), 0, (size_t)a.nbins[1] * sizeof(uint32_t), ctx->stream));
    a.hist[1] = hist.get<uint32_t>();
    const int hb = (int)std::min<uint64_t>((v->n + kHistBlock - 1) / kHistBlock,
                                           2ull * (uint64_t)device_cus(ctx));
    hipLaunchKernelGGL(hist3_kernel, dim3(hb), dim3(kHistBlock), 0, ctx->stream, v->triples(),
                       v->n, a);
    TID_HIP(hipGetLastError());
    std::vector<uint32_t> hh(a.nbins[1]);
    TID_HIP(hipMemcpyAsync(hh.data(), hist.get(), hh.size() * sizeof(uint32_t),
                           hipMemcpyDeviceToHost, ctx->stream));
    TID_HIP(hipStreamSynchronize(ctx->stream));
    auto &c = v->cdf[1];
    c.assign((size_t)a.nbins[1] + 1, 0);
    for (uint32_t i = 0; i < a.nbins[1]; ++i) c[i + 1] = c[i] + hh[i];
}

}  // namespace tid

uint64_t tid_graph::count_in(int pos, uint64_t lo, uint64_t hi) const {
    if (hi <= lo) return 0;
    const auto &c = cdf[pos];
    if (c.empty()) return bounds_from ? std::min(n, bounds_from->count_in(pos, lo, hi)) : n;
    const uint64_t last = c.size() - 1;  // c[last] = n
    const uint64_t a = std::min<uint64_t>(lo, last), b = std::min<uint64_t>(hi, last);
    return c[b] - c[a];
}

#include <mutex>

namespace tid {
int resident_blocks(const void *kernel, int block, size_t lds) {
    static std::mutex mu;
    static std::map<std::pair<const void *, size_t>, int> cache;
    static std::map<const void *, size_t> allowed;
    std::lock_guard<std::mutex> lock(mu);
    // above 64 KB of dynamic LDS a kernel must be allowed that much first
    // (its static LDS counts against the same 160 KB)
    if (lds > 65536 && lds > allowed[kernel]) {
        TID_HIP(hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        allowed[kernel] = lds;
    }
    auto key = std::make_pair(kernel, lds);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int nb = 0;
    TID_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, block, lds));
    nb = std::max(nb, 1);
    cache[key] = nb;
    return nb;
}

int device_cus(tid_ctx *ctx) {
    if (ctx->num_cus <= 0) {
        int n = 0;
        TID_HIP(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, ctx->device));
        ctx->num_cus = n > 0 ? n : 1;
    }
    return ctx->num_cus;
}
}  // namespace tid

uint64_t tid_table::rows() {
    if (!count_known) {
        tid_table *self = this;
        tid::resolve_counts(ctx, &self, 1);
    }
    return nrows;
}
