// batch.hip -- the small joins and the final sorts of many plans, each kind
// in one launch per round of a batch (the lockstep rounds of
// tid_query_batch): one workgroup per job, the job table in device memory.
// A plan's join whose sides both have at most kSmallRows rows does not launch
// its own hash build, scans, probe and expansion; it is a job of the round's
// one count launch, then of the next round's one expansion launch.  A plan's
// final lexicographic sort of at most kSortRows rows is likewise a job of one
// sort launch.  A job's hash table lives in the workgroup's LDS.
//
// Join job (Sec. 4.2: an equi-join on the shared variable, done here with a
// hash table in LDS): the R side's keys go into an open-addressing table
// (slot = key, count, first position of its rows in a per-slot row list);
// each L row finds its key's slot and pairs with the slot's R rows that also
// agree on every other shared variable (natural join).  The count launch
// writes each L row's exclusive output offset and the job's total.  Without
// other shared variables it also leaves its grouping of R's rows by key in
// device memory, and the expansion is one launch of output tiles over it;
// otherwise the expansion launch rebuilds the table and each L row's thread
// writes its pairs.  The order of rows within a join's output is not
// defined (a plan's result is always sorted at its end).
#include "batch.hpp"
#include "device_common.hpp"

#include <algorithm>

namespace tid {

namespace {

// Device-memory access through a pointer the compiler only knows as generic
// (one read from a job table): as a global access it is counted apart from
// LDS and scalar loads, so the waits those need do not also wait for it, as
// they would for a flat access.  p must point to device memory.
__device__ __forceinline__ uint32_t gload(const uint32_t *p) {
    return *(const __attribute__((address_space(1))) uint32_t *)p;
}
__device__ __forceinline__ void gstore(uint32_t *p, uint32_t v) {
    *(__attribute__((address_space(1))) uint32_t *)p = v;
}

__device__ __forceinline__ uint32_t pow2_at_least(uint32_t x) {
    uint32_t p = 64;
    while (p < x) p <<= 1;
    return p;
}

// exclusive scan of v over a block of BLOCK threads in thread order; returns
// this thread's prefix and leaves the total in *total
template <int BLOCK = kBatchBlock>
__device__ __forceinline__ uint32_t block_exclusive(uint32_t v, uint32_t *s_w, uint32_t *total) {
    constexpr int NW = BLOCK / dev::kWave;
    const int lane = threadIdx.x % dev::kWave, wave = threadIdx.x / dev::kWave;
    const uint32_t incl = dev::wave_inclusive_sum(v);
    if (lane == dev::kWave - 1) s_w[wave] = incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (int w = 0; w < NW; ++w) {
        if (w < wave) before += s_w[w];
        all += s_w[w];
    }
    __syncthreads();
    *total = all;
    return before + incl - v;
}

struct Table {
    uint32_t *key, *cnt, *start, *rows;
    uint32_t mask;
};

constexpr uint32_t kRowsPerThread = kSmallRows / kJoinBlock;  // 4

// R's keys into the LDS table: slot counts, slot starts, rows grouped by slot.
// The key equal to the empty marker (kEmptyKey, a valid ID) has a slot of its
// own past the probed ones, slot mask + 1, placed last.  Each thread loads its
// (up to kRowsPerThread) keys at once, then inserts them.  The lanes of a
// wave that share the key of its first row (a hub key fills whole waves)
// insert, count and reserve places through that row's lane: one LDS atomic
// for the group instead of one per lane on one word.
__device__ void build_table(const JoinJob &j, Table &t, uint32_t *s_w) {
    const uint32_t ts = pow2_at_least(2 * j.nr);
    t.mask = ts - 1;
    uint32_t rk[kRowsPerThread];
#pragma unroll
    for (uint32_t u = 0; u < kRowsPerThread; ++u) {
        const uint32_t r = u * kJoinBlock + threadIdx.x;
        rk[u] = r < j.nr ? gload(j.rkey + r) : kEmptyKey;
    }
    for (uint32_t s = threadIdx.x; s <= ts; s += kJoinBlock) {
        t.key[s] = kEmptyKey;
        t.cnt[s] = 0;
    }
    __syncthreads();
    const int lane = dev::lane_id();
#pragma unroll
    for (uint32_t u = 0; u < kRowsPerThread; ++u) {  // u is uniform: every lane takes the ballots
        const bool live = u * kJoinBlock + threadIdx.x < j.nr;
        const uint32_t k = rk[u];
        const uint64_t lv = dev::ballot(live);
        if (lv == 0) continue;  // the whole wave is past the end
        const int lead = __builtin_ctzll(lv);
        const uint32_t lk = __shfl(k, lead);
        const uint64_t same = dev::ballot(live && k == lk);
        if (live && (k != lk || lane == lead)) {
            uint32_t h = ts;
            if (k != kEmptyKey) {
                h = dev::hash32(k) & t.mask;
                for (;;) {  // ends: the table has more slots than keys
                    const uint32_t prev = atomicCAS(&t.key[h], kEmptyKey, k);
                    if (prev == kEmptyKey || prev == k) break;
                    h = (h + 1) & t.mask;
                }
            }
            atomicAdd(&t.cnt[h], k == lk ? (uint32_t)__popcll(same) : 1u);
        }
    }
    __syncthreads();
    // slot starts: each thread scans a contiguous run of ts / block slots
    const uint32_t per = ts / kJoinBlock > 0 ? ts / kJoinBlock : 1;
    const uint32_t s0 = threadIdx.x * per;
    uint32_t local = 0;
    for (uint32_t s = s0; s < s0 + per && s < ts; ++s) local += t.cnt[s];
    uint32_t all;
    uint32_t run = block_exclusive<kJoinBlock>(local, s_w, &all);
    for (uint32_t s = s0; s < s0 + per && s < ts; ++s) {
        t.start[s] = run;
        run += t.cnt[s];
        t.cnt[s] = 0;  // counts again while the rows are placed
    }
    if (threadIdx.x == 0) {  // the slot of kEmptyKey comes last
        t.start[ts] = all;
        t.cnt[ts] = 0;
    }
    __syncthreads();
#pragma unroll
    for (uint32_t u = 0; u < kRowsPerThread; ++u) {
        const uint32_t r = u * kJoinBlock + threadIdx.x;
        const bool live = r < j.nr;
        const uint32_t k = rk[u];
        const uint64_t lv = dev::ballot(live);
        if (lv == 0) continue;
        const int lead = __builtin_ctzll(lv);
        const uint32_t lk = __shfl(k, lead);
        const uint64_t same = dev::ballot(live && k == lk);
        uint32_t at = 0;
        if (live && (k != lk || lane == lead)) {
            uint32_t h = ts;
            if (k != kEmptyKey) {
                h = dev::hash32(k) & t.mask;
                while (t.key[h] != k) h = (h + 1) & t.mask;
            }
            at = t.start[h] + atomicAdd(&t.cnt[h], k == lk ? (uint32_t)__popcll(same) : 1u);
        }
        const uint32_t group_at = __shfl(at, lead);
        if (live) t.rows[k == lk ? group_at + dev::rank_in_mask(same) : at] = r;
    }
    __syncthreads();
}

// the slot of key k, or kEmptyKey if R does not hold k
__device__ __forceinline__ uint32_t find_slot(const Table &t, uint32_t k) {
    if (k == kEmptyKey) return t.cnt[t.mask + 1] ? t.mask + 1 : kEmptyKey;
    uint32_t h = dev::hash32(k) & t.mask;
    for (;;) {
        const uint32_t x = t.key[h];
        if (x == k) return h;
        if (x == kEmptyKey) return kEmptyKey;
        h = (h + 1) & t.mask;
    }
}

__device__ __forceinline__ bool agree(const JoinJob &j, uint32_t l, uint32_t r) {
    bool ok = true;
    for (int e = 0; e < j.neq; ++e) ok &= gload(j.eq_l[e] + l) == gload(j.eq_r[e] + r);
    return ok;
}

__shared__ uint32_t s_key[kSmallSlots + 1], s_cnt[kSmallSlots + 1], s_start[kSmallSlots + 1];
__shared__ uint32_t s_rows[kSmallRows];
__shared__ uint32_t s_w[kJoinBlock / dev::kWave];

}  // namespace

__global__ __launch_bounds__(kJoinBlock) void batch_join_count(const JoinJob *jobs) {
    const JoinJob &j = jobs[blockIdx.x];
    Table t{s_key, s_cnt, s_start, s_rows, 0};
    build_table(j, t, s_w);
    // each thread a contiguous run of L rows, so offsets follow row order;
    // the keys are loaded at once, the offsets (and group starts) stored after
    uint32_t c[kRowsPerThread], lb[kRowsPerThread], lk[kRowsPerThread];
    const uint32_t i0 = threadIdx.x * kRowsPerThread;
#pragma unroll
    for (uint32_t u = 0; u < kRowsPerThread; ++u) lk[u] = i0 + u < j.nl ? gload(j.lkey + i0 + u) : 0u;
    uint32_t local = 0;
#pragma unroll
    for (uint32_t u = 0; u < kRowsPerThread; ++u) {
        c[u] = lb[u] = 0;  // a row without a match owns no output
        if (i0 + u >= j.nl) continue;
        const uint32_t h = find_slot(t, lk[u]);
        if (h == kEmptyKey) continue;
        const uint32_t a = t.start[h], b = a + t.cnt[h];
        lb[u] = a;
        if (j.neq == 0) {
            c[u] = b - a;
        } else {
            for (uint32_t m = a; m < b; ++m) c[u] += agree(j, i0 + u, t.rows[m]);
        }
        local += c[u];
    }
    uint32_t all;
    uint32_t run = block_exclusive<kJoinBlock>(local, s_w, &all);
#pragma unroll
    for (uint32_t u = 0; u < kRowsPerThread; ++u) {
        const uint32_t i = i0 + u;
        if (i < j.nl) {
            gstore(j.off + i, run);
            if (j.neq == 0) gstore(j.lbase + i, lb[u]);
        }
        run += c[u];
    }
    if (threadIdx.x == 0) {
        gstore(j.off + j.nl, all);
        *j.total = all;
    }
    if (j.neq == 0)  // the expansion pairs through this table's grouping
        for (uint32_t m = threadIdx.x; m < j.nr; m += kJoinBlock)
            gstore(j.grp + m, t.rows[m]);
}

// Expansion.  With no other shared variable, L row i owns the output rows
// [off[i], off[i+1]), paired in turn with the R rows of its key, so each
// output row is one thread's: its L row by a binary search of the offsets,
// its R row the matching entry of the key's group; consecutive threads write
// consecutive rows.  (Giving each L row to a thread instead makes the thread
// of a hub key walk hundreds of pairs, a global load after the other.)  With
// other shared variables, a row's pairs are those that also agree on them,
// and each L row's thread writes its pairs.
namespace {
__shared__ uint32_t s_off[kSmallRows], s_lb[kSmallRows];

// the last row i in [lo, hi] with off[i] <= o (off non-decreasing, off[lo] <= o)
__device__ __forceinline__ uint32_t owner_row(const uint32_t *off, uint32_t lo, uint32_t hi,
                                              uint32_t o) {
    uint32_t n = hi - lo + 1, a = lo;
    while (n > 1) {
        const uint32_t half = n / 2;
        if (off[a + half] <= o) a += half;
        n -= half;
    }
    return a;
}

constexpr int kUnroll = 4;

// Output rows [o0, o1) of a job without other shared variables, thread-
// parallel: the L rows i0 + k own [loff[k], loff[k+1]) (loff in LDS, i0..i1),
// each paired in turn with the entries of its key's group of R rows, which
// start at lb[k] in grp.  The loads of kUnroll rows are issued before their
// stores.
__device__ __forceinline__ void expand_rows(const JoinJob &j, const uint32_t *loff,
                                            const uint32_t *lb, const uint32_t *grp,
                                            uint32_t i0, uint32_t i1, uint32_t o0,
                                            uint32_t o1) {
    for (uint32_t base = o0; base < o1; base += kBatchBlock * kUnroll) {
        uint32_t li[kUnroll], ri[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const uint32_t o = base + u * kBatchBlock + threadIdx.x;
            li[u] = ri[u] = 0;
            if (o < o1) {
                const uint32_t k = owner_row(loff, 0, i1 - i0, o);
                li[u] = i0 + k;
                ri[u] = gload(grp + lb[k] + (o - loff[k]));
            }
        }
        for (int c = 0; c < j.nlc + j.nrc; ++c) {
            const bool left = c < j.nlc;
            const uint32_t *src = left ? j.lcol[c] : j.rcol[c - j.nlc];
            uint32_t v[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u)
                v[u] = base + u * kBatchBlock + threadIdx.x < o1
                           ? gload(src + (left ? li[u] : ri[u])) : 0u;
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const uint32_t o = base + u * kBatchBlock + threadIdx.x;
                if (o < o1) gstore(j.out[c] + o, v[u]);
            }
        }
    }
}
}  // namespace

// a job with other shared variables: each L row's thread writes its pairs
__global__ __launch_bounds__(kJoinBlock) void batch_join_expand(const JoinJob *jobs) {
    const JoinJob &j = jobs[blockIdx.x];
    Table t{s_key, s_cnt, s_start, s_rows, 0};
    build_table(j, t, s_w);
    for (uint32_t i = threadIdx.x; i < j.nl; i += kJoinBlock) {
        const uint32_t h = find_slot(t, gload(j.lkey + i));
        if (h == kEmptyKey) continue;
        uint32_t o = gload(j.off + i);
        const uint32_t a = t.start[h], b = a + t.cnt[h];
        for (uint32_t m = a; m < b; ++m) {
            const uint32_t r = t.rows[m];
            if (!agree(j, i, r)) continue;
            for (int c = 0; c < j.nlc; ++c) gstore(j.out[c] + o, gload(j.lcol[c] + i));
            for (int c = 0; c < j.nrc; ++c)
                gstore(j.out[j.nlc + c] + o, gload(j.rcol[c] + r));
            ++o;
        }
    }
}

// a job without other shared variables: tiles of kSplitTile output rows, a
// workgroup each, over the grouping the count launch left (lbase, grp); a
// tile stages the offsets and group starts of the L rows that own it
__global__ __launch_bounds__(kBatchBlock) void batch_join_split(const SplitJob *jobs, int nj,
                                                                uint32_t tile_base) {
    const uint32_t tile = tile_base + blockIdx.x;
    int lo = 0, hi = nj - 1;  // the job: the last one whose first tile is <= tile
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (jobs[mid].tile0 <= tile) lo = mid; else hi = mid - 1;
    }
    const SplitJob &x = jobs[lo];
    const JoinJob &j = x.j;
    const uint32_t o0 = (tile - x.tile0) * kSplitTile;
    const uint32_t o1 = min(o0 + kSplitTile, j.nout);
    // the L rows owning [o0, o1): i0..i1 (at most nl of them)
    const uint32_t i0 = owner_row(j.off, 0, j.nl - 1, o0);
    const uint32_t i1 = owner_row(j.off, i0, j.nl - 1, o1 - 1);
    for (uint32_t k = threadIdx.x; k <= i1 - i0; k += kBatchBlock) {
        s_off[k] = gload(j.off + i0 + k);
        s_lb[k] = gload(j.lbase + i0 + k);
    }
    __syncthreads();
    expand_rows(j, s_off, s_lb, j.grp, i0, i1, o0, o1);
}

// ---------------------------------------------------------------------------
// batched sort: rows into LDS (column-major), a bitonic sort of row indices
// with the lexicographic order over all columns, rows written out in that
// order (DISTINCT: only rows differing from their predecessor)
// ---------------------------------------------------------------------------

namespace {
__shared__ uint32_t s_vals[kSortWords];
__shared__ uint16_t s_idx[kSortRows], s_pos[kSortRows];
__shared__ uint32_t s_sw[kBatchSortBlock / dev::kWave];
constexpr uint16_t kDropped = 0xFFFF;  // s_pos of a row DISTINCT leaves out

__device__ __forceinline__ bool row_less(uint32_t a, uint32_t b, uint32_t n, int ncols) {
    if (a >= n) return false;      // padding sorts last
    if (b >= n) return true;
    for (int c = 0; c < ncols; ++c) {
        const uint32_t x = s_vals[c * n + a], y = s_vals[c * n + b];
        if (x != y) return x < y;
    }
    return a < b;                  // equal rows keep their order: a total order
}

__device__ __forceinline__ bool row_equal(uint32_t a, uint32_t b, uint32_t n, int ncols) {
    for (int c = 0; c < ncols; ++c)
        if (s_vals[c * n + a] != s_vals[c * n + b]) return false;
    return true;
}
}  // namespace

// A workgroup of kBatchSortBlock threads per job.  Each step of the bitonic
// network compares p/2 disjoint pairs (i, i + d), i with bit d clear; thread
// q's pairs are numbered q, q + kBatchSortBlock, ... so that no thread idles.
__global__ __launch_bounds__(kBatchSortBlock) void batch_sort(const SortJob *jobs) {
    const SortJob &j = jobs[blockIdx.x];
    const uint32_t n = j.n;
    for (int c = 0; c < j.ncols; ++c)
        for (uint32_t i = threadIdx.x; i < n; i += kBatchSortBlock)
            s_vals[c * n + i] = gload(j.in[c] + i);
    uint32_t p = 1;
    while (p < n) p <<= 1;
    for (uint32_t i = threadIdx.x; i < p; i += kBatchSortBlock) s_idx[i] = (uint16_t)i;
    __syncthreads();
    const uint32_t pairs = p >> 1;
    for (uint32_t k = 2; k <= p; k <<= 1) {
        for (uint32_t d = k >> 1; d > 0; d >>= 1) {
            for (uint32_t q = threadIdx.x; q < pairs; q += kBatchSortBlock) {
                const uint32_t i = ((q & ~(d - 1)) << 1) | (q & (d - 1));
                const uint32_t x = i | d;
                const uint32_t a = s_idx[i], b = s_idx[x];
                const bool up = (i & k) == 0;
                if (row_less(b, a, n, j.ncols) == up) {
                    s_idx[i] = (uint16_t)b;
                    s_idx[x] = (uint16_t)a;
                }
            }
            __syncthreads();
        }
    }
    // output positions: all rows, or (DISTINCT) the first of each run of equal
    // rows; a thread counts a contiguous run of sorted rows, then the rows are
    // written in sorted-position order across the threads
    constexpr uint32_t kPer = kSortRows / kBatchSortBlock;  // 8
    const uint32_t i0 = threadIdx.x * kPer;
    bool kept[kPer];
    uint32_t keep = 0;
#pragma unroll
    for (uint32_t u = 0; u < kPer; ++u) {
        const uint32_t i = i0 + u;
        kept[u] = i < n && (!j.distinct || i == 0 || !row_equal(s_idx[i], s_idx[i - 1], n, j.ncols));
        keep += kept[u];
    }
    uint32_t all;
    uint32_t o = block_exclusive<kBatchSortBlock>(keep, s_sw, &all);
#pragma unroll
    for (uint32_t u = 0; u < kPer; ++u) {
        if (i0 + u >= n) break;
        s_pos[i0 + u] = kept[u] ? (uint16_t)o++ : kDropped;
    }
    __syncthreads();
    for (int c = 0; c < j.ncols; ++c)
        for (uint32_t i = threadIdx.x; i < n; i += kBatchSortBlock)
            if (s_pos[i] != kDropped) gstore(j.out[c] + s_pos[i], s_vals[c * n + s_idx[i]]);
    if (threadIdx.x == 0) *j.count = all;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

template <class Job>
static const Job *upload(tid_ctx *ctx, BatchState &bs, const std::vector<Job> &jobs) {
    const size_t bytes = jobs.size() * sizeof(Job);
    bs.host_keep.emplace_back(reinterpret_cast<const char *>(jobs.data()),
                              reinterpret_cast<const char *>(jobs.data()) + bytes);
    bs.keep.emplace_back(ctx, bytes);
    TID_HIP(hipMemcpyAsync(bs.keep.back().get(), bs.host_keep.back().data(), bytes,
                           hipMemcpyHostToDevice, ctx->stream));
    return bs.keep.back().get<const Job>();
}

// the expansions of jobs without other shared variables: one launch of
// output tiles; returns the other jobs
static std::vector<JoinJob> expand_split_jobs(tid_ctx *ctx, BatchState &bs,
                                              const std::vector<JoinJob> &jobs) {
    std::vector<JoinJob> rest;
    std::vector<SplitJob> split;
    uint64_t tiles = 0;
    for (const JoinJob &j : jobs) {
        if (j.neq != 0) {
            rest.push_back(j);
            continue;
        }
        SplitJob x{};
        x.j = j;
        x.tile0 = (uint32_t)tiles;
        tiles += (j.nout + kSplitTile - 1) / kSplitTile;
        split.push_back(x);
    }
    if (split.empty()) return rest;
    TID_REQUIRE(tiles < (1ull << 32), TID_E_UNSUPPORTED, "batched joins: output too large");
    const SplitJob *d = upload(ctx, bs, split);
    for (uint64_t t0 = 0; t0 < tiles; t0 += 1u << 20) {
        const unsigned g = (unsigned)std::min<uint64_t>(1u << 20, tiles - t0);
        hipLaunchKernelGGL(batch_join_split, dim3(g), dim3(kBatchBlock), 0, ctx->stream, d,
                           (int)split.size(), (uint32_t)t0);
        TID_HIP(hipGetLastError());
    }
    return rest;
}

void flush_join_jobs(tid_ctx *ctx, BatchState &bs, bool expand) {
    std::vector<JoinJob> &all = expand ? bs.expand_jobs : bs.count_jobs;
    if (all.empty()) return;
    std::vector<JoinJob> rest;
    if (expand) rest = expand_split_jobs(ctx, bs, all);
    std::vector<JoinJob> &jobs = expand ? rest : all;
    if (jobs.empty()) {
        all.clear();
        return;
    }
    const JoinJob *d = upload(ctx, bs, jobs);
    for (size_t j0 = 0; j0 < jobs.size(); j0 += 65535) {
        const unsigned g = (unsigned)std::min<size_t>(65535, jobs.size() - j0);
        if (expand)
            hipLaunchKernelGGL(batch_join_expand, dim3(g), dim3(kJoinBlock), 0, ctx->stream,
                               d + j0);
        else
            hipLaunchKernelGGL(batch_join_count, dim3(g), dim3(kJoinBlock), 0, ctx->stream,
                               d + j0);
        TID_HIP(hipGetLastError());
    }
    all.clear();
}

void flush_sort_jobs(tid_ctx *ctx, BatchState &bs) {
    if (!bs.row_sorts.empty()) {
        sort_rows_batched(ctx, bs.row_sorts, bs.keep, bs.host_keep);
        bs.row_sorts.clear();
    }
    if (bs.sort_jobs.empty()) return;
    const SortJob *d = upload(ctx, bs, bs.sort_jobs);
    for (size_t j0 = 0; j0 < bs.sort_jobs.size(); j0 += 65535) {
        const unsigned g = (unsigned)std::min<size_t>(65535, bs.sort_jobs.size() - j0);
        hipLaunchKernelGGL(batch_sort, dim3(g), dim3(kBatchSortBlock), 0, ctx->stream, d + j0);
        TID_HIP(hipGetLastError());
    }
    bs.sort_jobs.clear();
}

}  // namespace tid

// ---------------------------------------------------------------------------
// larger joins of a batch
// ---------------------------------------------------------------------------

namespace tid {

void exclusive_scan_async(tid_ctx *ctx, const uint32_t *in, uint64_t n, uint64_t *out);
int device_cus(tid_ctx *ctx);

namespace {

constexpr int kBigBlock = 256;
constexpr int kBigIPT = 4;
constexpr uint64_t kBigTile = (uint64_t)kBigBlock * kBigIPT;
constexpr int kBigLds = 2048;       // LDS rank table entries (> rows per tile)
constexpr uint32_t kNoSlot32 = 0xFFFFFFFFu;

// index j with base[j] <= x < base[j + 1] (base non-decreasing, base[0] = 0)
__device__ __forceinline__ int job_of(const uint64_t *base, int J, uint64_t x) {
    int lo = 0, hi = J;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (base[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Build: R rows, tile by tile from a work counter (tiles of all joins
// concatenated; tbase = tile prefix per join).  Each row finds or claims its
// key's slot; ranks within a slot are reserved per tile through an LDS table
// (one global atomic per slot present in the tile, not per row).
__global__ __launch_bounds__(kBigBlock) void big_insert(const BigCount *jobs, int J,
                                                        const uint64_t *tbase, uint64_t ntiles,
                                                        uint32_t *work, uint64_t *slots,
                                                        uint32_t *cnt, uint32_t *slot_of,
                                                        uint32_t *rank_of) {
    __shared__ uint32_t s_slot[kBigLds], s_cnt[kBigLds], s_base[kBigLds];
    __shared__ uint64_t s_tile;
    for (int x = threadIdx.x; x < kBigLds; x += kBigBlock) {
        s_slot[x] = kNoSlot32;
        s_cnt[x] = 0;
    }
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_tile = atomicAdd(work, 1u);
        __syncthreads();
        const uint64_t t = s_tile;
        if (t >= ntiles) break;
        const int j = job_of(tbase, J, t);
        const BigCount &b = jobs[j];
        const uint64_t r0 = (t - tbase[j]) * kBigTile;
        uint32_t h[kBigIPT], e[kBigIPT], local[kBigIPT];
#pragma unroll
        for (int u = 0; u < kBigIPT; ++u) {
            const uint64_t r = r0 + (uint64_t)u * kBigBlock + threadIdx.x;
            if (r >= b.nr) continue;
            const uint32_t key = b.rkey[r];
            const uint64_t want = (uint64_t)key + 1ull;
            uint32_t hh = dev::hash32(key) & b.mask;
            for (uint32_t probe = 0; probe <= b.mask; ++probe) {  // ends: free slots remain
                unsigned long long *w = (unsigned long long *)&slots[b.sbase + hh];
                unsigned long long cur = *w;
                if (cur == 0ull) cur = atomicCAS(w, 0ull, (unsigned long long)want);
                if (cur == 0ull || cur == want) break;
                hh = (hh + 1) & b.mask;
            }
            const uint32_t gs = (uint32_t)(b.sbase + hh);
            uint32_t ee = gs & (kBigLds - 1);
            for (;;) {  // ends: fewer distinct slots per tile than entries
                const uint32_t prev = atomicCAS(&s_slot[ee], kNoSlot32, gs);
                if (prev == kNoSlot32 || prev == gs) break;
                ee = (ee + 1) & (kBigLds - 1);
            }
            h[u] = gs;
            e[u] = ee;
            local[u] = atomicAdd(&s_cnt[ee], 1u);
        }
        __syncthreads();
        for (int x = threadIdx.x; x < kBigLds; x += kBigBlock) {
            const uint32_t sl = s_slot[x];
            if (sl != kNoSlot32) {
                s_base[x] = atomicAdd(&cnt[sl], s_cnt[x]);
                s_slot[x] = kNoSlot32;
                s_cnt[x] = 0;
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kBigIPT; ++u) {
            const uint64_t r = r0 + (uint64_t)u * kBigBlock + threadIdx.x;
            if (r >= b.nr) continue;
            slot_of[b.rbase + r] = h[u];
            rank_of[b.rbase + r] = s_base[e[u]] + local[u];
        }
    }
}

__global__ void big_fill(const BigCount *jobs, int J, const uint64_t *rbase, uint64_t nrows,
                         const uint32_t *slot_of, const uint32_t *rank_of, const uint64_t *start,
                         uint32_t *rows) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < nrows; g += stride) {
        const int j = job_of(rbase, J, g);
        rows[start[slot_of[g]] + rank_of[g]] = (uint32_t)(g - jobs[j].rbase);
    }
}

__device__ __forceinline__ bool big_agree(const uint32_t *const *el, const uint32_t *const *er,
                                          int neq, uint64_t l, uint32_t r) {
    bool ok = true;
    for (int e = 0; e < neq; ++e) ok &= el[e][l] == er[e][r];
    return ok;
}

__global__ void big_probe(const BigCount *jobs, int J, const uint64_t *lbase, uint64_t nrows,
                          const uint64_t *slots, const uint32_t *cnt, const uint64_t *start,
                          const uint32_t *rows, uint32_t *lslot, uint32_t *lcount) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < nrows; g += stride) {
        const int j = job_of(lbase, J, g);
        const BigCount &b = jobs[j];
        const uint64_t l = g - b.lbase;
        const uint32_t key = b.lkey[l];
        const uint64_t want = (uint64_t)key + 1ull;
        uint32_t h = dev::hash32(key) & b.mask;
        uint32_t slot = kNoSlot32, c = 0;
        for (uint32_t probe = 0; probe <= b.mask; ++probe) {
            const uint64_t cur = slots[b.sbase + h];
            if (cur == want) {
                slot = (uint32_t)(b.sbase + h);
                break;
            }
            if (cur == 0ull) break;
            h = (h + 1) & b.mask;
        }
        if (slot != kNoSlot32) {
            if (b.neq == 0) {
                c = cnt[slot];
            } else {
                const uint64_t a = start[slot];
                for (uint32_t m = 0; m < cnt[slot]; ++m)
                    c += big_agree(b.eq_l, b.eq_r, b.neq, l, rows[a + m]);
            }
        }
        lslot[g] = slot;
        lcount[g] = c;
    }
}

__global__ void big_totals(const BigCount *jobs, int J, const uint64_t *loff, uint64_t *tot) {
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < J; j += gridDim.x * blockDim.x)
        tot[j] = loff[jobs[j].lbase + jobs[j].nl] - loff[jobs[j].lbase];
}

// one output row per thread: its join, its L row (binary search over the
// join's slice of the offsets), the k-th partner in the L row's slot
__global__ void big_expand(const BigExpand *jobs, int J, const uint64_t *obase, uint64_t ntotal,
                           const uint64_t *loff, const uint32_t *lslot, const uint32_t *cnt,
                           const uint64_t *start, const uint32_t *rows) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < ntotal; g += stride) {
        const int j = job_of(obase, J, g);
        const BigExpand &b = jobs[j];
        const uint64_t o = g - b.obase;
        const uint64_t base = loff[b.lbase];
        uint64_t lo = 0, hi = b.nl;  // last L row i with loff[i] - base <= o
        while (hi - lo > 1) {
            const uint64_t mid = (lo + hi) >> 1;
            if (loff[b.lbase + mid] - base <= o) lo = mid;
            else hi = mid;
        }
        const uint64_t i = lo;
        uint64_t k = o - (loff[b.lbase + i] - base);
        const uint32_t slot = lslot[b.lbase + i];
        const uint64_t a = start[slot];
        uint32_t r;
        if (b.neq == 0) {
            r = rows[a + k];
        } else {  // the k-th partner that also agrees on the other shared variables
            uint32_t m = 0;
            for (;; ++m) {
                r = rows[a + m];
                if (big_agree(b.eq_l, b.eq_r, b.neq, i, r)) {
                    if (k == 0) break;
                    --k;
                }
            }
        }
        // the probe side is L or R; output columns are L's, then R's kept ones
        const uint64_t li = b.probe_is_left ? i : r, ri = b.probe_is_left ? r : i;
        for (int c = 0; c < b.nlc; ++c) b.out[c][o] = b.lcol[c][li];
        for (int c = 0; c < b.nrc; ++c) b.out[b.nlc + c][o] = b.rcol[c][ri];
    }
}

unsigned grid_cap(uint64_t n, uint64_t cap = 16384) {
    return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((n + 255) / 256, cap));
}

}  // namespace

void flush_big_count(tid_ctx *ctx, std::vector<BigJoinReq> &reqs,
                     std::shared_ptr<BigArena> *arena_out) {
    if (reqs.empty()) return;
    const int J = (int)reqs.size();
    std::vector<BigCount> jobs(J);
    std::vector<uint64_t> tbase(J + 1, 0), rbase(J + 1, 0), lbase(J + 1, 0);
    uint64_t S = 0;
    for (int j = 0; j < J; ++j) {
        BigCount &b = jobs[j];
        b = reqs[j].c;
        uint64_t cap = 64;
        while (cap < 2 * b.nr) cap <<= 1;
        b.mask = (uint32_t)(cap - 1);
        b.sbase = S;
        S += cap;
        b.rbase = rbase[j];
        b.lbase = lbase[j];
        rbase[j + 1] = rbase[j] + b.nr;
        lbase[j + 1] = lbase[j] + b.nl;
        tbase[j + 1] = tbase[j] + (b.nr + kBigTile - 1) / kBigTile;
    }
    const uint64_t NR = rbase[J], NL = lbase[J], T = tbase[J];
    TID_REQUIRE(S < (1ull << 32) && NR < (1ull << 32), TID_E_UNSUPPORTED,
                "batched joins: too many build rows in one round");
    // one arena: job table and prefixes, then the per-slot and per-row arrays
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += align_up(std::max<size_t>(bytes, 8));
        return at;
    };
    const size_t o_jobs = take(J * sizeof(BigCount)), o_tb = take((J + 1) * 8),
                 o_rb = take((J + 1) * 8), o_lb = take((J + 1) * 8), o_work = take(8),
                 o_slots = take(S * 8), o_cnt = take(S * 4), o_start = take((S + 1) * 8),
                 o_slotof = take(NR * 4), o_rank = take(NR * 4), o_rows = take(NR * 4),
                 o_lslot = take(NL * 4), o_lcnt = take(NL * 4), o_loff = take((NL + 1) * 8),
                 o_tot = take(J * 8);
    auto arena = std::make_shared<BigArena>();
    arena->buf = DevBuf(ctx, off);
    char *base = arena->buf.get<char>();
    arena->slots = reinterpret_cast<uint64_t *>(base + o_slots);
    arena->cnt = reinterpret_cast<uint32_t *>(base + o_cnt);
    arena->start = reinterpret_cast<uint64_t *>(base + o_start);
    arena->rows = reinterpret_cast<uint32_t *>(base + o_rows);
    arena->lslot = reinterpret_cast<uint32_t *>(base + o_lslot);
    arena->loff = reinterpret_cast<uint64_t *>(base + o_loff);
    arena->tot = reinterpret_cast<uint64_t *>(base + o_tot);
    // host tables: one staging copy, then one upload
    std::vector<char> host(o_slots);
    std::memcpy(host.data() + o_jobs, jobs.data(), J * sizeof(BigCount));
    std::memcpy(host.data() + o_tb, tbase.data(), (J + 1) * 8);
    std::memcpy(host.data() + o_rb, rbase.data(), (J + 1) * 8);
    std::memcpy(host.data() + o_lb, lbase.data(), (J + 1) * 8);
    std::memset(host.data() + o_work, 0, 8);
    TID_HIP(hipMemcpyAsync(base, host.data(), o_slots, hipMemcpyHostToDevice, ctx->stream));
    // slot words and counts start at zero (one clear of the contiguous run)
    TID_HIP(hipMemsetAsync(base + o_slots, 0, o_start - o_slots, ctx->stream));
    const BigCount *dj = reinterpret_cast<const BigCount *>(base + o_jobs);
    const uint64_t *dtb = reinterpret_cast<const uint64_t *>(base + o_tb);
    const uint64_t *drb = reinterpret_cast<const uint64_t *>(base + o_rb);
    const uint64_t *dlb = reinterpret_cast<const uint64_t *>(base + o_lb);
    uint32_t *slot_of = reinterpret_cast<uint32_t *>(base + o_slotof);
    uint32_t *rank_of = reinterpret_cast<uint32_t *>(base + o_rank);
    uint32_t *lcount = reinterpret_cast<uint32_t *>(base + o_lcnt);
    const unsigned workers = (unsigned)std::max<uint64_t>(
        1, std::min<uint64_t>(T, 4ull * (uint64_t)device_cus(ctx)));
    if (T)
        hipLaunchKernelGGL(big_insert, dim3(workers), dim3(kBigBlock), 0, ctx->stream, dj, J,
                           dtb, T, reinterpret_cast<uint32_t *>(base + o_work), arena->slots,
                           arena->cnt, slot_of, rank_of);
    TID_HIP(hipGetLastError());
    exclusive_scan_async(ctx, arena->cnt, S, arena->start);
    if (NR)
        hipLaunchKernelGGL(big_fill, dim3(grid_cap(NR)), dim3(256), 0, ctx->stream, dj, J, drb,
                           NR, slot_of, rank_of, arena->start, arena->rows);
    TID_HIP(hipGetLastError());
    if (NL)
        hipLaunchKernelGGL(big_probe, dim3(grid_cap(NL)), dim3(256), 0, ctx->stream, dj, J, dlb,
                           NL, arena->slots, arena->cnt, arena->start, arena->rows, arena->lslot,
                           lcount);
    TID_HIP(hipGetLastError());
    exclusive_scan_async(ctx, lcount, NL, arena->loff);
    hipLaunchKernelGGL(big_totals, dim3(grid_cap(J)), dim3(256), 0, ctx->stream, dj, J,
                       arena->loff, arena->tot);
    TID_HIP(hipGetLastError());
    for (int j = 0; j < J; ++j) {
        reqs[j].pj->total_ptr = arena->tot + j;
        reqs[j].pj->big_lbase = lbase[j];
        reqs[j].pj->big_arena = arena;
    }
    reqs.clear();
    *arena_out = arena;
}

void flush_big_expand(tid_ctx *ctx, const BigArena &arena, std::vector<BigExpand> &jobs,
                      BatchState &bs) {
    if (jobs.empty()) return;
    const int J = (int)jobs.size();
    // jobs arrive with obase = their output's first row in the concatenated
    // output space; bs.big_out_total is that space's size
    std::vector<uint64_t> obase(J + 1, 0);
    for (int j = 0; j < J; ++j) obase[j] = jobs[j].obase;
    const uint64_t total = bs.big_out_total;
    obase[J] = total;
    const size_t bytes_jobs = align_up(J * sizeof(BigExpand));
    std::vector<char> host(bytes_jobs + (J + 1) * 8);
    std::memcpy(host.data(), jobs.data(), J * sizeof(BigExpand));
    std::memcpy(host.data() + bytes_jobs, obase.data(), (J + 1) * 8);
    bs.host_keep.push_back(std::move(host));
    bs.keep.emplace_back(ctx, bs.host_keep.back().size());
    char *d = bs.keep.back().get<char>();
    TID_HIP(hipMemcpyAsync(d, bs.host_keep.back().data(), bs.host_keep.back().size(),
                           hipMemcpyHostToDevice, ctx->stream));
    if (total)
        hipLaunchKernelGGL(big_expand, dim3(grid_cap(total)), dim3(256), 0, ctx->stream,
                           reinterpret_cast<const BigExpand *>(d), J,
                           reinterpret_cast<const uint64_t *>(d + bytes_jobs), total, arena.loff,
                           arena.lslot, arena.cnt, arena.start, arena.rows);
    TID_HIP(hipGetLastError());
    jobs.clear();
    bs.big_out_total = 0;
}

}  // namespace tid

namespace tid {

namespace {
__global__ void batch_copy_kernel(const CopyJob *jobs, const uint64_t *base, int J,
                                  uint64_t total) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += stride) {
        const int j = job_of(base, J, g);
        const uint64_t i = g - base[j];
        jobs[j].dst[i] = jobs[j].src[i];
    }
}
}  // namespace

void batch_copy(tid_ctx *ctx, const std::vector<CopyJob> &jobs, BatchState &bs) {
    std::vector<CopyJob> nz;
    for (const CopyJob &c : jobs)
        if (c.n) nz.push_back(c);
    if (nz.empty()) return;
    const int J = (int)nz.size();
    std::vector<uint64_t> base(J + 1, 0);
    for (int j = 0; j < J; ++j) base[j + 1] = base[j] + nz[j].n;
    const size_t bj = align_up(J * sizeof(CopyJob));
    std::vector<char> host(bj + (J + 1) * 8);
    std::memcpy(host.data(), nz.data(), J * sizeof(CopyJob));
    std::memcpy(host.data() + bj, base.data(), (J + 1) * 8);
    bs.host_keep.push_back(std::move(host));
    bs.keep.emplace_back(ctx, bs.host_keep.back().size());
    char *d = bs.keep.back().get<char>();
    TID_HIP(hipMemcpyAsync(d, bs.host_keep.back().data(), bs.host_keep.back().size(),
                           hipMemcpyHostToDevice, ctx->stream));
    hipLaunchKernelGGL(batch_copy_kernel, dim3(grid_cap(base[J])), dim3(256), 0, ctx->stream,
                       reinterpret_cast<const CopyJob *>(d),
                       reinterpret_cast<const uint64_t *>(d + bj), J, base[J]);
    TID_HIP(hipGetLastError());
}

}  // namespace tid
