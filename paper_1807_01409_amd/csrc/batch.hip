// batch.hip -- the small joins and the final sorts of many plans, each kind
// in one launch per round of a batch (the lockstep rounds of
// tid_query_batch): one workgroup per job, the job table in device memory.
// A plan's join whose sides both have at most kSmallRows rows does not launch
// its own hash build, scans, probe and expansion; it is a job of the round's
// one count launch, then of the next round's one expansion launch.  A plan's
// final lexicographic sort of at most kSortRows rows is likewise a job of one
// sort launch.  Everything a job touches besides its inputs and outputs lives
// in the workgroup's LDS.
//
// Join job (Sec. 4.2: an equi-join on the shared variable, done here with a
// hash table in LDS): the R side's keys go into an open-addressing table
// (slot = key, count, first position of its rows in a per-slot row list);
// each L row finds its key's slot and pairs with the slot's R rows that also
// agree on every other shared variable (natural join).  The count launch
// writes each L row's exclusive output offset and the job's total; the
// expansion launch rebuilds the table and writes the rows.  The order of
// rows within a join's output is not defined (a plan's result is always
// sorted at its end).
#include "batch.hpp"
#include "device_common.hpp"

#include <algorithm>

namespace tid {

namespace {

__device__ __forceinline__ uint32_t pow2_at_least(uint32_t x) {
    uint32_t p = 64;
    while (p < x) p <<= 1;
    return p;
}

// exclusive scan of v over the block in thread order; returns this thread's
// prefix and leaves the total in *total
__device__ __forceinline__ uint32_t block_exclusive(uint32_t v, uint32_t *s_w, uint32_t *total) {
    constexpr int NW = kBatchBlock / dev::kWave;
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

// R's keys into the LDS table: slot counts, slot starts, rows grouped by slot
__device__ void build_table(const JoinJob &j, Table &t, uint32_t *s_w) {
    const uint32_t ts = pow2_at_least(2 * j.nr);
    t.mask = ts - 1;
    for (uint32_t s = threadIdx.x; s < ts; s += kBatchBlock) {
        t.key[s] = kEmptyKey;
        t.cnt[s] = 0;
    }
    __syncthreads();
    for (uint32_t r = threadIdx.x; r < j.nr; r += kBatchBlock) {
        const uint32_t k = j.rkey[r];
        uint32_t h = dev::hash32(k) & t.mask;
        for (;;) {  // ends: the table has more slots than keys
            const uint32_t prev = atomicCAS(&t.key[h], kEmptyKey, k);
            if (prev == kEmptyKey || prev == k) break;
            h = (h + 1) & t.mask;
        }
        atomicAdd(&t.cnt[h], 1u);
    }
    __syncthreads();
    // slot starts: each thread scans a contiguous run of ts / block slots
    const uint32_t per = ts / kBatchBlock > 0 ? ts / kBatchBlock : 1;
    const uint32_t s0 = threadIdx.x * per;
    uint32_t local = 0;
    for (uint32_t s = s0; s < s0 + per && s < ts; ++s) local += t.cnt[s];
    uint32_t all;
    uint32_t run = block_exclusive(local, s_w, &all);
    for (uint32_t s = s0; s < s0 + per && s < ts; ++s) {
        t.start[s] = run;
        run += t.cnt[s];
        t.cnt[s] = 0;  // counts again while the rows are placed
    }
    __syncthreads();
    for (uint32_t r = threadIdx.x; r < j.nr; r += kBatchBlock) {
        const uint32_t k = j.rkey[r];
        uint32_t h = dev::hash32(k) & t.mask;
        while (t.key[h] != k) h = (h + 1) & t.mask;
        t.rows[t.start[h] + atomicAdd(&t.cnt[h], 1u)] = r;
    }
    __syncthreads();
}

// the slot of key k, or kEmptyKey
__device__ __forceinline__ uint32_t find_slot(const Table &t, uint32_t k) {
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
    for (int e = 0; e < j.neq; ++e) ok &= j.eq_l[e][l] == j.eq_r[e][r];
    return ok;
}

constexpr uint32_t kRowsPerThread = kSmallRows / kBatchBlock;  // 16

__shared__ uint32_t s_key[kSmallSlots], s_cnt[kSmallSlots], s_start[kSmallSlots];
__shared__ uint32_t s_rows[kSmallRows];
__shared__ uint32_t s_w[kBatchBlock / dev::kWave];

}  // namespace

__global__ __launch_bounds__(kBatchBlock) void batch_join_count(const JoinJob *jobs) {
    const JoinJob &j = jobs[blockIdx.x];
    Table t{s_key, s_cnt, s_start, s_rows, 0};
    build_table(j, t, s_w);
    // each thread a contiguous run of L rows, so offsets follow row order
    uint32_t c[kRowsPerThread];
    uint32_t local = 0;
    const uint32_t i0 = threadIdx.x * kRowsPerThread;
#pragma unroll
    for (uint32_t u = 0; u < kRowsPerThread; ++u) {
        const uint32_t i = i0 + u;
        c[u] = 0;
        if (i >= j.nl) continue;
        const uint32_t h = find_slot(t, j.lkey[i]);
        if (h == kEmptyKey) continue;
        const uint32_t a = t.start[h], b = a + t.cnt[h];
        if (j.neq == 0) {
            c[u] = b - a;
        } else {
            for (uint32_t m = a; m < b; ++m) c[u] += agree(j, i, t.rows[m]);
        }
        local += c[u];
    }
    uint32_t all;
    uint32_t run = block_exclusive(local, s_w, &all);
#pragma unroll
    for (uint32_t u = 0; u < kRowsPerThread; ++u) {
        const uint32_t i = i0 + u;
        if (i < j.nl) j.off[i] = run;
        run += c[u];
    }
    if (threadIdx.x == 0) {
        j.off[j.nl] = all;
        *j.total = all;
    }
}

__global__ __launch_bounds__(kBatchBlock) void batch_join_expand(const JoinJob *jobs) {
    const JoinJob &j = jobs[blockIdx.x];
    Table t{s_key, s_cnt, s_start, s_rows, 0};
    build_table(j, t, s_w);
    for (uint32_t i = threadIdx.x; i < j.nl; i += kBatchBlock) {
        const uint32_t h = find_slot(t, j.lkey[i]);
        if (h == kEmptyKey) continue;
        uint32_t o = j.off[i];
        const uint32_t a = t.start[h], b = a + t.cnt[h];
        for (uint32_t m = a; m < b; ++m) {
            const uint32_t r = t.rows[m];
            if (j.neq && !agree(j, i, r)) continue;
            for (int c = 0; c < j.nlc; ++c) j.out[c][o] = j.lcol[c][i];
            for (int c = 0; c < j.nrc; ++c) j.out[j.nlc + c][o] = j.rcol[c][r];
            ++o;
        }
    }
}

// ---------------------------------------------------------------------------
// batched sort: rows into LDS (column-major), a bitonic sort of row indices
// with the lexicographic order over all columns, rows written out in that
// order (DISTINCT: only rows differing from their predecessor)
// ---------------------------------------------------------------------------

namespace {
__shared__ uint32_t s_vals[kSortWords];
__shared__ uint16_t s_idx[kSortRows];
__shared__ uint32_t s_sw[kBatchBlock / dev::kWave];

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

__global__ __launch_bounds__(kBatchBlock) void batch_sort(const SortJob *jobs) {
    const SortJob &j = jobs[blockIdx.x];
    const uint32_t n = j.n;
    for (int c = 0; c < j.ncols; ++c)
        for (uint32_t i = threadIdx.x; i < n; i += kBatchBlock) s_vals[c * n + i] = j.in[c][i];
    uint32_t p = 1;
    while (p < n) p <<= 1;
    for (uint32_t i = threadIdx.x; i < p; i += kBatchBlock) s_idx[i] = (uint16_t)i;
    __syncthreads();
    for (uint32_t k = 2; k <= p; k <<= 1) {
        for (uint32_t d = k >> 1; d > 0; d >>= 1) {
            for (uint32_t i = threadIdx.x; i < p; i += kBatchBlock) {
                const uint32_t x = i ^ d;
                if (x > i) {
                    const uint32_t a = s_idx[i], b = s_idx[x];
                    const bool up = (i & k) == 0;
                    if (row_less(b, a, n, j.ncols) == up) {
                        s_idx[i] = (uint16_t)b;
                        s_idx[x] = (uint16_t)a;
                    }
                }
            }
            __syncthreads();
        }
    }
    // output positions: all rows, or (DISTINCT) the first of each run of equal rows
    constexpr uint32_t kPer = kSortRows / kBatchBlock;  // 32
    const uint32_t i0 = threadIdx.x * kPer;
    uint32_t keep = 0;
    for (uint32_t u = 0; u < kPer; ++u) {
        const uint32_t i = i0 + u;
        if (i < n && (!j.distinct || i == 0 || !row_equal(s_idx[i], s_idx[i - 1], n, j.ncols)))
            ++keep;
    }
    uint32_t all;
    uint32_t o = block_exclusive(keep, s_sw, &all);
    for (uint32_t u = 0; u < kPer; ++u) {
        const uint32_t i = i0 + u;
        if (i < n && (!j.distinct || i == 0 || !row_equal(s_idx[i], s_idx[i - 1], n, j.ncols))) {
            for (int c = 0; c < j.ncols; ++c) j.out[c][o] = s_vals[c * n + s_idx[i]];
            ++o;
        }
    }
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

void flush_join_jobs(tid_ctx *ctx, BatchState &bs, bool expand) {
    std::vector<JoinJob> &jobs = expand ? bs.expand_jobs : bs.count_jobs;
    if (jobs.empty()) return;
    const JoinJob *d = upload(ctx, bs, jobs);
    for (size_t j0 = 0; j0 < jobs.size(); j0 += 65535) {
        const unsigned g = (unsigned)std::min<size_t>(65535, jobs.size() - j0);
        if (expand)
            hipLaunchKernelGGL(batch_join_expand, dim3(g), dim3(kBatchBlock), 0, ctx->stream,
                               d + j0);
        else
            hipLaunchKernelGGL(batch_join_count, dim3(g), dim3(kBatchBlock), 0, ctx->stream,
                               d + j0);
        TID_HIP(hipGetLastError());
    }
    jobs.clear();
}

void flush_sort_jobs(tid_ctx *ctx, BatchState &bs) {
    if (bs.sort_jobs.empty()) return;
    const SortJob *d = upload(ctx, bs, bs.sort_jobs);
    for (size_t j0 = 0; j0 < bs.sort_jobs.size(); j0 += 65535) {
        const unsigned g = (unsigned)std::min<size_t>(65535, bs.sort_jobs.size() - j0);
        hipLaunchKernelGGL(batch_sort, dim3(g), dim3(kBatchBlock), 0, ctx->stream, d + j0);
        TID_HIP(hipGetLastError());
    }
    bs.sort_jobs.clear();
}

}  // namespace tid
