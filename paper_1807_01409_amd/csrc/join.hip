// join.hip -- inner equi-join of two binding tables on one column pair
// (Sec. 4.2: any of the nine relation types of Table 3 is a choice of the two
// columns).  The paper sorts both key vectors, merge-joins them into pairs of
// positions with equal keys, and gathers the value parts through those pairs.
// Both algorithms here produce the pairs implicitly, as per-row match counts,
// their exclusive scan (output offsets), and an expansion in which every
// output row finds its (left, right) pair by binary search over the offsets:
//   sort-merge  radix-sort both sides on the key; each left key finds its
//               run in the sorted right keys by binary search;
//   hash        build an open-addressing table of distinct keys on the
//               smaller side, with each key's rows laid out contiguously
//               (count, scan, fill), and probe it with the other side.
// Output rows are then put in lexicographic order by the caller.
#include "compact.hpp"

#include <algorithm>

namespace tid {

// from sort.hip
bool radix_sort_pairs(tid_ctx *ctx, uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1,
                      uint64_t n, int bits);
void iota(tid_ctx *ctx, uint32_t *p, uint64_t n);
void fill(tid_ctx *ctx, uint32_t *p, uint64_t n, uint32_t v);
std::unique_ptr<tid_table> sort_rows(tid_ctx *ctx, const tid_table *t, uint64_t n, int distinct);

static unsigned grid_of(uint64_t n, unsigned block = 256, unsigned cap = 8192) {
    return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((n + block - 1) / block, cap));
}

// ---------------------------------------------------------------------------
// device-wide exclusive scan: uint32 counts -> uint64 offsets (n + 1 entries)
// ---------------------------------------------------------------------------

constexpr int kScanBlock = 256;
constexpr int kScanIPT = 4;
constexpr uint64_t kScanTile = (uint64_t)kScanBlock * kScanIPT;

__global__ __launch_bounds__(kScanBlock) void range_sums(const uint32_t *__restrict__ in,
                                                          uint64_t n, uint64_t range,
                                                          uint64_t *sums) {
    __shared__ uint64_t s_w[kScanBlock / dev::kWave];
    const int tid = threadIdx.x, wave = tid / dev::kWave, lane = tid % dev::kWave;
    const uint64_t r0 = (uint64_t)blockIdx.x * range, r1 = min(n, r0 + range);
    uint64_t s = 0;
    for (uint64_t i = r0 + tid; i < r1; i += kScanBlock) s += in[i];
    s = dev::wave_sum(s);
    if (lane == 0) s_w[wave] = s;
    __syncthreads();
    if (tid == 0) {
        uint64_t t = 0;
        for (int w = 0; w < kScanBlock / dev::kWave; ++w) t += s_w[w];
        sums[blockIdx.x] = t;
    }
}

// exclusive scan of P <= 4096 uint64 in one workgroup; base[P] = total
__global__ __launch_bounds__(1024) void small_exclusive_scan(const uint64_t *in, uint64_t *base,
                                                              uint32_t P) {
    __shared__ uint64_t s_w[16];
    const int tid = threadIdx.x, wave = tid / dev::kWave, lane = tid % dev::kWave;
    const uint32_t chunk = (P + 1023) / 1024;
    const uint32_t a = min(P, tid * chunk), b = min(P, a + chunk);
    uint64_t sum = 0;
    for (uint32_t i = a; i < b; ++i) sum += in[i];
    const uint64_t incl = dev::wave_inclusive_sum(sum);
    if (lane == dev::kWave - 1) s_w[wave] = incl;
    __syncthreads();
    uint64_t before = 0;
    for (int w = 0; w < wave; ++w) before += s_w[w];
    uint64_t run = before + incl - sum;
    for (uint32_t i = a; i < b; ++i) {
        base[i] = run;
        run += in[i];
    }
    if (tid == 1023) base[P] = before + incl;
}

__global__ __launch_bounds__(kScanBlock) void range_scan(const uint32_t *__restrict__ in,
                                                          uint64_t n, uint64_t range,
                                                          const uint64_t *base, uint64_t *out) {
    __shared__ uint64_t s_w[kScanBlock / dev::kWave];
    __shared__ uint64_t s_run;
    const int tid = threadIdx.x, wave = tid / dev::kWave, lane = tid % dev::kWave;
    const uint64_t r0 = (uint64_t)blockIdx.x * range, r1 = min(n, r0 + range);
    if (tid == 0) s_run = base[blockIdx.x];
    __syncthreads();
    for (uint64_t t0 = r0; t0 < r1; t0 += kScanTile) {
        uint32_t v[kScanIPT];
        uint64_t local = 0;
#pragma unroll
        for (int u = 0; u < kScanIPT; ++u) {
            const uint64_t i = t0 + (uint64_t)tid * kScanIPT + u;
            v[u] = i < r1 ? in[i] : 0u;
            local += v[u];
        }
        const uint64_t incl = dev::wave_inclusive_sum(local);
        if (lane == dev::kWave - 1) s_w[wave] = incl;
        __syncthreads();
        uint64_t before = s_run;
        for (int w = 0; w < wave; ++w) before += s_w[w];
        uint64_t run = before + incl - local;
#pragma unroll
        for (int u = 0; u < kScanIPT; ++u) {
            const uint64_t i = t0 + (uint64_t)tid * kScanIPT + u;
            if (i < r1) out[i] = run;
            run += v[u];
        }
        __syncthreads();
        if (tid == kScanBlock - 1) s_run = run;
        __syncthreads();
    }
    if (blockIdx.x == gridDim.x - 1 && tid == 0) out[n] = s_run;
}

__global__ void set_zero_u64(uint64_t *p) { *p = 0; }

// The whole scan in one workgroup, tile by tile (small inputs: one launch).
constexpr int kOneBlock = 1024;
constexpr uint64_t kOneTile = (uint64_t)kOneBlock * kScanIPT;
constexpr uint64_t kOneMax = 8 * kOneTile;
__global__ __launch_bounds__(kOneBlock) void one_block_scan(const uint32_t *__restrict__ in,
                                                            uint64_t n, uint64_t *out) {
    __shared__ uint64_t s_w[kOneBlock / dev::kWave];
    const int tid = threadIdx.x, wave = tid / dev::kWave, lane = tid % dev::kWave;
    uint64_t carry = 0;
    for (uint64_t t0 = 0; t0 < n; t0 += kOneTile) {
        uint32_t v[kScanIPT];
        uint64_t local = 0;
#pragma unroll
        for (int u = 0; u < kScanIPT; ++u) {
            const uint64_t i = t0 + (uint64_t)tid * kScanIPT + u;
            v[u] = i < n ? in[i] : 0u;
            local += v[u];
        }
        const uint64_t incl = dev::wave_inclusive_sum(local);
        if (lane == dev::kWave - 1) s_w[wave] = incl;
        __syncthreads();
        uint64_t before = carry, tile = 0;
        for (int w = 0; w < kOneBlock / dev::kWave; ++w) {
            if (w < wave) before += s_w[w];
            tile += s_w[w];
        }
        uint64_t run = before + incl - local;
#pragma unroll
        for (int u = 0; u < kScanIPT; ++u) {
            const uint64_t i = t0 + (uint64_t)tid * kScanIPT + u;
            if (i < n) out[i] = run;
            run += v[u];
        }
        carry += tile;
        __syncthreads();  // s_w is rewritten by the next tile
    }
    if (tid == 0) out[n] = carry;
}

// out[0..n] = exclusive prefix sums of in[0..n); out[n] = total, left on the device.
void exclusive_scan_async(tid_ctx *ctx, const uint32_t *in, uint64_t n, uint64_t *out) {
    if (n == 0) {
        hipLaunchKernelGGL(set_zero_u64, dim3(1), dim3(1), 0, ctx->stream, out);
        TID_HIP(hipGetLastError());
        return;
    }
    if (n <= kOneMax) {
        hipLaunchKernelGGL(one_block_scan, dim3(1), dim3(kOneBlock), 0, ctx->stream, in, n, out);
        TID_HIP(hipGetLastError());
        return;
    }
    const uint64_t tiles = (n + kScanTile - 1) / kScanTile;
    uint64_t P = std::max<uint64_t>(1, std::min<uint64_t>(tiles, 4096));
    const uint64_t range = (tiles + P - 1) / P * kScanTile;
    P = (n + range - 1) / range;
    DevBuf sums(ctx, P * 8), base(ctx, (P + 1) * 8);
    hipLaunchKernelGGL(range_sums, dim3((uint32_t)P), dim3(kScanBlock), 0, ctx->stream, in, n,
                       range, sums.get<uint64_t>());
    TID_HIP(hipGetLastError());
    hipLaunchKernelGGL(small_exclusive_scan, dim3(1), dim3(1024), 0, ctx->stream,
                       sums.get<const uint64_t>(), base.get<uint64_t>(), (uint32_t)P);
    TID_HIP(hipGetLastError());
    hipLaunchKernelGGL(range_scan, dim3((uint32_t)P), dim3(kScanBlock), 0, ctx->stream, in, n,
                       range, base.get<const uint64_t>(), out);
    TID_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// sort-merge matching
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint64_t lower_bound_u64(const uint64_t *a, uint64_t n, uint64_t x) {
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ uint64_t upper_bound_u64(const uint64_t *a, uint64_t n, uint64_t x) {
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (a[mid] <= x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// for each sorted probe key: where its run starts in the sorted build keys, and its length
__global__ void merge_counts(const uint64_t *qk, uint64_t nq, const uint64_t *bk, uint64_t nb,
                             uint32_t *start, uint32_t *count) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nq; i += stride) {
        const uint64_t x = qk[i];
        const uint64_t lo = lower_bound_u64(bk, nb, x);
        start[i] = (uint32_t)lo;
        count[i] = (uint32_t)upper_bound_u64(bk + lo, nb - lo, x);
    }
}

// ---------------------------------------------------------------------------
// hash build and probe
// ---------------------------------------------------------------------------


// Build: every build row finds (or claims) its key's slot -- slot words hold
// key + 1, 0 = empty -- and takes a rank among the rows of that slot.  The
// ranks are reserved per workgroup round, not per row: the round's rows are
// grouped by slot in an LDS table, and one global atomic per slot present
// reserves that group's ranks, so a key held by many rows (a hub) costs one
// global atomic per round instead of one per row.
constexpr int kHashBlock = 256;
constexpr int kHashIPT = 4;
constexpr int kHashLds = 2048;  // entries; a round holds at most 1024 distinct slots
constexpr uint32_t kNoSlot = 0xFFFFFFFFu;
// largest build side the automatic choice sends to the hash join (2^23 rows:
// 2^24 slots of 12 B = 192 MB)
constexpr uint64_t kHashAutoMaxRows = 1ull << 23;

__global__ __launch_bounds__(kHashBlock) void hash_insert(const uint32_t *keys, uint64_t n,
                                                          unsigned long long *slots, uint32_t mask,
                                                          uint32_t *slot_of, uint32_t *rank_of,
                                                          uint32_t *slot_count) {
    __shared__ uint32_t s_slot[kHashLds], s_cnt[kHashLds], s_base[kHashLds];
    for (int x = threadIdx.x; x < kHashLds; x += kHashBlock) {
        s_slot[x] = kNoSlot;
        s_cnt[x] = 0;
    }
    __syncthreads();
    const uint64_t per_round = (uint64_t)kHashBlock * kHashIPT;
    // the trip count is the same for every thread of the workgroup
    for (uint64_t i0 = (uint64_t)blockIdx.x * per_round; i0 < n;
         i0 += (uint64_t)gridDim.x * per_round) {
        uint32_t h[kHashIPT], e[kHashIPT], local[kHashIPT];
#pragma unroll
        for (int u = 0; u < kHashIPT; ++u) {
            const uint64_t i = i0 + (uint64_t)u * kHashBlock + threadIdx.x;
            if (i >= n) continue;
            const uint32_t key = keys[i];
            const unsigned long long want = (unsigned long long)key + 1ull;
            uint32_t hh = dev::hash32(key) & mask;
            for (uint32_t probe = 0; probe <= mask; ++probe) {
                unsigned long long cur = slots[hh];
                if (cur == 0ull) cur = atomicCAS(&slots[hh], 0ull, want);
                if (cur == 0ull || cur == want) break;
                hh = (hh + 1) & mask;
            }
            uint32_t ee = hh & (kHashLds - 1);
            for (;;) {  // ends: fewer distinct slots per round than entries
                const uint32_t prev = atomicCAS(&s_slot[ee], kNoSlot, hh);
                if (prev == kNoSlot || prev == hh) break;
                ee = (ee + 1) & (kHashLds - 1);
            }
            h[u] = hh;
            e[u] = ee;
            local[u] = atomicAdd(&s_cnt[ee], 1u);
        }
        __syncthreads();
        // reserve each group's ranks and clear the entry for the next round
        for (int x = threadIdx.x; x < kHashLds; x += kHashBlock) {
            const uint32_t sl = s_slot[x];
            if (sl != kNoSlot) {
                s_base[x] = atomicAdd(&slot_count[sl], s_cnt[x]);
                s_slot[x] = kNoSlot;
                s_cnt[x] = 0;
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kHashIPT; ++u) {
            const uint64_t i = i0 + (uint64_t)u * kHashBlock + threadIdx.x;
            if (i >= n) continue;
            slot_of[i] = h[u];
            rank_of[i] = s_base[e[u]] + local[u];
        }
        // s_base is next written after the next round's first barrier
    }
}

__global__ void hash_fill(const uint32_t *slot_of, const uint32_t *rank_of, uint64_t n,
                          const uint64_t *slot_start, uint32_t *rows) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        rows[slot_start[slot_of[i]] + rank_of[i]] = (uint32_t)i;
}

__global__ void hash_probe(const uint32_t *keys, uint64_t n, const unsigned long long *slots,
                           uint32_t mask, const uint32_t *slot_count, const uint64_t *slot_start,
                           uint32_t *start, uint32_t *count) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const unsigned long long want = (unsigned long long)keys[i] + 1ull;
        uint32_t h = dev::hash32(keys[i]) & mask;
        uint32_t c = 0, s = 0;
        for (uint32_t probe = 0; probe <= mask; ++probe) {
            const unsigned long long cur = slots[h];
            if (cur == want) {
                c = slot_count[h];
                s = (uint32_t)slot_start[h];
                break;
            }
            if (cur == 0ull) break;
            h = (h + 1) & mask;
        }
        start[i] = s;
        count[i] = c;
    }
}

// ---------------------------------------------------------------------------
// expansion: output row o -> (probe position a, build position j)
// ---------------------------------------------------------------------------

struct ExpandArgs {
    const uint64_t *off;    // nq + 1 output offsets per probe position
    const uint32_t *start;  // per probe position: first matching build position
    const uint32_t *qrow;   // probe position -> probe table row (null: identity)
    const uint32_t *brow;   // build position -> build table row
    const uint32_t *matches;  // left outer join: true match count per probe position
    uint64_t nq, total;
    int probe_is_left;
    const uint32_t *lcol[TID_MAX_COLS];
    const uint32_t *rcol[TID_MAX_COLS];
    uint32_t *out[TID_MAX_COLS];
    int nl, nr;  // output columns taken from left rows, then from right rows
};

__global__ void join_expand(ExpandArgs a) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t o = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; o < a.total; o += stride) {
        // last probe position whose offset is <= o
        uint64_t lo = 0, hi = a.nq;
        while (hi - lo > 1) {
            const uint64_t mid = (lo + hi) >> 1;
            if (a.off[mid] <= o) lo = mid;
            else hi = mid;
        }
        const uint32_t pr = a.qrow ? a.qrow[lo] : (uint32_t)lo;
        if (a.matches && a.matches[lo] == 0) {  // a left row with no partner
            for (int c = 0; c < a.nl; ++c) a.out[c][o] = a.lcol[c][pr];
            for (int c = 0; c < a.nr; ++c) a.out[a.nl + c][o] = 0u;
            continue;
        }
        const uint64_t j = a.start[lo] + (o - a.off[lo]);
        const uint32_t br = a.brow[j];
        const uint32_t lr = a.probe_is_left ? pr : br;
        const uint32_t rr = a.probe_is_left ? br : pr;
        for (int c = 0; c < a.nl; ++c) a.out[c][o] = a.lcol[c][lr];
        for (int c = 0; c < a.nr; ++c) a.out[a.nl + c][o] = a.rcol[c][rr];
    }
}

__global__ void at_least_one(const uint32_t *in, uint64_t n, uint32_t *out) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = max(in[i], 1u);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

__global__ void widen_kernel(const uint32_t *in, uint64_t n, uint64_t *out) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = in[i];
}

void widen_u32(tid_ctx *ctx, const uint32_t *in, uint64_t n, uint64_t *out) {
    hipLaunchKernelGGL(widen_kernel, dim3(grid_of(n)), dim3(256), 0, ctx->stream, in, n, out);
    TID_HIP(hipGetLastError());
}


static int bitw(uint32_t v) { return v ? 32 - __builtin_clz(v) : 0; }
std::vector<uint32_t> column_maxima(tid_ctx *ctx, const tid_table *t, uint64_t n);

// Count the matches of L[lc] = R[rc] on the device (no synchronisation).
std::unique_ptr<PendingJoin> join_begin(tid_ctx *ctx, const tid_table *L, uint64_t nl, int lc,
                                        const tid_table *R, uint64_t nr, int rc, int algo,
                                        const JoinPlan &jp, int kind) {
    auto pj = std::make_unique<PendingJoin>();
    pj->L = L;
    pj->R = R;
    pj->lc = lc;
    pj->rc = rc;
    pj->jp = jp;
    for (int c : jp.lkeep) pj->vars.push_back(L->vars[c]);
    for (int c : jp.rkeep) pj->vars.push_back(R->vars[c]);
    TID_REQUIRE(pj->vars.size() <= TID_MAX_COLS, TID_E_SCHEMA, "join: too many output columns");
    TID_REQUIRE(kind == kJoinInner || kind == kJoinLeft, TID_E_INTERNAL, "join: bad kind");
    // an inner join with an empty side is empty; so is any join of an empty L
    if (nl == 0 || (nr == 0 && kind == kJoinInner)) {
        pj->total = 0;
        pj->total_known = true;
        return pj;
    }
    if (nr == 0) algo = 1;  // left join of L with nothing: every L row, padded
    TID_REQUIRE(nl < (1ull << 32) && nr < (1ull << 32), TID_E_UNSUPPORTED,
                "join: inputs of 2^32 rows or more");
    // automatic choice by size: a hash table over the smaller side while its
    // slot words and counts (12 B per slot, at least two slots per build row)
    // fit the 256 MB last-level cache, so probes mostly stay on chip;
    // sort-merge above that, where the sorts stream both sides through HBM
    // instead of probing it at random
    if (algo == 0) algo = std::min(nl, nr) <= kHashAutoMaxRows ? 1 : 2;
    if (algo == 2) {
        // sort both sides on the key, then find each left key's run on the right
        uint32_t ml, mr;
        if (L->maxv_known && R->maxv_known) {
            ml = L->maxv[lc];
            mr = R->maxv[rc];
        } else {
            ml = column_maxima(ctx, L, nl)[lc];
            mr = column_maxima(ctx, R, nr)[rc];
        }
        const int bits = bitw(std::max(ml, mr));
        auto sort_side = [&](const tid_table *T, uint64_t n, int col,
                             int slot) -> std::pair<uint64_t *, uint32_t *> {
            DevBuf &k = pj->keys[slot], &k2 = pj->keys[slot + 1];
            DevBuf &v = pj->vals[slot], &v2 = pj->vals[slot + 1];
            k = DevBuf(ctx, n * 8);
            v = DevBuf(ctx, n * 4);
            k2 = DevBuf(ctx, n * 8);
            v2 = DevBuf(ctx, n * 4);
            widen_u32(ctx, T->col[col], n, k.get<uint64_t>());  // key = value, 64 bits wide
            iota(ctx, v.get<uint32_t>(), n);
            const bool moved = radix_sort_pairs(ctx, k.get<uint64_t>(), v.get<uint32_t>(),
                                                k2.get<uint64_t>(), v2.get<uint32_t>(), n, bits);
            return moved ? std::make_pair(k2.get<uint64_t>(), v2.get<uint32_t>())
                         : std::make_pair(k.get<uint64_t>(), v.get<uint32_t>());
        };
        auto [lk, lv] = sort_side(L, nl, lc, 0);
        auto [rk, rv] = sort_side(R, nr, rc, 2);
        pj->nq = nl;
        pj->start = DevBuf(ctx, nl * 4);
        pj->count = DevBuf(ctx, nl * 4);
        hipLaunchKernelGGL(merge_counts, dim3(grid_of(nl)), dim3(256), 0, ctx->stream, lk, nl, rk,
                           nr, pj->start.get<uint32_t>(), pj->count.get<uint32_t>());
        TID_HIP(hipGetLastError());
        pj->qrow = lv;
        pj->brow = rv;
        pj->probe_is_left = 1;
    } else {
        // build on the smaller side; a left join probes with L
        const bool build_right = kind == kJoinLeft || nr <= nl;
        const tid_table *B = build_right ? R : L;
        const tid_table *Q = build_right ? L : R;
        const uint64_t nb = build_right ? nr : nl;
        const uint64_t nq = build_right ? nl : nr;
        const uint32_t *bkey = B->col[build_right ? rc : lc];
        const uint32_t *qkey = Q->col[build_right ? lc : rc];
        uint64_t cap = 1024;
        while (cap < 2 * nb) cap <<= 1;
        TID_REQUIRE(cap <= (1ull << 31), TID_E_UNSUPPORTED, "join: hash table too large");
        const uint32_t mask = (uint32_t)(cap - 1);
        // slot words (cap x 8 B) then slot counts (cap x 4 B): one clear
        pj->slots = DevBuf(ctx, cap * 12);
        unsigned long long *slots = pj->slots.get<unsigned long long>();
        uint32_t *slot_count = reinterpret_cast<uint32_t *>(slots + cap);
        pj->rank = DevBuf(ctx, nb * 4);
        pj->slot_of = DevBuf(ctx, nb * 4);
        pj->slot_start = DevBuf(ctx, (cap + 1) * 8);
        pj->rows = DevBuf(ctx, nb * 4);
        TID_HIP(hipMemsetAsync(slots, 0, cap * 12, ctx->stream));
        hipLaunchKernelGGL(hash_insert, dim3(grid_of(nb, kHashBlock * kHashIPT)),
                           dim3(kHashBlock), 0, ctx->stream, bkey, nb, slots, mask,
                           pj->slot_of.get<uint32_t>(), pj->rank.get<uint32_t>(), slot_count);
        TID_HIP(hipGetLastError());
        exclusive_scan_async(ctx, slot_count, cap, pj->slot_start.get<uint64_t>());
        hipLaunchKernelGGL(hash_fill, dim3(grid_of(nb)), dim3(256), 0, ctx->stream,
                           pj->slot_of.get<const uint32_t>(), pj->rank.get<const uint32_t>(), nb,
                           pj->slot_start.get<const uint64_t>(), pj->rows.get<uint32_t>());
        TID_HIP(hipGetLastError());
        pj->nq = nq;
        pj->start = DevBuf(ctx, nq * 4);
        pj->count = DevBuf(ctx, nq * 4);
        hipLaunchKernelGGL(hash_probe, dim3(grid_of(nq)), dim3(256), 0, ctx->stream, qkey, nq,
                           pj->slots.get<const unsigned long long>(), mask, slot_count,
                           pj->slot_start.get<const uint64_t>(), pj->start.get<uint32_t>(),
                           pj->count.get<uint32_t>());
        TID_HIP(hipGetLastError());
        pj->qrow = nullptr;
        pj->brow = pj->rows.get<uint32_t>();
        pj->probe_is_left = build_right ? 1 : 0;
    }
    if (kind == kJoinLeft) {
        // a probe row with no partner still takes one output row
        pj->outer = true;
        pj->matches = std::move(pj->count);
        pj->count = DevBuf(ctx, pj->nq * 4);
        hipLaunchKernelGGL(at_least_one, dim3(grid_of(pj->nq)), dim3(256), 0, ctx->stream,
                           pj->matches.get<const uint32_t>(), pj->nq, pj->count.get<uint32_t>());
        TID_HIP(hipGetLastError());
    }
    pj->off = DevBuf(ctx, (pj->nq + 1) * 8);
    exclusive_scan_async(ctx, pj->count.get<const uint32_t>(), pj->nq, pj->off.get<uint64_t>());
    return pj;
}

// Materialise a counted join once its output size is on the host.
std::unique_ptr<tid_table> join_finish(tid_ctx *ctx, PendingJoin &pj) {
    TID_REQUIRE(pj.total_known, TID_E_INTERNAL, "join: output size not read yet");
    const tid_table *L = pj.L, *R = pj.R;
    const uint64_t total = pj.total;
    auto out = make_table(ctx, (int)pj.vars.size(), pj.vars.data(), total);
    out->maxv_known = L->maxv_known && R->maxv_known;
    if (out->maxv_known) {
        copy_bounds(out.get(), L, pj.jp.lkeep.data(), (int)pj.jp.lkeep.size(), 0);
        copy_bounds(out.get(), R, pj.jp.rkeep.data(), (int)pj.jp.rkeep.size(),
                    (int)pj.jp.lkeep.size());
    }
    if (total) {
        TID_REQUIRE(total < (1ull << 40), TID_E_UNSUPPORTED, "join: output too large");
        ExpandArgs ea{};
        ea.off = pj.off.get<const uint64_t>();
        ea.start = pj.start.get<const uint32_t>();
        ea.qrow = pj.qrow;
        ea.brow = pj.brow;
        ea.matches = pj.outer ? pj.matches.get<const uint32_t>() : nullptr;
        ea.probe_is_left = pj.probe_is_left;
        ea.nq = pj.nq;
        ea.total = total;
        ea.nl = (int)pj.jp.lkeep.size();
        ea.nr = (int)pj.jp.rkeep.size();
        for (int c = 0; c < ea.nl; ++c) ea.lcol[c] = L->col[pj.jp.lkeep[c]];
        for (int c = 0; c < ea.nr; ++c) ea.rcol[c] = R->col[pj.jp.rkeep[c]];
        for (int c = 0; c < (int)pj.vars.size(); ++c) ea.out[c] = out->col[c];
        hipLaunchKernelGGL(join_expand, dim3(grid_of(total, 256, 16384)), dim3(256), 0,
                           ctx->stream, ea);
        TID_HIP(hipGetLastError());
    }
    set_count(ctx, out.get(), total);
    return out;
}

// Matches of L[lc] = R[rc] as an unsorted table of the columns lkeep of L
// followed by the columns rkeep of R.
std::unique_ptr<tid_table> join_unsorted(tid_ctx *ctx, const tid_table *L, uint64_t nl, int lc,
                                         const tid_table *R, uint64_t nr, int rc, int algo,
                                         const JoinPlan &jp, int kind = kJoinInner) {
    auto pj = join_begin(ctx, L, nl, lc, R, nr, rc, algo, jp, kind);
    if (!pj->total_known) {
        read_words(ctx, {pj->d_total()}, &pj->total);
        pj->total_known = true;
    }
    return join_finish(ctx, *pj);
}

// R rows whose key has no partner in L, as rows of the join's schema (L's
// columns, then R's without rc): L's cells 0 except lc, which takes the R
// row's key.  `matches` holds, per R row, its partner count.
struct UnmatchedSrc {
    const uint32_t *matches;
    const uint32_t *rkey;
    const uint32_t *rcol[TID_MAX_COLS];
    uint64_t n;
    int nl, lc;
    using Item = uint32_t;
    __device__ __forceinline__ Item load(uint64_t i) const { return matches[i]; }
    __device__ __forceinline__ bool match(int, Item m) const { return m == 0; }
    __device__ __forceinline__ uint32_t value(int, int c, Item, uint64_t i) const {
        return c < nl ? (c == lc ? rkey[i] : 0u) : rcol[c - nl][i];
    }
};

static std::unique_ptr<tid_table> unmatched_right(tid_ctx *ctx, const tid_table *l, uint64_t nl,
                                                  int lc, const tid_table *r, uint64_t nr,
                                                  int rc, const std::vector<int32_t> &vars) {
    // partner counts of R's rows: a left join of R against L probes R in
    // row order (hash join, built on L)
    JoinPlan none;
    auto pj = join_begin(ctx, r, nr, rc, l, nl, lc, 1, none, kJoinLeft);
    auto out = make_table(ctx, (int)vars.size(), vars.data(), nr);
    if (nr == 0) {
        set_count(ctx, out.get(), 0);
        return out;
    }
    UnmatchedSrc src{};
    src.matches = pj->matches.get<const uint32_t>();
    src.rkey = r->col[rc];
    int k = 0;
    for (int c = 0; c < r->ncols; ++c)
        if (c != rc) src.rcol[k++] = r->col[c];
    src.n = nr;
    src.nl = l->ncols;
    src.lc = lc;
    CompactArgs<1, TID_MAX_COLS> a{};
    for (int c = 0; c < out->ncols; ++c) a.out[0].col[c] = out->col[c];
    a.out[0].cap = out->cap;
    a.out[0].count = out->d_count;
    a.out[0].ncols = out->ncols;
    launch_compact<UnmatchedSrc, 256, 16, 1, TID_MAX_COLS>(ctx, src, a, 1, 16384u);
    return out;
}

// Outer joins (Sec. 4.2 kinds): rows in lexicographic order over L's columns
// then R's without rc; an unbound cell is 0.
std::unique_ptr<tid_table> join_tables_kind(tid_ctx *ctx, const tid_table *l, int lcol,
                                            const tid_table *r, int rcol, int kind, int algo) {
    TID_REQUIRE(lcol >= 0 && lcol < l->ncols && rcol >= 0 && rcol < r->ncols, TID_E_INVALID_ARG,
                "join: column out of range");
    TID_REQUIRE(l->ncols + r->ncols - 1 <= TID_MAX_COLS, TID_E_SCHEMA, "join: too many columns");
    TID_REQUIRE(kind >= kJoinInner && kind <= kJoinFull, TID_E_INVALID_ARG, "join: bad kind");
    tid_table *both[2] = {const_cast<tid_table *>(l), const_cast<tid_table *>(r)};
    resolve_counts(ctx, both, 2);
    JoinPlan jp;
    for (int c = 0; c < l->ncols; ++c) jp.lkeep.push_back(c);
    for (int c = 0; c < r->ncols; ++c)
        if (c != rcol) jp.rkeep.push_back(c);
    std::vector<int32_t> vars;
    for (int c : jp.lkeep) vars.push_back(l->vars[c]);
    for (int c : jp.rkeep) vars.push_back(r->vars[c]);
    std::unique_ptr<tid_table> raw;
    if (kind == kJoinRight) {
        // the left join of R with L, its columns put back in this join's order
        JoinPlan sw;
        for (int c = 0; c < r->ncols; ++c) sw.lkeep.push_back(c);
        for (int c = 0; c < l->ncols; ++c)
            if (c != lcol) sw.rkeep.push_back(c);
        auto t = join_unsorted(ctx, r, r->nrows, rcol, l, l->nrows, lcol, algo, sw, kJoinLeft);
        // position in t of each output column
        std::vector<int> from;
        for (int c = 0; c < l->ncols; ++c) {
            if (c == lcol) {
                from.push_back(rcol);
            } else {
                const int at = (int)(std::find(sw.rkeep.begin(), sw.rkeep.end(), c) -
                                     sw.rkeep.begin());
                from.push_back(r->ncols + at);
            }
        }
        for (int c : jp.rkeep) from.push_back(c);
        raw = std::make_unique<tid_table>();
        raw->ctx = ctx;
        raw->ncols = (int)from.size();
        raw->cap = t->cap;
        raw->nrows = t->nrows;
        raw->count_known = t->count_known;
        raw->d_count = t->d_count;
        raw->maxv_known = t->maxv_known;
        for (int c = 0; c < raw->ncols; ++c) {
            raw->vars[c] = vars[c];
            raw->col[c] = t->col[from[c]];
            raw->maxv[c] = t->maxv[from[c]];
        }
        raw->block = std::move(t->block);
    } else {
        raw = join_unsorted(ctx, l, l->nrows, lcol, r, r->nrows, rcol, algo, jp,
                            kind == kJoinInner ? kJoinInner : kJoinLeft);
        if (kind == kJoinFull) {
            auto un = unmatched_right(ctx, l, l->nrows, lcol, r, r->nrows, rcol, vars);
            if (raw->maxv_known) copy_bounds(un.get(), raw.get(), nullptr, raw->ncols);
            un->maxv_known = raw->maxv_known;
            // rows of both parts, one schema (which may name a variable twice,
            // so this is a plain concatenation, not a union over variables)
            tid_table *parts[2] = {raw.get(), un.get()};
            resolve_counts(ctx, parts, 2);
            auto both = make_table(ctx, raw->ncols, raw->vars, raw->nrows + un->nrows);
            both->maxv_known = raw->maxv_known;
            copy_bounds(both.get(), raw.get(), nullptr, raw->ncols);
            for (int c = 0; c < raw->ncols; ++c) {
                if (raw->nrows)
                    TID_HIP(hipMemcpyAsync(both->col[c], raw->col[c], raw->nrows * 4,
                                           hipMemcpyDeviceToDevice, ctx->stream));
                if (un->nrows)
                    TID_HIP(hipMemcpyAsync(both->col[c] + raw->nrows, un->col[c], un->nrows * 4,
                                           hipMemcpyDeviceToDevice, ctx->stream));
            }
            set_count(ctx, both.get(), raw->nrows + un->nrows);
            raw = std::move(both);
        }
    }
    tid_table *rp = raw.get();
    resolve_counts(ctx, &rp, 1);
    return sort_rows(ctx, raw.get(), raw->nrows, 0);
}

std::unique_ptr<tid_table> join_tables(tid_ctx *ctx, const tid_table *l, int lcol,
                                       const tid_table *r, int rcol, int algo) {
    TID_REQUIRE(lcol >= 0 && lcol < l->ncols && rcol >= 0 && rcol < r->ncols, TID_E_INVALID_ARG,
                "join: column out of range");
    TID_REQUIRE(l->ncols + r->ncols - 1 <= TID_MAX_COLS, TID_E_SCHEMA, "join: too many columns");
    tid_table *both[2] = {const_cast<tid_table *>(l), const_cast<tid_table *>(r)};
    resolve_counts(ctx, both, 2);
    JoinPlan jp;
    for (int c = 0; c < l->ncols; ++c) jp.lkeep.push_back(c);
    for (int c = 0; c < r->ncols; ++c)
        if (c != rcol) jp.rkeep.push_back(c);
    auto raw = join_unsorted(ctx, l, l->nrows, lcol, r, r->nrows, rcol, algo, jp);
    return sort_rows(ctx, raw.get(), raw->nrows, 0);
}

}  // namespace tid
