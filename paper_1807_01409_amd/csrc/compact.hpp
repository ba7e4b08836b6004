// compact.hpp -- order-preserving stream compaction in one pass over the
// input, shaped for MI355X.
//
// Why not a chained (look-back) scan: on MI355X each XCD has its own L2, so
// the tile-state words of a chained scan are read with device-scope loads that
// go out to memory; the prefix frontier then advances by one window of
// predecessors per memory round trip, which caps a 600 MB scan far below HBM
// speed.  Here the grid is sized to the resident capacity of the chip and each
// workgroup owns one contiguous range of the input:
//   phase 1  stream the range tile by tile, test every item, and stage the
//            compacted outputs of each pattern in LDS (in item order);
//   prefix   publish the range's match count, then read the counts of all
//            earlier ranges at once (one memory round trip, not a chain);
//   phase 2  copy the staged rows to their final place with coalesced
//            stores; if a pattern's staging area filled up, re-read the rest
//            of the range from the first unstaged tile and write directly.
// Workgroups take their range index from an atomic counter, so a workgroup
// only ever waits on ranges handed out before its own, whose workgroups are
// already running: every wait ends.  The workgroup that finishes last clears
// the sync words for the next launch.
#pragma once

#include "device_common.hpp"
#include "internal.hpp"

#include <algorithm>

namespace tid {

template <int MAXC>
struct OutDesc {
    uint32_t *col[MAXC];
    uint64_t cap;        // rows allocated in the output columns
    uint64_t *count;     // device row count, written by the last range
    int32_t ncols;
    uint32_t stage_off;  // first LDS word of this output's staging area
    uint32_t stage_cap;  // rows its staging area holds
};

template <int MAXK, int MAXC>
struct CompactArgs {
    OutDesc<MAXC> out[MAXK];
    int32_t k;
    uint32_t P;       // number of ranges (= workgroups)
    uint64_t range;   // items per range, a multiple of the tile
};

constexpr uint64_t kNoTile = ~0ull;
constexpr uint64_t kPublished = 1ull << 63;
constexpr uint32_t kSpinLimit = 1u << 22;
constexpr int kPrefixPer = 8;  // ranges per thread in the prefix read: P <= BLOCK * 8

namespace dev {

// Load one tile of items (striped: item `it` of thread `tid` is
// t0 + it*BLOCK + tid), test them, and leave per-(item, wave) match counts of
// every pattern in s_off.  Returns the match bits in mb.
template <class Src, int BLOCK, int IPT>
__device__ __forceinline__ void tile_load(const Src &src, uint64_t t0, uint64_t r1,
                                          typename Src::Item *item) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int it = 0; it < IPT; ++it) {
        const uint64_t i = t0 + (uint64_t)it * BLOCK + tid;
        item[it] = i < r1 ? src.load(i) : typename Src::Item{};
    }
}

// Test a loaded tile and leave the per-(item, wave) match counts in s_off.
template <class Src, int BLOCK, int IPT, int MAXK>
__device__ __forceinline__ void tile_test(const Src &src, int k, uint64_t t0, uint64_t r1,
                                          const typename Src::Item *item, uint32_t *mb,
                                          uint32_t (*s_off)[IPT * (BLOCK / kWave)]) {
    constexpr int NW = BLOCK / kWave;
    const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
#pragma unroll
    for (int j = 0; j < MAXK; ++j) mb[j] = 0;
#pragma unroll
    for (int it = 0; it < IPT; ++it) {
        const bool valid = t0 + (uint64_t)it * BLOCK + tid < r1;
#pragma unroll
        for (int j = 0; j < MAXK; ++j)
            if (j < k && valid && src.match(j, item[it])) mb[j] |= 1u << it;
    }
#pragma unroll
    for (int j = 0; j < MAXK; ++j) {
        if (j >= k) break;
#pragma unroll
        for (int it = 0; it < IPT; ++it) {
            const uint64_t b = ballot((mb[j] >> it) & 1u);
            if (lane == 0) s_off[j][it * NW + wave] = (uint32_t)__popcll(b);
        }
    }
}

template <class Src, int BLOCK, int IPT, int MAXK>
__device__ __forceinline__ void tile_matches(const Src &src, int k, uint64_t t0, uint64_t r1,
                                             typename Src::Item *item, uint32_t *mb,
                                             uint32_t (*s_off)[IPT * (BLOCK / kWave)]) {
    tile_load<Src, BLOCK, IPT>(src, t0, r1, item);
    tile_test<Src, BLOCK, IPT, MAXK>(src, k, t0, r1, item, mb, s_off);
}

// exclusive offsets (in item order) of NV counts, in place; returns the total
template <int NV>
__device__ __forceinline__ uint32_t offsets_in_place(uint32_t *s) {
    constexpr int V = (NV + kWave - 1) / kWave;
    const int lane = lane_id();
    uint32_t vals[V];
    uint32_t local = 0;
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const int idx = lane * V + v;
        vals[v] = idx < NV ? s[idx] : 0u;
        local += vals[v];
    }
    const uint32_t incl = wave_inclusive_sum(local);
    uint32_t run = incl - local;
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const int idx = lane * V + v;
        if (idx < NV) s[idx] = run;
        run += vals[v];
    }
    return __shfl(incl, kWave - 1, kWave);
}

}  // namespace dev

template <class Src, int BLOCK, int IPT, int MAXK, int MAXC, bool PREFETCH = false>
__global__ __launch_bounds__(BLOCK) void compact_kernel(Src src, CompactArgs<MAXK, MAXC> a,
                                                         uint64_t *sync, uint32_t *flags) {
    constexpr int NW = BLOCK / dev::kWave;
    constexpr int NV = IPT * NW;
    constexpr uint64_t TILE = (uint64_t)BLOCK * IPT;
    static_assert(IPT <= 32, "match bits live in one 32-bit word per pattern");
    extern __shared__ uint32_t stage[];
    __shared__ uint32_t s_off[MAXK][NV];
    __shared__ uint32_t s_tot[MAXK];
    __shared__ uint64_t s_cnt[MAXK], s_staged[MAXK], s_ovf[MAXK], s_pre[MAXK], s_run[MAXK];
    __shared__ uint64_t s_red[MAXK][NW];
    __shared__ uint32_t s_wg;

    const int tid = threadIdx.x, wave = tid / dev::kWave, lane = tid % dev::kWave;
    const int k = MAXK == 1 ? 1 : a.k;
    const uint32_t P = a.P;
    uint32_t *counters = reinterpret_cast<uint32_t *>(sync + (size_t)k * P);
    if (tid == 0) s_wg = atomicAdd(&counters[0], 1u);
    if (tid < k) {
        s_cnt[tid] = 0;
        s_staged[tid] = 0;
        s_ovf[tid] = kNoTile;
    }
    __syncthreads();
    const uint32_t wg = s_wg;
    const uint64_t r0 = (uint64_t)wg * a.range;
    const uint64_t r1 = min(src.n, r0 + a.range);

    typename Src::Item item[IPT];
    typename Src::Item next[PREFETCH ? IPT : 1];
    uint32_t mb[MAXK];

    // ---- phase 1: test the range, stage compacted outputs in LDS ----------
    // With PREFETCH the loads of tile t+1 are issued before tile t is tested,
    // so the workgroup keeps memory busy through its barriers.
    if (PREFETCH && r0 < r1) dev::tile_load<Src, BLOCK, IPT>(src, r0, r1, next);
    for (uint64_t t0 = r0; t0 < r1; t0 += TILE) {
        if (PREFETCH) {
#pragma unroll
            for (int it = 0; it < IPT; ++it) item[it] = next[PREFETCH ? it : 0];
            if (t0 + TILE < r1) dev::tile_load<Src, BLOCK, IPT>(src, t0 + TILE, r1, next);
            dev::tile_test<Src, BLOCK, IPT, MAXK>(src, k, t0, r1, item, mb, s_off);
        } else {
            dev::tile_matches<Src, BLOCK, IPT, MAXK>(src, k, t0, r1, item, mb, s_off);
        }
        __syncthreads();
        for (int j = wave; j < k; j += NW) {
            const uint32_t tot = dev::offsets_in_place<NV>(s_off[j]);
            if (lane == 0) s_tot[j] = tot;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < MAXK; ++j) {
            if (j >= k) break;
            const OutDesc<MAXC> &o = a.out[j];
            const uint64_t cnt = s_cnt[j];
            if (s_ovf[j] != kNoTile || cnt + s_tot[j] > o.stage_cap) continue;
#pragma unroll
            for (int it = 0; it < IPT; ++it) {
                const bool bit = (mb[j] >> it) & 1u;
                const uint64_t b = dev::ballot(bit);
                if (bit) {
                    const uint32_t r =
                        (uint32_t)cnt + s_off[j][it * NW + wave] + dev::rank_in_mask(b);
                    const uint64_t i = t0 + (uint64_t)it * BLOCK + tid;
                    for (int c = 0; c < o.ncols; ++c)
                        stage[o.stage_off + (uint32_t)c * o.stage_cap + r] =
                            src.value(j, c, item[it], i);
                }
            }
        }
        __syncthreads();
        if (tid < k) {
            if (s_ovf[tid] == kNoTile && s_cnt[tid] + s_tot[tid] > a.out[tid].stage_cap) {
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
        dev::publish(&sync[(size_t)tid * P + wg], kPublished | s_cnt[tid]);
    }
    // all predecessor counts are requested at once (kPrefixPer per thread),
    // then any not yet published are polled again
    for (int j = 0; j < k; ++j) {
        uint64_t w[kPrefixPer];
#pragma unroll
        for (int u = 0; u < kPrefixPer; ++u) {
            const uint32_t i = tid + u * BLOCK;
            w[u] = i < wg ? dev::peek(&sync[(size_t)j * P + i]) : kPublished;
        }
        uint64_t part = 0;
#pragma unroll
        for (int u = 0; u < kPrefixPer; ++u) {
            const uint32_t i = tid + u * BLOCK;
            uint32_t spins = 0;
            while (!(w[u] & kPublished)) {
                if (++spins > kSpinLimit) {
                    atomicOr(&flags[0], 1u);
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
                w[u] = dev::peek(&sync[(size_t)j * P + i]);
            }
            part += w[u] & ~kPublished;
        }
        part = dev::wave_sum(part);
        if (lane == 0) s_red[j][wave] = part;
    }
    __syncthreads();
    if (tid < k) {
        uint64_t s = 0;
        for (int w = 0; w < NW; ++w) s += s_red[tid][w];
        s_pre[tid] = s;
        s_run[tid] = s_staged[tid];
    }
    __syncthreads();

    // ---- phase 2: write staged rows, re-read what did not fit --------------
    for (int j = 0; j < k; ++j) {
        const OutDesc<MAXC> &o = a.out[j];
        if (o.ncols == 0) continue;
        const uint64_t pre = s_pre[j];
        const uint32_t st = (uint32_t)s_staged[j];
        for (uint32_t r = tid; r < st; r += BLOCK) {
            const uint64_t dst = pre + r;
            if (dst < o.cap) {
                for (int c = 0; c < o.ncols; ++c)
                    o.col[c][dst] = stage[o.stage_off + (uint32_t)c * o.stage_cap + r];
            } else {
                atomicOr(&flags[1], 1u);
            }
        }
    }
    uint64_t first = kNoTile;
    for (int j = 0; j < k; ++j) first = min(first, s_ovf[j]);
    for (uint64_t t0 = first; t0 < r1; t0 += TILE) {
        dev::tile_matches<Src, BLOCK, IPT, MAXK>(src, k, t0, r1, item, mb, s_off);
        __syncthreads();
        for (int j = wave; j < k; j += NW) {
            const uint32_t tot = dev::offsets_in_place<NV>(s_off[j]);
            if (lane == 0) s_tot[j] = tot;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < MAXK; ++j) {
            if (j >= k) break;
            if (s_ovf[j] > t0) continue;
            const OutDesc<MAXC> &o = a.out[j];
            const uint64_t base = s_pre[j] + s_run[j];
#pragma unroll
            for (int it = 0; it < IPT; ++it) {
                const bool bit = (mb[j] >> it) & 1u;
                const uint64_t b = dev::ballot(bit);
                if (bit) {
                    const uint64_t dst = base + s_off[j][it * NW + wave] + dev::rank_in_mask(b);
                    const uint64_t i = t0 + (uint64_t)it * BLOCK + tid;
                    if (dst < o.cap) {
                        for (int c = 0; c < o.ncols; ++c) o.col[c][dst] = src.value(j, c, item[it], i);
                    } else {
                        atomicOr(&flags[1], 1u);
                    }
                }
            }
        }
        __syncthreads();
        if (tid < k && s_ovf[tid] <= t0) s_run[tid] += s_tot[tid];
    }
    if (wg == P - 1 && tid < k) *a.out[tid].count = s_pre[tid] + s_cnt[tid];
    dev::release_state(sync, (size_t)k * P, counters, P);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

int device_cus(tid_ctx *ctx);
// Workgroups of `kernel` (BLOCK threads, `lds` dynamic LDS bytes) resident per
// CU; cached per (kernel, lds) and safe to call from several host threads.
int resident_blocks(const void *kernel, int block, size_t lds);

// Launch the compaction of `n` items over the resident-capacity grid.  The
// caller fills a.out[0..k) (columns, caps, counts, ncols); staging areas are
// laid out here over `stage_words` words of LDS.
template <class Src, int BLOCK, int IPT, int MAXK, int MAXC, bool PREFETCH = false>
void launch_compact(tid_ctx *ctx, const Src &src, CompactArgs<MAXK, MAXC> &a, int k,
                    uint32_t stage_words) {
    constexpr uint64_t TILE = (uint64_t)BLOCK * IPT;
    auto kern = compact_kernel<Src, BLOCK, IPT, MAXK, MAXC, PREFETCH>;
    const size_t lds = (size_t)stage_words * sizeof(uint32_t);
    const int blocks_per_cu = resident_blocks((const void *)kern, BLOCK, lds);
    const uint64_t n = src.n;
    if (n == 0) return;
    uint64_t cols_total = 0;
    for (int j = 0; j < k; ++j) cols_total += (uint64_t)a.out[j].ncols;
    const uint32_t rows_per = (uint32_t)(stage_words / std::max<uint64_t>(cols_total, 1));
    uint32_t off = 0;
    for (int j = 0; j < k; ++j) {
        a.out[j].stage_off = off;
        a.out[j].stage_cap = a.out[j].ncols ? rows_per : 0xFFFFFFFFu;
        off += rows_per * (uint32_t)a.out[j].ncols;
    }
    const uint64_t tiles = (n + TILE - 1) / TILE;
    const uint64_t resident = (uint64_t)blocks_per_cu * (uint64_t)device_cus(ctx);
    uint64_t P = std::max<uint64_t>(1, std::min({tiles, resident, (uint64_t)BLOCK * kPrefixPer}));
    const uint64_t range = (tiles + P - 1) / P * TILE;
    P = (n + range - 1) / range;
    TID_REQUIRE(P < (1ull << 31), TID_E_UNSUPPORTED, "compaction: input too large");
    a.k = k;
    a.P = (uint32_t)P;
    a.range = range;
    uint64_t *sync =
        static_cast<uint64_t *>(ctx->lookback_state(((size_t)k * P + 1) * sizeof(uint64_t)));
    hipLaunchKernelGGL(kern, dim3((uint32_t)P), dim3(BLOCK), lds, ctx->stream, src, a, sync,
                       ctx->d_flags);
    TID_HIP(hipGetLastError());
}

}  // namespace tid
