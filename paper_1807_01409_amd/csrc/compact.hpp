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
// already running: every wait ends.  Range counts carry the launch's epoch
// stamp, so they need no clearing, and the workgroup that finishes last
// resets the ticket and done counters with relaxed atomics: no release fence,
// which on MI355X would write back the XCD's L2 once per workgroup.
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
    uint32_t P;          // number of ranges (= workgroups)
    uint64_t range;      // block-ranged kernel: items per range, a multiple of the tile
    // chunked kernel: chunk t < q_big holds big_tiles tiles, later chunks one
    // tile; q chunks in all; two staging buffers of buf_words LDS words
    uint64_t q_big, q;
    uint32_t big_tiles;
    uint32_t buf_words;
    uint32_t epoch;      // stamp of this launch's count slots
};

constexpr uint64_t kNoTile = ~0ull;
constexpr uint32_t kSpinLimit = 1u << 22;
constexpr int kPrefixPer = 8;  // ranges per thread in the prefix read: P <= BLOCK * 8
constexpr int kEpochShift = 40;                  // count slot: epoch << 40 | rows
constexpr uint64_t kRowsMask = (1ull << kEpochShift) - 1;

namespace dev {

// Load one tile of items (striped: item `it` of thread `tid` is
// t0 + it*BLOCK + tid); items past r1 are left empty.
template <class Src, int BLOCK, int IPT>
__device__ __forceinline__ void tile_load(const Src &src, uint64_t t0, uint64_t r1,
                                          typename Src::Item *item) {
    const int tid = threadIdx.x;
    if (t0 + (uint64_t)BLOCK * IPT <= r1) {  // a whole tile: no bounds tests
#pragma unroll
        for (int it = 0; it < IPT; ++it) item[it] = src.load(t0 + (uint64_t)it * BLOCK + tid);
        return;
    }
#pragma unroll
    for (int it = 0; it < IPT; ++it) {
        const uint64_t i = t0 + (uint64_t)it * BLOCK + tid;
        item[it] = i < r1 ? src.load(i) : typename Src::Item{};
    }
}

// Test a loaded tile: bal[j][it] is the wave's match mask of pattern j for
// item `it` (a ballot, so lane l matched iff bit l is set), and the
// per-(item, wave) match counts go to s_off.
template <class Src, int BLOCK, int IPT, int MAXK>
__device__ __forceinline__ void tile_test(const Src &src, int k, uint64_t t0, uint64_t r1,
                                          const typename Src::Item *item, uint64_t (*bal)[IPT],
                                          uint32_t (*s_off)[IPT * (BLOCK / kWave)]) {
    constexpr int NW = BLOCK / kWave;
    const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
    if (t0 + (uint64_t)BLOCK * IPT <= r1) {  // a whole tile: every item is valid
#pragma unroll
        for (int it = 0; it < IPT; ++it) {
#pragma unroll
            for (int j = 0; j < MAXK; ++j)
                bal[j][it] = j < k ? ballot(src.match(j, item[it])) : 0ull;
        }
    } else {
#pragma unroll
        for (int it = 0; it < IPT; ++it) {
            const bool valid = t0 + (uint64_t)it * BLOCK + tid < r1;
#pragma unroll
            for (int j = 0; j < MAXK; ++j)
                bal[j][it] = j < k ? ballot(valid && src.match(j, item[it])) : 0ull;
        }
    }
#pragma unroll
    for (int j = 0; j < MAXK; ++j) {
        if (j >= k) break;
#pragma unroll
        for (int it = 0; it < IPT; ++it)
            if (lane == 0) s_off[j][it * NW + wave] = (uint32_t)__popcll(bal[j][it]);
    }
}

template <class Src, int BLOCK, int IPT, int MAXK>
__device__ __forceinline__ void tile_matches(const Src &src, int k, uint64_t t0, uint64_t r1,
                                             typename Src::Item *item, uint64_t (*bal)[IPT],
                                             uint32_t (*s_off)[IPT * (BLOCK / kWave)]) {
    tile_load<Src, BLOCK, IPT>(src, t0, r1, item);
    tile_test<Src, BLOCK, IPT, MAXK>(src, k, t0, r1, item, bal, s_off);
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
                                                         uint64_t *sync, uint32_t *counters,
                                                         uint32_t *flags) {
    constexpr int NW = BLOCK / dev::kWave;
    constexpr int NV = IPT * NW;
    constexpr uint64_t TILE = (uint64_t)BLOCK * IPT;
    extern __shared__ uint32_t stage[];
    __shared__ uint32_t s_off[MAXK][NV];
    __shared__ uint32_t s_tot[MAXK];
    __shared__ uint64_t s_cnt[MAXK], s_staged[MAXK], s_ovf[MAXK], s_pre[MAXK], s_run[MAXK];
    __shared__ uint64_t s_red[MAXK][NW];
    __shared__ uint32_t s_wg;

    const int tid = threadIdx.x, wave = tid / dev::kWave, lane = tid % dev::kWave;
    const int k = MAXK == 1 ? 1 : a.k;
    const uint32_t P = a.P;
    const uint64_t stamp = (uint64_t)a.epoch << kEpochShift;
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
    uint64_t bal[MAXK][IPT];  // match masks of the tile being placed

    // ---- phase 1: test the range, stage compacted outputs in LDS ----------
    // With PREFETCH the loads of tile t+1 are issued before tile t is tested,
    // so the workgroup keeps memory busy through its barriers.
    if (PREFETCH && r0 < r1) dev::tile_load<Src, BLOCK, IPT>(src, r0, r1, next);
    for (uint64_t t0 = r0; t0 < r1; t0 += TILE) {
        if (PREFETCH) {
#pragma unroll
            for (int it = 0; it < IPT; ++it) item[it] = next[PREFETCH ? it : 0];
            if (t0 + TILE < r1) dev::tile_load<Src, BLOCK, IPT>(src, t0 + TILE, r1, next);
            dev::tile_test<Src, BLOCK, IPT, MAXK>(src, k, t0, r1, item, bal, s_off);
        } else {
            dev::tile_matches<Src, BLOCK, IPT, MAXK>(src, k, t0, r1, item, bal, s_off);
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
                const uint64_t b = bal[j][it];
                const bool bit = (b >> lane) & 1u;
                if (bit) {
                    const uint32_t r =
                        (uint32_t)cnt + s_off[j][it * NW + wave] + dev::rank_in_mask(b);
                    const uint64_t i = t0 + (uint64_t)it * BLOCK + tid;
                    TID_FOR_COLS(MAXC, c, o.ncols)
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
        dev::publish(&sync[(size_t)tid * P + wg], stamp | s_cnt[tid]);
    }
    // all predecessor counts are requested at once (kPrefixPer per thread),
    // then any not yet published are polled again
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
        // thread slots start at the 32-row (128-byte) boundary below pre, so
        // each wave's stores cover whole cache lines
        const uint32_t lead = (uint32_t)(pre & 31u);
        for (uint32_t x = tid; x < st + lead; x += BLOCK) {
            if (x < lead) continue;
            const uint32_t r = x - lead;
            const uint64_t dst = pre + r;
            if (dst < o.cap) {
                TID_FOR_COLS(MAXC, c, o.ncols)
                    dev::put(&o.col[c][dst], stage[o.stage_off + (uint32_t)c * o.stage_cap + r]);
            } else {
                atomicOr(&flags[1], 1u);
            }
        }
    }
    uint64_t first = kNoTile;
    for (int j = 0; j < k; ++j) first = min(first, s_ovf[j]);
    for (uint64_t t0 = first; t0 < r1; t0 += TILE) {
        dev::tile_matches<Src, BLOCK, IPT, MAXK>(src, k, t0, r1, item, bal, s_off);
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
                const uint64_t b = bal[j][it];
                const bool bit = (b >> lane) & 1u;
                if (bit) {
                    const uint64_t dst = base + s_off[j][it * NW + wave] + dev::rank_in_mask(b);
                    const uint64_t i = t0 + (uint64_t)it * BLOCK + tid;
                    if (dst < o.cap) {
                        TID_FOR_COLS(MAXC, c, o.ncols)
                            dev::put(&o.col[c][dst], src.value(j, c, item[it], i));
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
    // the last workgroup out resets the ticket and done counters (the count
    // words carry this launch's epoch and need no clearing)
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
// Chunked compaction with dynamic work distribution.  The input is cut into
// q chunks (big ones first, single tiles at the end so the tail is short);
// workgroups take chunks from an atomic ticket, in input order.  A workgroup
// streams its chunk tile by tile, staging the compacted rows in one of two LDS
// buffers, publishes the chunk's row count (publishing never waits, so every
// wait below ends), and then places its PREVIOUS chunk: by that time the chunks before it have been counted by their owners,
// so the offset (the sum of the counts between the workgroup's frontier and
// that chunk) is read in one round trip with little or no waiting, and the
// rows are written while the chunk just streamed waits its turn.  Fast
// workgroups simply take more chunks, so the kernel ends when the bytes are
// read, not when the slowest fixed share is.  Rows past a full staging buffer
// are found again by re-reading the rest of their chunk when it is placed.
//
// Chunks are handed out by one counter in increasing order and only to
// running workgroups, and each workgroup's chunks increase, so a workgroup
// never waits for a chunk that is not handed out or that a waiting workgroup
// holds: every wait ends.  Count slots carry the launch's epoch in their upper
// bits, so they never need clearing; the ticket and done counters are touched
// only by atomics whose results are consumed, and the last workgroup resets
// them without a cache write-back.
// ---------------------------------------------------------------------------
namespace dev {
template <class A>
__device__ __forceinline__ void chunk_bounds(const A &a, uint64_t t, uint64_t n,
                                             uint64_t tile, uint64_t &c0, uint64_t &c1) {
    const uint64_t big = tile * a.big_tiles;
    c0 = t < a.q_big ? t * big : a.q_big * big + (t - a.q_big) * tile;
    c1 = min(n, c0 + (t < a.q_big ? big : tile));
}
}  // namespace dev

template <class Src, int BLOCK, int IPT, int MAXK, int MAXC>
__global__ __launch_bounds__(BLOCK) void chunk_compact_kernel(Src src, CompactArgs<MAXK, MAXC> a,
                                                               uint64_t *slots, uint32_t *counters,
                                                               uint32_t *flags) {
    constexpr int NW = BLOCK / dev::kWave;
    constexpr int NV = IPT * NW;
    constexpr uint64_t TILE = (uint64_t)BLOCK * IPT;
    extern __shared__ uint32_t stage[];
    __shared__ uint32_t s_off[MAXK][NV];
    __shared__ uint32_t s_tot[MAXK];
    __shared__ uint64_t s_cnt[MAXK], s_stg[MAXK], s_ovf[MAXK];     // chunk being streamed
    __shared__ uint64_t s_pcnt[MAXK], s_pstg[MAXK], s_povf[MAXK];  // chunk waiting for placement
    __shared__ uint64_t s_fsum[MAXK];  // rows of all chunks before s_front
    __shared__ uint64_t s_pre[MAXK], s_run[MAXK];
    __shared__ uint64_t s_red[MAXK][NW];
    __shared__ uint64_t s_tk, s_front, s_pend;

    const int tid = threadIdx.x, wave = tid / dev::kWave, lane = tid % dev::kWave;
    const int k = MAXK == 1 ? 1 : a.k;
    const uint64_t Q = a.q;
    const uint64_t stamp = (uint64_t)a.epoch << kEpochShift;
    constexpr uint64_t kNone = ~0ull;

    if (tid == 0) {
        s_tk = atomicAdd(&counters[0], 1u);
        s_front = 0;
        s_pend = kNone;
    }
    if (tid < k) s_fsum[tid] = 0;
    __syncthreads();

    typename Src::Item item[IPT], next[IPT];
    uint64_t bal[MAXK][IPT];  // match masks of the tile being placed

    // Count slots are chunk-major (the k counts of chunk i at slots[i*k ..]),
    // so one round trip fetches every output's counts of a window of
    // kSlotsPer * BLOCK chunks.  The first window between the frontier and
    // the pending chunk is requested before the next tile's loads, so that
    // reading it does not wait for that tile.
    constexpr int kSlotsPer = MAXK == 1 ? 2 : 1;
    auto request_slots = [&](uint64_t (*w)[kSlotsPer]) {
        const uint64_t p = s_pend, f = s_front;
#pragma unroll
        for (int u = 0; u < kSlotsPer; ++u) {
            const uint64_t i = f + tid + (uint64_t)u * BLOCK;
#pragma unroll
            for (int j = 0; j < MAXK; ++j)
                if (j < k) w[j][u] = i < p ? dev::peek(&slots[i * k + j]) : stamp;
        }
    };
    // Place the pending chunk (staged in buffer `pb`): offset from the count
    // slots, staged rows out, overflow re-read, frontier advanced.
    auto place = [&](const uint32_t *pb, uint64_t (*w)[kSlotsPer]) {
        const uint64_t p = s_pend, f = s_front;
        uint64_t c0, c1;
        dev::chunk_bounds(a, p, src.n, TILE, c0, c1);
        uint64_t part[MAXK];
#pragma unroll
        for (int j = 0; j < MAXK; ++j) part[j] = 0;
        for (uint64_t base = f; base < p; base += (uint64_t)BLOCK * kSlotsPer) {
            if (base != f) {
#pragma unroll
                for (int u = 0; u < kSlotsPer; ++u) {
                    const uint64_t i = base + tid + (uint64_t)u * BLOCK;
#pragma unroll
                    for (int j = 0; j < MAXK; ++j)
                        if (j < k) w[j][u] = i < p ? dev::peek(&slots[i * k + j]) : stamp;
                }
            }
#pragma unroll
            for (int u = 0; u < kSlotsPer; ++u) {
                const uint64_t i = base + tid + (uint64_t)u * BLOCK;
#pragma unroll
                for (int j = 0; j < MAXK; ++j) {
                    if (j >= k) break;
                    uint32_t spins = 0;
                    while ((w[j][u] >> kEpochShift) != a.epoch) {
                        if (++spins > kSpinLimit) {
                            atomicOr(&flags[0], 1u);
                            break;
                        }
                        __builtin_amdgcn_s_sleep(2);
                        w[j][u] = dev::peek(&slots[i * k + j]);
                    }
                    part[j] += w[j][u] & kRowsMask;
                }
            }
        }
#pragma unroll
        for (int j = 0; j < MAXK; ++j) {
            if (j >= k) break;
            const uint64_t v = dev::wave_sum(part[j]);
            if (lane == 0) s_red[j][wave] = v;
        }
        __syncthreads();
        if (tid < k) {
            uint64_t s = s_fsum[tid];
            for (int w = 0; w < NW; ++w) s += s_red[tid][w];
            s_pre[tid] = s;
            s_run[tid] = s_pstg[tid];
        }
        __syncthreads();
        for (int j = 0; j < k; ++j) {
            const OutDesc<MAXC> &o = a.out[j];
            if (o.ncols == 0) continue;
            const uint64_t pre = s_pre[j];
            const uint32_t stg = (uint32_t)s_pstg[j];
            // from the 32-row boundary below pre: whole cache lines per wave
            const uint32_t lead = (uint32_t)(pre & 31u);
            for (uint32_t x = tid; x < stg + lead; x += BLOCK) {
                if (x < lead) continue;
                const uint32_t r = x - lead;
                const uint64_t dst = pre + r;
                if (dst < o.cap) {
                    TID_FOR_COLS(MAXC, c, o.ncols)
                        dev::put(&o.col[c][dst], pb[o.stage_off + (uint32_t)c * o.stage_cap + r]);
                } else {
                    atomicOr(&flags[1], 1u);
                }
            }
        }
        uint64_t first = kNoTile;
        for (int j = 0; j < k; ++j) first = min(first, s_povf[j]);
        for (uint64_t t0 = first; t0 < c1; t0 += TILE) {
            dev::tile_matches<Src, BLOCK, IPT, MAXK>(src, k, t0, c1, item, bal, s_off);
            __syncthreads();
            for (int j = wave; j < k; j += NW) {
                const uint32_t tot = dev::offsets_in_place<NV>(s_off[j]);
                if (lane == 0) s_tot[j] = tot;
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < MAXK; ++j) {
                if (j >= k) break;
                if (s_povf[j] > t0) continue;
                const OutDesc<MAXC> &o = a.out[j];
                const uint64_t base = s_pre[j] + s_run[j];
#pragma unroll
                for (int it = 0; it < IPT; ++it) {
                    const uint64_t b = bal[j][it];
                    const bool bit = (b >> lane) & 1u;
                    if (bit) {
                        const uint64_t dst =
                            base + s_off[j][it * NW + wave] + dev::rank_in_mask(b);
                        const uint64_t i = t0 + (uint64_t)it * BLOCK + tid;
                        if (dst < o.cap) {
                            TID_FOR_COLS(MAXC, c, o.ncols)
                                dev::put(&o.col[c][dst], src.value(j, c, item[it], i));
                        } else {
                            atomicOr(&flags[1], 1u);
                        }
                    }
                }
            }
            __syncthreads();
            if (tid < k && s_povf[tid] <= t0) s_run[tid] += s_tot[tid];
        }
        if (tid < k) {
            s_fsum[tid] = s_pre[tid] + s_pcnt[tid];
            if (p == Q - 1) *a.out[tid].count = s_pre[tid] + s_pcnt[tid];
        }
        if (tid == 0) s_front = p + 1;
        __syncthreads();
    };

    // The next chunk's ticket is taken while the last tile of the current one
    // is tested (its result is not waited for until the tile is done), and its
    // first tile is loaded before the previous chunk is placed, so the
    // placement round trip overlaps loads in flight.
    int buf = 0;
    uint32_t ticket = 0;
    if (s_tk < Q) {
        uint64_t c0, c1;
        dev::chunk_bounds(a, s_tk, src.n, TILE, c0, c1);
        dev::tile_load<Src, BLOCK, IPT>(src, c0, c1, next);
    }
    for (;;) {
        const uint64_t t = s_tk;
        if (t >= Q) break;
        uint64_t c0, c1;
        dev::chunk_bounds(a, t, src.n, TILE, c0, c1);
        uint32_t *st = stage + (uint32_t)buf * a.buf_words;
        if (tid < k) {
            s_cnt[tid] = 0;
            s_stg[tid] = 0;
            s_ovf[tid] = kNoTile;
        }
        __syncthreads();
        for (uint64_t t0 = c0; t0 < c1; t0 += TILE) {
#pragma unroll
            for (int it = 0; it < IPT; ++it) item[it] = next[it];
            if (t0 + TILE < c1)
                dev::tile_load<Src, BLOCK, IPT>(src, t0 + TILE, c1, next);
            else if (tid == 0)
                ticket = atomicAdd(&counters[0], 1u);  // result first used after the loop
            dev::tile_test<Src, BLOCK, IPT, MAXK>(src, k, t0, c1, item, bal, s_off);
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
                    const uint64_t b = bal[j][it];
                    const bool bit = (b >> lane) & 1u;
                    if (bit) {
                        const uint32_t r =
                            (uint32_t)cnt + s_off[j][it * NW + wave] + dev::rank_in_mask(b);
                        const uint64_t i = t0 + (uint64_t)it * BLOCK + tid;
                        TID_FOR_COLS(MAXC, c, o.ncols)
                            st[o.stage_off + (uint32_t)c * o.stage_cap + r] =
                                src.value(j, c, item[it], i);
                    }
                }
            }
            __syncthreads();
            if (tid < k) {
                if (s_ovf[tid] == kNoTile && s_cnt[tid] + s_tot[tid] > a.out[tid].stage_cap) {
                    s_ovf[tid] = t0;
                    s_stg[tid] = s_cnt[tid];
                }
                s_cnt[tid] += s_tot[tid];
            }
        }
        __syncthreads();
        if (tid == 0) s_tk = ticket;
        if (tid < k) {
            if (s_ovf[tid] == kNoTile) s_stg[tid] = s_cnt[tid];
            dev::publish(&slots[t * k + tid], stamp | s_cnt[tid]);
        }
        __syncthreads();
        const bool pending = s_pend != kNone;
        uint64_t w0[MAXK][kSlotsPer];
        if (pending) request_slots(w0);
        const uint64_t tn = s_tk;  // next chunk (taken during the last tile)
        if (tn < Q) {
            uint64_t n0, n1;
            dev::chunk_bounds(a, tn, src.n, TILE, n0, n1);
            dev::tile_load<Src, BLOCK, IPT>(src, n0, n1, next);
        }
        if (pending) place(stage + (uint32_t)(buf ^ 1) * a.buf_words, w0);
        if (tid < k) {
            s_pcnt[tid] = s_cnt[tid];
            s_pstg[tid] = s_stg[tid];
            s_povf[tid] = s_ovf[tid];
        }
        if (tid == 0) s_pend = t;
        buf ^= 1;
        __syncthreads();
    }
    if (s_pend != kNone) {
        uint64_t w0[MAXK][kSlotsPer];
        request_slots(w0);
        place(stage + (uint32_t)(buf ^ 1) * a.buf_words, w0);
    }

    // the last workgroup out resets the ticket and done counters
    __syncthreads();
    if (tid == 0) {
        const uint32_t d = __hip_atomic_fetch_add(&counters[1], 1u, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
        if (d == gridDim.x - 1) {
            __hip_atomic_store(&counters[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&counters[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

int device_cus(tid_ctx *ctx);
// Workgroups of `kernel` (BLOCK threads, `lds` dynamic LDS bytes) resident per
// CU; cached per (kernel, lds) and safe to call from several host threads.
int resident_blocks(const void *kernel, int block, size_t lds);

// tiles per chunk before the single-tile tail
constexpr uint64_t kMinBigTiles = 4;
constexpr uint64_t kMaxBigTiles = 32;

template <class Src, int BLOCK, int IPT, int MAXK, int MAXC>
void launch_chunked(tid_ctx *ctx, const Src &src, CompactArgs<MAXK, MAXC> &a, int k,
                    uint32_t stage_words) {
    constexpr uint64_t TILE = (uint64_t)BLOCK * IPT;
    auto kern = chunk_compact_kernel<Src, BLOCK, IPT, MAXK, MAXC>;
    const size_t lds = (size_t)stage_words * sizeof(uint32_t);
    const int blocks_per_cu = resident_blocks((const void *)kern, BLOCK, lds);
    const uint64_t n = src.n;
    if (n == 0) return;
    uint64_t cols_total = 0;
    for (int j = 0; j < k; ++j) cols_total += (uint64_t)a.out[j].ncols;
    a.buf_words = stage_words / 2;
    const uint32_t rows_per = (uint32_t)(a.buf_words / std::max<uint64_t>(cols_total, 1));
    uint32_t off = 0;
    for (int j = 0; j < k; ++j) {
        a.out[j].stage_off = off;
        a.out[j].stage_cap = a.out[j].ncols ? rows_per : 0xFFFFFFFFu;
        off += rows_per * (uint32_t)a.out[j].ncols;
    }
    const uint64_t resident = (uint64_t)blocks_per_cu * (uint64_t)device_cus(ctx);
    const uint64_t tiles = (n + TILE - 1) / TILE;
    const uint64_t tail = std::min<uint64_t>(tiles, 2 * resident);
    // Chunk length: about an eighth of a workgroup's share of the tiles, so
    // that every workgroup still takes several chunks (fast ones more), within
    // [kMinBigTiles, kMaxBigTiles]: each chunk costs one placement round trip
    // during which only its successor's first tile is in flight, so long
    // inputs take long chunks.  Then as long as the rows the output bounds
    // allow per chunk fit 80% of a staging buffer: fewer placements for sparse
    // outputs, no overflow re-reads for dense ones.
    uint64_t big = std::min<uint64_t>(kMaxBigTiles,
                                      std::max<uint64_t>(kMinBigTiles, tiles / (8 * resident)));
    for (int j = 0; j < k; ++j) {
        const OutDesc<MAXC> &o = a.out[j];
        if (o.ncols == 0 || o.cap == 0) continue;
        const double rows_per_tile = (double)std::min<uint64_t>(o.cap, n) * TILE / (double)n;
        big = std::min<uint64_t>(big, (uint64_t)(0.8 * o.stage_cap / rows_per_tile));
    }
    big = std::max<uint64_t>(big, 1);
    a.big_tiles = (uint32_t)big;
    a.q_big = (tiles - tail) / big;
    a.q = a.q_big + (tiles - a.q_big * big);
    TID_REQUIRE(a.q + resident < (1ull << 32), TID_E_UNSUPPORTED, "compaction: input too large");
    a.k = k;
    const uint64_t P = std::max<uint64_t>(1, std::min<uint64_t>(resident, a.q));
    a.P = (uint32_t)P;
    // state: the ticket and done counters (one u64 word), then k * q count slots
    constexpr size_t kCounterWords = 1;
    uint64_t *state = nullptr;
    a.epoch = ctx->next_epoch(((size_t)k * a.q + kCounterWords) * sizeof(uint64_t), &state);
    hipLaunchKernelGGL(kern, dim3((uint32_t)P), dim3(BLOCK), lds, ctx->stream, src, a,
                       state + kCounterWords, reinterpret_cast<uint32_t *>(state), ctx->d_flags);
    TID_HIP(hipGetLastError());
}

// Block-ranged compaction, in two steps so that callers may bring their own
// cross-workgroup state: block_ranged_layout lays out the staging areas over
// `stage_words` words of LDS, fixes the ranges (a.P, a.range, a.k) and
// returns the state words the launch needs (the ticket and done counters in
// one word, then k * P count words); block_ranged_launch starts the kernel
// with that state and a.epoch, and `flags` (2 words: spin limit, overflow).
template <class Src, int BLOCK, int IPT, int MAXK, int MAXC, bool PREFETCH = false>
size_t block_ranged_layout(tid_ctx *ctx, const Src &src, CompactArgs<MAXK, MAXC> &a, int k,
                           uint32_t stage_words) {
    constexpr uint64_t TILE = (uint64_t)BLOCK * IPT;
    auto kern = compact_kernel<Src, BLOCK, IPT, MAXK, MAXC, PREFETCH>;
    const size_t lds = (size_t)stage_words * sizeof(uint32_t);
    const int blocks_per_cu = resident_blocks((const void *)kern, BLOCK, lds);
    const uint64_t n = src.n;
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
    const uint64_t resident = (uint64_t)blocks_per_cu * (uint64_t)device_cus(ctx) *
                              (uint64_t)std::max<int64_t>(1, ctx->opt.range_factor);
    uint64_t P = std::max<uint64_t>(1, std::min({tiles, resident, (uint64_t)BLOCK * kPrefixPer}));
    const uint64_t range = (tiles + P - 1) / P * TILE;
    P = (n + range - 1) / range;
    TID_REQUIRE(P < (1ull << 31), TID_E_UNSUPPORTED, "compaction: input too large");
    a.k = k;
    a.P = (uint32_t)P;
    a.range = range;
    return (size_t)k * P + 1;
}

template <class Src, int BLOCK, int IPT, int MAXK, int MAXC, bool PREFETCH = false>
void block_ranged_launch(tid_ctx *ctx, const Src &src, CompactArgs<MAXK, MAXC> &a,
                         uint32_t stage_words, uint64_t *state, uint32_t *flags) {
    auto kern = compact_kernel<Src, BLOCK, IPT, MAXK, MAXC, PREFETCH>;
    const size_t lds = (size_t)stage_words * sizeof(uint32_t);
    hipLaunchKernelGGL(kern, dim3(a.P), dim3(BLOCK), lds, ctx->stream, src, a, state + 1,
                       reinterpret_cast<uint32_t *>(state), flags);
    TID_HIP(hipGetLastError());
}

// Launch the compaction of `n` items over the resident-capacity grid.  The
// caller fills a.out[0..k) (columns, caps, counts, ncols); staging areas are
// laid out here over `stage_words` words of LDS.  The context's
// compact_kernel option picks the kernel: 1 block-ranged (PREFETCH picks its
// prefetching variant), 2 chunked, 0 (default) by the output bounds (below).
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
    int kind = (int)ctx->opt.compact_kernel;
    if (kind == 0) {
        const uint64_t ranges = std::max<uint64_t>(
            1, std::min<uint64_t>({(n + TILE - 1) / TILE,
                                   (uint64_t)blocks_per_cu * (uint64_t)device_cus(ctx) *
                                       (uint64_t)std::max<int64_t>(1, ctx->opt.range_factor),
                                   (uint64_t)BLOCK * kPrefixPer}));
        // One output: chunked where the block-ranged staging would overflow
        // (that kernel would then re-read the graph); block-ranged otherwise
        // (it has no per-chunk placements and, without a release fence, no
        // fixed cost at its end beyond one round trip).  Several outputs:
        // block-ranged (measured faster on the batched query mix).
        kind = 1;
        if (MAXK == 1 && a.out[0].ncols && a.out[0].cap / ranges > rows_per) kind = 2;
    }
    if (kind == 2) {
        launch_chunked<Src, BLOCK, IPT, MAXK, MAXC>(ctx, src, a, k, stage_words);
        return;
    }
    // epoch state: the ticket and done counters (one u64 word), then k * P count words
    const size_t words = block_ranged_layout<Src, BLOCK, IPT, MAXK, MAXC, PREFETCH>(
        ctx, src, a, k, stage_words);
    uint64_t *state = nullptr;
    a.epoch = ctx->next_epoch(words * sizeof(uint64_t), &state);
    block_ranged_launch<Src, BLOCK, IPT, MAXK, MAXC, PREFETCH>(ctx, src, a, stage_words, state,
                                                               ctx->d_flags);
}

}  // namespace tid
