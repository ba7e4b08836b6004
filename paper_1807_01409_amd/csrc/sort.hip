// sort.hip -- stable LSD radix sort of (64-bit key, 32-bit value) pairs, the
// canonical lexicographic row order of tables, DISTINCT, and union.
//
// The paper sorts subquery results before joining them and merges final
// results to distinct values (Sec. 4.2 step 3 with Mgpu's mergesort, Sec. 4.3
// DISTINCT).  Here every ordering is an LSD radix sort written for wave64:
//   hist     each workgroup owns one contiguous range of the input and counts
//            the digits of its range (wave-private LDS histograms, updated
//            by the leader lane of each group of lanes holding one digit);
//   offsets  one workgroup per digit scans that digit's counts over the
//            ranges; the scatter kernel adds the bases of the smaller digits
//            (a scan of the 256 digit totals) to find, for every (range,
//            digit), the place where its first element goes;
//   scatter  each workgroup walks its range tile by tile and writes every
//            element at its digit's running offset plus its stable rank,
//            found with ballots that group the lanes holding equal digits.
// Up to 8192 pairs are sorted by one workgroup instead, every pass in LDS,
// in one launch (small sorts are otherwise bound by launches, three a pass).
// A row of k columns is sorted as one or more packed 64-bit keys (as many
// leading columns as fit their bit widths), least significant group first,
// carrying the row permutation as the value.
#include "batch.hpp"
#include "compact.hpp"

#include <algorithm>
#include <mutex>
#include <numeric>

namespace tid {

constexpr int kRadixBits = 8;
constexpr uint32_t kRadix = 1u << kRadixBits;
constexpr int kSortBlock = 256;
constexpr int kSortIPT = 16;
constexpr int kSortNW = kSortBlock / dev::kWave;
constexpr uint64_t kSortTile = (uint64_t)kSortBlock * kSortIPT;

// lanes (among the valid ones) that hold the same digit as the calling lane
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid) {
    uint64_t peers = dev::ballot(valid);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t m = dev::ballot(bit);
        peers &= bit ? m : ~m;
    }
    return valid ? peers : 0ull;
}

// item `it` of lane `lane` in wave `wave` of the tile at t0: each wave owns 64*IPT
// consecutive items, so every load instruction reads 64 consecutive keys
__device__ __forceinline__ uint64_t sort_item(uint64_t t0, int wave, int it, int lane) {
    return t0 + (uint64_t)wave * (dev::kWave * kSortIPT) + (uint64_t)it * dev::kWave + lane;
}

__global__ __launch_bounds__(kSortBlock) void radix_hist(const uint64_t *__restrict__ keys,
                                                          uint64_t n, uint64_t range, int shift,
                                                          uint32_t *counts) {
    __shared__ uint32_t s_h[kSortNW][kRadix];
    const int tid = threadIdx.x, wave = tid / dev::kWave, lane = tid % dev::kWave;
    for (uint32_t d = tid; d < kSortNW * kRadix; d += kSortBlock) (&s_h[0][0])[d] = 0;
    __syncthreads();
    const uint32_t w = blockIdx.x;
    const uint64_t r0 = (uint64_t)w * range, r1 = min(n, r0 + range);
    for (uint64_t t0 = r0; t0 < r1; t0 += kSortTile) {
        uint32_t d[kSortIPT];
#pragma unroll
        for (int it = 0; it < kSortIPT; ++it) {
            const uint64_t i = sort_item(t0, wave, it, lane);
            d[it] = i < r1 ? (uint32_t)(keys[i] >> shift) & (kRadix - 1) : 0u;
        }
#pragma unroll
        for (int it = 0; it < kSortIPT; ++it) {
            const bool valid = sort_item(t0, wave, it, lane) < r1;
            const uint64_t peers = match_digit(d[it], valid);
            if (valid && lane == __builtin_ctzll(peers)) s_h[wave][d[it]] += (uint32_t)__popcll(peers);
        }
    }
    __syncthreads();
    for (uint32_t dd = tid; dd < kRadix; dd += kSortBlock) {
        uint32_t s = 0;
        for (int ww = 0; ww < kSortNW; ++ww) s += s_h[ww][dd];
        counts[(size_t)w * kRadix + dd] = s;
    }
}

// Where each (range, digit) goes is offs[w][d] = base[d] + scan[w][d]: base[d]
// counts every element of a smaller digit, scan[w][d] the elements of digit d
// in ranges before w.  One workgroup per digit scans its column of the
// range-major count matrix and writes the digit's total; the scatter kernel
// turns the 256 totals into bases itself.
constexpr int kColThreads = 256;
__global__ __launch_bounds__(kColThreads) void digit_scan(const uint32_t *__restrict__ counts,
                                                           uint32_t *__restrict__ scan,
                                                           uint32_t *__restrict__ totals,
                                                           uint32_t P) {
    __shared__ uint32_t s_w[kColThreads / dev::kWave];
    const uint32_t d = blockIdx.x;
    const int tid = threadIdx.x, wave = tid / dev::kWave, lane = tid % dev::kWave;
    const uint32_t per = (P + kColThreads - 1) / kColThreads;
    const uint32_t w0 = min(P, (uint32_t)tid * per), w1 = min(P, w0 + per);
    uint32_t sum = 0;
    for (uint32_t w = w0; w < w1; ++w) sum += counts[(size_t)w * kRadix + d];
    const uint32_t incl = dev::wave_inclusive_sum(sum);
    if (lane == dev::kWave - 1) s_w[wave] = incl;
    __syncthreads();
    uint32_t run = incl - sum;
    for (int x = 0; x < wave; ++x) run += s_w[x];
    for (uint32_t w = w0; w < w1; ++w) {
        const uint32_t c = counts[(size_t)w * kRadix + d];
        scan[(size_t)w * kRadix + d] = run;
        run += c;
    }
    if (tid == kColThreads - 1) totals[d] = run;
}

__global__ __launch_bounds__(kSortBlock) void radix_scatter(
    const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin, uint64_t *__restrict__ kout,
    uint32_t *__restrict__ vout, uint64_t n, uint64_t range, int shift, const uint32_t *scan,
    const uint32_t *totals) {
    constexpr int kPer = kRadix / dev::kWave;  // digits per lane in the base scan
    __shared__ uint32_t s_run[kRadix];
    __shared__ uint32_t s_wh[kSortNW][kRadix];
    const int tid = threadIdx.x, wave = tid / dev::kWave, lane = tid % dev::kWave;
    const uint32_t w = blockIdx.x;
    // digit bases: exclusive scan of the digit totals (wave 0, kPer digits a lane)
    if (wave == 0) {
        uint32_t v[kPer], loc = 0;
#pragma unroll
        for (int x = 0; x < kPer; ++x) {
            v[x] = totals[lane * kPer + x];
            loc += v[x];
        }
        uint32_t run = dev::wave_inclusive_sum(loc) - loc;
#pragma unroll
        for (int x = 0; x < kPer; ++x) {
            s_run[lane * kPer + x] = run;
            run += v[x];
        }
    }
    __syncthreads();
    for (uint32_t d = tid; d < kRadix; d += kSortBlock) s_run[d] += scan[(size_t)w * kRadix + d];
    const uint64_t r0 = (uint64_t)w * range, r1 = min(n, r0 + range);
    const uint64_t lt = (1ull << lane) - 1ull;
    for (uint64_t t0 = r0; t0 < r1; t0 += kSortTile) {
        uint64_t key[kSortIPT];
        uint32_t val[kSortIPT], rank[kSortIPT];
#pragma unroll
        for (int it = 0; it < kSortIPT; ++it) {
            const uint64_t i = sort_item(t0, wave, it, lane);
            key[it] = i < r1 ? kin[i] : 0ull;
            val[it] = i < r1 ? vin[i] : 0u;
        }
        for (uint32_t d = lane; d < kRadix; d += dev::kWave) s_wh[wave][d] = 0;
#pragma unroll
        for (int it = 0; it < kSortIPT; ++it) {
            const bool valid = sort_item(t0, wave, it, lane) < r1;
            const uint32_t d = (uint32_t)(key[it] >> shift) & (kRadix - 1);
            const uint64_t peers = match_digit(d, valid);
            const uint32_t before = valid ? s_wh[wave][d] : 0u;
            rank[it] = before + (uint32_t)__popcll(peers & lt);
            if (valid && lane == __builtin_ctzll(peers)) s_wh[wave][d] = before + (uint32_t)__popcll(peers);
        }
        __syncthreads();
        // per-wave counts -> per-wave bases (waves in item order)
        for (uint32_t d = tid; d < kRadix; d += kSortBlock) {
            uint32_t run = s_run[d];
            for (int ww = 0; ww < kSortNW; ++ww) {
                const uint32_t c = s_wh[ww][d];
                s_wh[ww][d] = run;
                run += c;
            }
            s_run[d] = run;
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < kSortIPT; ++it) {
            if (sort_item(t0, wave, it, lane) < r1) {
                const uint32_t d = (uint32_t)(key[it] >> shift) & (kRadix - 1);
                const uint32_t pos = s_wh[wave][d] + rank[it];
                kout[pos] = key[it];
                vout[pos] = val[it];
            }
        }
        __syncthreads();
    }
}

// One workgroup sorts n <= kSmallBlock * kSmallIPT pairs on key bits
// [0, bits), in place: the pairs stay in LDS between passes, and each pass
// ranks items like the scatter kernel (waves in item order, ballots within a
// wave) and writes them back to LDS at their new places.
constexpr int kSmallBlock = 1024;
constexpr int kSmallIPT = 8;
constexpr int kSmallNW = kSmallBlock / dev::kWave;
constexpr uint64_t kSmallMax = (uint64_t)kSmallBlock * kSmallIPT;
constexpr size_t kSmallLds = kSmallMax * 12 + (size_t)kSmallNW * kRadix * 4 + kRadix * 4;

// item `it` of lane `lane` in wave `wave`: each wave owns 64 * kSmallIPT
// consecutive items
__device__ __forceinline__ uint32_t small_item(int wave, int it, int lane) {
    return (uint32_t)(wave * (dev::kWave * kSmallIPT) + it * dev::kWave + lane);
}

__global__ __launch_bounds__(kSmallBlock) void small_sort(uint64_t *keys, uint32_t *vals,
                                                          uint32_t n, int bits) {
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    uint64_t *s_key = reinterpret_cast<uint64_t *>(lds);
    uint32_t *s_val = lds + 2 * kSmallMax;
    uint32_t(*s_wh)[kRadix] = reinterpret_cast<uint32_t(*)[kRadix]>(s_val + kSmallMax);
    uint32_t *s_run = s_val + kSmallMax + kSmallNW * kRadix;
    const int tid = threadIdx.x, wave = tid / dev::kWave, lane = tid % dev::kWave;
    const uint64_t lt = (1ull << lane) - 1ull;
    constexpr int kPer = kRadix / dev::kWave;
    for (int shift = 0; shift < bits; shift += kRadixBits) {
        uint64_t key[kSmallIPT];
        uint32_t val[kSmallIPT], rank[kSmallIPT];
#pragma unroll
        for (int it = 0; it < kSmallIPT; ++it) {
            const uint32_t i = small_item(wave, it, lane);
            key[it] = 0;
            val[it] = 0;
            if (i < n) {
                key[it] = shift == 0 ? keys[i] : s_key[i];
                val[it] = shift == 0 ? vals[i] : s_val[i];
            }
        }
        for (uint32_t d = lane; d < kRadix; d += dev::kWave) s_wh[wave][d] = 0;
#pragma unroll
        for (int it = 0; it < kSmallIPT; ++it) {
            const bool valid = small_item(wave, it, lane) < n;
            const uint32_t d = (uint32_t)(key[it] >> shift) & (kRadix - 1);
            const uint64_t peers = match_digit(d, valid);
            const uint32_t before = valid ? s_wh[wave][d] : 0u;
            rank[it] = before + (uint32_t)__popcll(peers & lt);
            if (valid && lane == __builtin_ctzll(peers)) s_wh[wave][d] = before + (uint32_t)__popcll(peers);
        }
        __syncthreads();  // every item is in registers and every wave has counted
        if (tid < (int)kRadix) {
            uint32_t t = 0;
            for (int w = 0; w < kSmallNW; ++w) t += s_wh[w][tid];
            s_run[tid] = t;
        }
        __syncthreads();
        if (wave == 0) {  // digit totals -> digit bases
            uint32_t v[kPer], loc = 0;
#pragma unroll
            for (int x = 0; x < kPer; ++x) {
                v[x] = s_run[lane * kPer + x];
                loc += v[x];
            }
            uint32_t run = dev::wave_inclusive_sum(loc) - loc;
#pragma unroll
            for (int x = 0; x < kPer; ++x) {
                s_run[lane * kPer + x] = run;
                run += v[x];
            }
        }
        __syncthreads();
        if (tid < (int)kRadix) {  // per-wave bases of each digit, waves in item order
            uint32_t run = s_run[tid];
            for (int w = 0; w < kSmallNW; ++w) {
                const uint32_t c = s_wh[w][tid];
                s_wh[w][tid] = run;
                run += c;
            }
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < kSmallIPT; ++it) {
            if (small_item(wave, it, lane) < n) {
                const uint32_t d = (uint32_t)(key[it] >> shift) & (kRadix - 1);
                const uint32_t pos = s_wh[wave][d] + rank[it];
                s_key[pos] = key[it];
                s_val[pos] = val[it];
            }
        }
        __syncthreads();  // the next pass reads the new order
    }
    for (uint32_t i = tid; i < n; i += kSmallBlock) {
        keys[i] = s_key[i];
        vals[i] = s_val[i];
    }
}

__global__ void iota_u32(uint32_t *v, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        v[i] = (uint32_t)i;
}

struct PackArgs {
    const uint32_t *col[TID_MAX_COLS];
    int shift[TID_MAX_COLS];
    int ncols;
};

// key[i] = concatenation of the group's columns of row perm[i] (or row i)
__global__ void pack_keys(PackArgs a, const uint32_t *perm, uint64_t n, uint64_t *key) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint64_t r = perm ? perm[i] : i;
        uint64_t k = 0;
        for (int c = 0; c < a.ncols; ++c) k |= (uint64_t)a.col[c][r] << a.shift[c];
        key[i] = k;
    }
}

struct GatherArgs {
    const uint32_t *in[TID_MAX_COLS];
    uint32_t *out[TID_MAX_COLS];
    int ncols;
};

__global__ void gather_rows(GatherArgs a, const uint32_t *perm, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t r = perm[i];
        for (int c = 0; c < a.ncols; ++c) a.out[c][i] = a.in[c][r];
    }
}

// per-column maximum: one atomic per workgroup after an LDS reduction
__global__ __launch_bounds__(256) void column_max(const uint32_t *const *cols, uint64_t n,
                                                   uint32_t *mx) {
    __shared__ uint32_t s_m[4];
    const uint32_t *col = cols[blockIdx.y];
    uint32_t m = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        m = max(m, col[i]);
    for (int d = 32; d >= 1; d >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, d, 64));
    if (dev::lane_id() == 0) s_m[threadIdx.x / 64] = m;
    __syncthreads();
    if (threadIdx.x == 0) atomicMax(&mx[blockIdx.y], max(max(s_m[0], s_m[1]), max(s_m[2], s_m[3])));
}

__global__ void fill_u32(uint32_t *p, uint64_t n, uint32_t v) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

// rows of a sorted table that differ from the row before them
struct UniqueSrc {
    const uint32_t *col[TID_MAX_COLS];
    int ncols;
    uint64_t n;
    using Item = uint64_t;
    __device__ __forceinline__ Item load(uint64_t i) const { return i; }
    __device__ __forceinline__ bool match(int, Item i) const {
        if (i == 0) return true;
        for (int c = 0; c < ncols; ++c)
            if (col[c][i] != col[c][i - 1]) return true;
        return false;
    }
    __device__ __forceinline__ uint32_t value(int, int c, Item i, uint64_t) const {
        return col[c][i];
    }
};

// ---------------------------------------------------------------------------
// Batched row sorts: the final sorts of many plans of one round share their
// launches.  Each job is one table's (key, value) pairs; a pass cuts every
// active job into ranges of whole tiles (the ranges of all jobs concatenated,
// rbase = a job's first range) and runs the three steps of the single sort
// above over all of them: per-range digit counts, one workgroup per job that
// turns its counts into output offsets (four quarters of its ranges in
// parallel), and the stable scatter of every range.
// ---------------------------------------------------------------------------

struct SegPass {
    const uint64_t *kin;
    const uint32_t *vin;
    uint64_t *kout;
    uint32_t *vout;
    uint64_t n;         // pairs
    uint64_t range;     // pairs per range, a multiple of the tile
    uint64_t rbase;     // the job's first range in this pass
    uint32_t nranges;
    int32_t shift;
};

// job j with jobs[j].rbase <= r < jobs[j + 1].rbase
__device__ __forceinline__ int seg_job_of(const SegPass *jobs, int J, uint64_t r) {
    int lo = 0, hi = J;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (jobs[mid].rbase <= r) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kSortBlock) void seg_hist(const SegPass *jobs, int J,
                                                        uint32_t *counts) {
    __shared__ uint32_t s_h[kSortNW][kRadix];
    const int tid = threadIdx.x, wave = tid / dev::kWave, lane = tid % dev::kWave;
    for (uint32_t d = tid; d < kSortNW * kRadix; d += kSortBlock) (&s_h[0][0])[d] = 0;
    __syncthreads();
    const uint64_t gr = blockIdx.x;
    const SegPass &p = jobs[seg_job_of(jobs, J, gr)];
    const uint64_t r0 = (gr - p.rbase) * p.range, r1 = min(p.n, r0 + p.range);
    for (uint64_t t0 = r0; t0 < r1; t0 += kSortTile) {
        uint32_t d[kSortIPT];
#pragma unroll
        for (int it = 0; it < kSortIPT; ++it) {
            const uint64_t i = sort_item(t0, wave, it, lane);
            d[it] = i < r1 ? (uint32_t)(p.kin[i] >> p.shift) & (kRadix - 1) : 0u;
        }
#pragma unroll
        for (int it = 0; it < kSortIPT; ++it) {
            const bool valid = sort_item(t0, wave, it, lane) < r1;
            const uint64_t peers = match_digit(d[it], valid);
            if (valid && lane == __builtin_ctzll(peers)) s_h[wave][d[it]] += (uint32_t)__popcll(peers);
        }
    }
    __syncthreads();
    for (uint32_t dd = tid; dd < kRadix; dd += kSortBlock) {
        uint32_t sum = 0;
        for (int ww = 0; ww < kSortNW; ++ww) sum += s_h[ww][dd];
        counts[gr * kRadix + dd] = sum;
    }
}

// In place: counts[range][d] -> the job-relative output position of the
// range's first pair of digit d (pairs of smaller digits, then those of
// digit d in earlier ranges).
constexpr int kSegParts = 4;
__global__ __launch_bounds__(kRadix * kSegParts) void seg_offsets(const SegPass *jobs,
                                                                   uint32_t *counts) {
    constexpr int kPer = kRadix / dev::kWave;
    __shared__ uint32_t s_part[kSegParts][kRadix];
    __shared__ uint32_t s_base[kRadix];
    const SegPass &p = jobs[blockIdx.x];
    const int d = threadIdx.x % kRadix, part = threadIdx.x / kRadix;
    const uint32_t R = p.nranges;
    const uint32_t per = (R + kSegParts - 1) / kSegParts;
    const uint32_t a = min(R, (uint32_t)part * per), b = min(R, a + per);
    uint32_t *c = counts + p.rbase * kRadix;
    uint32_t sum = 0;
    for (uint32_t r = a; r < b; ++r) sum += c[(size_t)r * kRadix + d];
    s_part[part][d] = sum;
    __syncthreads();
    if (part == 0) {
        uint32_t tot = 0;
#pragma unroll
        for (int x = 0; x < kSegParts; ++x) tot += s_part[x][d];
        s_base[d] = tot;
    }
    __syncthreads();
    if (threadIdx.x < dev::kWave) {  // digit totals -> digit bases
        const int lane = threadIdx.x;
        uint32_t v[kPer], loc = 0;
#pragma unroll
        for (int x = 0; x < kPer; ++x) {
            v[x] = s_base[lane * kPer + x];
            loc += v[x];
        }
        uint32_t run = dev::wave_inclusive_sum(loc) - loc;
#pragma unroll
        for (int x = 0; x < kPer; ++x) {
            s_base[lane * kPer + x] = run;
            run += v[x];
        }
    }
    __syncthreads();
    uint32_t run = s_base[d];
    for (int x = 0; x < part; ++x) run += s_part[x][d];
    for (uint32_t r = a; r < b; ++r) {
        const uint32_t v = c[(size_t)r * kRadix + d];
        c[(size_t)r * kRadix + d] = run;
        run += v;
    }
}

__global__ __launch_bounds__(kSortBlock) void seg_scatter(const SegPass *jobs, int J,
                                                           const uint32_t *offs) {
    __shared__ uint32_t s_run[kRadix];
    __shared__ uint32_t s_wh[kSortNW][kRadix];
    const int tid = threadIdx.x, wave = tid / dev::kWave, lane = tid % dev::kWave;
    const uint64_t gr = blockIdx.x;
    const SegPass &p = jobs[seg_job_of(jobs, J, gr)];
    for (uint32_t d = tid; d < kRadix; d += kSortBlock) s_run[d] = offs[gr * kRadix + d];
    const uint64_t r0 = (gr - p.rbase) * p.range, r1 = min(p.n, r0 + p.range);
    const uint64_t lt = (1ull << lane) - 1ull;
    __syncthreads();
    for (uint64_t t0 = r0; t0 < r1; t0 += kSortTile) {
        uint64_t key[kSortIPT];
        uint32_t val[kSortIPT], rank[kSortIPT];
#pragma unroll
        for (int it = 0; it < kSortIPT; ++it) {
            const uint64_t i = sort_item(t0, wave, it, lane);
            key[it] = i < r1 ? p.kin[i] : 0ull;
            val[it] = i < r1 ? p.vin[i] : 0u;
        }
        for (uint32_t d = lane; d < kRadix; d += dev::kWave) s_wh[wave][d] = 0;
#pragma unroll
        for (int it = 0; it < kSortIPT; ++it) {
            const bool valid = sort_item(t0, wave, it, lane) < r1;
            const uint32_t d = (uint32_t)(key[it] >> p.shift) & (kRadix - 1);
            const uint64_t peers = match_digit(d, valid);
            const uint32_t before = valid ? s_wh[wave][d] : 0u;
            rank[it] = before + (uint32_t)__popcll(peers & lt);
            if (valid && lane == __builtin_ctzll(peers)) s_wh[wave][d] = before + (uint32_t)__popcll(peers);
        }
        __syncthreads();
        for (uint32_t d = tid; d < kRadix; d += kSortBlock) {
            uint32_t run = s_run[d];
            for (int ww = 0; ww < kSortNW; ++ww) {
                const uint32_t c = s_wh[ww][d];
                s_wh[ww][d] = run;
                run += c;
            }
            s_run[d] = run;
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < kSortIPT; ++it) {
            if (sort_item(t0, wave, it, lane) < r1) {
                const uint32_t d = (uint32_t)(key[it] >> p.shift) & (kRadix - 1);
                const uint32_t pos = s_wh[wave][d] + rank[it];
                p.kout[pos] = key[it];
                p.vout[pos] = val[it];
            }
        }
        __syncthreads();
    }
}

// Keys of one column group for every job: key[i] = the group's columns of
// row perm[i] (or of row i, when perm is null: the first group, which also
// writes the identity permutation).  One y-row of the grid per job.
struct SegPack {
    const uint32_t *col[TID_MAX_COLS];
    int32_t shift[TID_MAX_COLS];
    int32_t ncols;
    const uint32_t *perm;
    uint32_t *iota;
    uint64_t *key;
    uint64_t n;
};

__global__ void seg_pack(const SegPack *jobs) {
    const SegPack &p = jobs[blockIdx.y];
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < p.n; i += stride) {
        const uint64_t r = p.perm ? p.perm[i] : i;
        if (!p.perm) p.iota[i] = (uint32_t)i;
        uint64_t k = 0;
        for (int c = 0; c < p.ncols; ++c) k |= (uint64_t)p.col[c][r] << p.shift[c];
        p.key[i] = k;
    }
}

// rows of every job's input in the order of its permutation
struct SegGather {
    const uint32_t *in[TID_MAX_COLS];
    uint32_t *out[TID_MAX_COLS];
    int32_t ncols;
    const uint32_t *perm;
    uint64_t n;
};

__global__ void seg_gather(const SegGather *jobs) {
    const SegGather &p = jobs[blockIdx.y];
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < p.n; i += stride) {
        const uint32_t r = p.perm[i];
        for (int c = 0; c < p.ncols; ++c) p.out[c][i] = p.in[c][r];
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

static unsigned grid_for(uint64_t n, unsigned block = 256, unsigned cap = 8192) {
    return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((n + block - 1) / block, cap));
}

void fill(tid_ctx *ctx, uint32_t *p, uint64_t n, uint32_t v) {
    if (!n) return;
    hipLaunchKernelGGL(fill_u32, dim3(grid_for(n)), dim3(256), 0, ctx->stream, p, n, v);
    TID_HIP(hipGetLastError());
}

void iota(tid_ctx *ctx, uint32_t *p, uint64_t n) {
    if (!n) return;
    hipLaunchKernelGGL(iota_u32, dim3(grid_for(n)), dim3(256), 0, ctx->stream, p, n);
    TID_HIP(hipGetLastError());
}

// Stable sort of n (key, value) pairs on key bits [0, bits).  The sorted pairs
// end in (k0, v0) if the return value is false, in (k1, v1) if true.
bool radix_sort_pairs(tid_ctx *ctx, uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1,
                      uint64_t n, int bits) {
    if (n <= 1 || bits <= 0) return false;
    TID_REQUIRE(n < (1ull << 32), TID_E_UNSUPPORTED, "sort: more than 2^32-1 rows");
    if (n <= kSmallMax) {
        // once per process, also when several host threads (serving workers,
        // each with its own context) reach the first small sort together
        static std::once_flag attr_once;
        std::call_once(attr_once, [] {
            TID_HIP(hipFuncSetAttribute((const void *)small_sort,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSmallLds));
        });
        hipLaunchKernelGGL(small_sort, dim3(1), dim3(kSmallBlock), kSmallLds, ctx->stream, k0, v0,
                           (uint32_t)n, bits);
        TID_HIP(hipGetLastError());
        return false;
    }
    const uint64_t tiles = (n + kSortTile - 1) / kSortTile;
    uint64_t P = std::max<uint64_t>(1, std::min<uint64_t>(tiles, 2ull * device_cus(ctx)));
    const uint64_t range = (tiles + P - 1) / P * kSortTile;
    P = (n + range - 1) / range;
    DevBuf counts(ctx, (size_t)kRadix * P * sizeof(uint32_t));
    DevBuf scan(ctx, (size_t)kRadix * (P + 1) * sizeof(uint32_t));  // then the digit totals
    uint32_t *totals = scan.get<uint32_t>() + (size_t)kRadix * P;
    bool flip = false;
    for (int shift = 0; shift < bits; shift += kRadixBits) {
        const uint64_t *ki = flip ? k1 : k0;
        const uint32_t *vi = flip ? v1 : v0;
        uint64_t *ko = flip ? k0 : k1;
        uint32_t *vo = flip ? v0 : v1;
        hipLaunchKernelGGL(radix_hist, dim3((uint32_t)P), dim3(kSortBlock), 0, ctx->stream, ki, n,
                           range, shift, counts.get<uint32_t>());
        TID_HIP(hipGetLastError());
        hipLaunchKernelGGL(digit_scan, dim3(kRadix), dim3(kColThreads), 0, ctx->stream,
                           counts.get<const uint32_t>(), scan.get<uint32_t>(), totals, (uint32_t)P);
        TID_HIP(hipGetLastError());
        hipLaunchKernelGGL(radix_scatter, dim3((uint32_t)P), dim3(kSortBlock), 0, ctx->stream, ki,
                           vi, ko, vo, n, range, shift, scan.get<const uint32_t>(), totals);
        TID_HIP(hipGetLastError());
        flip = !flip;
    }
    return flip;
}

std::vector<uint32_t> column_maxima(tid_ctx *ctx, const tid_table *t, uint64_t n) {
    std::vector<uint32_t> mx(t->ncols, 0);
    if (n == 0 || t->ncols == 0) return mx;
    DevBuf cols(ctx, sizeof(uint32_t *) * t->ncols);
    DevBuf dmx(ctx, sizeof(uint32_t) * t->ncols);
    TID_HIP(hipMemcpyAsync(cols.get(), t->col, sizeof(uint32_t *) * t->ncols,
                           hipMemcpyHostToDevice, ctx->stream));
    TID_HIP(hipMemsetAsync(dmx.get(), 0, sizeof(uint32_t) * t->ncols, ctx->stream));
    hipLaunchKernelGGL(column_max, dim3(grid_for(n, 256, 512), t->ncols), dim3(256), 0,
                       ctx->stream, cols.get<const uint32_t *const>(), n, dmx.get<uint32_t>());
    TID_HIP(hipGetLastError());
    TID_HIP(hipMemcpyAsync(mx.data(), dmx.get(), sizeof(uint32_t) * t->ncols,
                           hipMemcpyDeviceToHost, ctx->stream));
    ctx->sync();
    return mx;
}

static int bit_width(uint32_t v) { return v ? 32 - __builtin_clz(v) : 0; }

// Permutation that puts the rows of t (n rows) in lexicographic order.
DevBuf sort_permutation(tid_ctx *ctx, const tid_table *t, uint64_t n) {
    // column bounds known on the host spare a device round trip
    const std::vector<uint32_t> mx =
        t->maxv_known ? std::vector<uint32_t>(t->maxv, t->maxv + t->ncols)
                      : column_maxima(ctx, t, n);
    // columns grouped from the most significant one while their widths fit 64 bits
    std::vector<std::pair<int, int>> groups;  // [first, last) columns
    int c = 0;
    while (c < t->ncols) {
        int width = 0, e = c;
        while (e < t->ncols && width + bit_width(mx[e]) <= 64) width += bit_width(mx[e++]);
        if (e == c) e = c + 1;  // unreachable: a column is at most 32 bits
        groups.emplace_back(c, e);
        c = e;
    }
    DevBuf ka(ctx, n * 8), kb(ctx, n * 8), va(ctx, n * 4), vb(ctx, n * 4);
    iota(ctx, va.get<uint32_t>(), n);
    bool perm_in_b = false;
    bool first = true;
    for (int g = (int)groups.size() - 1; g >= 0; --g) {
        PackArgs pa{};
        int shift = 0;
        for (int x = groups[g].second - 1; x >= groups[g].first; --x) {
            pa.col[pa.ncols] = t->col[x];
            pa.shift[pa.ncols] = shift;
            ++pa.ncols;
            shift += bit_width(mx[x]);
        }
        if (shift == 0) continue;  // all-zero columns order nothing
        uint32_t *perm = perm_in_b ? vb.get<uint32_t>() : va.get<uint32_t>();
        uint64_t *keys = perm_in_b ? kb.get<uint64_t>() : ka.get<uint64_t>();
        hipLaunchKernelGGL(pack_keys, dim3(grid_for(n)), dim3(256), 0, ctx->stream, pa,
                           first ? (const uint32_t *)nullptr : perm, n, keys);
        TID_HIP(hipGetLastError());
        first = false;
        const bool moved = perm_in_b
                               ? radix_sort_pairs(ctx, kb.get<uint64_t>(), vb.get<uint32_t>(),
                                                  ka.get<uint64_t>(), va.get<uint32_t>(), n, shift)
                               : radix_sort_pairs(ctx, ka.get<uint64_t>(), va.get<uint32_t>(),
                                                  kb.get<uint64_t>(), vb.get<uint32_t>(), n, shift);
        if (moved) perm_in_b = !perm_in_b;
    }
    return perm_in_b ? std::move(vb) : std::move(va);
}

// rows of src (n rows) placed in the order given by perm, into dst
void gather_table(tid_ctx *ctx, const tid_table *src, const uint32_t *perm, uint64_t n,
                  tid_table *dst) {
    if (!n || !src->ncols) return;
    GatherArgs ga{};
    ga.ncols = src->ncols;
    for (int c = 0; c < src->ncols; ++c) {
        ga.in[c] = src->col[c];
        ga.out[c] = dst->col[c];
    }
    hipLaunchKernelGGL(gather_rows, dim3(grid_for(n)), dim3(256), 0, ctx->stream, ga, perm, n);
    TID_HIP(hipGetLastError());
}

// drop rows equal to their predecessor in a sorted table
std::unique_ptr<tid_table> unique_sorted(tid_ctx *ctx, const tid_table *t, uint64_t n) {
    auto out = make_table(ctx, t->ncols, t->vars, n);
    out->maxv_known = t->maxv_known;
    copy_bounds(out.get(), t, nullptr, t->ncols);
    if (n == 0) {
        set_count(ctx, out.get(), 0);
        return out;
    }
    UniqueSrc src{};
    for (int c = 0; c < t->ncols; ++c) src.col[c] = t->col[c];
    src.ncols = t->ncols;
    src.n = n;
    CompactArgs<1, TID_MAX_COLS> a{};
    for (int c = 0; c < t->ncols; ++c) a.out[0].col[c] = out->col[c];
    a.out[0].cap = n;
    a.out[0].count = out->d_count;
    a.out[0].ncols = t->ncols;
    launch_compact<UniqueSrc, 256, 16, 1, TID_MAX_COLS>(ctx, src, a, 1, 8192);
    return out;
}

std::unique_ptr<tid_table> sort_rows(tid_ctx *ctx, const tid_table *t, uint64_t n, int distinct) {
    if (t->ncols == 0) {
        // zero-width rows are all equal
        auto out = make_table(ctx, 0, t->vars, 0);
        set_count(ctx, out.get(), distinct ? std::min<uint64_t>(n, 1) : n);
        return out;
    }
    auto sorted = make_table(ctx, t->ncols, t->vars, n);
    sorted->maxv_known = t->maxv_known;
    copy_bounds(sorted.get(), t, nullptr, t->ncols);
    if (n <= 1) {
        for (int c = 0; c < t->ncols && n; ++c)
            TID_HIP(hipMemcpyAsync(sorted->col[c], t->col[c], n * 4, hipMemcpyDeviceToDevice,
                                   ctx->stream));
        set_count(ctx, sorted.get(), n);
        return sorted;
    }
    DevBuf perm = sort_permutation(ctx, t, n);
    gather_table(ctx, t, perm.get<const uint32_t>(), n, sorted.get());
    set_count(ctx, sorted.get(), n);
    if (!distinct) return sorted;
    return unique_sorted(ctx, sorted.get(), n);
}

// Row sorts of many tables in shared launches (see the batched kernels
// above).  Every table needs its column bounds on the host and fewer than
// 2^32 rows; each output table is allocated by the caller with n rows.  The
// job tables, key arrays and permutations go into `keep` / `host_keep`,
// which the caller holds until the stream has passed these launches.
void sort_rows_batched(tid_ctx *ctx, const std::vector<RowSortJob> &jobs,
                       std::vector<DevBuf> &keep, std::vector<std::vector<char>> &host_keep) {
    if (jobs.empty()) return;
    if (jobs.size() == 1) {
        // one table (a single plan): the sort of one table, whose passes
        // spread over up to two ranges per compute unit
        const RowSortJob &job = jobs[0];
        TID_REQUIRE(job.in->maxv_known && job.n < (1ull << 32) && job.in->ncols > 0,
                    TID_E_INTERNAL, "batched sort: bad job");
        keep.push_back(sort_permutation(ctx, job.in, job.n));
        gather_table(ctx, job.in, keep.back().get<const uint32_t>(), job.n, job.out);
        return;
    }
    constexpr uint64_t kChunkRows = 1ull << 27;  // rows per arena fill
    struct Plan {
        std::vector<std::pair<int, int>> groups;  // [first, last) columns, most significant first
        std::vector<int> width;
    };
    auto upload = [&](const void *data, size_t bytes) -> const void * {
        host_keep.emplace_back(reinterpret_cast<const char *>(data),
                               reinterpret_cast<const char *>(data) + bytes);
        keep.emplace_back(ctx, bytes);
        TID_HIP(hipMemcpyAsync(keep.back().get(), host_keep.back().data(), bytes,
                               hipMemcpyHostToDevice, ctx->stream));
        return keep.back().get();
    };
    // chunks of jobs in order, each within kChunkRows rows (a larger job alone)
    size_t j0 = 0;
    uint64_t most = 0;
    std::vector<std::pair<size_t, size_t>> chunks;
    while (j0 < jobs.size()) {
        size_t j1 = j0;
        uint64_t rows = 0;
        while (j1 < jobs.size() && (j1 == j0 || rows + jobs[j1].n <= kChunkRows))
            rows += jobs[j1++].n;
        chunks.emplace_back(j0, j1);
        most = std::max(most, rows);
        j0 = j1;
    }
    // one arena for every chunk (stream order keeps the fills apart): per
    // job two key and two value arrays
    DevBuf arena(ctx, std::max<uint64_t>(most, 1) * 24 + 4 * kAlign * jobs.size());
    char *const base = arena.get<char>();
    for (const auto &ch : chunks) {
        const int J = (int)(ch.second - ch.first);
        std::vector<Plan> plans(J);
        std::vector<uint64_t *> ka(J), kb(J);
        std::vector<uint32_t *> va(J), vb(J);
        size_t at = 0;
        int max_groups = 0;
        for (int j = 0; j < J; ++j) {
            const RowSortJob &job = jobs[ch.first + j];
            const tid_table *t = job.in;
            TID_REQUIRE(t->maxv_known && job.n < (1ull << 32) && t->ncols > 0, TID_E_INTERNAL,
                        "batched sort: bad job");
            Plan &pl = plans[j];
            int c = 0;
            while (c < t->ncols) {
                int w = 0, e = c;
                while (e < t->ncols && w + bit_width(t->maxv[e]) <= 64) w += bit_width(t->maxv[e++]);
                if (e == c) e = c + 1;
                pl.groups.emplace_back(c, e);
                pl.width.push_back(w);
                c = e;
            }
            max_groups = std::max(max_groups, (int)pl.groups.size());
            ka[j] = reinterpret_cast<uint64_t *>(base + at);
            at += align_up(job.n * 8);
            kb[j] = reinterpret_cast<uint64_t *>(base + at);
            at += align_up(job.n * 8);
            va[j] = reinterpret_cast<uint32_t *>(base + at);
            at += align_up(job.n * 4);
            vb[j] = reinterpret_cast<uint32_t *>(base + at);
            at += align_up(job.n * 4);
        }
        // the whole schedule on the host: per step (column group, least
        // significant first) the packs, then its digit passes
        std::vector<SegPack> packs;
        std::vector<std::pair<size_t, size_t>> step_packs;  // [first, last) in packs
        std::vector<SegPass> passes;
        struct PassLaunch { size_t first; int J; uint64_t ranges; };
        std::vector<std::vector<PassLaunch>> step_passes;
        std::vector<int> cur(J, 0);  // 0: (ka, va) hold the current pairs, 1: (kb, vb)
        uint64_t most_ranges = 0;
        for (int st = 0; st < max_groups; ++st) {
            const size_t p0 = packs.size();
            std::vector<int> npass(J, 0);
            for (int j = 0; j < J; ++j) {
                const Plan &pl = plans[j];
                const int G = (int)pl.groups.size();
                if (st >= G) continue;
                const int g = G - 1 - st;
                const int w = pl.width[g];
                if (w == 0 && st > 0) continue;  // all-zero columns order nothing
                const tid_table *t = jobs[ch.first + j].in;
                SegPack pk{};
                int shift = 0;
                for (int x = pl.groups[g].second - 1; x >= pl.groups[g].first; --x) {
                    pk.col[pk.ncols] = t->col[x];
                    pk.shift[pk.ncols] = shift;
                    ++pk.ncols;
                    shift += bit_width(t->maxv[x]);
                }
                pk.perm = st == 0 ? nullptr : (cur[j] ? vb[j] : va[j]);
                pk.iota = cur[j] ? vb[j] : va[j];
                pk.key = cur[j] ? kb[j] : ka[j];
                pk.n = jobs[ch.first + j].n;
                packs.push_back(pk);
                npass[j] = (w + kRadixBits - 1) / kRadixBits;
            }
            step_packs.emplace_back(p0, packs.size());
            std::vector<PassLaunch> pl_launch;
            for (int pass = 0;; ++pass) {
                uint64_t active = 0;
                for (int j = 0; j < J; ++j)
                    if (npass[j] > pass) active += jobs[ch.first + j].n;
                if (active == 0) break;
                const uint64_t tile = kSortTile;
                const uint64_t g_range =
                    std::max<uint64_t>(tile, (active / 4096 + tile - 1) / tile * tile);
                PassLaunch L{passes.size(), 0, 0};
                for (int j = 0; j < J; ++j) {
                    if (npass[j] <= pass) continue;
                    const uint64_t n = jobs[ch.first + j].n;
                    SegPass sp{};
                    sp.kin = cur[j] ? kb[j] : ka[j];
                    sp.vin = cur[j] ? vb[j] : va[j];
                    sp.kout = cur[j] ? ka[j] : kb[j];
                    sp.vout = cur[j] ? va[j] : vb[j];
                    sp.n = n;
                    sp.range = std::max<uint64_t>(g_range, ((n + 255) / 256 + tile - 1) / tile * tile);
                    sp.nranges = (uint32_t)((n + sp.range - 1) / sp.range);
                    sp.rbase = L.ranges;
                    sp.shift = pass * kRadixBits;
                    L.ranges += sp.nranges;
                    ++L.J;
                    passes.push_back(sp);
                    cur[j] ^= 1;
                }
                most_ranges = std::max(most_ranges, L.ranges);
                pl_launch.push_back(L);
            }
            step_passes.push_back(std::move(pl_launch));
        }
        std::vector<SegGather> gathers(J);
        uint64_t most_n = 0;
        for (int j = 0; j < J; ++j) {
            const RowSortJob &job = jobs[ch.first + j];
            SegGather &g = gathers[j];
            g.ncols = job.in->ncols;
            for (int c = 0; c < g.ncols; ++c) {
                g.in[c] = job.in->col[c];
                g.out[c] = job.out->col[c];
            }
            g.perm = cur[j] ? vb[j] : va[j];
            g.n = job.n;
            most_n = std::max(most_n, job.n);
        }
        TID_REQUIRE(!packs.empty(), TID_E_INTERNAL, "batched sort: nothing to pack");
        const SegPack *d_pack = reinterpret_cast<const SegPack *>(
            upload(packs.data(), packs.size() * sizeof(SegPack)));
        const SegPass *d_pass = passes.empty() ? nullptr
                                               : reinterpret_cast<const SegPass *>(upload(
                                                     passes.data(), passes.size() * sizeof(SegPass)));
        const SegGather *d_gather = reinterpret_cast<const SegGather *>(
            upload(gathers.data(), gathers.size() * sizeof(SegGather)));
        keep.emplace_back(ctx, std::max<uint64_t>(most_ranges, 1) * kRadix * sizeof(uint32_t));
        uint32_t *counts = keep.back().get<uint32_t>();
        auto grid_x = [](uint64_t n) {
            return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((n + 255) / 256, 1024));
        };
        for (int st = 0; st < max_groups; ++st) {
            const size_t a = step_packs[st].first, b = step_packs[st].second;
            uint64_t mn = 0;
            for (size_t x = a; x < b; ++x) mn = std::max(mn, packs[x].n);
            for (size_t y0 = a; y0 < b; y0 += 65535) {
                const unsigned gy = (unsigned)std::min<size_t>(65535, b - y0);
                hipLaunchKernelGGL(seg_pack, dim3(grid_x(mn), gy), dim3(256), 0, ctx->stream,
                                   d_pack + y0);
                TID_HIP(hipGetLastError());
            }
            for (const PassLaunch &L : step_passes[st]) {
                hipLaunchKernelGGL(seg_hist, dim3((unsigned)L.ranges), dim3(kSortBlock), 0,
                                   ctx->stream, d_pass + L.first, L.J, counts);
                TID_HIP(hipGetLastError());
                hipLaunchKernelGGL(seg_offsets, dim3((unsigned)L.J), dim3(kRadix * kSegParts), 0,
                                   ctx->stream, d_pass + L.first, counts);
                TID_HIP(hipGetLastError());
                hipLaunchKernelGGL(seg_scatter, dim3((unsigned)L.ranges), dim3(kSortBlock), 0,
                                   ctx->stream, d_pass + L.first, L.J, (const uint32_t *)counts);
                TID_HIP(hipGetLastError());
            }
        }
        for (int y0 = 0; y0 < J; y0 += 65535) {
            const unsigned gy = (unsigned)std::min(65535, J - y0);
            hipLaunchKernelGGL(seg_gather, dim3(grid_x(most_n), gy), dim3(256), 0, ctx->stream,
                               d_gather + y0);
            TID_HIP(hipGetLastError());
        }
    }
    keep.push_back(std::move(arena));
}

std::unique_ptr<tid_table> sort_table(tid_ctx *ctx, const tid_table *t, int distinct) {
    const uint64_t n = const_cast<tid_table *>(t)->rows();
    return sort_rows(ctx, t, n, distinct);
}

// Outer union: schema = ordered union of the inputs' variables; unbound cells 0.
std::unique_ptr<tid_table> union_tables(tid_ctx *ctx, const tid_table *const *ts, int k,
                                        int dedupe) {
    std::vector<int32_t> vars;
    for (int j = 0; j < k; ++j)
        for (int c = 0; c < ts[j]->ncols; ++c)
            if (std::find(vars.begin(), vars.end(), ts[j]->vars[c]) == vars.end())
                vars.push_back(ts[j]->vars[c]);
    TID_REQUIRE((int)vars.size() <= TID_MAX_COLS, TID_E_SCHEMA, "union: too many columns");
    std::vector<tid_table *> raw(k);
    for (int j = 0; j < k; ++j) raw[j] = const_cast<tid_table *>(ts[j]);
    resolve_counts(ctx, raw.data(), k);
    uint64_t total = 0;
    for (int j = 0; j < k; ++j) total += ts[j]->nrows;
    auto out = make_table(ctx, (int)vars.size(), vars.data(), total);
    out->maxv_known = true;
    for (size_t c = 0; c < vars.size(); ++c) {
        uint32_t m = 0;
        for (int j = 0; j < k; ++j)
            for (int x = 0; x < ts[j]->ncols; ++x)
                if (ts[j]->vars[x] == vars[c]) m = std::max(m, ts[j]->maxv[x]);
        out->maxv[c] = m;
    }
    for (int j = 0; j < k; ++j) out->maxv_known &= ts[j]->maxv_known;
    uint64_t at = 0;
    for (int j = 0; j < k; ++j) {
        const uint64_t n = ts[j]->nrows;
        if (!n) continue;
        for (size_t c = 0; c < vars.size(); ++c) {
            int src = -1;
            for (int x = 0; x < ts[j]->ncols; ++x)
                if (ts[j]->vars[x] == vars[c]) src = x;
            if (src >= 0)
                TID_HIP(hipMemcpyAsync(out->col[c] + at, ts[j]->col[src], n * 4,
                                       hipMemcpyDeviceToDevice, ctx->stream));
            else
                fill(ctx, out->col[c] + at, n, 0u);
        }
        at += n;
    }
    set_count(ctx, out.get(), total);
    if (!dedupe) return out;
    return sort_rows(ctx, out.get(), total, 1);
}

}  // namespace tid
