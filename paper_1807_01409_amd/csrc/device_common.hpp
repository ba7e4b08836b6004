// device_common.hpp -- wave64 primitives and the cross-workgroup sync words
// used by the single-pass kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

// Loop over the first n of at most MAXC output columns.  For small MAXC the
// loop is unrolled to MAXC steps with a guard, so that per-column constants
// indexed by c (source positions, column pointers) are loop-invariant loads
// the compiler can hoist, rather than loads repeated for every staged row.
#define TID_FOR_COLS(MAXC, c, n) \
    _Pragma("unroll") for (int c = 0; c < ((MAXC) <= 4 ? (MAXC) : (n)); ++c) if (c < (n))

namespace tid {
namespace dev {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// number of set bits of `mask` in lanes below the calling lane
__device__ __forceinline__ uint32_t rank_in_mask(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// 32-bit finaliser of MurmurHash3 (Appleby): every input bit affects every
// output bit
__device__ __forceinline__ uint32_t hash32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x85ebca6bu;
    x ^= x >> 13;
    x *= 0xc2b2ae35u;
    x ^= x >> 16;
    return x;
}

// Word-blocked Bloom filter of (mask + 1) bits, a power of two >= 32: a value
// sets two bits of one 32-bit word (the word from one hash, the two bit
// positions from a second), so a test is one load.  At 16 bits per value its
// false-positive rate is close to that of two independent positions.
__device__ __forceinline__ uint32_t bloom_word_bits(uint32_t x) {
    const uint32_t h2 = hash32(x ^ 0x9E3779B9u);
    return (1u << (h2 & 31u)) | (1u << ((h2 >> 8) & 31u));
}

__device__ __forceinline__ bool bloom_has(const uint32_t *bits, uint32_t mask, uint32_t x) {
    const uint32_t want = bloom_word_bits(x);
    return (bits[(hash32(x) & mask) >> 5] & want) == want;
}

__device__ __forceinline__ void bloom_add(uint32_t *bits, uint32_t mask, uint32_t x) {
    atomicOr(&bits[(hash32(x) & mask) >> 5], bloom_word_bits(x));
}

// Output rows of a compaction are written once and read by a later kernel:
// non-temporal stores, so they stream to memory instead of taking L2 lines
// that the graph's next tiles would use.
__device__ __forceinline__ void put(uint32_t *p, uint32_t v) { __builtin_nontemporal_store(v, p); }

// inclusive prefix sum across the wave
template <class T>
__device__ __forceinline__ T wave_inclusive_sum(T v) {
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        T o = __shfl_up(v, d, kWave);
        if (lane >= d) v += o;
    }
    return v;
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

// Words shared between workgroups of one kernel are written and read with
// agent-scope atomics so that workgroups on different XCDs (each with its own
// L2) see each other.
__device__ __forceinline__ void publish(uint64_t *word, uint64_t v) {
    __hip_atomic_store(word, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t peek(const uint64_t *word) {
    return __hip_atomic_load(const_cast<uint64_t *>(word), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace dev
}  // namespace tid
