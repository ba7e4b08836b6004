// device_common.hpp -- wave64 primitives and the cross-workgroup sync words
// used by the single-pass kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

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

// End of a kernel that uses sync words, called by every thread of every
// workgroup.  The sync words are all zero when a kernel starts: the workgroup
// that finishes last (counted on counters[1]) clears the `nwords` words and
// the `ncounters` counter words for the next launch.  Every other workgroup has made its last state access
// before its increment of done.
__device__ __forceinline__ void release_state(uint64_t *state, size_t nwords,
                                              uint32_t *counters, uint32_t num_tiles,
                                              int ncounters = 2) {
    __shared__ int s_last;
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const uint32_t d = __hip_atomic_fetch_add(&counters[1], 1u, __ATOMIC_ACQ_REL,
                                                  __HIP_MEMORY_SCOPE_AGENT);
        s_last = d == num_tiles - 1;
    }
    __syncthreads();
    if (s_last) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        for (size_t i = threadIdx.x; i < nwords; i += blockDim.x) state[i] = 0;
        for (int i = threadIdx.x; i < ncounters; i += blockDim.x) counters[i] = 0;
    }
}

}  // namespace dev
}  // namespace tid
