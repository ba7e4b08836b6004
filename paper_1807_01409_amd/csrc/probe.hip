// probe.hip -- a plain streaming read of device memory, the ceiling the scan
// is measured against.  It reads the same bytes the scan reads with the same
// access shape (one 12-byte non-temporal load per lane per triple, tiles of
// 512 x 8 triples, one contiguous range per resident workgroup), or with one
// 16-byte load per lane, and does nothing with them beyond an xor folded into
// one word, so its time is the time of the reads alone.
#include "device_common.hpp"
#include "internal.hpp"

#include <algorithm>

namespace tid {

int device_cus(tid_ctx *ctx);
int resident_blocks(const void *kernel, int block, size_t lds);

namespace {

constexpr int kProbeBlock = 512;
constexpr int kProbeItems = 8;

// mode 0: n items of 12 bytes (triples); mode 1: n items of 16 bytes
template <int MODE>
__global__ __launch_bounds__(kProbeBlock) void read_probe_kernel(const uint32_t *__restrict__ p,
                                                                 uint64_t n, uint64_t range,
                                                                 uint32_t *sink) {
    constexpr uint64_t TILE = (uint64_t)kProbeBlock * kProbeItems;
    const uint64_t r0 = (uint64_t)blockIdx.x * range;
    const uint64_t r1 = min(n, r0 + range);
    uint32_t acc = 0;
    for (uint64_t t0 = r0; t0 < r1; t0 += TILE) {
#pragma unroll
        for (int it = 0; it < kProbeItems; ++it) {
            const uint64_t i = t0 + (uint64_t)it * kProbeBlock + threadIdx.x;
            if (i >= r1) continue;
            if (MODE == 0) {
                acc ^= __builtin_nontemporal_load(p + 3 * i) ^
                       __builtin_nontemporal_load(p + 3 * i + 1) ^
                       __builtin_nontemporal_load(p + 3 * i + 2);
            } else {
                typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
                const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p) + i);
                acc ^= v.x ^ v.y ^ v.z ^ v.w;
            }
        }
    }
    // one word per launch; a value no read can produce keeps the loads live
    if (acc == 0x9E3779B9u) atomicXor(sink, acc);
}

}  // namespace

void read_probe(tid_ctx *ctx, const void *ptr, uint64_t bytes, int mode) {
    TID_REQUIRE(mode == 0 || mode == 1, TID_E_INVALID_ARG, "read probe: mode must be 0 or 1");
    TID_REQUIRE(ptr || bytes == 0, TID_E_INVALID_ARG, "read probe: null pointer");
    const uint64_t item = mode == 0 ? 12 : 16;
    const uint64_t n = bytes / item;
    if (n == 0) return;
    TID_REQUIRE(mode == 0 || reinterpret_cast<uintptr_t>(ptr) % 16 == 0, TID_E_INVALID_ARG,
                "read probe: 16-byte loads need a 16-byte aligned pointer");
    auto kern = mode == 0 ? read_probe_kernel<0> : read_probe_kernel<1>;
    const uint64_t tile = (uint64_t)kProbeBlock * kProbeItems;
    const uint64_t tiles = (n + tile - 1) / tile;
    const uint64_t resident =
        (uint64_t)resident_blocks((const void *)kern, kProbeBlock, 0) * (uint64_t)device_cus(ctx);
    uint64_t P = std::max<uint64_t>(1, std::min(tiles, resident));
    const uint64_t range = (tiles + P - 1) / P * tile;
    P = (n + range - 1) / range;
    hipLaunchKernelGGL(kern, dim3((uint32_t)P), dim3(kProbeBlock), 0, ctx->stream,
                       static_cast<const uint32_t *>(ptr), n, range, ctx->d_flags + 2);
    TID_HIP(hipGetLastError());
}

}  // namespace tid
