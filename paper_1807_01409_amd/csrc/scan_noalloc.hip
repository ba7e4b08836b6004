// scan_noalloc.hip -- the single-pattern scan of Sec. 3 (GPUSearch) for
// callers that cannot allocate device memory: code under HIP graph capture,
// tight serving loops, harnesses that forbid allocation.  The caller brings
// the output columns and the row-count word; the kernel's cross-workgroup
// state lives in a fixed file-scope device array.
#include "scan_common.hpp"

#include <map>
#include <mutex>

namespace tid {

// ---------------------------------------------------------------------------
// Allocation-free scan.  The
// block-ranged kernel's cross-workgroup state (ticket and done counters, one
// epoch-stamped count word per range) and its two flag words live in a
// file-scope device array.  Its address is looked up once per device at
// context creation and kept; host code never passes the array's own name.
// Every call on a device shares the array: calls that overlap on one device
// (two streams, two threads) race and must not be issued.
// ---------------------------------------------------------------------------

// words: [0] ticket and done counters; [1, 1 + 4096] one count word per range
// (at most 512 x 8 = 4096 ranges per launch); [kNoAllocFlagWord] two flags
constexpr size_t kNoAllocRanges = 512 * kPrefixPer;
constexpr size_t kNoAllocFlagWord = 1 + kNoAllocRanges;
constexpr size_t kNoAllocWords = kNoAllocFlagWord + 1;
static __device__ __align__(256) uint64_t scratch[kNoAllocWords];

__global__ void fill_words(uint64_t *p, uint64_t n, uint64_t v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

namespace {
struct NoAllocDevice {
    uint64_t *ptr = nullptr;  // the device address of `scratch` on this device
};
std::mutex g_noalloc_mu;
std::map<int, NoAllocDevice> g_noalloc;
}  // namespace

// Once per device, with that device current: find the array's device
// address and clear it (a fill kernel, not a memset, so that the same code
// may run under graph capture).
void noalloc_init(tid_ctx *ctx) {
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    NoAllocDevice &d = g_noalloc[ctx->device];
    if (d.ptr) return;
    void *ptr = nullptr;
    TID_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    TID_REQUIRE(ptr != nullptr, TID_E_HIP, "no device address for the scan scratch array");
    hipLaunchKernelGGL(fill_words, dim3(8), dim3(256), 0, ctx->stream,
                       static_cast<uint64_t *>(ptr), (uint64_t)kNoAllocWords, 0ull);
    TID_HIP(hipGetLastError());
    TID_HIP(hipStreamSynchronize(ctx->stream));
    d.ptr = static_cast<uint64_t *>(ptr);
}

void scan_noalloc(tid_ctx *ctx, const tid_graph *g, const tid_pattern &p,
                  uint32_t *const *cols, int ncols, uint64_t cap, uint64_t *d_count) {
    int32_t vars[3], src[3];
    const int nc = pattern_schema(p, vars, src);
    TID_REQUIRE(ncols == nc, TID_E_INVALID_ARG,
                "scan_noalloc: ncols must be the pattern's column count");
    TID_REQUIRE(d_count, TID_E_INVALID_ARG, "scan_noalloc: null count pointer");
    for (int c = 0; c < nc; ++c)
        TID_REQUIRE(cols && cols[c], TID_E_INVALID_ARG, "scan_noalloc: null output column");
    uint64_t *base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_noalloc_mu);
        auto it = g_noalloc.find(ctx->device);
        TID_REQUIRE(it != g_noalloc.end() && it->second.ptr, TID_E_INTERNAL,
                    "scan_noalloc: scratch not set up on this device");
        base = it->second.ptr;
    }
    if (g->n == 0) {
        hipLaunchKernelGGL(fill_words, dim3(1), dim3(64), 0, ctx->stream, d_count, 1ull, 0ull);
        TID_HIP(hipGetLastError());
        return;
    }
    ScanSrc<1, false> sc{};
    CompactArgs<1, 3> a{};
    sc.g = g->triples();
    sc.n = g->n;
    sc.pat[0] = compile_pattern(p);
    for (int c = 0; c < nc; ++c) a.out[0].col[c] = cols[c];
    a.out[0].cap = cap;
    a.out[0].count = d_count;
    a.out[0].ncols = nc;
    const uint32_t sw = 16384u;
    const size_t words = block_ranged_layout<ScanSrc<1, false>, 512, 8, 1, 3, true>(ctx, sc, a, 1,
                                                                                     sw);
    TID_REQUIRE(words <= kNoAllocFlagWord, TID_E_CAPACITY,
                "scan_noalloc: the launch needs more ranges than the scratch array holds");
    // Every call clears the words its launch uses (a fill kernel, not a
    // memset) and stamps them with epoch 1: the same launch sequence is then
    // correct when recorded once in a HIP graph and replayed, whatever ran on
    // the device in between.
    hipLaunchKernelGGL(fill_words, dim3(8), dim3(256), 0, ctx->stream, base, (uint64_t)words, 0ull);
    TID_HIP(hipGetLastError());
    a.epoch = 1;
    block_ranged_launch<ScanSrc<1, false>, 512, 8, 1, 3, true>(
        ctx, sc, a, sw, base, reinterpret_cast<uint32_t *>(base + kNoAllocFlagWord));
}

}  // namespace tid
