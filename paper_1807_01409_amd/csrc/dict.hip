// dict.hip -- dictionary encoding of string triples into TripleID rows, and
// decoding of IDs back to strings (Sec. 3: the conversion of an RDF file into
// ID dictionaries and rows of three 32-bit IDs, done there in one linear pass
// with hash tables on the host).
//
// Encoding on the GPU, one shared dictionary, IDs from 1 in order of first
// appearance when the terms are read s, p, o, triple by triple:
//   1. hash every term (64-bit FNV-1a over its bytes);
//   2. radix-sort (hash, term index) pairs -- stable, so each group of equal
//      hashes lists its terms in reading order and its first element is the
//      term's first appearance;
//   3. check that every term of a group is byte-equal to the group's first
//      (a 64-bit collision between different strings is reported as an
//      error, never silently merged);
//   4. sort the groups' first appearances: a group's rank in that order is
//      its ID - 1; scatter each term's ID to its row and position;
//   5. copy each distinct term's bytes, in ID order, into the dictionary.
// Decoding gathers the strings of a column of IDs (lengths, offsets by an
// exclusive scan, bytes).
#include "compact.hpp"

#include <algorithm>

namespace tid {

bool radix_sort_pairs(tid_ctx *ctx, uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1,
                      uint64_t n, int bits);
void iota(tid_ctx *ctx, uint32_t *p, uint64_t n);
void exclusive_scan_async(tid_ctx *ctx, const uint32_t *in, uint64_t n, uint64_t *out);
void read_words(tid_ctx *ctx, const std::vector<const uint64_t *> &src, uint64_t *dst);

namespace {

unsigned grid_of(uint64_t n) {
    return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((n + 255) / 256, 16384));
}

#define TID_GRID_LOOP(i, n)                                                              \
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n);          \
         i += (uint64_t)gridDim.x * blockDim.x)

// FNV-1a, 64 bits (Fowler, Noll, Vo)
__global__ void hash_terms(const uint8_t *bytes, const uint64_t *off, uint64_t m, uint64_t *h,
                           uint32_t *idx) {
    TID_GRID_LOOP(t, m) {
        uint64_t x = 0xcbf29ce484222325ull;
        for (uint64_t b = off[t]; b < off[t + 1]; ++b) {
            x ^= bytes[b];
            x *= 0x100000001b3ull;
        }
        h[t] = x;
        idx[t] = (uint32_t)t;
    }
}

// first[i] = 1 where sorted position i starts a group of equal hashes
__global__ void group_starts(const uint64_t *h, uint64_t m, uint32_t *first) {
    TID_GRID_LOOP(i, m) first[i] = (i == 0 || h[i] != h[i - 1]) ? 1u : 0u;
}

// gstart (exclusive scan of `first`): group g starts at the i with
// first[i] = 1 and gstart[i] = g; lead[g] = the term index there
__global__ void group_leads(const uint32_t *first, const uint64_t *gstart, const uint32_t *term,
                            uint64_t m, uint32_t *lead) {
    TID_GRID_LOOP(i, m) if (first[i]) lead[gstart[i]] = term[i];
}

__device__ __forceinline__ uint64_t group_of(const uint32_t *first, const uint64_t *gstart,
                                             uint64_t i) {
    return gstart[i] + first[i] - 1;  // inclusive count of group starts, minus one
}

// every term byte-equal to its group's first term; flag set otherwise
__global__ void check_groups(const uint8_t *bytes, const uint64_t *off, const uint32_t *first,
                             const uint64_t *gstart, const uint32_t *term, const uint32_t *lead,
                             uint64_t m, uint32_t *flag) {
    TID_GRID_LOOP(i, m) {
        if (first[i]) continue;
        const uint32_t a = term[i], b = lead[group_of(first, gstart, i)];
        const uint64_t la = off[a + 1] - off[a], lb = off[b + 1] - off[b];
        bool eq = la == lb;
        for (uint64_t k = 0; eq && k < la; ++k) eq = bytes[off[a] + k] == bytes[off[b] + k];
        if (!eq) atomicOr(flag, 1u);
    }
}

__global__ void widen_leads(const uint32_t *lead, uint64_t d, uint64_t *key, uint32_t *val) {
    TID_GRID_LOOP(g, d) {
        key[g] = lead[g];
        val[g] = (uint32_t)g;
    }
}

// group_sorted[r] = the group whose first appearance has rank r: its ID is r + 1
__global__ void group_ids(const uint32_t *group_sorted, uint64_t d, uint32_t *id_of) {
    TID_GRID_LOOP(r, d) id_of[group_sorted[r]] = (uint32_t)(r + 1);
}

__global__ void scatter_ids(const uint32_t *first, const uint64_t *gstart, const uint32_t *term,
                            const uint32_t *id_of, uint64_t m, uint32_t *rows) {
    TID_GRID_LOOP(i, m) rows[term[i]] = id_of[group_of(first, gstart, i)];
}

// lengths of the distinct terms in ID order (term of ID r + 1 is first[r])
__global__ void id_lengths(const uint64_t *first_sorted, const uint64_t *off, uint64_t d,
                           uint32_t *len) {
    TID_GRID_LOOP(r, d) {
        const uint64_t t = first_sorted[r];
        len[r] = (uint32_t)(off[t + 1] - off[t]);
    }
}

__global__ void copy_terms(const uint64_t *first_sorted, const uint8_t *bytes, const uint64_t *off,
                           const uint64_t *doff, uint64_t d, uint8_t *dbytes) {
    TID_GRID_LOOP(r, d) {
        const uint64_t t = first_sorted[r];
        for (uint64_t k = 0; k < off[t + 1] - off[t]; ++k) dbytes[doff[r] + k] = bytes[off[t] + k];
    }
}

__global__ void decode_lengths(const uint32_t *ids, uint64_t n, const uint64_t *doff,
                               uint64_t nterms, uint32_t *len, uint32_t *flag) {
    TID_GRID_LOOP(i, n) {
        const uint32_t id = ids[i];
        if (id == 0 || id > nterms) {
            atomicOr(flag, 1u);
            len[i] = 0;
        } else {
            len[i] = (uint32_t)(doff[id] - doff[id - 1]);
        }
    }
}

__global__ void decode_copy(const uint32_t *ids, uint64_t n, const uint64_t *doff,
                            const uint8_t *dbytes, uint64_t nterms, const uint64_t *out_off,
                            uint8_t *out) {
    TID_GRID_LOOP(i, n) {
        const uint32_t id = ids[i];
        if (id == 0 || id > nterms) continue;
        const uint64_t a = doff[id - 1], l = doff[id] - a;
        for (uint64_t k = 0; k < l; ++k) out[out_off[i] + k] = dbytes[a + k];
    }
}

int bitw64(uint64_t v) { return v ? 64 - __builtin_clzll(v) : 0; }

}  // namespace

std::unique_ptr<tid_dict> encode(tid_ctx *ctx, const uint8_t *bytes, uint64_t nbytes,
                                 const uint64_t *offsets, uint64_t n, int on_device,
                                 uint32_t *rows) {
    TID_REQUIRE(n < (1ull << 32) / 3, TID_E_UNSUPPORTED, "encode: too many triples");
    TID_REQUIRE(n == 0 || (offsets && rows), TID_E_INVALID_ARG, "encode: null argument");
    TID_REQUIRE(nbytes == 0 || bytes, TID_E_INVALID_ARG, "encode: null bytes");
    const uint64_t m = 3 * n;
    auto dict = std::make_unique<tid_dict>();
    dict->ctx = ctx;
    // inputs on the device
    DevBuf dbytes_in(ctx, std::max<uint64_t>(nbytes, 1)), doff_in(ctx, (m + 1) * 8);
    const auto kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    if (nbytes) TID_HIP(hipMemcpyAsync(dbytes_in.get(), bytes, nbytes, kind, ctx->stream));
    if (n) {
        TID_HIP(hipMemcpyAsync(doff_in.get(), offsets, (m + 1) * 8, kind, ctx->stream));
        // offsets must rise and stay within the bytes: checked on the host copy
        std::vector<uint64_t> ho(m + 1);
        TID_HIP(hipMemcpyAsync(ho.data(), doff_in.get(), (m + 1) * 8, hipMemcpyDeviceToHost,
                               ctx->stream));
        TID_HIP(hipStreamSynchronize(ctx->stream));
        for (uint64_t t = 0; t < m; ++t)
            TID_REQUIRE(ho[t] <= ho[t + 1], TID_E_INVALID_ARG, "encode: offsets must not fall");
        TID_REQUIRE(ho[m] <= nbytes, TID_E_INVALID_ARG, "encode: offsets past the bytes");
    }
    if (m == 0) {
        dict->offsets = DevBuf(ctx, 8);
        TID_HIP(hipMemsetAsync(dict->offsets.get(), 0, 8, ctx->stream));
        TID_HIP(hipStreamSynchronize(ctx->stream));
        return dict;
    }
    const uint8_t *B = dbytes_in.get<const uint8_t>();
    const uint64_t *O = doff_in.get<const uint64_t>();
    // 1-2: hash, then sort (hash, term) pairs
    DevBuf h0(ctx, m * 8), h1(ctx, m * 8), t0(ctx, m * 4), t1(ctx, m * 4);
    hipLaunchKernelGGL(hash_terms, dim3(grid_of(m)), dim3(256), 0, ctx->stream, B, O, m,
                       h0.get<uint64_t>(), t0.get<uint32_t>());
    TID_HIP(hipGetLastError());
    const bool moved = radix_sort_pairs(ctx, h0.get<uint64_t>(), t0.get<uint32_t>(),
                                        h1.get<uint64_t>(), t1.get<uint32_t>(), m, 64);
    const uint64_t *H = moved ? h1.get<const uint64_t>() : h0.get<const uint64_t>();
    const uint32_t *T = moved ? t1.get<const uint32_t>() : t0.get<const uint32_t>();
    // groups of equal hashes and their first terms
    DevBuf first(ctx, m * 4), gstart(ctx, (m + 1) * 8);
    hipLaunchKernelGGL(group_starts, dim3(grid_of(m)), dim3(256), 0, ctx->stream, H, m,
                       first.get<uint32_t>());
    TID_HIP(hipGetLastError());
    exclusive_scan_async(ctx, first.get<const uint32_t>(), m, gstart.get<uint64_t>());
    uint64_t d = 0;
    read_words(ctx, {gstart.get<const uint64_t>() + m}, &d);
    DevBuf lead(ctx, d * 4);
    hipLaunchKernelGGL(group_leads, dim3(grid_of(m)), dim3(256), 0, ctx->stream,
                       first.get<const uint32_t>(), gstart.get<const uint64_t>(), T, m,
                       lead.get<uint32_t>());
    TID_HIP(hipGetLastError());
    // 3: every term equal to its group's first (no silent collision)
    DevBuf flag(ctx, 8);
    TID_HIP(hipMemsetAsync(flag.get(), 0, 8, ctx->stream));
    hipLaunchKernelGGL(check_groups, dim3(grid_of(m)), dim3(256), 0, ctx->stream, B, O,
                       first.get<const uint32_t>(), gstart.get<const uint64_t>(), T,
                       lead.get<const uint32_t>(), m, flag.get<uint32_t>());
    TID_HIP(hipGetLastError());
    uint64_t bad = 0;
    read_words(ctx, {flag.get<const uint64_t>()}, &bad);
    TID_REQUIRE(bad == 0, TID_E_UNSUPPORTED,
                "encode: two different terms share a 64-bit hash; not encoded");
    // 4: IDs by first appearance
    DevBuf k0(ctx, d * 8), k1(ctx, d * 8), g0(ctx, d * 4), g1(ctx, d * 4);
    hipLaunchKernelGGL(widen_leads, dim3(grid_of(d)), dim3(256), 0, ctx->stream,
                       lead.get<const uint32_t>(), d, k0.get<uint64_t>(), g0.get<uint32_t>());
    TID_HIP(hipGetLastError());
    const bool mv = radix_sort_pairs(ctx, k0.get<uint64_t>(), g0.get<uint32_t>(),
                                     k1.get<uint64_t>(), g1.get<uint32_t>(), d, bitw64(m));
    const uint64_t *first_sorted = mv ? k1.get<const uint64_t>() : k0.get<const uint64_t>();
    const uint32_t *group_sorted = mv ? g1.get<const uint32_t>() : g0.get<const uint32_t>();
    DevBuf id_of(ctx, d * 4);
    hipLaunchKernelGGL(group_ids, dim3(grid_of(d)), dim3(256), 0, ctx->stream, group_sorted, d,
                       id_of.get<uint32_t>());
    TID_HIP(hipGetLastError());
    hipLaunchKernelGGL(scatter_ids, dim3(grid_of(m)), dim3(256), 0, ctx->stream,
                       first.get<const uint32_t>(), gstart.get<const uint64_t>(), T,
                       id_of.get<const uint32_t>(), m, rows);
    TID_HIP(hipGetLastError());
    // 5: the dictionary, terms in ID order
    DevBuf len(ctx, d * 4);
    dict->offsets = DevBuf(ctx, (d + 1) * 8);
    hipLaunchKernelGGL(id_lengths, dim3(grid_of(d)), dim3(256), 0, ctx->stream, first_sorted, O,
                       d, len.get<uint32_t>());
    TID_HIP(hipGetLastError());
    exclusive_scan_async(ctx, len.get<const uint32_t>(), d, dict->offsets.get<uint64_t>());
    uint64_t total = 0;
    read_words(ctx, {dict->offsets.get<const uint64_t>() + d}, &total);
    dict->bytes = DevBuf(ctx, std::max<uint64_t>(total, 1));
    hipLaunchKernelGGL(copy_terms, dim3(grid_of(d)), dim3(256), 0, ctx->stream, first_sorted, B,
                       O, dict->offsets.get<const uint64_t>(), d, dict->bytes.get<uint8_t>());
    TID_HIP(hipGetLastError());
    TID_HIP(hipStreamSynchronize(ctx->stream));
    dict->n_terms = d;
    dict->n_bytes = total;
    return dict;
}

// Strings of n IDs, to host buffers: out_off gets n + 1 offsets (always);
// the bytes only if they fit cap_bytes (else TID_E_CAPACITY, the total in
// out_off[n]).  An ID of 0 or above the dictionary's size is refused.
void decode(tid_ctx *ctx, const tid_dict *dict, const uint32_t *ids, uint64_t n, int on_device,
            uint64_t *out_off, uint8_t *out, uint64_t cap_bytes) {
    TID_REQUIRE(out_off, TID_E_INVALID_ARG, "decode: null offsets");
    if (n == 0) {
        out_off[0] = 0;
        return;
    }
    TID_REQUIRE(ids, TID_E_INVALID_ARG, "decode: null ids");
    DevBuf did;
    const uint32_t *I = ids;
    if (!on_device) {
        did = DevBuf(ctx, n * 4);
        TID_HIP(hipMemcpyAsync(did.get(), ids, n * 4, hipMemcpyHostToDevice, ctx->stream));
        I = did.get<const uint32_t>();
    }
    DevBuf len(ctx, n * 4), off(ctx, (n + 1) * 8), flag(ctx, 8);
    TID_HIP(hipMemsetAsync(flag.get(), 0, 8, ctx->stream));
    hipLaunchKernelGGL(decode_lengths, dim3(grid_of(n)), dim3(256), 0, ctx->stream, I, n,
                       dict->offsets.get<const uint64_t>(), dict->n_terms, len.get<uint32_t>(),
                       flag.get<uint32_t>());
    TID_HIP(hipGetLastError());
    exclusive_scan_async(ctx, len.get<const uint32_t>(), n, off.get<uint64_t>());
    TID_HIP(hipMemcpyAsync(out_off, off.get(), (n + 1) * 8, hipMemcpyDeviceToHost, ctx->stream));
    uint64_t bad = 0;
    TID_HIP(hipMemcpyAsync(&bad, flag.get(), 8, hipMemcpyDeviceToHost, ctx->stream));
    TID_HIP(hipStreamSynchronize(ctx->stream));
    TID_REQUIRE(bad == 0, TID_E_INVALID_ARG, "decode: an ID is 0 or not in the dictionary");
    const uint64_t total = out_off[n];
    TID_REQUIRE(total <= cap_bytes, TID_E_CAPACITY, "decode: the strings need more bytes");
    if (total == 0) return;
    TID_REQUIRE(out, TID_E_INVALID_ARG, "decode: null output bytes");
    DevBuf dout(ctx, total);
    hipLaunchKernelGGL(decode_copy, dim3(grid_of(n)), dim3(256), 0, ctx->stream, I, n,
                       dict->offsets.get<const uint64_t>(), dict->bytes.get<const uint8_t>(),
                       dict->n_terms, off.get<const uint64_t>(), dout.get<uint8_t>());
    TID_HIP(hipGetLastError());
    TID_HIP(hipMemcpyAsync(out, dout.get(), total, hipMemcpyDeviceToHost, ctx->stream));
    TID_HIP(hipStreamSynchronize(ctx->stream));
}

}  // namespace tid
