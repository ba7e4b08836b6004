// capi.hip -- the extern "C" boundary declared in include/tid.h.  Each entry
// point validates its arguments, runs the library code, and turns any
// internal error into a status code plus a message on the context.
#include "internal.hpp"

#include <cstdio>
#include <fstream>

using tid::Error;

namespace {

template <class F>
tid_status guarded(tid_ctx *ctx, F &&f) {
    try {
        f();
        if (ctx) ctx->last_error.clear();
        return TID_OK;
    } catch (const Error &e) {
        if (ctx) ctx->last_error = e.what();
        return e.code;
    } catch (const std::bad_alloc &) {
        if (ctx) ctx->last_error = "host allocation failed";
        return TID_E_OOM;
    } catch (const std::exception &e) {
        if (ctx) ctx->last_error = e.what();
        return TID_E_INTERNAL;
    }
}

void check_ctx(tid_ctx *ctx) {
    if (!ctx) throw Error(TID_E_INVALID_ARG, "null context");
    TID_HIP(hipSetDevice(ctx->device));
}

}  // namespace

namespace tid {
// operators implemented in other translation units (stubs until built)
std::unique_ptr<tid_table> join_tables(tid_ctx *, const tid_table *, int, const tid_table *, int,
                                       int);
std::unique_ptr<tid_table> union_tables(tid_ctx *, const tid_table *const *, int, int);
std::unique_ptr<tid_table> scan_keyed(tid_ctx *, const tid_graph *, const tid_pattern &, int,
                                      const uint32_t *, uint64_t);
std::unique_ptr<tid_table> entail(tid_ctx *, const tid_graph *, int, const uint32_t *);
void partition_graph(tid_ctx *, tid_graph *, bool);
tid_server *serve_open(tid_ctx *, const tid_graph *, uint32_t, uint32_t);
uint64_t serve_submit(tid_server *, const tid_plan *);
std::vector<uint64_t> serve_step(tid_server *);
void serve_free(tid_server *);
tid_ctx *serve_ctx(const tid_server *);
uint32_t serve_slots(const tid_server *);
void serve_info(const tid_server *, int32_t *, int32_t *, int32_t *);
tid_status serve_take(tid_server *, uint64_t, tid_table **, std::string *);
std::unique_ptr<tid_dict> encode(tid_ctx *, const uint8_t *, uint64_t, const uint64_t *, uint64_t,
                                 int, uint32_t *);
void decode(tid_ctx *, const tid_dict *, const uint32_t *, uint64_t, int, uint64_t *, uint8_t *,
            uint64_t);
std::unique_ptr<tid_table> join_tables_kind(tid_ctx *, const tid_table *, int, const tid_table *,
                                            int, int, int);
std::unique_ptr<tid_table> sort_table(tid_ctx *, const tid_table *, int);
std::unique_ptr<tid_table> run_query(tid_ctx *, const tid_graph *, const tid_plan *);
std::vector<std::unique_ptr<tid_table>> run_plans(
    tid_ctx *, const tid_graph *, const tid_plan *const *, int,
    std::vector<std::vector<std::unique_ptr<tid_table>>> * = nullptr);
uint64_t estimate_plan_bytes(const tid_graph *, const tid_plan *);
void read_probe(tid_ctx *, const void *, uint64_t, int);
void noalloc_init(tid_ctx *);
void scan_noalloc(tid_ctx *, const tid_graph *, const tid_pattern &, uint32_t *const *, int,
                  uint64_t, uint64_t *);
std::unique_ptr<tid_table> copy_columns(tid_ctx *, const uint32_t *const *, int32_t,
                                        const int32_t *, uint64_t, int);
}  // namespace tid

extern "C" {

tid_status tid_ctx_create(int device, void *stream, tid_alloc_fn alloc, tid_free_fn free_fn,
                          void *user, tid_ctx **out) {
    if (!out) return TID_E_INVALID_ARG;
    if ((alloc == nullptr) != (free_fn == nullptr)) return TID_E_INVALID_ARG;
    tid_ctx *ctx = new (std::nothrow) tid_ctx();
    if (!ctx) return TID_E_OOM;
    tid_status st = guarded(ctx, [&] {
        int ndev = 0;
        TID_HIP(hipGetDeviceCount(&ndev));
        TID_REQUIRE(device >= 0 && device < ndev, TID_E_INVALID_ARG, "no such device");
        ctx->device = device;
        TID_HIP(hipSetDevice(device));
        if (stream) {
            ctx->stream = static_cast<hipStream_t>(stream);
        } else {
            TID_HIP(hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking));
            ctx->own_stream = true;
        }
        ctx->alloc_fn = alloc;
        ctx->free_fn = free_fn;
        ctx->user = user;
        // words 0-1: error and overflow flags; word 2: the read probe's sink
        ctx->d_flags = static_cast<uint32_t *>(ctx->alloc(4 * sizeof(uint32_t)));
        TID_HIP(hipMemsetAsync(ctx->d_flags, 0, 4 * sizeof(uint32_t), ctx->stream));
        TID_HIP(hipStreamSynchronize(ctx->stream));
        // once per device: the allocation-free scan's state array
        tid::noalloc_init(ctx);
    });
    if (st != TID_OK) {
        tid_ctx_destroy(ctx);
        return st;
    }
    *out = ctx;
    return TID_OK;
}

void tid_ctx_destroy(tid_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    if (ctx->ep_state) ctx->free(ctx->ep_state, ctx->ep_bytes);
    if (ctx->d_flags) ctx->free(ctx->d_flags, 4 * sizeof(uint32_t));
    if (ctx->rw_dev) ctx->free(ctx->rw_dev, ctx->rw_cap * 16);
    if (ctx->rw_host_ptrs) (void)hipHostFree(ctx->rw_host_ptrs);
    if (ctx->rw_host_vals) (void)hipHostFree(ctx->rw_host_vals);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

const char *tid_last_error(const tid_ctx *ctx) { return ctx ? ctx->last_error.c_str() : ""; }

tid_status tid_ctx_synchronize(tid_ctx *ctx) {
    return guarded(ctx, [&] {
        check_ctx(ctx);
        ctx->sync();
    });
}

tid_status tid_ctx_set_option(tid_ctx *ctx, const char *key, int64_t value) {
    return guarded(ctx, [&] {
        check_ctx(ctx);
        TID_REQUIRE(key, TID_E_INVALID_ARG, "null option name");
        const std::string k(key);
        if (k == "capacity_override") {
            TID_REQUIRE(value >= 0, TID_E_INVALID_ARG, "capacity_override must be >= 0");
            ctx->opt.capacity_override = value;
        } else if (k == "retry") {
            ctx->opt.retry = value ? 1 : 0;
        } else if (k == "scan_items") {
            ctx->opt.scan_items = value;
        } else if (k == "scan_block") {
            ctx->opt.scan_block = value;
        } else if (k == "multi_kernel") {
            TID_REQUIRE(value == 0 || value == 1, TID_E_INVALID_ARG, "multi_kernel is 0 or 1");
            ctx->opt.multi_kernel = value;
        } else if (k == "multi_shape") {
            TID_REQUIRE(value >= 0 && value <= 3, TID_E_INVALID_ARG, "multi_shape is 0..3");
            ctx->opt.multi_shape = value;
        } else if (k == "range_factor") {
            TID_REQUIRE(value >= 1 && value <= 8, TID_E_INVALID_ARG, "range_factor is 1..8");
            ctx->opt.range_factor = value;
        } else if (k == "semijoin") {
            ctx->opt.semijoin = value ? 1 : 0;
        } else if (k == "semijoin_min") {
            TID_REQUIRE(value >= 0, TID_E_INVALID_ARG, "semijoin_min must be >= 0");
            ctx->opt.semijoin_min = value;
        } else if (k == "wide_slice") {
            ctx->opt.wide_slice = value ? 1 : 0;
        } else if (k == "slice_rows") {
            TID_REQUIRE(value >= 0, TID_E_INVALID_ARG, "slice_rows must be >= 0");
            ctx->opt.slice_rows = value;
        } else if (k == "layout") {
            TID_REQUIRE(value == 0 || value == 1, TID_E_INVALID_ARG, "layout must be 0 or 1");
            ctx->opt.layout = value;
        } else if (k == "index_semijoin") {
            TID_REQUIRE(value == 0 || value == 1, TID_E_INVALID_ARG,
                        "index_semijoin must be 0 or 1");
            ctx->opt.index_semijoin = value;
        } else if (k == "index_ratio") {
            TID_REQUIRE(value >= 0 && value <= (1 << 20), TID_E_INVALID_ARG,
                        "index_ratio must be in 0..2^20");
            ctx->opt.index_ratio = value;
        } else if (k == "chunk_epoch") {
            TID_REQUIRE(value >= 0 && value <= (int64_t)tid::kEpochMax, TID_E_INVALID_ARG,
                        "chunk_epoch is 0..2^23-1");
            ctx->epoch = (uint32_t)value;
        } else if (k == "compact_kernel") {
            TID_REQUIRE(value >= 0 && value <= 2, TID_E_INVALID_ARG, "compact_kernel is 0, 1 or 2");
            ctx->opt.compact_kernel = value;
        } else if (k == "scan_prefetch") {
            ctx->opt.scan_prefetch = value < 0 ? -1 : (value ? 1 : 0);
        } else if (k == "wide_min") {
            TID_REQUIRE(value >= 0, TID_E_INVALID_ARG, "wide_min must be >= 0");
            ctx->opt.wide_min = value;
        } else if (k == "stage_words") {
            TID_REQUIRE(value >= 0 && value <= 40448, TID_E_INVALID_ARG,
                        "stage_words must be in 0..40448");
            ctx->opt.stage_words = value;
        } else {
            throw Error(TID_E_INVALID_ARG, "unknown option " + k);
        }
    });
}

tid_status tid_ctx_get_option(tid_ctx *ctx, const char *key, int64_t *value) {
    return guarded(ctx, [&] {
        check_ctx(ctx);
        TID_REQUIRE(key && value, TID_E_INVALID_ARG, "null argument");
        const std::string k(key);
        if (k == "capacity_override") *value = ctx->opt.capacity_override;
        else if (k == "retry") *value = ctx->opt.retry;
        else if (k == "scan_items") *value = ctx->opt.scan_items;
        else if (k == "scan_block") *value = ctx->opt.scan_block;
        else if (k == "stage_words") *value = ctx->opt.stage_words;
        else if (k == "wide_min") *value = ctx->opt.wide_min;
        else if (k == "scan_prefetch") *value = ctx->opt.scan_prefetch;
        else if (k == "multi_kernel") *value = ctx->opt.multi_kernel;
        else if (k == "multi_shape") *value = ctx->opt.multi_shape;
        else if (k == "compact_kernel") *value = ctx->opt.compact_kernel;
        else if (k == "chunk_epoch") *value = ctx->epoch;
        else if (k == "semijoin") *value = ctx->opt.semijoin;
        else if (k == "range_factor") *value = ctx->opt.range_factor;
        else if (k == "semijoin_min") *value = ctx->opt.semijoin_min;
        else if (k == "wide_slice") *value = ctx->opt.wide_slice;
        else if (k == "slice_rows") *value = ctx->opt.slice_rows;
        else if (k == "layout") *value = ctx->opt.layout;
        else if (k == "index_semijoin") *value = ctx->opt.index_semijoin;
        else if (k == "index_ratio") *value = ctx->opt.index_ratio;
        else throw Error(TID_E_INVALID_ARG, "unknown option " + k);
    });
}

tid_status tid_load(tid_ctx *ctx, const uint32_t *triples, uint64_t n, int src_on_device,
                    tid_graph **out) {
    std::unique_ptr<tid_graph> g;
    tid_status st = guarded(ctx, [&] {
        check_ctx(ctx);
        TID_REQUIRE(out, TID_E_INVALID_ARG, "null output");
        TID_REQUIRE(n == 0 || triples, TID_E_INVALID_ARG, "null triples");
        g = std::make_unique<tid_graph>();
        g->ctx = ctx;
        g->n = n;
        const size_t bytes = (size_t)n * 12;
        g->data = tid::DevBuf(ctx, bytes + 64);
        if (bytes)
            TID_HIP(hipMemcpyAsync(g->data.get(), triples, bytes,
                                   src_on_device ? hipMemcpyDeviceToDevice
                                                 : hipMemcpyHostToDevice,
                                   ctx->stream));
        TID_HIP(hipMemsetAsync(g->data.get<char>() + bytes, 0, 64, ctx->stream));
        tid::build_stats(ctx, g.get());
        ctx->sync();
    });
    if (st == TID_OK) *out = g.release();
    return st;
}

tid_status tid_load_file(tid_ctx *ctx, const char *path, tid_graph **out) {
    std::vector<uint32_t> host;
    tid_status st = guarded(ctx, [&] {
        check_ctx(ctx);
        TID_REQUIRE(path && out, TID_E_INVALID_ARG, "null argument");
        std::ifstream f(path, std::ios::binary | std::ios::ate);
        TID_REQUIRE(f.good(), TID_E_INVALID_ARG, std::string("cannot open ") + path);
        const std::streamoff sz = f.tellg();
        TID_REQUIRE(sz % 12 == 0, TID_E_INVALID_ARG, "file size is not a multiple of 12 bytes");
        host.resize((size_t)sz / 4);
        f.seekg(0);
        if (sz) f.read(reinterpret_cast<char *>(host.data()), sz);
        TID_REQUIRE(f.good(), TID_E_INVALID_ARG, "short read");
    });
    if (st != TID_OK) return st;
    return tid_load(ctx, host.data(), host.size() / 3, 0, out);
}

tid_status tid_graph_info(const tid_graph *g, uint64_t *n, const uint32_t **device_triples) {
    if (!g) return TID_E_INVALID_ARG;
    if (n) *n = g->n;
    if (device_triples) *device_triples = g->data.get<const uint32_t>();
    return TID_OK;
}

tid_status tid_graph_count(const tid_graph *g, int32_t pos, uint32_t lo, uint32_t hi,
                           uint64_t *count) {
    if (!g || !count || pos < 0 || pos > 2) return TID_E_INVALID_ARG;
    if (g->n && g->cdf[pos].empty()) return TID_E_UNSUPPORTED;
    *count = g->n ? g->count_in(pos, lo, hi) : 0;
    return TID_OK;
}

tid_status tid_graph_partition(tid_ctx *ctx, tid_graph *g, int32_t enable) {
    return guarded(ctx, [&] {
        check_ctx(ctx);
        TID_REQUIRE(g, TID_E_INVALID_ARG, "null graph");
        tid::partition_graph(ctx, g, enable != 0);
    });
}

tid_status tid_serve_open(tid_ctx *ctx, const tid_graph *g, int32_t chunks, int32_t slots,
                          tid_server **out) {
    tid_server *sv = nullptr;
    tid_status st = guarded(ctx, [&] {
        check_ctx(ctx);
        TID_REQUIRE(g && out, TID_E_INVALID_ARG, "null argument");
        TID_REQUIRE(chunks >= 1 && slots >= 1, TID_E_INVALID_ARG, "serve: chunks, slots >= 1");
        sv = tid::serve_open(ctx, g, (uint32_t)chunks, (uint32_t)slots);
    });
    if (st == TID_OK) *out = sv;
    return st;
}

tid_status tid_serve_submit(tid_server *s, const tid_plan *plan, uint64_t *ticket) {
    if (!s || !ticket) return TID_E_INVALID_ARG;
    tid_ctx *ctx = tid::serve_ctx(s);
    return guarded(ctx, [&] {
        check_ctx(ctx);
        *ticket = tid::serve_submit(s, plan);
    });
}

tid_status tid_serve_step(tid_server *s, uint64_t *done, int32_t cap, int32_t *n_done) {
    if (!s || !n_done || (cap > 0 && !done)) return TID_E_INVALID_ARG;
    tid_ctx *ctx = tid::serve_ctx(s);
    return guarded(ctx, [&] {
        check_ctx(ctx);
        TID_REQUIRE(cap >= (int32_t)tid::serve_slots(s), TID_E_INVALID_ARG,
                    "serve: cap must be at least the slot count");
        const auto fin = tid::serve_step(s);
        for (size_t i = 0; i < fin.size(); ++i) done[i] = fin[i];
        *n_done = (int32_t)fin.size();
    });
}

tid_status tid_serve_result(tid_server *s, uint64_t ticket, tid_table **out) {
    if (!s || !out) return TID_E_INVALID_ARG;
    std::string msg;
    const tid_status st = tid::serve_take(s, ticket, out, &msg);
    if (st != TID_OK) tid::serve_ctx(s)->last_error = msg;
    return st;
}

tid_status tid_serve_info(const tid_server *s, int32_t *waiting, int32_t *active,
                          int32_t *next_chunk) {
    if (!s) return TID_E_INVALID_ARG;
    tid::serve_info(s, waiting, active, next_chunk);
    return TID_OK;
}

void tid_serve_close(tid_server *s) {
    if (!s) return;
    tid_ctx *ctx = tid::serve_ctx(s);
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    tid::serve_free(s);
}

tid_status tid_encode(tid_ctx *ctx, const uint8_t *bytes, uint64_t nbytes,
                      const uint64_t *offsets, uint64_t n, int on_device, uint32_t *rows_out,
                      tid_dict **dict) {
    std::unique_ptr<tid_dict> d;
    tid_status st = guarded(ctx, [&] {
        check_ctx(ctx);
        TID_REQUIRE(dict, TID_E_INVALID_ARG, "null output");
        d = tid::encode(ctx, bytes, nbytes, offsets, n, on_device, rows_out);
    });
    if (st == TID_OK) *dict = d.release();
    return st;
}

tid_status tid_dict_info(const tid_dict *dict, uint64_t *n_terms, uint64_t *n_bytes) {
    if (!dict) return TID_E_INVALID_ARG;
    if (n_terms) *n_terms = dict->n_terms;
    if (n_bytes) *n_bytes = dict->n_bytes;
    return TID_OK;
}

tid_status tid_decode(tid_ctx *ctx, const tid_dict *dict, const uint32_t *ids, uint64_t n,
                      int on_device, uint64_t *offsets_out, uint8_t *bytes_out,
                      uint64_t cap_bytes) {
    return guarded(ctx, [&] {
        check_ctx(ctx);
        TID_REQUIRE(dict, TID_E_INVALID_ARG, "null dictionary");
        tid::decode(ctx, dict, ids, n, on_device, offsets_out, bytes_out, cap_bytes);
    });
}

void tid_dict_free(tid_dict *dict) {
    if (!dict) return;
    (void)hipSetDevice(dict->ctx->device);
    delete dict;
}

tid_status tid_read_probe(tid_ctx *ctx, const void *device_ptr, uint64_t bytes, int32_t mode) {
    return guarded(ctx, [&] {
        check_ctx(ctx);
        tid::read_probe(ctx, device_ptr, bytes, mode);
    });
}

void tid_graph_free(tid_graph *g) {
    if (!g) return;
    (void)hipSetDevice(g->ctx->device);
    delete g;
}

tid_status tid_table_info(tid_ctx *ctx, tid_table *t, uint64_t *nrows, int32_t *ncols,
                          int32_t *vars) {
    return guarded(ctx, [&] {
        check_ctx(ctx);
        TID_REQUIRE(t, TID_E_INVALID_ARG, "null table");
        if (nrows) *nrows = t->rows();
        if (ncols) *ncols = t->ncols;
        if (vars)
            for (int c = 0; c < t->ncols; ++c) vars[c] = t->vars[c];
    });
}

tid_status tid_table_column(const tid_table *t, int32_t col, const uint32_t **device_ptr) {
    if (!t || !device_ptr || col < 0 || col >= t->ncols) return TID_E_INVALID_ARG;
    *device_ptr = t->col[col];
    return TID_OK;
}

tid_status tid_table_to_host(tid_ctx *ctx, tid_table *t, uint32_t *host, uint64_t cap_rows) {
    return guarded(ctx, [&] {
        check_ctx(ctx);
        TID_REQUIRE(t, TID_E_INVALID_ARG, "null table");
        const uint64_t n = t->rows();
        TID_REQUIRE(cap_rows >= n, TID_E_CAPACITY, "host buffer too small");
        if (n == 0 || t->ncols == 0) return;
        TID_REQUIRE(host, TID_E_INVALID_ARG, "null host buffer");
        // columns land next to each other, then are interleaved on the host
        std::vector<uint32_t> colmajor((size_t)n * t->ncols);
        for (int c = 0; c < t->ncols; ++c)
            TID_HIP(hipMemcpyAsync(colmajor.data() + (size_t)c * n, t->col[c], n * 4,
                                   hipMemcpyDeviceToHost, ctx->stream));
        ctx->sync();
        const int k = t->ncols;
        for (uint64_t r = 0; r < n; ++r)
            for (int c = 0; c < k; ++c) host[r * k + c] = colmajor[(size_t)c * n + r];
    });
}

tid_status tid_table_from_columns(tid_ctx *ctx, const uint32_t *const *cols, int32_t ncols,
                                  const int32_t *vars, uint64_t nrows, int on_device,
                                  tid_table **out) {
    std::unique_ptr<tid_table> t;
    tid_status st = guarded(ctx, [&] {
        check_ctx(ctx);
        TID_REQUIRE(out, TID_E_INVALID_ARG, "null output");
        TID_REQUIRE(ncols >= 0 && ncols <= TID_MAX_COLS, TID_E_INVALID_ARG, "bad column count");
        TID_REQUIRE(ncols == 0 || (cols && vars), TID_E_INVALID_ARG, "null columns");
        t = tid::copy_columns(ctx, cols, ncols, vars, nrows, on_device);
    });
    if (st == TID_OK) *out = t.release();
    return st;
}

void tid_table_free(tid_table *t) {
    if (!t) return;
    (void)hipSetDevice(t->ctx->device);
    delete t;
}

tid_status tid_scan(tid_ctx *ctx, const tid_graph *g, const tid_pattern *pattern,
                    tid_table **out) {
    std::unique_ptr<tid_table> t;
    tid_status st = guarded(ctx, [&] {
        check_ctx(ctx);
        TID_REQUIRE(g && pattern && out, TID_E_INVALID_ARG, "null argument");
        tid::scan_multi(ctx, g, pattern, 1, &t);
    });
    if (st == TID_OK) *out = t.release();
    return st;
}

tid_status tid_scan_noalloc(tid_ctx *ctx, const tid_graph *g, const tid_pattern *pattern,
                            uint32_t *const *out_cols, int32_t ncols, uint64_t cap_rows,
                            uint64_t *d_count) {
    return guarded(ctx, [&] {
        check_ctx(ctx);
        TID_REQUIRE(g && pattern, TID_E_INVALID_ARG, "null argument");
        tid::scan_noalloc(ctx, g, *pattern, out_cols, ncols, cap_rows, d_count);
    });
}

tid_status tid_scan_keyed(tid_ctx *ctx, const tid_graph *g, const tid_pattern *pattern,
                          int32_t key_pos, const tid_table *keys, int32_t key_col,
                          tid_table **out) {
    std::unique_ptr<tid_table> t;
    tid_status st = guarded(ctx, [&] {
        check_ctx(ctx);
        TID_REQUIRE(g && pattern && keys && out, TID_E_INVALID_ARG, "null argument");
        TID_REQUIRE(key_col >= 0 && key_col < keys->ncols, TID_E_INVALID_ARG,
                    "keyed scan: key column out of range");
        const uint64_t nk = const_cast<tid_table *>(keys)->rows();
        t = tid::scan_keyed(ctx, g, *pattern, key_pos, keys->col[key_col], nk);
    });
    if (st == TID_OK) *out = t.release();
    return st;
}

tid_status tid_entail(tid_ctx *ctx, const tid_graph *g, int32_t rule, const uint32_t *vocab,
                      tid_table **out) {
    std::unique_ptr<tid_table> t;
    tid_status st = guarded(ctx, [&] {
        check_ctx(ctx);
        TID_REQUIRE(g && vocab && out, TID_E_INVALID_ARG, "null argument");
        t = tid::entail(ctx, g, rule, vocab);
    });
    if (st == TID_OK) *out = t.release();
    return st;
}

tid_status tid_scan_multi(tid_ctx *ctx, const tid_graph *g, const tid_pattern *patterns,
                          int32_t k, tid_table **outs) {
    std::vector<std::unique_ptr<tid_table>> ts;
    tid_status st = guarded(ctx, [&] {
        check_ctx(ctx);
        TID_REQUIRE(g && patterns && outs, TID_E_INVALID_ARG, "null argument");
        TID_REQUIRE(k >= 1 && k <= TID_MAX_MULTI, TID_E_INVALID_ARG, "k must be in 1..16");
        ts.resize(k);
        tid::scan_multi(ctx, g, patterns, k, ts.data());
    });
    if (st == TID_OK)
        for (int j = 0; j < k; ++j) outs[j] = ts[j].release();
    return st;
}

tid_status tid_filter(tid_ctx *ctx, const tid_table *t, int32_t col, uint32_t lo, uint32_t hi,
                      tid_table **out) {
    std::unique_ptr<tid_table> r;
    tid_status st = guarded(ctx, [&] {
        check_ctx(ctx);
        TID_REQUIRE(t && out, TID_E_INVALID_ARG, "null argument");
        r = tid::filter_range(ctx, t, col, lo, hi);
    });
    if (st == TID_OK) *out = r.release();
    return st;
}

tid_status tid_join(tid_ctx *ctx, const tid_table *l, int32_t lcol, const tid_table *r,
                    int32_t rcol, int32_t algo, tid_table **out) {
    std::unique_ptr<tid_table> res;
    tid_status st = guarded(ctx, [&] {
        check_ctx(ctx);
        TID_REQUIRE(l && r && out, TID_E_INVALID_ARG, "null argument");
        TID_REQUIRE(algo >= 0 && algo <= 2, TID_E_INVALID_ARG, "algo must be 0, 1 or 2");
        res = tid::join_tables(ctx, l, lcol, r, rcol, algo);
    });
    if (st == TID_OK) *out = res.release();
    return st;
}

tid_status tid_join_outer(tid_ctx *ctx, const tid_table *l, int32_t lcol, const tid_table *r,
                          int32_t rcol, int32_t kind, int32_t algo, tid_table **out) {
    std::unique_ptr<tid_table> t;
    tid_status st = guarded(ctx, [&] {
        check_ctx(ctx);
        TID_REQUIRE(l && r && out, TID_E_INVALID_ARG, "null argument");
        TID_REQUIRE(algo >= 0 && algo <= 2, TID_E_INVALID_ARG, "join: algo must be 0, 1 or 2");
        t = tid::join_tables_kind(ctx, l, lcol, r, rcol, kind, algo);
    });
    if (st == TID_OK) *out = t.release();
    return st;
}

tid_status tid_union(tid_ctx *ctx, const tid_table *const *ts, int32_t k, int32_t dedupe,
                     tid_table **out) {
    std::unique_ptr<tid_table> res;
    tid_status st = guarded(ctx, [&] {
        check_ctx(ctx);
        TID_REQUIRE(ts && out && k >= 1, TID_E_INVALID_ARG, "bad arguments");
        for (int j = 0; j < k; ++j) TID_REQUIRE(ts[j], TID_E_INVALID_ARG, "null table");
        res = tid::union_tables(ctx, ts, k, dedupe ? 1 : 0);
    });
    if (st == TID_OK) *out = res.release();
    return st;
}

tid_status tid_sort(tid_ctx *ctx, const tid_table *t, int32_t distinct, tid_table **out) {
    std::unique_ptr<tid_table> res;
    tid_status st = guarded(ctx, [&] {
        check_ctx(ctx);
        TID_REQUIRE(t && out, TID_E_INVALID_ARG, "null argument");
        res = tid::sort_table(ctx, t, distinct ? 1 : 0);
    });
    if (st == TID_OK) *out = res.release();
    return st;
}

tid_status tid_query(tid_ctx *ctx, const tid_graph *g, const tid_plan *plan, tid_table **out) {
    std::unique_ptr<tid_table> res;
    tid_status st = guarded(ctx, [&] {
        check_ctx(ctx);
        TID_REQUIRE(g && plan && out, TID_E_INVALID_ARG, "null argument");
        res = tid::run_query(ctx, g, plan);
    });
    if (st == TID_OK) *out = res.release();
    return st;
}

tid_status tid_plan_estimate(tid_ctx *ctx, const tid_graph *g, const tid_plan *plan,
                             uint64_t *bytes) {
    return guarded(ctx, [&] {
        check_ctx(ctx);
        TID_REQUIRE(g && plan && bytes, TID_E_INVALID_ARG, "null argument");
        *bytes = tid::estimate_plan_bytes(g, plan);
    });
}

tid_status tid_query_batch(tid_ctx *ctx, const tid_graph *g, const tid_plan *const *plans,
                           int32_t nq, tid_table **outs) {
    std::vector<std::unique_ptr<tid_table>> res;
    tid_status st = guarded(ctx, [&] {
        check_ctx(ctx);
        TID_REQUIRE(g && outs && nq >= 0 && (nq == 0 || plans), TID_E_INVALID_ARG,
                    "null argument");
        res = tid::run_plans(ctx, g, plans, nq);
    });
    if (st == TID_OK)
        for (int i = 0; i < nq; ++i) outs[i] = res[i].release();
    return st;
}

}  // extern "C"
