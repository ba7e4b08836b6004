// internal.hpp -- host-side runtime structures of libtid (context, device
// buffers, graphs, tables, error plumbing).  Included by every .hip file.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <exception>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/tid.h"

namespace tid {

// An error carrying a tid_status; thrown inside the library and turned into a
// return code at the C boundary.
struct Error : std::runtime_error {
    tid_status code;
    Error(tid_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define TID_HIP(call)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            throw ::tid::Error(TID_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define TID_REQUIRE(cond, code, msg)                        \
    do {                                                    \
        if (!(cond)) throw ::tid::Error((code), (msg));     \
    } while (0)

// Size-class caching pool over hipMalloc, used when the caller gives no
// allocator.  Blocks are reused in stream order on the context's one stream,
// so a freed block may be handed out again at once.
class Pool {
  public:
    ~Pool();
    void *alloc(size_t bytes);
    void free(void *p, size_t bytes);
    void release_all();

  private:
    static size_t size_class(size_t bytes);
    std::multimap<size_t, void *> free_;
    std::map<void *, size_t> live_;
};

struct Options {
    int64_t capacity_override = 0;
    int64_t retry = 1;
    int64_t scan_items = 0;   // 0 = built-in default
    int64_t scan_block = 0;
    int64_t stage_words = 0;  // LDS staging words per workgroup (0 = default)
    int64_t wide_min = 0;     // patterns needed before wide passes are used (0 = 8)
    int64_t scan_prefetch = -1;  // -1 built-in default, 0 off, 1 prefetch the next tile
    int64_t multi_kernel = 0;    // 0 passes of <= 4 unrolled patterns, 1 LDS pattern loop
    int64_t multi_shape = 0;     // launch shape index of the chosen multi-pattern kernel
    int64_t compact_kernel = 0;  // 0 auto, 1 block-ranged, 2 chunked compaction
    int64_t semijoin = 1;        // filter scans of conjunctive plans by join values
    int64_t range_factor = 1;    // block-ranged kernel: ranges per resident workgroup
    int64_t semijoin_min = 1 << 16;  // rows a scan's bound needs before it is filtered
    int64_t wide_slice = 1;      // wide passes slice predicates shared by patterns
    int64_t slice_rows = 0;      // rows a predicate needs to be sliced (0 = default)
    int64_t layout = 1;          // 1: scans use a graph's partitioned layout if built; 0: never
    int64_t batch_small = 1;     // 1: small joins and final sorts of plans batched per round
    int64_t index_semijoin = 1;  // 1: small semi-join sources look their keys up in the
                                 // partitioned layout's sorted copies; 0: Bloom filters
    int64_t index_ratio = 4;     // "small": index_ratio x source rows <= the predicate's rows
};

}  // namespace tid

struct tid_ctx {
    int device = 0;
    int num_cus = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    tid_alloc_fn alloc_fn = nullptr;
    tid_free_fn free_fn = nullptr;
    void *user = nullptr;
    tid::Pool pool;
    std::string last_error;
    tid::Options opt;
    // cross-workgroup state of the compaction kernels: a ticket and a done
    // counter, then epoch-stamped count words; zeroed when grown and when the
    // epoch wraps
    void *ep_state = nullptr;
    size_t ep_bytes = 0;
    uint32_t epoch = 0;
    uint32_t *d_flags = nullptr;      // device error/overflow flags (2 words)
    // staging for read_words: pinned pointer list and values, device copies
    const uint64_t **rw_host_ptrs = nullptr;
    uint64_t *rw_host_vals = nullptr;
    void *rw_dev = nullptr;
    size_t rw_cap = 0;

    void *alloc(size_t bytes);
    void free(void *p, size_t bytes);
    // stamp for the next chunked launch; *state gets the slot area of `bytes`
    uint32_t next_epoch(size_t bytes, uint64_t **state);
    void sync();
    // device row-count words whose values the host already knows, written
    // together by tid::flush_counts (one launch per 128)
    std::vector<std::pair<uint64_t *, uint64_t>> pending_counts;
};

namespace tid {

// RAII device allocation through the context's allocator.
class DevBuf {
  public:
    DevBuf() = default;
    DevBuf(tid_ctx *c, size_t bytes) : ctx_(c), bytes_(bytes) {
        if (bytes) ptr_ = c->alloc(bytes);
    }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept { *this = std::move(o); }
    DevBuf &operator=(DevBuf &&o) noexcept {
        reset();
        ctx_ = o.ctx_;
        ptr_ = o.ptr_;
        bytes_ = o.bytes_;
        o.ptr_ = nullptr;
        o.bytes_ = 0;
        return *this;
    }
    ~DevBuf() { reset(); }
    void reset() {
        if (ptr_ && ctx_) ctx_->free(ptr_, bytes_);
        ptr_ = nullptr;
        bytes_ = 0;
    }
    template <class T = void> T *get() const { return static_cast<T *>(ptr_); }
    size_t bytes() const { return bytes_; }
    void *release() {
        void *p = ptr_;
        ptr_ = nullptr;
        bytes_ = 0;
        return p;
    }

  private:
    tid_ctx *ctx_ = nullptr;
    void *ptr_ = nullptr;
    size_t bytes_ = 0;
};

constexpr size_t kAlign = 256;
// Chunked-compaction launch stamps run 1..kEpochMax; then the slots are zeroed.
constexpr uint32_t kEpochMax = (1u << 23) - 1;
inline size_t align_up(size_t x, size_t a = kAlign) { return (x + a - 1) / a * a; }

}  // namespace tid

// Per-position ID histograms kept on the host as cumulative counts:
// cdf[x][id] = number of triples whose position x holds an ID < id.  Used to
// bound scan output sizes without a device round trip.
struct tid_graph {
    tid_ctx *ctx = nullptr;
    uint64_t n = 0;
    tid::DevBuf data;                 // n*12 bytes (+ padding), AoS s,p,o
    std::vector<uint64_t> cdf[3];     // empty if the position's max ID is too large
    uint32_t max_id[3] = {0, 0, 0};
    // Optional layout variant: the triples stably sorted by predicate, as two
    // columns (subject, object); predicate p's triples are rows
    // [cdf[1][p], cdf[1][p + 1]) in ascending triple position.  Scans with a
    // constant predicate then read only that slice (8 B per triple of p).
    tid::DevBuf part_s, part_o;
    // The same rows ordered by (predicate, subject) and by (predicate,
    // object), ties in triple order, as (subject, object) columns: predicate
    // p's rows are the same [cdf[1][p], cdf[1][p + 1]) in both.  A semi-join
    // on a pattern's subject or object looks its keys up in these.
    tid::DevBuf ps_s, ps_o, po_s, po_o;
    bool partitioned = false;
    // A chunk of another graph (circular serving scan): `view` is its first
    // triple (not owned); positions without a histogram here take their
    // bounds from `bounds_from`.
    const uint32_t *view = nullptr;
    const tid_graph *bounds_from = nullptr;
    const uint32_t *triples() const { return view ? view : data.get<const uint32_t>(); }
    // number of triples with lo <= position value < hi (n if no histogram)
    uint64_t count_in(int pos, uint64_t lo, uint64_t hi) const;
};

// A term dictionary on the device: term ID k (1-based) is bytes
// [offsets[k-1], offsets[k]).
struct tid_dict {
    tid_ctx *ctx = nullptr;
    uint64_t n_terms = 0;        // distinct terms = the largest ID
    uint64_t n_bytes = 0;
    tid::DevBuf offsets;         // n_terms + 1 uint64
    tid::DevBuf bytes;
};

struct tid_table {
    tid_ctx *ctx = nullptr;
    int32_t ncols = 0;
    int32_t vars[TID_MAX_COLS] = {};
    uint64_t cap = 0;                 // rows allocated per column
    uint64_t nrows = 0;               // valid when count_known
    bool count_known = false;
    // columns (each align_up(cap*4)) + 8-byte device count; shared by the
    // tables that alias one result (tables are never written after they are
    // produced)
    std::shared_ptr<tid::DevBuf> block;
    uint32_t *col[TID_MAX_COLS] = {};
    uint64_t *d_count = nullptr;
    // host-side upper bound of every column's values (valid when maxv_known);
    // lets sorts size their passes without reading the device
    uint32_t maxv[TID_MAX_COLS] = {};
    bool maxv_known = false;

    uint64_t rows();                  // host row count (may synchronise)
};

namespace tid {

// Allocate a table with `cap` rows per column and the given schema; the
// device count word is not initialised.
std::unique_ptr<tid_table> make_table(tid_ctx *ctx, int32_t ncols, const int32_t *vars,
                                      uint64_t cap);
// Read a batch of device counts into table->nrows with one synchronisation;
// also checks the device error flag.
void resolve_counts(tid_ctx *ctx, tid_table *const *ts, int k);
// Write a known row count to the table's device word and host copy.
void set_count(tid_ctx *ctx, tid_table *t, uint64_t n);
// The same, with the device word written by the next flush_counts (the host
// copy at once); for the many tables of a batch round, whose device words no
// kernel reads before the round's end.
void set_count_later(tid_ctx *ctx, tid_table *t, uint64_t n);
void flush_counts(tid_ctx *ctx);
// Drops the counts still pending when a call fails (their tables may be
// freed with the error); on success the call has flushed them itself.
struct PendingCountsGuard {
    tid_ctx *ctx;
    int exc;
    explicit PendingCountsGuard(tid_ctx *c) : ctx(c), exc(std::uncaught_exceptions()) {}
    ~PendingCountsGuard() {
        if (std::uncaught_exceptions() > exc) ctx->pending_counts.clear();
    }
};
// Column value bounds: dst column c takes the bound of src column map[c].
void copy_bounds(tid_table *dst, const tid_table *src, const int *map, int n, int dst_off = 0);

// ---- launchers implemented in the .hip files ------------------------------

// Values one position of a pattern may take (Sec. 4.2: a union of scans that
// differ only in that constant, evaluated as one scan).  The pattern keeps a
// constant there so that its schema is that of each scan of the union.
constexpr int kMaxSet = 16;
struct PatternSet {
    int32_t pos = -1;  // -1: none
    int32_t n = 0;
    uint32_t v[kMaxSet] = {};
};

// A membership filter on one position of a pattern: a Bloom filter of
// (mask + 1) bits over the values another scan of the same conjunctive plan
// binds to the variable at that position.  A row whose value is not in it
// cannot take part in the plan's join; a false positive only keeps a row that
// the join then drops.
//
// With exact = 1 the filter is instead a bitmap over IDs 0..mask (one bit per
// ID, set for the members): a multi-key search (Sec. 4.1 keysArray; Sec. 5.7,
// the second search of an entailment rule) with no false positives.
struct ScanFilter {
    const uint32_t *bits = nullptr;
    uint32_t mask = 0;
    int32_t pos = -1;  // -1: none
    int32_t exact = 0;
    // index = 1: no bits; the rows are those of the pattern's predicate whose
    // value at `pos` is one of the `nkeys` values at `keys` (device, any
    // order, repeats allowed), found in the sorted copies of the partitioned
    // layout (index_semijoin); rows then come grouped by key
    const uint32_t *keys = nullptr;
    uint64_t nkeys = 0;
    uint32_t key_max = 0;  // bound of the key values
    int32_t index = 0;
};

// Scan: fill `outs[j]` for k patterns in one pass.  Tables are allocated here.
// sets, filters (each may be null): per pattern, a set of values for one
// position, and a membership filter on one position.
void scan_multi(tid_ctx *ctx, const tid_graph *g, const tid_pattern *pats, int k,
                std::unique_ptr<tid_table> *outs, const PatternSet *sets = nullptr,
                const ScanFilter *filters = nullptr);
// any number of patterns, in as few passes over the graph as the kernels allow
void scan_many(tid_ctx *ctx, const tid_graph *g, const tid_pattern *pats, int k,
               std::unique_ptr<tid_table> *outs, const PatternSet *sets = nullptr,
               const ScanFilter *filters = nullptr);
// rows a pattern (with its set, if any) can produce, from the load-time histograms
uint64_t pattern_output_bound(const tid_graph *g, const tid_pattern &p,
                              const PatternSet *set = nullptr);
std::unique_ptr<tid_table> filter_range(tid_ctx *ctx, const tid_table *t, int col, uint32_t lo,
                                        uint32_t hi);
// columns of L and of R kept, in that order, in a join's output
struct JoinPlan {
    std::vector<int> lkeep, rkeep;
};

// A join whose matches are counted on the device but whose output size has
// not reached the host yet (the split lets many joins share one round trip).
struct PendingJoin {
    const tid_table *L = nullptr, *R = nullptr;
    std::unique_ptr<tid_table> own_l, own_r;  // inputs kept alive until expanded
    int lc = 0, rc = 0;
    JoinPlan jp;
    std::vector<int32_t> vars;
    DevBuf start, count, off, keys[4], vals[4];
    DevBuf slots, slot_of, rank, slot_start, rows;  // slots: slot words, then counts
    const uint32_t *qrow = nullptr, *brow = nullptr;
    int probe_is_left = 1;
    // left outer join (probe side = L): each probe row with no partner still
    // gives one output row, R's cells 0; `count` then holds max(matches, 1)
    // and `matches` the true counts
    bool outer = false;
    DevBuf matches;
    uint64_t nq = 0;
    uint64_t total = 0;
    bool total_known = false;
    // a small join of a batch (batch.hip): counted and expanded as one job
    // of a round's launch; sj_off holds its L rows' output offsets (then,
    // without other shared variables, their key groups' starts and R's rows
    // grouped by key), sj_total its size, small_result its rows once expanded
    bool small = false;
    DevBuf sj_off, sj_total;
    std::unique_ptr<tid_table> small_result;
    // a larger join of a batch (batch.hip): counted with the round's other
    // larger joins in one arena; total_ptr is its size word there
    bool big = false;
    std::shared_ptr<void> big_arena;
    const uint64_t *total_ptr = nullptr;
    uint64_t big_lbase = 0;
    const uint64_t *d_total() const {
        if (total_ptr) return total_ptr;
        return small ? sj_total.get<const uint64_t>() : off.get<const uint64_t>() + nq;
    }
};
// join kinds (Sec. 4.2: the join library's Inner, Left, Right and Outer)
constexpr int kJoinInner = 0, kJoinLeft = 1, kJoinRight = 2, kJoinFull = 3;
// kind: kJoinInner or kJoinLeft (the probe side is then L)
std::unique_ptr<PendingJoin> join_begin(tid_ctx *ctx, const tid_table *L, uint64_t nl, int lc,
                                        const tid_table *R, uint64_t nr, int rc, int algo,
                                        const JoinPlan &jp, int kind = kJoinInner);
std::unique_ptr<tid_table> join_finish(tid_ctx *ctx, PendingJoin &pj);

// Read device words (counts, totals) to the host with one copy and one
// synchronisation; also checks the device error flag.
void read_words(tid_ctx *ctx, const std::vector<const uint64_t *> &src, uint64_t *dst);

// validate and return the schema of a pattern; throws on a malformed pattern
int pattern_schema(const tid_pattern &p, int32_t *vars, int32_t *src);
// per-position histograms (device) -> host cdf
void build_stats(tid_ctx *ctx, tid_graph *g);
void check_no_zero(tid_ctx *ctx, const tid_graph *g);

}  // namespace tid
