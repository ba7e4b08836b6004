// batch.hpp -- job descriptors of the batched small joins and sorts
// (batch.hip): one workgroup per job, many plans' jobs in one launch.
#pragma once

#include "internal.hpp"

namespace tid {

constexpr int kBatchBlock = 256;
constexpr int kJoinBlock = 1024;             // threads of a small join's count or expansion (LDS table)
constexpr uint32_t kSmallRows = 4096;       // rows per side of a batched join
constexpr uint32_t kSmallSlots = 8192;      // LDS hash slots (>= 2 * kSmallRows)
constexpr int kSmallCols = 8;               // columns per side of a batched join
constexpr int kSmallEq = 4;                 // other shared variables of a batched join
constexpr uint32_t kSortRows = 8192;        // rows of a batched sort
constexpr int kBatchSortBlock = 1024;       // threads of a batched sort's workgroup
constexpr uint32_t kSortWords = 24576;      // rows x columns of a batched sort
constexpr int kSortCols = 16;
constexpr uint32_t kEmptyKey = 0xFFFFFFFFu;  // empty LDS hash slot (the ID itself has its own slot)
// A join job without other shared variables is expanded in tiles of
// kSplitTile output rows, a workgroup each.
constexpr uint32_t kSplitTile = 2048;

struct JoinJob {
    const uint32_t *lkey, *rkey;
    uint32_t nl, nr;
    int32_t neq, nlc, nrc;
    const uint32_t *eq_l[kSmallEq], *eq_r[kSmallEq];
    const uint32_t *lcol[kSmallCols], *rcol[kSmallCols];
    uint32_t *out[2 * kSmallCols];
    uint32_t *off;     // nl + 1 entries
    uint32_t *lbase;   // neq == 0: nl entries, where each L row's key group starts in grp
    uint32_t *grp;     // neq == 0: nr entries, R row indices grouped by key
    uint64_t *total;
    uint32_t nout;     // output rows (set on the host for the expansion)
};

// A join job expanded in tiles (neq == 0), with its first tile in the
// expansion launch.
struct SplitJob {
    JoinJob j;
    uint32_t tile0;
};

// A table to put in lexicographic row order with the round's other larger
// sorts (sort_rows_batched, sort.hip): input, output (n rows allocated).
struct RowSortJob {
    const tid_table *in;
    tid_table *out;
    uint64_t n;
};
void sort_rows_batched(tid_ctx *ctx, const std::vector<RowSortJob> &jobs,
                       std::vector<DevBuf> &keep, std::vector<std::vector<char>> &host_keep);

struct SortJob {
    const uint32_t *in[kSortCols];
    uint32_t *out[kSortCols];
    uint32_t n;
    int32_t ncols, distinct;
    uint64_t *count;
};

// Jobs of one round of a batch, launched together; the device job tables
// and the host copies they came from are kept until the round's wait.
struct BatchState {
    std::vector<JoinJob> count_jobs, expand_jobs;
    std::vector<SortJob> sort_jobs;
    std::vector<RowSortJob> row_sorts;
    std::vector<DevBuf> keep;
    std::vector<std::vector<char>> host_keep;
    std::vector<std::unique_ptr<tid_table>> keep_tables;  // inputs of queued sorts
    uint64_t big_out_total = 0;   // rows of the queued larger-join expansions
    std::vector<struct BigJoinReq> big_reqs;
    std::vector<struct BigExpand> big_expand_jobs;
};
// launch and clear the queued jobs of one kind
void flush_join_jobs(tid_ctx *ctx, BatchState &bs, bool expand);
void flush_sort_jobs(tid_ctx *ctx, BatchState &bs);  // small sorts, then the larger ones

}  // namespace tid

namespace tid {

// Larger hash joins of a batch (sides above kSmallRows rows): every join of
// a round in the same few launches, each a persistent kernel over the
// concatenation of all the joins' rows.  Count phase: build (insert with
// per-workgroup rank reservation in LDS, slot scan, fill), probe, offsets,
// per-join totals; expansion phase (next round): one output-row-parallel
// launch for all joins.
constexpr int kBigCols = TID_MAX_COLS;
// largest build side of a batched larger join (as the automatic choice of
// tid_join: 2^23 rows, 2^24 slots)
constexpr uint64_t kBigBuildMax = 1ull << 23;

// "l" is the probe side and "r" the build side here (the build is the
// smaller table, which may be the join's L or R); eq_l / eq_r are columns of
// the probe / build side that must agree (the join's other shared variables).
struct BigCount {
    const uint32_t *lkey, *rkey;
    uint64_t nl, nr;
    uint64_t lbase, rbase;     // offsets in the concatenated probe and build rows
    uint64_t sbase;            // first slot in the concatenated slot arrays
    uint32_t mask;             // slots - 1 (a power of two minus one)
    int32_t neq;
    const uint32_t *eq_l[kSmallEq], *eq_r[kSmallEq];
};

struct BigExpand {
    uint64_t lbase, nl, obase;   // probe rows (as in BigCount), first output row
    int32_t neq, nlc, nrc;       // nlc / nrc: output columns from the join's L / R
    int32_t probe_is_left;
    const uint32_t *eq_l[kSmallEq], *eq_r[kSmallEq];
    const uint32_t *lcol[kBigCols], *rcol[kBigCols];
    uint32_t *out[kBigCols];
};

// The device state of one round's larger joins, kept until their expansion.
struct BigArena {
    DevBuf buf;
    uint64_t *slots = nullptr;     // key + 1 per slot, 0 = empty
    uint32_t *cnt = nullptr;       // rows per slot
    uint64_t *start = nullptr;     // first row of each slot in `rows`
    uint32_t *rows = nullptr;      // R rows grouped by slot (local row numbers)
    uint32_t *lslot = nullptr;     // per L row: its key's slot, or ~0u
    uint64_t *loff = nullptr;      // per L row: exclusive output offset (global)
    uint64_t *tot = nullptr;       // per join: its output rows
};

struct BigJoinReq {
    BigCount c;
    PendingJoin *pj;
};

// Count phase of the queued larger joins: launches, and points each
// PendingJoin's total at its word in the new arena.
void flush_big_count(tid_ctx *ctx, std::vector<BigJoinReq> &reqs,
                     std::shared_ptr<BigArena> *arena_out);
// Expansion of larger joins whose totals are known (each job's lbase refers
// to `arena`).
void flush_big_expand(tid_ctx *ctx, const BigArena &arena, std::vector<BigExpand> &jobs,
                      BatchState &bs);

}  // namespace tid

namespace tid {

// Many device-to-device copies of uint32 runs in one launch.
struct CopyJob {
    const uint32_t *src;
    uint32_t *dst;
    uint64_t n;
};
void batch_copy(tid_ctx *ctx, const std::vector<CopyJob> &jobs, BatchState &bs);

}  // namespace tid
