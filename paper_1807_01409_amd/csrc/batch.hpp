// batch.hpp -- job descriptors of the batched small joins and sorts
// (batch.hip): one workgroup per job, many plans' jobs in one launch.
#pragma once

#include "internal.hpp"

namespace tid {

constexpr int kBatchBlock = 256;
constexpr uint32_t kSmallRows = 4096;       // rows per side of a batched join
constexpr uint32_t kSmallSlots = 8192;      // LDS hash slots (>= 2 * kSmallRows)
constexpr int kSmallCols = 8;               // columns per side of a batched join
constexpr int kSmallEq = 4;                 // other shared variables of a batched join
constexpr uint32_t kSortRows = 8192;        // rows of a batched sort
constexpr uint32_t kSortWords = 24576;      // rows x columns of a batched sort
constexpr int kSortCols = 16;
constexpr uint32_t kEmptyKey = 0xFFFFFFFFu;

struct JoinJob {
    const uint32_t *lkey, *rkey;
    uint32_t nl, nr;
    int32_t neq, nlc, nrc;
    const uint32_t *eq_l[kSmallEq], *eq_r[kSmallEq];
    const uint32_t *lcol[kSmallCols], *rcol[kSmallCols];
    uint32_t *out[2 * kSmallCols];
    uint32_t *off;     // nl + 1 entries
    uint64_t *total;
};

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
    std::vector<DevBuf> keep;
    std::vector<std::vector<char>> host_keep;
    std::vector<std::unique_ptr<tid_table>> keep_tables;  // inputs of queued sorts
};
// launch and clear the queued jobs of one kind
void flush_join_jobs(tid_ctx *ctx, BatchState &bs, bool expand);
void flush_sort_jobs(tid_ctx *ctx, BatchState &bs);

}  // namespace tid
