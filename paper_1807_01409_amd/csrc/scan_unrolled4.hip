// scan_unrolled4.hip -- passes of up to 4 patterns in one unrolled kernel
// (a translation unit of its own, compiled in parallel with the others).
#include "scan_common.hpp"

namespace tid {

void run_unrolled_shape4(tid_ctx *ctx, const tid_graph *g, const tid_pattern *pats, int k,
                         tid_table *const *outs, int shape, const PatternSet *sets,
                         const ScanFilter *filters) {
    run_unrolled_shape<4>(ctx, g, pats, k, outs, shape, sets, filters);
}

}  // namespace tid
