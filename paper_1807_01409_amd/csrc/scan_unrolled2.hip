// scan_unrolled2.hip -- passes of up to 2 patterns in one unrolled kernel
// (a translation unit of its own, compiled in parallel with the others).
#include "scan_common.hpp"

namespace tid {

void run_unrolled_shape2(tid_ctx *ctx, const tid_graph *g, const tid_pattern *pats, int k,
                         tid_table *const *outs, int shape, const PatternSet *sets,
                         const ScanFilter *filters) {
    run_unrolled_shape<2>(ctx, g, pats, k, outs, shape, sets, filters);
}

}  // namespace tid
