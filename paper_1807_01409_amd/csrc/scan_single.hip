// scan_single.hip -- one-pattern scans in every launch shape the autotuner
// may pick (a translation unit of its own: these are most of the scan
// kernels' instantiations).
#include "scan_common.hpp"

namespace tid {

void run_scan1(tid_ctx *ctx, const tid_graph *g, const tid_pattern *pats, int k,
               tid_table *const *outs, const PatternSet *sets, const ScanFilter *filters) {
    run_scan<1>(ctx, g, pats, k, outs, sets, filters);
}

}  // namespace tid
