// ops_stub.hip -- operators not yet built return TID_E_UNSUPPORTED.
#include "internal.hpp"

namespace tid {
std::unique_ptr<tid_table> join_tables(tid_ctx *, const tid_table *, int, const tid_table *, int,
                                       int) {
    throw Error(TID_E_UNSUPPORTED, "join: not built yet");
}
std::unique_ptr<tid_table> union_tables(tid_ctx *, const tid_table *const *, int, int) {
    throw Error(TID_E_UNSUPPORTED, "union: not built yet");
}
std::unique_ptr<tid_table> sort_table(tid_ctx *, const tid_table *, int) {
    throw Error(TID_E_UNSUPPORTED, "sort: not built yet");
}
std::unique_ptr<tid_table> run_query(tid_ctx *, const tid_graph *, const tid_plan *) {
    throw Error(TID_E_UNSUPPORTED, "query: not built yet");
}
}  // namespace tid
