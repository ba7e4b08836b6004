"""MI355X-native TripleID-Q query path: resident TripleID graph, triple-pattern
scan with order-preserving compaction, filter, join, union, DISTINCT and
query plans, all in hand-written HIP kernels for gfx950 behind the C ABI of
include/tid.h."""
from .tid import (Context, Graph, Table, TidError, tid_filter, tid_graph_count, tid_join, tid_join_outer,
                  tid_load, tid_entail, tid_scan_keyed, tid_encode, tid_decode,
                  tid_load_file, tid_query, tid_query_batch, tid_scan, tid_scan_multi, tid_sort,
                  tid_table_from_columns, tid_union)

__all__ = ["Context", "Graph", "Table", "TidError", "tid_filter", "tid_graph_count", "tid_join", "tid_join_outer",
           "tid_load", "tid_entail", "tid_scan_keyed", "tid_encode", "tid_decode",
           "tid_load_file", "tid_query", "tid_query_batch", "tid_scan", "tid_scan_multi", "tid_sort",
           "tid_table_from_columns", "tid_union"]
