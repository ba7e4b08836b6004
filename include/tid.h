/*
 * tid.h -- C ABI of libtid.so, the MI355X (gfx950) TripleID-Q query library.
 *
 * The method (Chantrapornchai & Choksuchat, "TripleID-Q: RDF Query Processing
 * Framework using GPU"): an RDF graph is dictionary-encoded into rows of three
 * 32-bit IDs (subject, predicate, object) -- the TripleID form of Sec. 3 --
 * and kept in GPU memory; a triple pattern is answered by testing every triple
 * in parallel with no index (Sec. 3, Algorithm 1, GPUSearch), and subquery
 * results are combined by union (Sec. 4.1), join on a shared variable
 * (Sec. 4.2, Table 3), filter, projection and DISTINCT (Sec. 4.3, Fig. 6).
 *
 * Conventions for every call:
 *  - Status: each call returns a tid_status; TID_OK (0) on success, a negative
 *    code otherwise.  On error no output handle is written and no device
 *    memory stays owned by the failed call; tid_last_error() describes it.
 *  - IDs: ID 0 is reserved for the free variable "?" (Sec. 3); graph triples
 *    must hold IDs in [1, 2^32-1].  One ID space is shared by all positions.
 *  - Device and stream: a context is bound to one device and one HIP stream.
 *    Every call enqueues its work on that stream and returns without waiting,
 *    except where a result count must reach the host (noted per call).
 *  - Ownership: the library owns every handle it returns; the caller releases
 *    it with the matching *_free.  Inputs are borrowed for the duration of the
 *    call only (tid_load copies the triples).  Handles must be released before
 *    their context is destroyed.
 *  - Threading: one host thread at a time per context.
 *  - There is no CPU fallback: every step runs in the library's HIP kernels.
 */
#ifndef TRIPLEID_TID_H
#define TRIPLEID_TID_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tid_status;
#define TID_OK             0
#define TID_E_INVALID_ARG (-1)  /* bad argument, pattern, plan or reserved ID 0 in a triple */
#define TID_E_OOM         (-2)  /* the allocator returned NULL */
#define TID_E_CAPACITY    (-3)  /* a result outgrew its buffer and retry is switched off */
#define TID_E_UNSUPPORTED (-4)  /* a valid request the library does not handle */
#define TID_E_SCHEMA      (-5)  /* a variable named by a plan or join is not in the table */
#define TID_E_HIP         (-6)  /* a HIP runtime call failed */
#define TID_E_INTERNAL    (-7)  /* a kernel reported an inconsistency (a bug) */

#define TID_MAX_COLS 32         /* widest table */
#define TID_MAX_MULTI 16        /* patterns per multi-pattern pass */

typedef struct tid_ctx tid_ctx;
typedef struct tid_graph tid_graph;
typedef struct tid_table tid_table;
typedef struct tid_dict tid_dict;
typedef struct tid_server tid_server;

/* Device-memory callbacks.  alloc returns a device pointer of at least
   `bytes` usable in stream order on `stream`, or NULL; free releases it.  Pass
   NULL for both to use the library's own caching pool over hipMalloc. */
typedef void *(*tid_alloc_fn)(void *user, size_t bytes, void *stream);
typedef void (*tid_free_fn)(void *user, void *ptr, size_t bytes, void *stream);

/* ---- context --------------------------------------------------------- */

/* Create a context on HIP device `device`, enqueueing on `stream` (a
   hipStream_t; NULL means the library creates and owns a stream). */
tid_status tid_ctx_create(int device, void *stream, tid_alloc_fn alloc, tid_free_fn free_fn,
                          void *user, tid_ctx **out);
void tid_ctx_destroy(tid_ctx *ctx);
/* Text of the last error on this context ("" if none); valid until the next call. */
const char *tid_last_error(const tid_ctx *ctx);
/* Wait for all work enqueued by this context. */
tid_status tid_ctx_synchronize(tid_ctx *ctx);
/* Tuning and test options, by name:
     "capacity_override"  >0: force every scan/filter output buffer to this many
                          rows (forces the overflow path in tests); 0 = off
     "retry"              1 (default): on overflow, resize and run again;
                          0: return TID_E_CAPACITY instead
     "scan_items"         triples per thread in the scan kernel (autotuner)
     "scan_block"         threads per workgroup in the scan kernel (autotuner)
     "scan_prefetch"      1: the scan loads tile t+1 before testing tile t;
                          0: it does not; -1: built-in default (autotuner)
     "stage_words"        LDS words per workgroup for staging compacted rows
                          (0 = default, at most 40448; above 20352 one
                          512-thread workgroup fits a compute unit)
     "multi_kernel"       multi-pattern scans: 0 passes of at most 4
                          patterns (unrolled), 1 one pass of up to 16
                          patterns (LDS pattern loop)      (autotuner)
     "multi_shape"        launch shape index 0..3 of that kernel (autotuner)
     "compact_kernel"     1: block-ranged compaction (one fixed range per
                          workgroup, placed after all ranges are counted);
                          2: chunked (workgroups take chunks of the input
                          from a ticket and place each chunk one chunk
                          later); 0 (default): block-ranged when the output
                          bound per range is small, chunked otherwise
     "range_factor"       block-ranged compaction: ranges per resident
                          workgroup, 1..8 (default 1; more ranges measured
                          slower on 50M and 200M triples)
     "semijoin"           1 (default): in a conjunctive plan (only SCAN, JOIN
                          and FILTER up to its last JOIN, no UNION), large
                          scans run after a smaller scan sharing a variable
                          and keep only rows whose value there passes a Bloom
                          filter of that scan's values (same result, smaller
                          joins); 0: every scan in one round, unfiltered
     "semijoin_min"       bound (rows, from the histograms) a scan needs
                          before it is filtered (default 65536)
     "chunk_epoch"        stamp of the last compaction launch; the next launch
                          uses stamp + 1 and, past 2^23 - 1, clears the
                          context's count slots and restarts at 1 (settable
                          so that tests can reach the wrap)
     "wide_min"           a round of plan scans with at least this many
                          patterns of constant predicate uses the bucketed
                          wide pass (0 = default 8: from 8 patterns on, its two
                          graph reads cost no more than passes of 4)
     "wide_slice"         1 (default): in a wide pass, a predicate that at
                          least two of its patterns share, with at least
                          "slice_rows" triples, is sliced: the graph pass
                          writes the predicate's (s, o) rows once, in triple
                          order, and a pass over that slice alone fills the
                          predicate's patterns (same tables); 0: every pattern
                          is tested in the graph pass
     "slice_rows"         triples a predicate needs to be sliced (0 = default:
                          the larger of 65536 and 1/4096 of the graph)
     "layout"             1 (default): scans use a graph's predicate-partitioned
                          layout when it is built (tid_graph_partition) and
                          pays; 0: scans always read the TripleID array
     "index_semijoin"     1 (default): in plans on a partitioned graph, a
                          scan filtered by a small semi-join source looks the
                          source's values up in the layout's (predicate,
                          subject) or (predicate, object) order instead of
                          testing every row of the predicate; 0: never
     "index_ratio"        a source is small when index_ratio times its rows
                          are at most the predicate's rows (default 4) */
tid_status tid_ctx_set_option(tid_ctx *ctx, const char *key, int64_t value);
tid_status tid_ctx_get_option(tid_ctx *ctx, const char *key, int64_t *value);

/* ---- graph (Sec. 3: the TripleID array kept in GPU memory) ----------- */

/* Copy n triples, row-major (s,p,o) uint32 (12 bytes per triple, the TripleID
   file layout), into device memory owned by the new graph.  `triples` is a
   host pointer (src_on_device = 0) or a device pointer on the context's device
   (src_on_device = 1).  Rejects any triple holding ID 0 with TID_E_INVALID_ARG.
   Builds per-position ID histograms used to size scan outputs.  Synchronises. */
tid_status tid_load(tid_ctx *ctx, const uint32_t *triples, uint64_t n, int src_on_device,
                    tid_graph **out);
/* Same, reading a raw TripleID file (n x 12 bytes, little-endian, no header). */
tid_status tid_load_file(tid_ctx *ctx, const char *path, tid_graph **out);
/* Number of triples and the device address of the resident array. */
tid_status tid_graph_info(const tid_graph *g, uint64_t *n, const uint32_t **device_triples);
/* Number of triples whose position `pos` (0 s, 1 p, 2 o) holds an ID in
   [lo, hi), from the per-position histograms built at load (Sec. 3: the
   TripleID array kept resident; these counts size scan outputs and bound
   plans).  lo >= hi gives 0.  Host only, no device work.  TID_E_UNSUPPORTED
   if the position has no histogram (its largest ID is 2^28 or more, or the
   graph holds 2^32 triples or more). */
tid_status tid_graph_count(const tid_graph *g, int32_t pos, uint32_t lo, uint32_t hi,
                           uint64_t *count);
/* Layout variant (the paper's ID assignment for pruning a search, Sec. 4.3):
   enable = 1 builds, beside the TripleID array, the triples stably sorted by
   predicate as two device columns (subject, object), and the same rows
   ordered by (predicate, subject) and by (predicate, object) for semi-join
   lookups: 24 B per triple more; enable = 0 drops them.  While they exist
   (and the context option "layout" is 1), scans whose patterns all have a
   constant predicate and whose slices add up to less than one read of the
   array read only those predicates' slices; results are identical
   (ascending triple position).  Plans and batches use the layout as well
   (see the options "layout" and "index_semijoin").  Needs the predicate
   histogram and fewer than 2^32 triples (TID_E_UNSUPPORTED otherwise).
   Synchronises. */
tid_status tid_graph_partition(tid_ctx *ctx, tid_graph *g, int32_t enable);
void tid_graph_free(tid_graph *g);

/* ---- triple pattern (Sec. 3: key with 0 as "?") ----------------------- */

typedef struct {
    uint32_t s, p, o;     /* constant ID >= 1, or 0 = free position */
    int32_t vs, vp, vo;   /* variable id (>= 0) naming a free position, or -1:
                             free and not projected.  A bound position must
                             carry -1.  Free positions sharing an id must hold
                             equal values. */
    int32_t range_pos;    /* -1, or the position (0 s, 1 p, 2 o) whose value must
                             lie in [lo, hi); lo >= hi matches nothing */
    uint32_t lo, hi;
} tid_pattern;

/* ---- tables ----------------------------------------------------------- */
/* A table is ncols device columns of uint32 (one per variable), nrows rows.
   Column c holds variable vars[c]; 0 marks an unbound cell after a union. */

/* Row count, column count and variable ids (vars must hold TID_MAX_COLS
   entries; may be NULL).  Synchronises if the count is still on the device. */
tid_status tid_table_info(tid_ctx *ctx, tid_table *t, uint64_t *nrows, int32_t *ncols,
                          int32_t *vars);
/* Device address of column `col` (valid while the table lives). */
tid_status tid_table_column(const tid_table *t, int32_t col, const uint32_t **device_ptr);
/* Copy the rows to host memory, row-major (nrows x ncols uint32).  Fails with
   TID_E_CAPACITY if cap_rows < nrows.  Synchronises. */
tid_status tid_table_to_host(tid_ctx *ctx, tid_table *t, uint32_t *host_rowmajor,
                             uint64_t cap_rows);
/* Build a table from caller data: ncols columns, each a pointer to nrows
   uint32 on the host (on_device = 0) or on the device (on_device = 1); the
   data is copied. */
tid_status tid_table_from_columns(tid_ctx *ctx, const uint32_t *const *cols, int32_t ncols,
                                  const int32_t *vars, uint64_t nrows, int on_device,
                                  tid_table **out);
void tid_table_free(tid_table *t);

/* ---- operators -------------------------------------------------------- */

/* Sec. 3 (GPUSearch, Algorithm 1): every triple is tested against the pattern;
   the bindings of the matching triples are returned in ascending triple
   position.  Output columns: the distinct variable ids of the pattern in
   s, p, o order (none if all free positions carry -1: the table then only
   counts matches). */
tid_status tid_scan(tid_ctx *ctx, const tid_graph *g, const tid_pattern *pattern,
                    tid_table **out);
/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid allocation): the rows
   tid_scan returns for `pattern`, written into caller buffers, with no device
   allocation and no host wait.
     out_cols  ncols device pointers, one per output column (the pattern's
               distinct variables in s, p, o order; ncols must equal that
               count; may be NULL when it is 0), each with room for cap_rows
               uint32 values; rows land in ascending triple position
     d_count   device pointer to one uint64 that receives the number of
               matching triples; if it exceeds cap_rows, rows past cap_rows
               are not written (size cap_rows from tid_graph_count to be safe)
   The kernel's cross-workgroup state is a fixed device array of the library
   (one per GPU, 32 KB, held until the process ends; at most 4096 ranges per
   launch, which every graph size fits).  All calls on one GPU share it:
   calls that overlap on one GPU (other streams or threads) race and must not
   be issued.  Asynchronous on the context's stream. */
tid_status tid_scan_noalloc(tid_ctx *ctx, const tid_graph *g, const tid_pattern *pattern,
                            uint32_t *const *out_cols, int32_t ncols, uint64_t cap_rows,
                            uint64_t *d_count);
/* Sec. 4.1 (keysArray / positionArray[i].query): k <= TID_MAX_MULTI patterns
   answered in one pass over the graph; outs[j] receives exactly what
   tid_scan would return for patterns[j]. */
tid_status tid_scan_multi(tid_ctx *ctx, const tid_graph *g, const tid_pattern *patterns,
                          int32_t k, tid_table **outs);
/* Sec. 4.1 (keysArray) and Sec. 5.7 (the second search of an entailment
   rule): tid_scan of `pattern`, keeping only triples whose value at position
   key_pos (0 s, 1 p, 2 o; a free position of the pattern) is one of the
   values in column key_col of `keys` (repeats allowed; the multi-key search
   of the paper's keysArray built from an earlier result).  Exact: no false
   positives.  Rows in ascending triple position. */
tid_status tid_scan_keyed(tid_ctx *ctx, const tid_graph *g, const tid_pattern *pattern,
                          int32_t key_pos, const tid_table *keys, int32_t key_col,
                          tid_table **out);
/* Sec. 5.7 (RDFS entailment, the rule table): the triples rule 2, 3, 5, 7, 9
   or 11 derives from the graph, as distinct (s, p, o) rows (variable ids 0, 1,
   2) in lexicographic order.  vocab[0..5) are the IDs of rdf:type,
   rdfs:subClassOf, rdfs:subPropertyOf, rdfs:domain and rdfs:range.  Two
   searches as in the paper: the rule's schema pattern, then the data pattern
   keyed by the values the first bound to the shared variable; then their
   join.  Synchronises. */
tid_status tid_entail(tid_ctx *ctx, const tid_graph *g, int32_t rule, const uint32_t *vocab,
                      tid_table **out);
/* Sec. 4.3 (FILTER, here on an ID range): the rows with lo <= row[col] < hi,
   in input order.  lo >= hi gives an empty table. */
tid_status tid_filter(tid_ctx *ctx, const tid_table *t, int32_t col, uint32_t lo, uint32_t hi,
                      tid_table **out);
/* Sec. 4.2 (join on the shared variable; any of the Table 3 position pairs):
   the inner equi-join of l and r on l[lcol] = r[rcol].  Output columns are
   l's columns followed by r's columns without rcol; rows are returned in
   lexicographic order over all output columns.  algo: 0 automatic, 1 hash
   join, 2 sort-merge join (same result).  Synchronises (output size). */
tid_status tid_join(tid_ctx *ctx, const tid_table *l, int32_t lcol, const tid_table *r,
                    int32_t rcol, int32_t algo, tid_table **out);
/* Sec. 4.2 (the join library's Left, Right and Outer kinds besides Inner):
   the join of l and r on l[lcol] = r[rcol] of the given kind, by hash or
   sort-merge (algo as in tid_join).  Columns and order as in tid_join.
     TID_JOIN_INNER  the matching pairs (same as tid_join)
     TID_JOIN_LEFT   also every l row with no partner, r's cells 0
     TID_JOIN_RIGHT  also every r row with no partner, l's cells 0 except
                     lcol, which holds the r row's key
     TID_JOIN_FULL   both
   Synchronises (output size). */
#define TID_JOIN_INNER 0
#define TID_JOIN_LEFT 1
#define TID_JOIN_RIGHT 2
#define TID_JOIN_FULL 3
tid_status tid_join_outer(tid_ctx *ctx, const tid_table *l, int32_t lcol, const tid_table *r,
                          int32_t rcol, int32_t kind, int32_t algo, tid_table **out);
/* Sec. 4.1 and Sec. 4.3 (union, DISTINCT): the schema is the ordered union of
   the inputs' variable ids (first appearance first), unbound cells are 0.
   dedupe = 0: the rows of ts[0], then ts[1], ... ; dedupe = 1: the distinct
   rows in lexicographic order.  Synchronises when dedupe = 1. */
tid_status tid_union(tid_ctx *ctx, const tid_table *const *ts, int32_t k, int32_t dedupe,
                     tid_table **out);
/* Lexicographic row order (the canonical order of query results); distinct = 1
   also drops repeated rows (Sec. 4.3, DISTINCT).  Synchronises. */
tid_status tid_sort(tid_ctx *ctx, const tid_table *t, int32_t distinct, tid_table **out);

/* ---- query plans (Sec. 4.3, Fig. 6) ----------------------------------- */

/* Postfix op words (uint32):
     TID_OP_SCAN i              push the bindings of patterns[i]
     TID_OP_JOIN v              pop R, pop L; push the join of L and R on variable
                                v; every other variable both hold must also
                                agree and is kept once
     TID_OP_UNION k d           pop k tables; push their union (d = 1: distinct)
     TID_OP_FILTER v lo hi      keep rows with lo <= v < hi
     TID_OP_PROJECT n v1..vn    keep variables v1..vn in that order
     TID_OP_DISTINCT            drop repeated rows
     TID_OP_OPTIONAL v          pop R, pop L; push the left outer join of L and R
                                on variable v (SPARQL OPTIONAL): L rows with no
                                partner are kept, R's cells 0; L and R may
                                share no other variable (TID_E_UNSUPPORTED)
   Exactly one table must remain; it is returned in lexicographic row order. */
#define TID_OP_SCAN 1
#define TID_OP_JOIN 2
#define TID_OP_UNION 3
#define TID_OP_FILTER 4
#define TID_OP_PROJECT 5
#define TID_OP_DISTINCT 6
#define TID_OP_OPTIONAL 7

typedef struct {
    int32_t n_patterns;
    const tid_pattern *patterns;
    int32_t n_ops;
    const uint32_t *ops;
} tid_plan;

/* Evaluate a plan: all its patterns in one pass over the graph, then its
   joins, unions, filters, projections and DISTINCT on the device.
   Synchronises (intermediate sizes). */
tid_status tid_query(tid_ctx *ctx, const tid_graph *g, const tid_plan *plan, tid_table **out);
/* Evaluate nq plans together: outs[i] receives exactly what tid_query would
   return for plans[i].  The patterns of all plans are searched in shared
   multi-pattern passes over the graph (Sec. 4.1 keysArray, at batch scale)
   and the plans' joins, unions and sorts advance in lockstep, so the host
   waits for the device once per round for the whole batch.  On error no
   output is written.  Synchronises. */
tid_status tid_query_batch(tid_ctx *ctx, const tid_graph *g, const tid_plan *const *plans,
                           int32_t nq, tid_table **outs);
/* Upper estimate of the device bytes a plan holds while it runs: the sum of
   its scans' output buffers (sized from the load-time histograms, Sec. 3's
   one-pass search) times two for join intermediates.  Host only, no device
   work; used to admit queries against a memory budget. */
tid_status tid_plan_estimate(tid_ctx *ctx, const tid_graph *g, const tid_plan *plan,
                             uint64_t *bytes);

/* ---- serving: a circular chunked shared scan --------------------------- */
/* The paper keeps the TripleID array resident and answers every query with a
   full search of it (Sec. 3, Algorithm 1, which loops over chunks of the
   array).  A server cuts the resident graph into `chunks` contiguous chunks
   and scans them one after another, round and round; each step scans the
   next chunk once for every admitted query.  A submitted query is admitted
   at the next chunk boundary into one of `slots` slots and has seen the whole
   graph one revolution later; its per-chunk results are then joined end to
   end in chunk order, so its scans equal scans of the whole graph, and its
   remaining ops (joins, unions, filters, projections, DISTINCT, OPTIONAL) run
   together with those of the other queries finishing at that step.  Every
   result equals tid_query's.  One host thread at a time per server; the
   server uses its context's stream.  tid_serve_open synchronises (it counts
   each chunk's predicates). */
tid_status tid_serve_open(tid_ctx *ctx, const tid_graph *g, int32_t chunks, int32_t slots,
                          tid_server **out);
/* Queue a plan (copied); *ticket names its result.  Checks the plan. */
tid_status tid_serve_submit(tid_server *s, const tid_plan *plan, uint64_t *ticket);
/* One step: admit waiting queries into free slots, scan the next chunk for all
   admitted queries, finish those that have seen every chunk.  Their tickets go
   to done[0..*n_done) (cap must be at least the slot count).  Synchronises. */
tid_status tid_serve_step(tid_server *s, uint64_t *done, int32_t cap, int32_t *n_done);
/* The result of a finished ticket (the caller frees the table), or the
   status its query failed with; TID_E_INVALID_ARG for a ticket that is not
   finished or was already taken. */
tid_status tid_serve_result(tid_server *s, uint64_t ticket, tid_table **out);
/* Queries waiting for a slot, queries in slots, the next chunk to scan. */
tid_status tid_serve_info(const tid_server *s, int32_t *waiting, int32_t *active,
                          int32_t *next_chunk);
void tid_serve_close(tid_server *s);

/* ---- dictionary (Sec. 3: conversion of RDF terms into TripleID rows) ---- */

/* Encode n triples of terms into TripleID rows on the GPU.  Term t (t < 3n) is
   bytes[offsets[t] .. offsets[t+1]); term 3i + x is position x (s, p, o) of
   triple i.  bytes, offsets (3n + 1 uint64, non-decreasing, within nbytes)
   are host (on_device = 0) or device (1) buffers.  One dictionary for all
   positions; IDs are handed out from 1 in order of first appearance, reading
   the terms s, p, o of triple 0, then triple 1, and so on.  rows_out (device,
   3n uint32) receives the rows (row-major, the tid_load layout); *dict the
   dictionary (device resident).  TID_E_UNSUPPORTED if two different terms
   share a 64-bit hash (checked, never merged).  Synchronises. */
tid_status tid_encode(tid_ctx *ctx, const uint8_t *bytes, uint64_t nbytes,
                      const uint64_t *offsets, uint64_t n, int on_device, uint32_t *rows_out,
                      tid_dict **dict);
/* Number of distinct terms (= the largest ID) and their total bytes. */
tid_status tid_dict_info(const tid_dict *dict, uint64_t *n_terms, uint64_t *n_bytes);
/* Decode n IDs (host or device buffer) to their terms, into host buffers:
   offsets_out (n + 1 uint64) always receives the offsets of the terms in the
   output; bytes_out receives the bytes if they fit cap_bytes, otherwise the
   call returns TID_E_CAPACITY with the needed size in offsets_out[n].  An ID
   of 0 or above the dictionary's size is TID_E_INVALID_ARG.  Synchronises. */
tid_status tid_decode(tid_ctx *ctx, const tid_dict *dict, const uint32_t *ids, uint64_t n,
                      int on_device, uint64_t *offsets_out, uint8_t *bytes_out,
                      uint64_t cap_bytes);
void tid_dict_free(tid_dict *dict);

/* ---- measurement ------------------------------------------------------ */

/* Read `bytes` of device memory at `device_ptr` once, as a streaming scan
   reads the TripleID array (Sec. 3: every triple tested in parallel), and do
   nothing with the values: the time of this call is the read ceiling a scan
   of the same bytes is measured against.  mode 0: one 12-byte load per lane
   per triple, the scan's own access shape; mode 1: one 16-byte load per lane
   (the pointer must be 16-byte aligned).  A tail shorter than one item is not
   read.  Asynchronous on the context's stream; writes nothing the caller can
   observe. */
tid_status tid_read_probe(tid_ctx *ctx, const void *device_ptr, uint64_t bytes, int32_t mode);

#ifdef __cplusplus
}
#endif
#endif
