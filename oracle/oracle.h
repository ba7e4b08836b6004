/*
 * oracle.h -- plain CPU oracle for the TripleID-Q query path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  It shares no code,
 * header, table or constant with the GPU library, and it never calls it.
 *
 * Definitions followed (Chantrapornchai & Choksuchat, "TripleID-Q: RDF Query
 * Processing Framework using GPU"):
 *   graph   -- N triples of 32-bit (subject, predicate, object) IDs, one
 *              triple per row; ID 0 is reserved for the free variable "?"
 *              (Sec. 3, the TripleID file and the key convention).  One
 *              shared ID space is used for all positions, since joins pair
 *              different positions (Sec. 4.2, Table 3) and the Rule-11
 *              example uses one ID as object and as subject (Sec. 5.7, Rule 11 example).
 *   scan    -- triple i matches when every bound key position equals the
 *              triple's value (Sec. 3, GPUSearch, Algorithm 1); matches are
 *              reported in ascending triple position (the positionArray is
 *              indexed by triple, Sec. 3).
 *   multi   -- a triple may answer several subqueries; its membership is a
 *              set of subquery indices (Sec. 4.1, keysArray and
 *              positionArray[i].query).
 *   join    -- inner equi-join of two result vectors on one key column
 *              (Sec. 4.2: relation types of Table 3, key/value vectors,
 *              sort then merge-join into index pairs, gather of values).
 *   union   -- rows of all subqueries over the union of their variables
 *              (Sec. 4.1); DISTINCT keeps one copy of each row (Sec. 4.3).
 *   filter  -- keep rows whose chosen column lies in [lo, hi): the ID-range
 *              stand-in for the paper's string FILTER (Sec. 4.3).
 *   query   -- subqueries are searched, filtered, joined left to right and
 *              merged to distinct values on request (Sec. 4.3, Fig. 6).
 * Every result table is row-major; results of join, union(distinct) and
 * query are in lexicographic row order.  Counts are 64-bit.
 */
#ifndef TRIPLEID_ORACLE_H
#define TRIPLEID_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_MAXCOLS 32

#define OR_OK 0
#define OR_E_INVALID (-1)
#define OR_E_OOM (-2)
#define OR_E_UNSUPPORTED (-4)
#define OR_E_SCHEMA (-5)

typedef struct {
    uint32_t c[3];     /* constant ID per position, 0 = free */
    int32_t  v[3];     /* variable id of a free position, -1 = not projected */
    int32_t  range_pos;/* -1 none, else position whose value must be in [lo,hi) */
    uint32_t lo, hi;
} or_pattern;

typedef struct {
    uint32_t *rows;    /* nrows * ncols, row-major, malloc-owned */
    uint64_t  nrows;
    int32_t   ncols;
    int32_t   vars[OR_MAXCOLS];
} or_table;

/* per-triple match flags (the positionArray of Algorithm 1) */
int or_scan_flags(const uint32_t *g, uint64_t n, const or_pattern *q, uint8_t *flags);
/* per-triple subquery membership bitmask for k <= 64 patterns (Sec. 4.1) */
int or_scan_multi(const uint32_t *g, uint64_t n, const or_pattern *qs, int32_t k,
                  uint64_t *member);
/* bindings of matching triples, ascending triple position */
int or_scan(const uint32_t *g, uint64_t n, const or_pattern *q, or_table *out);
/* multi-key search (Sec. 4.1 keysArray; Sec. 5.7, the second search of an
   entailment rule): the bindings of the triples matching q whose value at
   position pos (0 s, 1 p, 2 o; a free position of q) is one of
   keys[0..nkeys); ascending triple position */
int or_scan_keyed(const uint32_t *g, uint64_t n, const or_pattern *q, int32_t pos,
                  const uint32_t *keys, uint64_t nkeys, or_table *out);
/* RDFS entailment (Sec. 5.7, the table of rules 2, 3, 5, 7, 9, 11): the
   triples the rule derives, as (s, p, o) rows (vars 0, 1, 2), distinct, in
   lexicographic order.  vocab = IDs of rdf:type, rdfs:subClassOf,
   rdfs:subPropertyOf, rdfs:domain, rdfs:range.  Two searches as in the
   paper: the rule's schema pattern, then the data pattern keyed by the
   distinct values the first bound to the shared variable; then their join. */
int or_entail(const uint32_t *g, uint64_t n, int32_t rule, const uint32_t *vocab, or_table *out);
/* rows with lo <= row[col] < hi, input order */
int or_filter(const or_table *t, int32_t col, uint32_t lo, uint32_t hi, or_table *out);
/* L join R on L[lc] = R[rc]; columns L ++ (R without rc); lexicographic order.
   _nested: the definition by nested loops.  _sortmerge: sort both key vectors,
   merge equal-key runs into index pairs, gather values (Sec. 4.2). */
int or_join_nested(const or_table *l, int32_t lc, const or_table *r, int32_t rc, or_table *out);
int or_join_sortmerge(const or_table *l, int32_t lc, const or_table *r, int32_t rc, or_table *out);
/* outer join kinds (Sec. 4.2: the join library's Left, Right and Outer
   kinds besides Inner); an unbound cell is 0, as in a union */
#define OR_JOIN_INNER 0
#define OR_JOIN_LEFT 1
#define OR_JOIN_RIGHT 2
#define OR_JOIN_FULL 3
/* L join R on L[lc] = R[rc] of the given kind, by nested loops; columns
   L ++ (R without rc); lexicographic order.  Left/full also keep each L row
   with no partner, R's columns 0; right/full also keep each R row with no
   partner, L's columns 0 except lc, which holds the R row's key. */
int or_join_outer(const or_table *l, int32_t lc, const or_table *r, int32_t rc, int32_t kind,
                  or_table *out);
/* outer union over the ordered union of variable ids, unbound cells 0.
   dedupe = 0: concatenation in input order; 1: sorted distinct rows. */
int or_union(const or_table *const *ts, int32_t k, int32_t dedupe, or_table *out);
/* in-place lexicographic sort; in-place sort + removal of repeated rows */
int or_sort_rows(or_table *t);
int or_distinct(or_table *t);
/* postfix plan evaluation; result in lexicographic row order */
int or_query(const uint32_t *g, uint64_t n, const or_pattern *pats, int32_t npats,
             const uint32_t *ops, int32_t nops, or_table *out);
void or_table_free(or_table *t);
/* plan joins above this many row pairs use sort-merge instead of nested loops */
void or_set_nested_join_limit(double pairs);

#ifdef __cplusplus
}
#endif
#endif
