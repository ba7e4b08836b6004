// query.hip -- evaluation of postfix query plans (Sec. 4.3, Fig. 6): the
// plans' subqueries are searched together in multi-pattern passes over the
// graph (the multi-key search of Sec. 4.1), filters on a scanned variable are
// applied during that search, then joins go left to right over the subquery
// results, followed by unions, projections and DISTINCT; every result is
// returned in lexicographic row order.  A batch of plans advances in
// lockstep, so the host waits for the device once per round for all plans.
#include "batch.hpp"

#include <deque>
#include "compact.hpp"

#include <map>
#include <string>

#include <algorithm>

namespace tid {

std::unique_ptr<tid_table> union_tables(tid_ctx *, const tid_table *const *, int, int);
std::unique_ptr<tid_table> sort_rows(tid_ctx *ctx, const tid_table *t, uint64_t n, int distinct);

// Rows whose column pairs (a[p], b[p]) are all equal, keeping the listed columns.
struct EqSrc {
    const uint32_t *in[TID_MAX_COLS];
    int keep[TID_MAX_COLS];
    int a[TID_MAX_COLS], b[TID_MAX_COLS];
    int npairs;
    uint64_t n;
    using Item = uint64_t;
    __device__ __forceinline__ Item load(uint64_t i) const { return i; }
    __device__ __forceinline__ bool match(int, Item i) const {
        for (int p = 0; p < npairs; ++p)
            if (in[a[p]][i] != in[b[p]][i]) return false;
        return true;
    }
    __device__ __forceinline__ uint32_t value(int, int c, Item i, uint64_t) const {
        return in[keep[c]][i];
    }
};

static std::unique_ptr<tid_table> select_equal(tid_ctx *ctx, const tid_table *t,
                                               const std::vector<std::pair<int, int>> &pairs,
                                               const std::vector<int> &keep) {
    const uint64_t n = const_cast<tid_table *>(t)->rows();
    std::vector<int32_t> vars;
    for (int c : keep) vars.push_back(t->vars[c]);
    auto out = make_table(ctx, (int)keep.size(), vars.data(), n);
    out->maxv_known = t->maxv_known;
    copy_bounds(out.get(), t, keep.data(), (int)keep.size());
    if (n == 0) {
        set_count(ctx, out.get(), 0);
        return out;
    }
    EqSrc src{};
    for (int c = 0; c < t->ncols; ++c) src.in[c] = t->col[c];
    for (size_t c = 0; c < keep.size(); ++c) src.keep[c] = keep[c];
    src.npairs = (int)pairs.size();
    for (size_t p = 0; p < pairs.size(); ++p) {
        src.a[p] = pairs[p].first;
        src.b[p] = pairs[p].second;
    }
    src.n = n;
    CompactArgs<1, TID_MAX_COLS> a{};
    for (size_t c = 0; c < keep.size(); ++c) a.out[0].col[c] = out->col[c];
    a.out[0].cap = n;
    a.out[0].count = out->d_count;
    a.out[0].ncols = (int)keep.size();
    launch_compact<EqSrc, 256, 16, 1, TID_MAX_COLS>(ctx, src, a, 1, 8192);
    return out;
}

static int col_of(const tid_table *t, int32_t var) {
    for (int c = 0; c < t->ncols; ++c)
        if (t->vars[c] == var) return c;
    return -1;
}

// Keep the listed variables, in that order, without copying: the columns of
// the consumed table are re-pointed.
static std::unique_ptr<tid_table> project(std::unique_ptr<tid_table> t,
                                          const std::vector<int32_t> &vars) {
    auto out = std::make_unique<tid_table>();
    out->ctx = t->ctx;
    out->ncols = (int32_t)vars.size();
    for (size_t j = 0; j < vars.size(); ++j) {
        const int c = col_of(t.get(), vars[j]);
        TID_REQUIRE(c >= 0, TID_E_SCHEMA, "project: variable not in the table");
        for (size_t i = 0; i < j; ++i)
            TID_REQUIRE(vars[i] != vars[j], TID_E_SCHEMA, "project: variable listed twice");
        out->vars[j] = vars[j];
        out->col[j] = t->col[c];
        out->maxv[j] = t->maxv[c];
    }
    out->maxv_known = t->maxv_known;
    out->cap = t->cap;
    out->nrows = t->nrows;
    out->count_known = t->count_known;
    out->d_count = t->d_count;
    out->block = std::move(t->block);
    return out;
}

struct Entry {
    std::unique_ptr<tid_table> t;
    bool sorted = false;
};

// One plan in flight: its compiled scans, its stack, and the join (if any)
// waiting for its output size.
// Where a scan sits in the semi-join rounds of its plan: the round it runs in,
// and the scan whose rows filter it on a shared variable (-1: unfiltered).
struct ScanRound {
    int round = 0;
    int src = -1;
    int32_t var = -1;
};

struct PlanRun {
    const tid_plan *plan = nullptr;
    std::vector<tid_pattern> scans;
    std::vector<PatternSet> sets;  // per scan: a value set for one position, if any
    std::vector<ScanRound> rounds; // per scan
    bool conjunctive = false;      // the result is the natural join of all its scans
    std::vector<int> scan_at_op;   // per op: scan index, or kAbsorbed for a fused union member
    std::vector<char> fused;       // per op: FILTER run inside its scan / UNION of one table
    std::vector<std::unique_ptr<tid_table>> scanned;
    int pc = 0;
    std::vector<Entry> st;
    std::unique_ptr<PendingJoin> pj;
    JoinJob sj{};                  // the job of pj when it is a small join
    BigExpand bx{};                // the expansion of pj when it is a larger batched join
    std::vector<std::pair<int, int>> pj_eq;
    std::vector<int> pj_keep;
    std::unique_ptr<tid_table> result;
    bool done = false;
};

struct Needs {
    std::vector<tid_table *> tables;
    std::vector<PendingJoin *> joins;
};

constexpr int kAbsorbed = -2;

// A UNION of the k scans just pushed (k consecutive SCAN ops right before it)
// whose patterns bind the same variables at the same positions, carry the
// same range, and differ in exactly one position, where each holds a
// distinct constant, is one scan of a pattern whose value there is any of
// those constants: no triple matches two of the scans, so the rows are the
// same multiset, found in one pass over the graph (the union's result is
// sorted afterwards either way).
static void fuse_union(PlanRun &r, int pc, int k) {
    const uint32_t *ops = r.plan->ops;
    if (k < 2 || k > kMaxSet || pc < 2 * k) return;
    for (int j = 0; j < k; ++j) {
        const int at = pc - 2 * k + 2 * j;
        if (ops[at] != TID_OP_SCAN || r.scan_at_op[at] < 0) return;
    }
    const int first = r.scan_at_op[pc - 2 * k];
    if (first + k != (int)r.scans.size()) return;
    const tid_pattern *q = &r.scans[first];
    for (int j = 0; j < k; ++j)
        if (r.sets[first + j].pos >= 0) return;
    auto consts = [](const tid_pattern &p, int x) { return x == 0 ? p.s : x == 1 ? p.p : p.o; };
    int pos = -1;
    for (int x = 0; x < 3; ++x)
        for (int j = 1; j < k; ++j)
            if (consts(q[j], x) != consts(q[0], x)) {
                if (pos >= 0 && pos != x) return;
                pos = x;
            }
    if (pos < 0) return;
    for (int j = 0; j < k; ++j) {
        if (q[j].vs != q[0].vs || q[j].vp != q[0].vp || q[j].vo != q[0].vo) return;
        if (q[j].range_pos != q[0].range_pos) return;
        if (q[0].range_pos >= 0 && (q[j].lo != q[0].lo || q[j].hi != q[0].hi)) return;
        if (consts(q[j], pos) == 0) return;
        for (int i = 0; i < j; ++i)
            if (consts(q[i], pos) == consts(q[j], pos)) return;
    }
    PatternSet set;
    set.pos = pos;
    set.n = k;
    for (int j = 0; j < k; ++j) set.v[j] = consts(q[j], pos);
    r.sets[first] = set;
    r.scans.resize(first + 1);
    r.sets.resize(first + 1);
    for (int j = 1; j < k; ++j) r.scan_at_op[pc - 2 * k + 2 * j] = kAbsorbed;
    r.fused[pc] = 1;
}

// Check the op stream and list one scan per SCAN op.  A FILTER right after a
// SCAN on a variable that the pattern binds (and with no range yet) becomes
// the pattern's range: the filter runs inside the search (Fig. 6).  A UNION
// of compatible scans becomes one scan (fuse_union).
static void compile_plan(const tid_plan *plan, PlanRun &r) {
    TID_REQUIRE(plan, TID_E_INVALID_ARG, "plan: null");
    TID_REQUIRE(plan->n_patterns >= 0 && plan->n_ops >= 0, TID_E_INVALID_ARG, "plan: bad sizes");
    TID_REQUIRE(plan->n_patterns == 0 || plan->patterns, TID_E_INVALID_ARG, "plan: no patterns");
    TID_REQUIRE(plan->n_ops > 0 && plan->ops, TID_E_INVALID_ARG, "plan: no ops");
    r.plan = plan;
    const uint32_t *ops = plan->ops;
    const int nops = plan->n_ops;
    r.scan_at_op.assign(nops, -1);
    r.fused.assign(nops, 0);
    int depth = 0;
    for (int pc = 0; pc < nops;) {
        const uint32_t op = ops[pc];
        auto need = [&](int words) {
            TID_REQUIRE(pc + words <= nops, TID_E_INVALID_ARG, "plan: truncated op");
        };
        if (op == TID_OP_SCAN) {
            need(2);
            const uint32_t i = ops[pc + 1];
            TID_REQUIRE(i < (uint32_t)plan->n_patterns, TID_E_INVALID_ARG,
                        "plan: pattern index out of range");
            int32_t vars[3], src[3];
            pattern_schema(plan->patterns[i], vars, src);
            tid_pattern p = plan->patterns[i];
            if (pc + 6 <= nops && ops[pc + 2] == TID_OP_FILTER && p.range_pos < 0) {
                const int32_t v = (int32_t)ops[pc + 3];
                const int32_t pv[3] = {p.vs, p.vp, p.vo};
                int pos = -1;
                for (int x = 0; x < 3; ++x)
                    if (pv[x] >= 0 && pv[x] == v) pos = x;
                if (pos >= 0) {
                    p.range_pos = pos;
                    p.lo = ops[pc + 4];
                    p.hi = ops[pc + 5];
                    r.fused[pc + 2] = 1;
                }
            }
            r.scan_at_op[pc] = (int)r.scans.size();
            r.scans.push_back(p);
            r.sets.emplace_back();
            ++depth;
            pc += 2;
        } else if (op == TID_OP_JOIN) {
            need(2);
            TID_REQUIRE(depth >= 2, TID_E_INVALID_ARG, "plan: JOIN needs two tables");
            --depth;
            pc += 2;
        } else if (op == TID_OP_OPTIONAL) {
            need(2);
            TID_REQUIRE(depth >= 2, TID_E_INVALID_ARG, "plan: OPTIONAL needs two tables");
            --depth;
            pc += 2;
        } else if (op == TID_OP_UNION) {
            need(3);
            const uint32_t k = ops[pc + 1];
            TID_REQUIRE(k >= 1 && (int)k <= depth, TID_E_INVALID_ARG, "plan: bad UNION arity");
            fuse_union(r, pc, (int)k);
            depth -= (int)k - 1;
            pc += 3;
        } else if (op == TID_OP_FILTER) {
            need(4);
            TID_REQUIRE(depth >= 1, TID_E_INVALID_ARG, "plan: FILTER on an empty stack");
            pc += 4;
        } else if (op == TID_OP_PROJECT) {
            need(2);
            const uint32_t n = ops[pc + 1];
            TID_REQUIRE(n <= TID_MAX_COLS, TID_E_INVALID_ARG, "plan: PROJECT too wide");
            need(2 + (int)n);
            TID_REQUIRE(depth >= 1, TID_E_INVALID_ARG, "plan: PROJECT on an empty stack");
            pc += 2 + (int)n;
        } else if (op == TID_OP_DISTINCT) {
            TID_REQUIRE(depth >= 1, TID_E_INVALID_ARG, "plan: DISTINCT on an empty stack");
            pc += 1;
        } else {
            throw Error(TID_E_INVALID_ARG, "plan: unknown op " + std::to_string(op));
        }
    }
    TID_REQUIRE(depth == 1, TID_E_INVALID_ARG, "plan: must leave exactly one table");
    r.scanned.resize(r.scans.size());
    r.rounds.assign(r.scans.size(), ScanRound{});
    // Conjunctive: at least one JOIN, no UNION, and nothing but SCAN, JOIN and
    // FILTER up to the last JOIN.  Every JOIN is a natural join (all shared
    // variables must agree) and filters only remove rows, so the result is
    // the natural join of all scans, filtered, then projected or deduplicated.
    int last_join = -1;
    for (int pc = 0; pc < nops;) {
        const uint32_t op = ops[pc];
        if (op == TID_OP_JOIN) last_join = pc;
        pc += op == TID_OP_SCAN || op == TID_OP_JOIN || op == TID_OP_OPTIONAL ? 2
            : op == TID_OP_UNION ? 3 : op == TID_OP_FILTER ? 4
            : op == TID_OP_PROJECT ? 2 + (int)ops[pc + 1] : 1;
    }
    // an OPTIONAL keeps rows without a partner: such a plan is not the natural
    // join of its scans, and no scan of it is filtered by another
    bool conj = last_join >= 0;
    for (int pc = 0; pc < nops && conj;) {
        const uint32_t op = ops[pc];
        if (op == TID_OP_UNION || op == TID_OP_OPTIONAL) conj = false;
        if (pc < last_join && op != TID_OP_SCAN && op != TID_OP_JOIN && op != TID_OP_FILTER)
            conj = false;
        pc += op == TID_OP_SCAN || op == TID_OP_JOIN || op == TID_OP_OPTIONAL ? 2
            : op == TID_OP_UNION ? 3 : op == TID_OP_FILTER ? 4
            : op == TID_OP_PROJECT ? 2 + (int)ops[pc + 1] : 1;
    }
    r.conjunctive = conj;
}

static bool binds(const tid_pattern &p, int32_t v) { return p.vs == v || p.vp == v || p.vo == v; }

static int position_of(const tid_pattern &p, int32_t v) {
    return p.vs == v ? 0 : p.vp == v ? 1 : p.vo == v ? 2 : -1;
}

// Semi-join rounds of a conjunctive plan (Sec. 4.2 joins, reduced first):
// the scan with the smallest bound runs unfiltered in round 0; going outward
// over the scans that share a variable, each large scan is filtered by the
// smallest already-placed scan it shares a variable with, one round after
// it.  A scan whose bound is under `min_rows`, or under 8x its filter
// source's, is not worth a round and runs unfiltered in round 0.
static void plan_rounds(const tid_graph *g, PlanRun &r, uint64_t min_rows) {
    const int n = (int)r.scans.size();
    if (!r.conjunctive || n < 2) return;
    std::vector<uint64_t> bound(n);
    for (int i = 0; i < n; ++i) bound[i] = pattern_output_bound(g, r.scans[i], &r.sets[i]);
    int seed = 0;
    for (int i = 1; i < n; ++i)
        if (bound[i] < bound[seed]) seed = i;
    std::vector<char> placed(n, 0);
    std::vector<int> queue{seed};
    placed[seed] = 1;
    for (size_t qi = 0; qi < queue.size(); ++qi) {
        const int u = queue[qi];
        const tid_pattern &pu = r.scans[u];
        const int32_t uv[3] = {pu.vs, pu.vp, pu.vo};
        for (int j = 0; j < n; ++j) {
            if (placed[j]) continue;
            bool shares = false;
            for (int x = 0; x < 3; ++x) shares |= uv[x] >= 0 && binds(r.scans[j], uv[x]);
            if (!shares) continue;
            // filter source: the smallest placed scan sharing a variable with j
            int src = -1;
            int32_t var = -1;
            for (int i = 0; i < n; ++i) {
                if (!placed[i]) continue;
                const tid_pattern &pi = r.scans[i];
                const int32_t iv[3] = {pi.vs, pi.vp, pi.vo};
                for (int x = 0; x < 3; ++x)
                    if (iv[x] >= 0 && binds(r.scans[j], iv[x]) &&
                        (src < 0 || bound[i] < bound[src])) {
                        src = i;
                        var = iv[x];
                    }
            }
            placed[j] = 1;
            queue.push_back(j);
            if (bound[j] >= min_rows && bound[j] >= 8 * bound[src])
                r.rounds[j] = ScanRound{r.rounds[src].round + 1, src, var};
        }
    }
}

// Scans that compute the same rows: the pattern with its variables renamed
// by first appearance, its value set and its filter.
static std::string scan_key(const tid_pattern &p, const PatternSet &set, const ScanFilter &f) {
    tid_pattern q = p;
    int32_t *v[3] = {&q.vs, &q.vp, &q.vo};
    int32_t seen[3] = {-1, -1, -1};
    int nseen = 0;
    for (int x = 0; x < 3; ++x) {
        if (*v[x] < 0) continue;
        int id = -1;
        for (int i = 0; i < nseen; ++i)
            if (seen[i] == *v[x]) id = i;
        if (id < 0) {
            seen[nseen] = *v[x];
            id = nseen++;
        }
        *v[x] = id;
    }
    std::string k(reinterpret_cast<const char *>(&q), sizeof q);
    k.append(reinterpret_cast<const char *>(&set.pos), sizeof set.pos);
    k.append(reinterpret_cast<const char *>(&set.n), sizeof set.n);
    k.append(reinterpret_cast<const char *>(set.v), sizeof(uint32_t) * (size_t)std::max(set.n, 0));
    k.append(reinterpret_cast<const char *>(&f.bits), sizeof f.bits);
    k.append(reinterpret_cast<const char *>(&f.mask), sizeof f.mask);
    k.append(reinterpret_cast<const char *>(&f.pos), sizeof f.pos);
    k.append(reinterpret_cast<const char *>(&f.index), sizeof f.index);
    k.append(reinterpret_cast<const char *>(&f.keys), sizeof f.keys);
    k.append(reinterpret_cast<const char *>(&f.nkeys), sizeof f.nkeys);
    return k;
}

// The same rows under the variable ids of pattern p (no copy: the columns
// are shared).
static std::unique_ptr<tid_table> alias_table(const tid_table *t, const tid_pattern &p) {
    auto out = std::make_unique<tid_table>(*t);
    int32_t vars[3], src[3];
    const int nc = pattern_schema(p, vars, src);
    TID_REQUIRE(nc == t->ncols, TID_E_INTERNAL, "scan alias: schema mismatch");
    for (int c = 0; c < nc; ++c) out->vars[c] = vars[c];
    return out;
}

// Whether a scan filtered on position `pos` by a source of `rows` rows is a
// semi-join by index (index_semijoin): the partitioned layout is built and
// used, the pattern has a constant predicate and a free subject and object
// (no other test), and the source is small against the predicate's rows
// (option index_ratio: a lookup per source value then costs less than
// testing every row).
static bool index_semijoin_ok(tid_ctx *ctx, const tid_graph *g, const tid_pattern &p,
                              const PatternSet &set, int pos, uint64_t rows) {
    if (!g->partitioned || !ctx->opt.layout || !ctx->opt.index_semijoin ||
        ctx->opt.capacity_override > 0 || g->cdf[1].empty())
        return false;
    if (p.p == 0 || p.s != 0 || p.o != 0 || p.range_pos >= 0 || (p.vs >= 0 && p.vs == p.vo) ||
        set.pos >= 0 || (pos != 0 && pos != 2) || rows >= (1ull << 32))
        return false;
    return (uint64_t)ctx->opt.index_ratio * rows <= g->count_in(1, p.p, (uint64_t)p.p + 1);
}

// One Bloom filter per job: the values of a table column.
struct BloomJob {
    const uint32_t *vals;
    uint64_t n;
    uint32_t *bits;
    uint32_t mask;
};

__global__ void bloom_build(const BloomJob *jobs) {
    const BloomJob j = jobs[blockIdx.y];
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < j.n; i += stride)
        dev::bloom_add(j.bits, j.mask, j.vals[i]);
}

static bool need_count(tid_table *t, Needs &needs) {
    if (t->count_known) return false;
    needs.tables.push_back(t);
    return true;
}

// Run the plan's ops until one needs a value that is still on the device.
static void advance(tid_ctx *ctx, PlanRun &r, Needs &needs, BatchState *bs) {
    const uint32_t *ops = r.plan->ops;
    const int nops = r.plan->n_ops;
    while (!r.done) {
        if (r.pj) {
            if (!r.pj->total_known) {
                needs.joins.push_back(r.pj.get());
                return;
            }
            if (r.pj->small || r.pj->big) {  // expanded by the round's batched launch
                TID_REQUIRE(r.pj->small_result, TID_E_INTERNAL, "batched join not expanded");
                auto t = std::move(r.pj->small_result);
                r.pj.reset();
                r.st.push_back({std::move(t), false});
                continue;
            }
            auto raw = join_finish(ctx, *r.pj);
            r.pj.reset();  // inputs go back to the allocator in stream order
            if (r.pj_eq.empty())
                r.st.push_back({std::move(raw), false});
            else
                r.st.push_back({select_equal(ctx, raw.get(), r.pj_eq, r.pj_keep), false});
            continue;
        }
        if (r.pc >= nops) {
            Entry &top = r.st.back();
            if (top.sorted) {
                r.result = std::move(top.t);
                r.done = true;
                return;
            }
            if (need_count(top.t.get(), needs)) return;
            const tid_table *T = top.t.get();
            if (bs && ctx->opt.batch_small && T->ncols > 0 && T->ncols <= kSortCols &&
                T->nrows > 1 && T->nrows <= kSortRows &&
                T->nrows * (uint64_t)T->ncols <= kSortWords) {
                // one job of the round's batched sort; the input stays alive
                // in the batch state until the round's wait
                auto out = make_table(ctx, T->ncols, T->vars, T->nrows);
                out->maxv_known = T->maxv_known;
                copy_bounds(out.get(), T, nullptr, T->ncols);
                SortJob j{};
                for (int c = 0; c < T->ncols; ++c) {
                    j.in[c] = T->col[c];
                    j.out[c] = out->col[c];
                }
                j.n = (uint32_t)T->nrows;
                j.ncols = T->ncols;
                j.distinct = 0;
                j.count = out->d_count;
                bs->sort_jobs.push_back(j);
                bs->keep_tables.push_back(std::move(top.t));
                r.result = std::move(out);
                r.done = true;
                return;
            }
            if (bs && ctx->opt.batch_small && T->ncols > 0 && T->maxv_known &&
                T->nrows > 1 && T->nrows < (1ull << 32)) {
                // one job of the round's batched larger sorts; the input stays
                // alive in the batch state until the round's wait
                auto out = make_table(ctx, T->ncols, T->vars, T->nrows);
                out->maxv_known = T->maxv_known;
                copy_bounds(out.get(), T, nullptr, T->ncols);
                set_count_later(ctx, out.get(), T->nrows);  // a result: not freed this round
                bs->row_sorts.push_back(RowSortJob{T, out.get(), T->nrows});
                bs->keep_tables.push_back(std::move(top.t));
                r.result = std::move(out);
                r.done = true;
                return;
            }
            r.result = sort_rows(ctx, top.t.get(), top.t->nrows, 0);
            r.done = true;
            return;
        }
        const int pc = r.pc;
        const uint32_t op = ops[pc];
        if (op == TID_OP_SCAN) {
            if (r.scan_at_op[pc] != kAbsorbed)
                r.st.push_back({std::move(r.scanned[r.scan_at_op[pc]]), false});
            r.pc += 2;
        } else if (op == TID_OP_JOIN) {
            tid_table *L = r.st[r.st.size() - 2].t.get();
            tid_table *R = r.st.back().t.get();
            const bool wl = need_count(L, needs), wr = need_count(R, needs);
            if (wl || wr) return;
            const int32_t v = (int32_t)ops[pc + 1];
            const int lc = col_of(L, v), rc = col_of(R, v);
            TID_REQUIRE(lc >= 0 && rc >= 0, TID_E_SCHEMA, "join: variable not bound on both sides");
            // every other variable both sides hold must agree; it is kept once
            JoinPlan jp;
            for (int c = 0; c < L->ncols; ++c) jp.lkeep.push_back(c);
            r.pj_eq.clear();
            r.pj_keep.clear();
            for (int c = 0; c < L->ncols; ++c) r.pj_keep.push_back(c);
            for (int c = 0; c < R->ncols; ++c) {
                if (c == rc) continue;
                const int out_col = L->ncols + (int)jp.rkeep.size();
                jp.rkeep.push_back(c);
                const int lmatch = col_of(L, R->vars[c]);
                if (lmatch >= 0)
                    r.pj_eq.emplace_back(lmatch, out_col);
                else
                    r.pj_keep.push_back(out_col);
            }
            const int nkeep = (int)r.pj_keep.size() - L->ncols;
            if (bs && ctx->opt.batch_small && L->nrows > 0 && R->nrows > 0 &&
                L->nrows <= kSmallRows && R->nrows <= kSmallRows && L->ncols <= kSmallCols &&
                nkeep <= kSmallCols && (int)r.pj_eq.size() <= kSmallEq) {
                // a job of this round's batched count; expanded next round
                auto pj = std::make_unique<PendingJoin>();
                pj->small = true;
                pj->L = L;
                pj->R = R;
                // offsets; without other shared variables also the L rows'
                // key group starts and R's rows grouped by key
                const uint64_t lists = r.pj_eq.empty() ? L->nrows + R->nrows : 0;
                pj->sj_off = DevBuf(ctx, (L->nrows + 1 + lists) * 4);
                pj->sj_total = DevBuf(ctx, 8);
                JoinJob &j = r.sj;
                j = JoinJob{};
                j.lkey = L->col[lc];
                j.rkey = R->col[rc];
                j.nl = (uint32_t)L->nrows;
                j.nr = (uint32_t)R->nrows;
                j.neq = (int)r.pj_eq.size();
                for (int e = 0; e < j.neq; ++e) {
                    j.eq_l[e] = L->col[r.pj_eq[e].first];
                    // the pair names an output column: L's columns, then R's kept ones
                    j.eq_r[e] = R->col[jp.rkeep[r.pj_eq[e].second - L->ncols]];
                }
                j.nlc = L->ncols;
                for (int c = 0; c < L->ncols; ++c) j.lcol[c] = L->col[c];
                j.nrc = 0;
                for (size_t k = L->ncols; k < r.pj_keep.size(); ++k)
                    j.rcol[j.nrc++] = R->col[jp.rkeep[r.pj_keep[k] - L->ncols]];
                j.off = pj->sj_off.get<uint32_t>();
                if (j.neq == 0) {
                    j.lbase = j.off + j.nl + 1;
                    j.grp = j.lbase + j.nl;
                }
                j.total = pj->sj_total.get<uint64_t>();
                for (int c = 0; c < L->ncols; ++c) pj->vars.push_back(L->vars[c]);
                for (int c = 0; c < j.nrc; ++c)
                    pj->vars.push_back(R->vars[jp.rkeep[r.pj_keep[L->ncols + c] - L->ncols]]);
                bs->count_jobs.push_back(j);
                r.pj = std::move(pj);
                r.pj_eq.clear();
                r.pj->own_r = std::move(r.st.back().t);
                r.st.pop_back();
                r.pj->own_l = std::move(r.st.back().t);
                r.st.pop_back();
                r.pc += 2;
                continue;
            }
            if (bs && ctx->opt.batch_small && L->nrows > 0 && R->nrows > 0 &&
                std::min(L->nrows, R->nrows) <= kBigBuildMax &&
                (int)r.pj_eq.size() <= kSmallEq && L->ncols + nkeep <= kBigCols) {
                // counted with this round's other larger joins, expanded next round;
                // the hash is built on the smaller side
                auto pj = std::make_unique<PendingJoin>();
                pj->big = true;
                pj->L = L;
                pj->R = R;
                const bool probe_left = R->nrows <= L->nrows;
                BigJoinReq q{};
                BigCount &c = q.c;
                c.lkey = probe_left ? L->col[lc] : R->col[rc];
                c.rkey = probe_left ? R->col[rc] : L->col[lc];
                c.nl = probe_left ? L->nrows : R->nrows;
                c.nr = probe_left ? R->nrows : L->nrows;
                c.neq = (int)r.pj_eq.size();
                BigExpand &x = r.bx;
                x = BigExpand{};
                x.nl = c.nl;
                x.neq = c.neq;
                x.probe_is_left = probe_left ? 1 : 0;
                for (int e = 0; e < c.neq; ++e) {
                    const uint32_t *lcol_e = L->col[r.pj_eq[e].first];
                    const uint32_t *rcol_e = R->col[jp.rkeep[r.pj_eq[e].second - L->ncols]];
                    c.eq_l[e] = x.eq_l[e] = probe_left ? lcol_e : rcol_e;
                    c.eq_r[e] = x.eq_r[e] = probe_left ? rcol_e : lcol_e;
                }
                x.nlc = L->ncols;
                for (int cc = 0; cc < L->ncols; ++cc) {
                    x.lcol[cc] = L->col[cc];
                    pj->vars.push_back(L->vars[cc]);
                }
                x.nrc = 0;
                for (size_t k = L->ncols; k < r.pj_keep.size(); ++k) {
                    const int rcx = jp.rkeep[r.pj_keep[k] - L->ncols];
                    x.rcol[x.nrc++] = R->col[rcx];
                    pj->vars.push_back(R->vars[rcx]);
                }
                q.pj = pj.get();
                bs->big_reqs.push_back(q);
                r.pj = std::move(pj);
                r.pj_eq.clear();
                r.pj->own_r = std::move(r.st.back().t);
                r.st.pop_back();
                r.pj->own_l = std::move(r.st.back().t);
                r.st.pop_back();
                r.pc += 2;
                continue;
            }
            r.pj = join_begin(ctx, L, L->nrows, lc, R, R->nrows, rc, 0, jp);
            r.pj->own_r = std::move(r.st.back().t);
            r.st.pop_back();
            r.pj->own_l = std::move(r.st.back().t);
            r.st.pop_back();
            r.pc += 2;
        } else if (op == TID_OP_OPTIONAL) {
            // SPARQL OPTIONAL: the left outer join on one shared variable
            tid_table *L = r.st[r.st.size() - 2].t.get();
            tid_table *R = r.st.back().t.get();
            const bool wl = need_count(L, needs), wr = need_count(R, needs);
            if (wl || wr) return;
            const int32_t v = (int32_t)ops[pc + 1];
            const int lc = col_of(L, v), rc = col_of(R, v);
            TID_REQUIRE(lc >= 0 && rc >= 0, TID_E_SCHEMA,
                        "optional: variable not bound on both sides");
            JoinPlan jp;
            for (int c = 0; c < L->ncols; ++c) jp.lkeep.push_back(c);
            for (int c = 0; c < R->ncols; ++c) {
                if (c == rc) continue;
                TID_REQUIRE(col_of(L, R->vars[c]) < 0, TID_E_UNSUPPORTED,
                            "optional: the two sides share a second variable");
                jp.rkeep.push_back(c);
            }
            r.pj_eq.clear();
            r.pj_keep.clear();
            r.pj = join_begin(ctx, L, L->nrows, lc, R, R->nrows, rc, 0, jp, kJoinLeft);
            r.pj->own_r = std::move(r.st.back().t);
            r.st.pop_back();
            r.pj->own_l = std::move(r.st.back().t);
            r.st.pop_back();
            r.pc += 2;
        } else if (op == TID_OP_UNION) {
            const int k = r.fused[pc] ? 1 : (int)ops[pc + 1];
            const int d = ops[pc + 2] ? 1 : 0;
            bool wait = false;
            std::vector<const tid_table *> ins;
            for (int j = 0; j < k; ++j) {
                tid_table *t = r.st[r.st.size() - k + j].t.get();
                wait |= need_count(t, needs);
                ins.push_back(t);
            }
            if (wait) return;
            auto u = union_tables(ctx, ins.data(), k, d);
            r.st.resize(r.st.size() - k);
            r.st.push_back({std::move(u), d == 1});
            r.pc += 3;
        } else if (op == TID_OP_FILTER) {
            if (!r.fused[pc]) {
                tid_table *t = r.st.back().t.get();
                if (need_count(t, needs)) return;
                const int c = col_of(t, (int32_t)ops[pc + 1]);
                TID_REQUIRE(c >= 0, TID_E_SCHEMA, "filter: variable not in the table");
                r.st.back().t = filter_range(ctx, t, c, ops[pc + 2], ops[pc + 3]);
            }
            r.pc += 4;  // filtering keeps row order
        } else if (op == TID_OP_PROJECT) {
            const int n = (int)ops[pc + 1];
            std::vector<int32_t> vars(ops + pc + 2, ops + pc + 2 + n);
            r.st.back().t = project(std::move(r.st.back().t), vars);
            r.st.back().sorted = false;
            r.pc += 2 + n;
        } else {  // DISTINCT
            tid_table *t = r.st.back().t.get();
            if (need_count(t, needs)) return;
            r.st.back().t = sort_rows(ctx, t, t->nrows, 1);
            r.st.back().sorted = true;
            r.pc += 1;
        }
    }
}

// Evaluate nq plans together: all their patterns in shared multi-pattern
// passes over the graph, then their remaining ops in lockstep, every round
// of device reads shared by all plans.
// pre (may be null): per plan, the tables of its compiled scans, already
// found (the circular serving scan); the plans then skip their scan rounds.
std::vector<std::unique_ptr<tid_table>> run_plans(
    tid_ctx *ctx, const tid_graph *g, const tid_plan *const *plans, int nq,
    std::vector<std::vector<std::unique_ptr<tid_table>>> *pre = nullptr) {
    PendingCountsGuard counts_guard(ctx);
    std::vector<PlanRun> runs(nq);
    int nrounds = pre ? 0 : 1;
    for (int i = 0; i < nq; ++i) {
        compile_plan(plans[i], runs[i]);
        if (pre) {
            TID_REQUIRE((*pre)[i].size() == runs[i].scans.size(), TID_E_INTERNAL,
                        "prescanned plan: scan count differs");
            for (size_t k = 0; k < runs[i].scans.size(); ++k)
                runs[i].scanned[k] = std::move((*pre)[i][k]);
            continue;
        }
        if (ctx->opt.semijoin) plan_rounds(g, runs[i], (uint64_t)ctx->opt.semijoin_min);
        for (const ScanRound &sr : runs[i].rounds) nrounds = std::max(nrounds, sr.round + 1);
    }
    // Scans in rounds: each round's patterns of all plans share passes over
    // the graph; a filtered scan's Bloom filter is built from its source
    // table, which an earlier round produced.
    for (int rd = 0; rd < nrounds; ++rd) {
        std::vector<tid_pattern> all;
        std::vector<PatternSet> all_sets;
        std::vector<ScanFilter> all_filters;
        std::vector<std::pair<int, int>> where;
        std::vector<tid_table *> sources;
        for (int i = 0; i < nq; ++i)
            for (size_t s = 0; s < runs[i].scans.size(); ++s) {
                const ScanRound &sr = runs[i].rounds[s];
                if (sr.round != rd) continue;
                all.push_back(runs[i].scans[s]);
                all_sets.push_back(runs[i].sets[s]);
                all_filters.emplace_back();
                where.emplace_back(i, (int)s);
                if (sr.src >= 0) sources.push_back(runs[i].scanned[sr.src].get());
            }
        if (all.empty()) continue;
        resolve_counts(ctx, sources.data(), (int)sources.size());
        // size the filters: 16 bits per source row, a power of two in [2^12, 2^28]
        std::vector<BloomJob> jobs;
        std::vector<size_t> at;
        size_t words = 0;
        for (size_t j = 0; j < all.size(); ++j) {
            const ScanRound &sr = runs[where[j].first].rounds[where[j].second];
            if (sr.src < 0) continue;
            const tid_table *S = runs[where[j].first].scanned[sr.src].get();
            const int c = col_of(S, sr.var);
            TID_REQUIRE(c >= 0, TID_E_INTERNAL, "semi-join: source lacks the variable");
            const int fpos = position_of(all[j], sr.var);
            if (index_semijoin_ok(ctx, g, all[j], all_sets[j], fpos, S->nrows)) {
                ScanFilter &f = all_filters[j];
                f.pos = fpos;
                f.index = 1;
                f.keys = S->col[c];
                f.nkeys = S->nrows;
                f.key_max = S->maxv_known ? S->maxv[c]
                                          : std::max({g->max_id[0], g->max_id[1], g->max_id[2]});
                continue;  // no Bloom filter
            }
            uint64_t bits = 4096;
            while (bits < 16 * S->nrows && bits < (1ull << 28)) bits <<= 1;
            jobs.push_back(BloomJob{S->col[c], S->nrows, nullptr, (uint32_t)(bits - 1)});
            at.push_back(j);
            all_filters[j].pos = position_of(all[j], sr.var);
            all_filters[j].mask = (uint32_t)(bits - 1);
            words += bits / 32;
        }
        DevBuf filter_bits(ctx, words * 4), job_table(ctx, jobs.size() * sizeof(BloomJob));
        if (!jobs.empty()) {
            size_t w = 0;
            uint64_t most = 0;
            for (size_t x = 0; x < jobs.size(); ++x) {
                jobs[x].bits = filter_bits.get<uint32_t>() + w;
                all_filters[at[x]].bits = jobs[x].bits;
                w += ((uint64_t)jobs[x].mask + 1) / 32;
                most = std::max(most, jobs[x].n);
            }
            TID_HIP(hipMemsetAsync(filter_bits.get(), 0, words * 4, ctx->stream));
            TID_HIP(hipMemcpyAsync(job_table.get(), jobs.data(), jobs.size() * sizeof(BloomJob),
                                   hipMemcpyHostToDevice, ctx->stream));
            const unsigned gx = (unsigned)std::max<uint64_t>(
                1, std::min<uint64_t>((most + 255) / 256, 256));
            for (size_t y0 = 0; y0 < jobs.size(); y0 += 65535) {
                const unsigned gy = (unsigned)std::min<size_t>(65535, jobs.size() - y0);
                hipLaunchKernelGGL(bloom_build, dim3(gx, gy), dim3(256), 0, ctx->stream,
                                   job_table.get<const BloomJob>() + y0);
                TID_HIP(hipGetLastError());
            }
        }
        // identical scans (across plans) run once; the others alias the result
        std::map<std::string, size_t> uniq;
        std::vector<size_t> rep(all.size());
        std::vector<tid_pattern> upats;
        std::vector<PatternSet> usets;
        std::vector<ScanFilter> ufilters;
        for (size_t j = 0; j < all.size(); ++j) {
            const auto ins =
                uniq.emplace(scan_key(all[j], all_sets[j], all_filters[j]), upats.size());
            rep[j] = ins.first->second;
            if (ins.second) {
                upats.push_back(all[j]);
                usets.push_back(all_sets[j]);
                ufilters.push_back(all_filters[j]);
            }
        }
        std::vector<std::unique_ptr<tid_table>> outs(upats.size());
        scan_many(ctx, g, upats.data(), (int)upats.size(), outs.data(), usets.data(),
                  ufilters.data());
        for (size_t j = 0; j < all.size(); ++j)
            runs[where[j].first].scanned[where[j].second] = alias_table(outs[rep[j]].get(), all[j]);
    }
    BatchState bs;
    for (;;) {
        // expand the small joins whose sizes reached the host: one launch
        for (auto &r : runs) {
            if (!r.pj || !r.pj->small || !r.pj->total_known || r.pj->small_result) continue;
            auto t = make_table(ctx, (int)r.pj->vars.size(), r.pj->vars.data(), r.pj->total);
            const tid_table *L = r.pj->own_l.get(), *R = r.pj->own_r.get();
            t->maxv_known = L->maxv_known && R->maxv_known;
            if (t->maxv_known) {
                for (int c = 0; c < r.sj.nlc; ++c) t->maxv[c] = L->maxv[c];
                for (int c = 0; c < r.sj.nrc; ++c)
                    for (int x = 0; x < R->ncols; ++x)
                        if (R->col[x] == r.sj.rcol[c]) t->maxv[r.sj.nlc + c] = R->maxv[x];
            }
            if (r.pj->total) {
                JoinJob j = r.sj;
                for (int c = 0; c < t->ncols; ++c) j.out[c] = t->col[c];
                j.nout = (uint32_t)r.pj->total;  // at most kSmallRows^2
                bs.expand_jobs.push_back(j);
            }
            set_count_later(ctx, t.get(), r.pj->total);
            r.pj->small_result = std::move(t);
        }
        flush_join_jobs(ctx, bs, true);
        // expand the larger joins whose sizes reached the host: one launch
        // (all were counted in the previous round, in one arena)
        std::shared_ptr<BigArena> arena;
        for (auto &r : runs) {
            if (!r.pj || !r.pj->big || !r.pj->total_known || r.pj->small_result) continue;
            arena = std::static_pointer_cast<BigArena>(r.pj->big_arena);
            auto t = make_table(ctx, (int)r.pj->vars.size(), r.pj->vars.data(), r.pj->total);
            const tid_table *L = r.pj->own_l.get(), *R = r.pj->own_r.get();
            t->maxv_known = L->maxv_known && R->maxv_known;
            if (t->maxv_known) {
                for (int c = 0; c < r.bx.nlc; ++c) t->maxv[c] = L->maxv[c];
                for (int c = 0; c < r.bx.nrc; ++c)
                    for (int x = 0; x < R->ncols; ++x)
                        if (R->col[x] == r.bx.rcol[c]) t->maxv[r.bx.nlc + c] = R->maxv[x];
            }
            if (r.pj->total) {
                TID_REQUIRE(r.pj->total < (1ull << 40), TID_E_UNSUPPORTED, "join: output too large");
                BigExpand x = r.bx;
                x.lbase = r.pj->big_lbase;
                x.obase = bs.big_out_total;
                for (int c = 0; c < t->ncols; ++c) x.out[c] = t->col[c];
                bs.big_out_total += r.pj->total;
                bs.big_expand_jobs.push_back(x);
            }
            set_count_later(ctx, t.get(), r.pj->total);
            r.pj->small_result = std::move(t);
        }
        if (arena) flush_big_expand(ctx, *arena, bs.big_expand_jobs, bs);
        flush_counts(ctx);  // before any plan can consume (and free) these tables
        Needs needs;
        bool all_done = true;
        for (auto &r : runs) {
            if (!r.done) advance(ctx, r, needs, &bs);
            all_done &= r.done;
        }
        flush_join_jobs(ctx, bs, false);
        flush_sort_jobs(ctx, bs);
        flush_counts(ctx);
        std::shared_ptr<BigArena> fresh;
        flush_big_count(ctx, bs.big_reqs, &fresh);
        if (all_done) break;
        std::vector<const uint64_t *> src;
        for (tid_table *t : needs.tables) src.push_back(t->d_count);
        for (PendingJoin *j : needs.joins) src.push_back(j->d_total());
        TID_REQUIRE(!src.empty(), TID_E_INTERNAL, "query: no progress");
        std::vector<uint64_t> v(src.size());
        read_words(ctx, src, v.data());
        bs.keep.clear();         // the round's launches have completed
        bs.host_keep.clear();
        bs.keep_tables.clear();
        size_t at = 0;
        for (tid_table *t : needs.tables) {
            t->nrows = v[at++];
            t->count_known = true;
        }
        for (PendingJoin *j : needs.joins) {
            j->total = v[at++];
            j->total_known = true;
        }
    }
    // the last round's batched sorts read tables kept in `bs`: wait for them
    // before those go back to the pool
    if (!bs.keep.empty() || !bs.keep_tables.empty()) ctx->sync();
    std::vector<std::unique_ptr<tid_table>> out(nq);
    for (int i = 0; i < nq; ++i) out[i] = std::move(runs[i].result);
    return out;
}

// Device bytes the plan's scans will hold (their outputs are sized by the
// load-time histograms), times two for the intermediate results of joins.
uint64_t estimate_plan_bytes(const tid_graph *g, const tid_plan *plan) {
    PlanRun r;
    compile_plan(plan, r);
    uint64_t bytes = 0;
    for (size_t i = 0; i < r.scans.size(); ++i) {
        int32_t vars[3], src[3];
        const int nc = pattern_schema(r.scans[i], vars, src);
        bytes += pattern_output_bound(g, r.scans[i], &r.sets[i]) * 4ull *
                 (uint64_t)std::max(nc, 1);
    }
    return 2 * bytes;
}

std::unique_ptr<tid_table> run_query(tid_ctx *ctx, const tid_graph *g, const tid_plan *plan) {
    auto v = run_plans(ctx, g, &plan, 1);
    return std::move(v[0]);
}

// ---------------------------------------------------------------------------
// Serving with a circular chunked shared scan.  The graph is cut into C
// contiguous chunks; one step scans the next chunk for the compiled scans of
// every admitted query (one shared pass, as a batch's scans share passes).  A
// query is admitted at a chunk boundary, into a free slot, and has seen the
// whole graph one revolution later; its per-chunk tables are then joined end
// to end in chunk order (so its scans equal a scan of the whole graph, rows
// in ascending triple position), and its remaining ops run with those of the
// other queries completing at the same step, in lockstep (run_plans).
// ---------------------------------------------------------------------------

void chunk_stats(tid_ctx *ctx, tid_graph *v);
void scan_many(tid_ctx *ctx, const tid_graph *g, const tid_pattern *pats, int k,
               std::unique_ptr<tid_table> *outs, const PatternSet *sets,
               const ScanFilter *filters);

struct ServeQuery {
    uint64_t ticket = 0;
    std::vector<tid_pattern> pats;
    std::vector<uint32_t> ops;
    tid_plan plan{};
    PlanRun pr;
    uint32_t seen = 0;
    std::vector<std::vector<std::unique_ptr<tid_table>>> parts;  // [scan][chunk]
};

}  // namespace tid

struct tid_server {
    tid_ctx *ctx = nullptr;
    const tid_graph *g = nullptr;
    uint32_t C = 1, slots = 1, next_chunk = 0;
    std::vector<std::unique_ptr<tid_graph>> views;
    std::deque<std::unique_ptr<tid::ServeQuery>> waiting;
    std::vector<std::unique_ptr<tid::ServeQuery>> active;
    std::map<uint64_t, std::unique_ptr<tid_table>> done;
    std::map<uint64_t, std::pair<tid_status, std::string>> failed;
    uint64_t next_ticket = 1;
};

namespace tid {

tid_server *serve_open(tid_ctx *ctx, const tid_graph *g, uint32_t chunks, uint32_t slots) {
    TID_REQUIRE(chunks >= 1 && chunks <= 4096, TID_E_INVALID_ARG, "serve: 1..4096 chunks");
    TID_REQUIRE(slots >= 1, TID_E_INVALID_ARG, "serve: at least one slot");
    auto s = std::make_unique<tid_server>();
    s->ctx = ctx;
    s->g = g;
    s->C = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(chunks, std::max<uint64_t>(g->n, 1)));
    s->slots = slots;
    for (uint32_t k = 0; k < s->C; ++k) {
        const uint64_t a = g->n * k / s->C, b = g->n * (k + 1) / s->C;
        auto v = std::make_unique<tid_graph>();
        v->ctx = ctx;
        v->n = b - a;
        v->view = g->triples() + 3 * a;
        v->bounds_from = g;
        for (int x = 0; x < 3; ++x) v->max_id[x] = g->max_id[x];
        chunk_stats(ctx, v.get());
        s->views.push_back(std::move(v));
    }
    return s.release();
}

void serve_free(tid_server *s) { delete s; }
tid_ctx *serve_ctx(const tid_server *s) { return s->ctx; }
uint32_t serve_slots(const tid_server *s) { return s->slots; }

void serve_info(const tid_server *s, int32_t *waiting, int32_t *active, int32_t *next_chunk) {
    if (waiting) *waiting = (int32_t)s->waiting.size();
    if (active) *active = (int32_t)s->active.size();
    if (next_chunk) *next_chunk = (int32_t)s->next_chunk;
}

// The result of a finished ticket, or the status its query failed with.
tid_status serve_take(tid_server *s, uint64_t ticket, tid_table **out, std::string *msg) {
    auto f = s->failed.find(ticket);
    if (f != s->failed.end()) {
        const tid_status code = f->second.first;
        *msg = f->second.second;
        s->failed.erase(f);
        return code;
    }
    auto it = s->done.find(ticket);
    if (it == s->done.end()) {
        *msg = "serve: ticket not finished or already taken";
        return TID_E_INVALID_ARG;
    }
    *out = it->second.release();
    s->done.erase(it);
    return TID_OK;
}

uint64_t serve_submit(tid_server *s, const tid_plan *plan) {
    auto q = std::make_unique<ServeQuery>();
    TID_REQUIRE(plan && plan->n_patterns >= 0 && plan->n_ops > 0 && plan->ops, TID_E_INVALID_ARG,
                "serve: bad plan");
    q->pats.assign(plan->patterns, plan->patterns + plan->n_patterns);
    q->ops.assign(plan->ops, plan->ops + plan->n_ops);
    q->plan.n_patterns = plan->n_patterns;
    q->plan.patterns = q->pats.data();
    q->plan.n_ops = plan->n_ops;
    q->plan.ops = q->ops.data();
    compile_plan(&q->plan, q->pr);  // checks the plan; lists its scans
    q->ticket = s->next_ticket++;
    const uint64_t t = q->ticket;
    s->waiting.push_back(std::move(q));
    return t;
}

// One step: admit into free slots, scan the next chunk for every admitted
// query, finish the queries that have seen every chunk.  Returns their tickets.
std::vector<uint64_t> serve_step(tid_server *s) {
    tid_ctx *ctx = s->ctx;
    while (!s->waiting.empty() && s->active.size() < s->slots) {
        auto q = std::move(s->waiting.front());
        s->waiting.pop_front();
        q->parts.clear();
        q->parts.resize(q->pr.scans.size());
        for (auto &per : q->parts) per.resize(s->C);
        s->active.push_back(std::move(q));
    }
    std::vector<uint64_t> finished;
    if (s->active.empty()) return finished;
    const uint32_t k = s->next_chunk;
    const tid_graph *view = s->views[k].get();
    // the chunk pass: identical scans across queries run once
    std::vector<tid_pattern> all;
    std::vector<PatternSet> sets;
    std::vector<std::pair<ServeQuery *, size_t>> where;
    std::map<std::string, size_t> uniq;
    std::vector<size_t> rep;
    for (auto &q : s->active)
        for (size_t j = 0; j < q->pr.scans.size(); ++j) {
            const auto ins = uniq.emplace(scan_key(q->pr.scans[j], q->pr.sets[j], ScanFilter{}),
                                          all.size());
            if (ins.second) {
                all.push_back(q->pr.scans[j]);
                sets.push_back(q->pr.sets[j]);
            }
            rep.push_back(ins.first->second);
            where.emplace_back(q.get(), j);
        }
    std::vector<std::unique_ptr<tid_table>> outs(all.size());
    if (!all.empty()) scan_many(ctx, view, all.data(), (int)all.size(), outs.data(), sets.data(),
                                nullptr);
    for (size_t w = 0; w < where.size(); ++w)
        where[w].first->parts[where[w].second][k] =
            alias_table(outs[rep[w]].get(), where[w].first->pr.scans[where[w].second]);
    for (auto &q : s->active) ++q->seen;
    s->next_chunk = (k + 1) % s->C;
    // queries with a full revolution
    std::vector<std::unique_ptr<ServeQuery>> complete, still;
    for (auto &q : s->active) (q->seen == s->C ? complete : still).push_back(std::move(q));
    s->active = std::move(still);
    if (complete.empty()) return finished;
    std::vector<tid_table *> counted;
    for (auto &q : complete)
        for (auto &per : q->parts)
            for (auto &t : per) counted.push_back(t.get());
    resolve_counts(ctx, counted.data(), (int)counted.size());
    // each scan's chunk tables end to end, in chunk (= triple position) order
    std::vector<std::vector<std::unique_ptr<tid_table>>> pre(complete.size());
    std::vector<CopyJob> copies;
    for (size_t i = 0; i < complete.size(); ++i) {
        ServeQuery &q = *complete[i];
        for (auto &per : q.parts) {
            uint64_t rows = 0;
            for (auto &t : per) rows += t->nrows;
            const tid_table *t0 = per[0].get();
            auto cat = make_table(ctx, t0->ncols, t0->vars, rows);
            cat->maxv_known = t0->maxv_known;
            copy_bounds(cat.get(), t0, nullptr, t0->ncols);
            uint64_t at = 0;
            for (auto &t : per) {
                for (int c = 0; c < t->ncols; ++c)
                    copies.push_back(CopyJob{t->col[c], cat->col[c] + at, t->nrows});
                at += t->nrows;
            }
            set_count(ctx, cat.get(), rows);
            pre[i].push_back(std::move(cat));
        }
    }
    BatchState bs;
    batch_copy(ctx, copies, bs);
    for (auto &q : complete) q->parts.clear();  // the chunk tables go back in stream order
    std::vector<const tid_plan *> plans;
    for (auto &q : complete) plans.push_back(&q->plan);
    try {
        auto res = run_plans(ctx, s->g, plans.data(), (int)plans.size(), &pre);
        for (size_t i = 0; i < complete.size(); ++i) {
            s->done[complete[i]->ticket] = std::move(res[i]);
            finished.push_back(complete[i]->ticket);
        }
    } catch (const Error &e) {
        // a group that fails (memory, ...) is not retried here: each query of
        // it reports the error
        for (auto &q : complete) {
            s->failed[q->ticket] = {e.code, e.what()};
            finished.push_back(q->ticket);
        }
    }
    ctx->sync();  // the copy job tables in `bs` are read by now
    return finished;
}

}  // namespace tid
