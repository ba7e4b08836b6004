// query.hip -- evaluation of postfix query plans (Sec. 4.3, Fig. 6): the
// plan's subqueries are searched together in one pass over the graph (the
// multi-key search of Sec. 4.1), filters on a scanned variable are applied
// during that search, then joins go left to right over the subquery results,
// followed by unions, projections and DISTINCT; the result is returned in
// lexicographic row order.
#include "compact.hpp"

#include <algorithm>

namespace tid {

std::unique_ptr<tid_table> union_tables(tid_ctx *, const tid_table *const *, int, int);
std::unique_ptr<tid_table> sort_rows(tid_ctx *ctx, const tid_table *t, uint64_t n, int distinct);
std::unique_ptr<tid_table> join_unsorted(tid_ctx *ctx, const tid_table *L, uint64_t nl, int lc,
                                         const tid_table *R, uint64_t nr, int rc, int algo,
                                         const JoinPlan &jp);

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

// Join on variable v; every other variable both sides hold must agree and is
// kept once (the left copy).
static std::unique_ptr<tid_table> natural_join(tid_ctx *ctx, tid_table *L, tid_table *R,
                                               int32_t v) {
    const int lc = col_of(L, v), rc = col_of(R, v);
    TID_REQUIRE(lc >= 0 && rc >= 0, TID_E_SCHEMA, "join: variable not bound on both sides");
    tid_table *both[2] = {L, R};
    resolve_counts(ctx, both, 2);
    JoinPlan jp;
    for (int c = 0; c < L->ncols; ++c) jp.lkeep.push_back(c);
    std::vector<std::pair<int, int>> eq;  // (left output column, right output column)
    std::vector<int> keep;
    for (int c = 0; c < L->ncols; ++c) keep.push_back(c);
    for (int c = 0; c < R->ncols; ++c) {
        if (c == rc) continue;
        const int out_col = L->ncols + (int)jp.rkeep.size();
        jp.rkeep.push_back(c);
        const int lmatch = col_of(L, R->vars[c]);
        if (lmatch >= 0)
            eq.emplace_back(lmatch, out_col);
        else
            keep.push_back(out_col);
    }
    auto raw = join_unsorted(ctx, L, L->nrows, lc, R, R->nrows, rc, 0, jp);
    if (eq.empty()) return raw;
    return select_equal(ctx, raw.get(), eq, keep);
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
    }
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

std::unique_ptr<tid_table> run_query(tid_ctx *ctx, const tid_graph *g, const tid_plan *plan) {
    TID_REQUIRE(plan->n_patterns >= 0 && plan->n_ops >= 0, TID_E_INVALID_ARG, "plan: bad sizes");
    TID_REQUIRE(plan->n_patterns == 0 || plan->patterns, TID_E_INVALID_ARG, "plan: no patterns");
    TID_REQUIRE(plan->n_ops > 0 && plan->ops, TID_E_INVALID_ARG, "plan: no ops");
    const uint32_t *ops = plan->ops;
    const int nops = plan->n_ops;

    // Pass 1: check the op stream, and list one scan per SCAN op.  A FILTER
    // right after a SCAN on a variable that the pattern binds at one position
    // (and with no range yet) becomes the pattern's range: the filter runs
    // inside the search (Fig. 6).
    std::vector<tid_pattern> scans;
    std::vector<int> scan_at_op(nops, -1);  // op index -> scan slot
    std::vector<char> fused(nops, 0);       // FILTER ops folded into their scan
    int depth = 0;
    for (int pc = 0; pc < nops;) {
        const uint32_t op = ops[pc];
        auto need = [&](int words) {
            TID_REQUIRE(pc + words < nops + 1, TID_E_INVALID_ARG, "plan: truncated op");
        };
        if (op == TID_OP_SCAN) {
            need(2);
            const uint32_t i = ops[pc + 1];
            TID_REQUIRE(i < (uint32_t)plan->n_patterns, TID_E_INVALID_ARG,
                        "plan: pattern index out of range");
            int32_t vars[3], src[3];
            pattern_schema(plan->patterns[i], vars, src);
            tid_pattern p = plan->patterns[i];
            // peephole: SCAN i; FILTER v lo hi
            if (pc + 6 <= nops && ops[pc + 2] == TID_OP_FILTER && p.range_pos < 0) {
                const int32_t v = (int32_t)ops[pc + 3];
                const int32_t pv[3] = {p.vs, p.vp, p.vo};
                int pos = -1, hits = 0;
                for (int x = 0; x < 3; ++x)
                    if (pv[x] >= 0 && pv[x] == v) {
                        pos = x;
                        ++hits;
                    }
                if (hits >= 1) {
                    p.range_pos = pos;
                    p.lo = ops[pc + 4];
                    p.hi = ops[pc + 5];
                    fused[pc + 2] = 1;
                }
            }
            scan_at_op[pc] = (int)scans.size();
            scans.push_back(p);
            ++depth;
            pc += 2;
        } else if (op == TID_OP_JOIN) {
            need(2);
            TID_REQUIRE(depth >= 2, TID_E_INVALID_ARG, "plan: JOIN needs two tables");
            --depth;
            pc += 2;
        } else if (op == TID_OP_UNION) {
            need(3);
            const uint32_t k = ops[pc + 1];
            TID_REQUIRE(k >= 1 && (int)k <= depth, TID_E_INVALID_ARG, "plan: bad UNION arity");
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

    // All subqueries searched together, up to 16 per pass over the graph.
    std::vector<std::unique_ptr<tid_table>> scanned(scans.size());
    for (size_t s0 = 0; s0 < scans.size(); s0 += TID_MAX_MULTI) {
        const int k = (int)std::min<size_t>(TID_MAX_MULTI, scans.size() - s0);
        scan_multi(ctx, g, scans.data() + s0, k, scanned.data() + s0);
    }

    // Pass 2: evaluate.
    std::vector<Entry> st;
    for (int pc = 0; pc < nops;) {
        const uint32_t op = ops[pc];
        if (op == TID_OP_SCAN) {
            st.push_back({std::move(scanned[scan_at_op[pc]]), false});
            pc += 2;
        } else if (op == TID_OP_JOIN) {
            const int32_t v = (int32_t)ops[pc + 1];
            Entry r = std::move(st.back());
            st.pop_back();
            Entry l = std::move(st.back());
            st.pop_back();
            st.push_back({natural_join(ctx, l.t.get(), r.t.get(), v), false});
            pc += 2;
        } else if (op == TID_OP_UNION) {
            const int k = (int)ops[pc + 1];
            const int d = ops[pc + 2] ? 1 : 0;
            std::vector<const tid_table *> ins;
            for (int j = 0; j < k; ++j) ins.push_back(st[st.size() - k + j].t.get());
            auto u = union_tables(ctx, ins.data(), k, d);
            st.resize(st.size() - k);
            st.push_back({std::move(u), d == 1});
            pc += 3;
        } else if (op == TID_OP_FILTER) {
            if (!fused[pc]) {
                const int32_t v = (int32_t)ops[pc + 1];
                const int c = col_of(st.back().t.get(), v);
                TID_REQUIRE(c >= 0, TID_E_SCHEMA, "filter: variable not in the table");
                auto f = filter_range(ctx, st.back().t.get(), c, ops[pc + 2], ops[pc + 3]);
                st.back().t = std::move(f);  // filtering keeps row order
            }
            pc += 4;
        } else if (op == TID_OP_PROJECT) {
            const int n = (int)ops[pc + 1];
            std::vector<int32_t> vars(ops + pc + 2, ops + pc + 2 + n);
            st.back().t = project(std::move(st.back().t), vars);
            st.back().sorted = false;
            pc += 2 + n;
        } else {  // DISTINCT
            tid_table *t = st.back().t.get();
            st.back().t = sort_rows(ctx, t, t->rows(), 1);
            st.back().sorted = true;
            pc += 1;
        }
    }
    Entry &res = st.back();
    if (res.sorted) return std::move(res.t);
    tid_table *t = res.t.get();
    return sort_rows(ctx, t, t->rows(), 0);
}

}  // namespace tid
