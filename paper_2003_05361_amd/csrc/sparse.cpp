// Sparse direct local solver, host side: fill-reducing ordering, symbolic and
// numeric Cholesky factorisation of each local matrix (Sec. 3.3.1: the local
// problems are factored once at setup and applied by triangular solves).
//
// Ordering: nested dissection on the local matrix graph.  A subset is split by
// the middle level of a breadth-first level structure rooted at a
// pseudo-peripheral vertex (a level set separates the levels before it from
// the levels after it); the two parts are ordered recursively and the
// separator last, so fill stays inside the parts and the separator block.
//
// Factorisation: elimination tree (parent of j = the first row below j whose
// factor row reaches j), row patterns of L as unions of elimination-tree paths,
// then an up-looking numeric factorisation: row k of L solves the triangular
// system with the rows above it, visiting its pattern in ascending order and
// scattering each finished entry along its column.
//
// Solve schedules: each triangular pass becomes a short sequence of parallel
// steps, dense separator blocks solved through the explicit inverses of their
// triangles (Alvarado and Schreiber, SIAM J. Sci. Comput. 14, 1993), and each
// step's records are dealt out to the lanes of one workgroup (the device's
// lane-stream layout).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <numeric>
#include <queue>
#include <string>
#include <utility>
#include <vector>

#include "device.hpp"
#include "plan.hpp"

namespace ras {

namespace {

struct LocalGraph {
    int32_t n = 0;
    std::vector<int64_t> ptr;   // [n + 1]
    std::vector<int32_t> adj;   // neighbours (local ids), no diagonal
    std::vector<double> val;    // matching values A_ij
    std::vector<double> diag;   // A_ii
};

LocalGraph local_graph(const Plan& plan, const Subdomain& sd) {
    LocalGraph G;
    G.n = static_cast<int32_t>(sd.omega.size());
    G.ptr.assign(G.n + 1, 0);
    G.diag.assign(G.n, 0.0);
    const double shift = robin_shift_factor(plan.local);  // Robin transmission (ORAS)
    for (int32_t i = 0; i < G.n; ++i) {
        const int32_t g = sd.omega[i];
        for (int64_t e = plan.row_ptr[g]; e < plan.row_ptr[g + 1]; ++e) {
            const int32_t c = plan.col[e];
            auto it = std::lower_bound(sd.omega.begin(), sd.omega.end(), c);
            if (it == sd.omega.end() || *it != c) {
                G.diag[i] -= shift * std::fabs(plan.val[e]);
                continue;
            }
            const int32_t j = static_cast<int32_t>(it - sd.omega.begin());
            if (j == i) {
                G.diag[i] += plan.val[e];
            } else {
                G.adj.push_back(j);
                G.val.push_back(plan.val[e]);
            }
        }
        G.ptr[i + 1] = static_cast<int64_t>(G.adj.size());
    }
    return G;
}

class Dissector {
public:
    explicit Dissector(const LocalGraph& G) : G_(G), member_(G.n, 0), seen_(G.n, 0), level_(G.n, 0) {}

    std::vector<int32_t> order() {
        std::vector<int32_t> all(G_.n);
        for (int32_t i = 0; i < G_.n; ++i) all[i] = i;
        out_.clear();
        out_.reserve(G_.n);
        split(all);
        return out_;
    }

private:
    static constexpr size_t kLeaf = 8;

    // breadth-first levels from s inside the current subset (member_ == id);
    // returns the vertices in visiting order, level_ holds their depth
    std::vector<int32_t> bfs(int32_t s, int32_t id, int32_t* depth) {
        const int32_t mark = ++stamp_;
        std::vector<int32_t> q{s};
        seen_[s] = mark;
        level_[s] = 0;
        for (size_t h = 0; h < q.size(); ++h) {
            const int32_t v = q[h];
            for (int64_t e = G_.ptr[v]; e < G_.ptr[v + 1]; ++e) {
                const int32_t u = G_.adj[e];
                if (member_[u] != id || seen_[u] == mark) continue;
                seen_[u] = mark;
                level_[u] = level_[v] + 1;
                q.push_back(u);
            }
        }
        *depth = level_[q.back()];
        return q;
    }

    int32_t degree_in(int32_t v, int32_t id) const {
        int32_t d = 0;
        for (int64_t e = G_.ptr[v]; e < G_.ptr[v + 1]; ++e) d += member_[G_.adj[e]] == id;
        return d;
    }

    void split(std::vector<int32_t>& S) {
        if (S.size() <= kLeaf) {
            std::sort(S.begin(), S.end());
            out_.insert(out_.end(), S.begin(), S.end());
            return;
        }
        const int32_t id = ++ids_;
        for (int32_t v : S) member_[v] = id;
        int32_t depth = 0;
        std::vector<int32_t> q = bfs(*std::min_element(S.begin(), S.end()), id, &depth);
        if (q.size() < S.size()) {
            // disconnected: find every component, then order each independently
            std::vector<std::vector<int32_t>> comps;
            std::sort(S.begin(), S.end());
            comps.push_back(std::move(q));
            for (int32_t v : comps.back()) member_[v] = -id;  // claimed by a component
            for (size_t k = 0; k < S.size(); ++k) {
                if (member_[S[k]] != id) continue;
                int32_t d = 0;
                comps.push_back(bfs(S[k], id, &d));
                for (int32_t v : comps.back()) member_[v] = -id;
            }
            S.clear();
            for (auto& c : comps) split(c);
            return;
        }
        // pseudo-peripheral root: restart from a least-degree vertex of the last level
        // while the level structure gets deeper
        for (int it = 0; it < 4; ++it) {
            int32_t best = -1, bd = 0;
            for (auto r = q.rbegin(); r != q.rend() && level_[*r] == depth; ++r) {
                const int32_t d = degree_in(*r, id);
                if (best < 0 || d < bd || (d == bd && *r < best)) {
                    best = *r;
                    bd = d;
                }
            }
            int32_t d2 = 0;
            std::vector<int32_t> q2 = bfs(best, id, &d2);
            if (d2 <= depth) {
                q = bfs(q.front(), id, &depth);  // restore the levels of the kept root
                break;
            }
            q.swap(q2);
            depth = d2;
        }
        if (depth < 2) {
            std::sort(S.begin(), S.end());
            out_.insert(out_.end(), S.begin(), S.end());
            return;
        }
        // separator: the first level at which half of the vertices lie before it
        std::vector<int64_t> count(depth + 1, 0);
        for (int32_t v : q) ++count[level_[v]];
        int32_t m = 1;
        int64_t before = count[0];
        while (m < depth - 1 && 2 * (before + count[m]) <= static_cast<int64_t>(S.size())) before += count[m++];
        std::vector<int32_t> a, b, sep;
        for (int32_t v : q) {
            if (level_[v] < m) a.push_back(v);
            else if (level_[v] == m) sep.push_back(v);
            else b.push_back(v);
        }
        S.clear();
        split(a);
        split(b);
        std::sort(sep.begin(), sep.end());
        out_.insert(out_.end(), sep.begin(), sep.end());
    }

    const LocalGraph& G_;
    std::vector<int32_t> member_, seen_, level_;
    std::vector<int32_t> out_;
    int32_t ids_ = 0, stamp_ = 0;
};

}  // namespace

void sparse_factor_one(const Plan& plan, Subdomain& sd, int32_t p) {
    const LocalGraph G = local_graph(plan, sd);
    const int32_t n = G.n;
    SparseFactor& F = sd.sf;
    F.perm = Dissector(G).order();
    std::vector<int32_t> inv(n);
    for (int32_t k = 0; k < n; ++k) inv[F.perm[k]] = k;

    // strictly lower part of the permuted matrix, by rows, columns ascending
    std::vector<int64_t> bp(n + 1, 0);
    std::vector<std::pair<int32_t, double>> bl;
    std::vector<double> bd(n);
    for (int32_t k = 0; k < n; ++k) {
        const int32_t i = F.perm[k];
        bd[k] = G.diag[i];
        const size_t s0 = bl.size();
        for (int64_t e = G.ptr[i]; e < G.ptr[i + 1]; ++e) {
            const int32_t c = inv[G.adj[e]];
            if (c < k) bl.emplace_back(c, G.val[e]);
        }
        std::sort(bl.begin() + s0, bl.end());
        bp[k + 1] = static_cast<int64_t>(bl.size());
    }

    // elimination tree, with path compression through `anc`
    std::vector<int32_t> parent(n, -1), anc(n, -1);
    for (int32_t k = 0; k < n; ++k)
        for (int64_t e = bp[k]; e < bp[k + 1]; ++e) {
            int32_t j = bl[e].first;
            while (j != -1 && j < k) {
                const int32_t next = anc[j];
                anc[j] = k;
                if (next == -1) parent[j] = k;
                j = next;
            }
        }

    // row patterns: row k reaches every vertex on the tree paths from its
    // entries up to k
    std::vector<int32_t> mark(n, -1);
    F.lp.assign(n + 1, 0);
    F.lj.clear();
    std::vector<int64_t> colcount(n, 0);
    for (int32_t k = 0; k < n; ++k) {
        mark[k] = k;
        const size_t s0 = F.lj.size();
        for (int64_t e = bp[k]; e < bp[k + 1]; ++e)
            for (int32_t j = bl[e].first; mark[j] != k; j = parent[j]) {
                mark[j] = k;
                F.lj.push_back(j);
            }
        std::sort(F.lj.begin() + s0, F.lj.end());
        for (size_t q = s0; q < F.lj.size(); ++q) ++colcount[F.lj[q]];
        F.lp[k + 1] = static_cast<int64_t>(F.lj.size());
    }

    // numeric, up-looking; columns of L are filled as rows complete
    F.cp.assign(n + 1, 0);
    for (int32_t j = 0; j < n; ++j) F.cp[j + 1] = F.cp[j] + colcount[j];
    F.ci.assign(F.cp[n], 0);
    F.cx.assign(F.cp[n], 0.0);
    std::vector<int64_t> fill(F.cp.begin(), F.cp.end() - 1);
    F.lx.assign(F.lj.size(), 0.0);
    F.d.assign(n, 0.0);
    std::vector<double> x(n, 0.0);
    for (int32_t k = 0; k < n; ++k) {
        for (int64_t e = bp[k]; e < bp[k + 1]; ++e) x[bl[e].first] = bl[e].second;
        double dk = bd[k];
        for (int64_t q = F.lp[k]; q < F.lp[k + 1]; ++q) {
            const int32_t j = F.lj[q];
            const double lkj = x[j] / F.d[j];
            x[j] = 0.0;
            for (int64_t c = F.cp[j]; c < fill[j]; ++c) x[F.ci[c]] -= F.cx[c] * lkj;
            dk -= lkj * lkj;
            F.lx[q] = lkj;
            F.ci[fill[j]] = k;
            F.cx[fill[j]++] = lkj;
        }
        if (!(dk > 0.0) || !std::isfinite(dk))
            throw Error{RAS_E_NOT_SPD, "non-positive pivot in subdomain " + std::to_string(p) + " at local row " +
                                           std::to_string(F.perm[k])};
        F.d[k] = std::sqrt(dk);
    }
}

// ---------------------------------------------------------------------------
// Triangular-solve schedules.  A level-scheduled pass takes one parallel step
// per level of the dependency graph, and a dense diagonal block of s rows
// (a separator of the dissection, eliminated last among its subtree) is a
// chain of s levels.  A block of at least min_block rows is solved in two
// steps instead (the partitioned-inverse form of Alvarado and Schreiber):
// first every row of the block subtracts its products with rows outside the
// block (one dot product per row, results into block slots), then every row
// takes its dot product with the explicit inverse of the block's triangle,
// computed here in float64 (forward: row k of T^{-1}; backward: column k).
// Singleton rows keep their one-step form y_k = (v_k - sum_j L_kj y_j) / L_kk.

std::vector<int32_t> dense_runs(const SparseFactor& F) {
    const int32_t n = static_cast<int32_t>(F.d.size());
    std::vector<int32_t> starts;
    int32_t s0 = 0;
    for (int32_t k = 0; k < n; ++k) {
        // row k continues the run iff its k - s0 largest columns are s0 .. k-1
        const int64_t need = k - s0;
        const bool cont = need > 0 && F.lp[k + 1] - F.lp[k] >= need && F.lj[F.lp[k + 1] - need] == s0;
        if (!cont) {
            starts.push_back(k);
            s0 = k;
        }
    }
    starts.push_back(n);
    return starts;
}

namespace {

struct PassShape {
    int32_t nsteps = 0;
    int32_t slots = 0;
};

// Steps of every row (singletons) and block (first step), and the slot
// capacities; a block's slots are live from its first step to its second, so
// blocks starting at even and at odd steps use two separate slot ranges.
PassShape schedule_steps(const SparseFactor& F, const std::vector<int32_t>& runs, int32_t min_block, bool forward,
                         std::vector<int32_t>& ready, std::vector<int32_t>& block_step) {
    const int32_t n = static_cast<int32_t>(F.d.size());
    const int32_t nruns = static_cast<int32_t>(runs.size()) - 1;
    ready.assign(n, -1);
    block_step.assign(nruns, -1);
    std::vector<int64_t> at_step;
    for (int32_t r = 0; r < nruns; ++r) {
        const int32_t ri = forward ? r : nruns - 1 - r;
        const int32_t a = runs[ri], b = runs[ri + 1];
        const bool block = min_block > 0 && b - a >= min_block;
        if (!block) {
            for (int32_t q = 0; q < b - a; ++q) {
                const int32_t k = forward ? a + q : b - 1 - q;
                int32_t st = 0;
                if (forward)
                    for (int64_t e = F.lp[k]; e < F.lp[k + 1]; ++e) st = std::max(st, ready[F.lj[e]] + 1);
                else
                    for (int64_t e = F.cp[k]; e < F.cp[k + 1]; ++e) st = std::max(st, ready[F.ci[e]] + 1);
                ready[k] = st;
            }
            continue;
        }
        int32_t st = 0;
        for (int32_t k = a; k < b; ++k) {
            if (forward)  // columns below a: all but the last k - a entries
                for (int64_t e = F.lp[k]; e < F.lp[k + 1] - (k - a); ++e) st = std::max(st, ready[F.lj[e]] + 1);
            else  // rows at or past b: all but the first b - 1 - k entries
                for (int64_t e = F.cp[k] + (b - 1 - k); e < F.cp[k + 1]; ++e) st = std::max(st, ready[F.ci[e]] + 1);
        }
        block_step[ri] = st;
        for (int32_t k = a; k < b; ++k) ready[k] = st + 1;
        if (static_cast<int32_t>(at_step.size()) <= st) at_step.resize(st + 1, 0);
        at_step[st] += b - a;
    }
    PassShape sh;
    for (int32_t k = 0; k < n; ++k) sh.nsteps = std::max(sh.nsteps, ready[k] + 1);
    int64_t cap[2] = {0, 0};
    for (size_t s = 0; s < at_step.size(); ++s) cap[s & 1] = std::max(cap[s & 1], at_step[s]);
    sh.slots = static_cast<int32_t>(cap[0] + cap[1]);
    return sh;
}

// inverse of the dense lower triangle T = L[a:b, a:b] (row-major s x s, lower part)
std::vector<double> block_inverse(const SparseFactor& F, int32_t a, int32_t b) {
    const int32_t s = b - a;
    std::vector<double> T(static_cast<size_t>(s) * s, 0.0), G(static_cast<size_t>(s) * s, 0.0);
    for (int32_t r = 0; r < s; ++r) {
        const int32_t k = a + r;
        for (int32_t c = 0; c < r; ++c) T[static_cast<size_t>(r) * s + c] = F.lx[F.lp[k + 1] - r + c];
        T[static_cast<size_t>(r) * s + r] = F.d[k];
    }
    for (int32_t c = 0; c < s; ++c) {
        G[static_cast<size_t>(c) * s + c] = 1.0 / T[static_cast<size_t>(c) * s + c];
        for (int32_t r = c + 1; r < s; ++r) {
            double acc = 0.0;
            for (int32_t m = c; m < r; ++m) acc += T[static_cast<size_t>(r) * s + m] * G[static_cast<size_t>(m) * s + c];
            G[static_cast<size_t>(r) * s + c] = -acc / T[static_cast<size_t>(r) * s + r];
        }
    }
    return G;
}

}  // namespace

void sparse_schedule(const SparseFactor& F, const std::vector<int32_t>& runs, int32_t min_block, bool forward,
                     SparseSchedule* out) {
    const int32_t n = static_cast<int32_t>(F.d.size());
    const int32_t nruns = static_cast<int32_t>(runs.size()) - 1;
    std::vector<int32_t> ready, block_step;
    const PassShape sh = schedule_steps(F, runs, min_block, forward, ready, block_step);
    // slot base of every block: n, then the even-step range, then the odd-step range
    std::vector<int64_t> at_step(sh.nsteps + 1, 0);
    int64_t cap_even = 0;
    for (int32_t r = 0; r < nruns; ++r)
        if (block_step[r] >= 0) at_step[block_step[r]] += runs[r + 1] - runs[r];
    for (int32_t s = 0; s < sh.nsteps; s += 2) cap_even = std::max(cap_even, at_step[s]);
    std::fill(at_step.begin(), at_step.end(), 0);
    std::vector<int32_t> base(nruns, -1);
    for (int32_t q = 0; q < nruns; ++q) {
        const int32_t r = forward ? q : nruns - 1 - q;
        const int32_t st = block_step[r];
        if (st < 0) continue;
        base[r] = static_cast<int32_t>(n + (st & 1 ? cap_even : 0) + at_step[st]);
        at_step[st] += runs[r + 1] - runs[r];
    }
    // records with their step, entries gathered per record, then emitted by step
    struct Rec {
        int32_t step, dest;
        int64_t e0, e1;
    };
    std::vector<Rec> recs;
    std::vector<int32_t> col;
    std::vector<double> val;
    recs.reserve(n);
    auto singleton = [&](int32_t k) {
        const double inv = 1.0 / F.d[k];
        Rec rc{ready[k], k, static_cast<int64_t>(col.size()), 0};
        col.push_back(k);
        val.push_back(inv);
        if (forward)
            for (int64_t e = F.lp[k]; e < F.lp[k + 1]; ++e) {
                col.push_back(F.lj[e]);
                val.push_back(-F.lx[e] * inv);
            }
        else
            for (int64_t e = F.cp[k]; e < F.cp[k + 1]; ++e) {
                col.push_back(F.ci[e]);
                val.push_back(-F.cx[e] * inv);
            }
        rc.e1 = static_cast<int64_t>(col.size());
        recs.push_back(rc);
    };
    for (int32_t q = 0; q < nruns; ++q) {
        const int32_t r = forward ? q : nruns - 1 - q;
        const int32_t a = runs[r], b = runs[r + 1];
        if (block_step[r] < 0) {
            for (int32_t i = 0; i < b - a; ++i) singleton(forward ? a + i : b - 1 - i);
            continue;
        }
        const int32_t st = block_step[r], s = b - a;
        // first step: v_k minus the products with rows outside the block
        for (int32_t k = a; k < b; ++k) {
            Rec rc{st, base[r] + (k - a), static_cast<int64_t>(col.size()), 0};
            col.push_back(k);
            val.push_back(1.0);
            if (forward)
                for (int64_t e = F.lp[k]; e < F.lp[k + 1] - (k - a); ++e) {
                    col.push_back(F.lj[e]);
                    val.push_back(-F.lx[e]);
                }
            else
                for (int64_t e = F.cp[k] + (b - 1 - k); e < F.cp[k + 1]; ++e) {
                    col.push_back(F.ci[e]);
                    val.push_back(-F.cx[e]);
                }
            rc.e1 = static_cast<int64_t>(col.size());
            recs.push_back(rc);
        }
        // second step: the inverse triangle (forward T^{-1}, backward T^{-T}) times the block slots
        const std::vector<double> G = block_inverse(F, a, b);
        for (int32_t i = 0; i < s; ++i) {
            Rec rc{st + 1, a + i, static_cast<int64_t>(col.size()), 0};
            if (forward)
                for (int32_t j = 0; j <= i; ++j) {
                    col.push_back(base[r] + j);
                    val.push_back(G[static_cast<size_t>(i) * s + j]);
                }
            else
                for (int32_t j = i; j < s; ++j) {
                    col.push_back(base[r] + j);
                    val.push_back(G[static_cast<size_t>(j) * s + i]);
                }
            rc.e1 = static_cast<int64_t>(col.size());
            recs.push_back(rc);
        }
    }
    std::stable_sort(recs.begin(), recs.end(), [](const Rec& x, const Rec& y) { return x.step < y.step; });
    out->step.assign(sh.nsteps + 1, 0);
    out->meta.assign(4 * recs.size(), 0);
    out->col.clear();
    out->val.clear();
    out->col.reserve(col.size());
    out->val.reserve(val.size());
    for (size_t t = 0; t < recs.size(); ++t) {
        const Rec& rc = recs[t];
        ++out->step[rc.step + 1];
        out->meta[4 * t] = rc.dest;
        out->meta[4 * t + 1] = static_cast<int32_t>(out->col.size());
        out->col.insert(out->col.end(), col.begin() + rc.e0, col.begin() + rc.e1);
        out->val.insert(out->val.end(), val.begin() + rc.e0, val.begin() + rc.e1);
        out->meta[4 * t + 2] = static_cast<int32_t>(out->col.size());
    }
    for (int32_t s = 0; s < sh.nsteps; ++s) out->step[s + 1] += out->step[s];
    out->slots = sh.slots;
}

namespace {

// Records dealt to ng groups, longest first, each to the least loaded group
// (ties: the lowest group); returns the largest group load in rounds.
int64_t deal(const std::vector<int32_t>& order, const std::vector<int64_t>& rounds, int32_t ng,
             std::vector<std::vector<int32_t>>* groups, std::vector<int64_t>* load) {
    using Slot = std::pair<int64_t, int32_t>;
    std::priority_queue<Slot, std::vector<Slot>, std::greater<Slot>> heap;
    for (int32_t g = 0; g < ng; ++g) heap.push({0, g});
    if (groups) groups->assign(ng, {});
    if (load) load->assign(ng, 0);
    int64_t most = 0;
    for (size_t k = 0; k < order.size(); ++k) {
        const Slot t = heap.top();
        heap.pop();
        const int64_t l = t.first + rounds[k];
        if (groups) (*groups)[t.second].push_back(order[k]);
        if (load) (*load)[t.second] = l;
        most = std::max(most, l);
        heap.push({l, t.second});
    }
    return most;
}

}  // namespace

void pack_schedule(const SparseSchedule& q, SparseLanes* out) {
    constexpr int W = kSparseWaves, NL = 64 * kSparseWaves;
    const int32_t nsteps = static_cast<int32_t>(q.step.size()) - 1;
    std::vector<std::vector<uint16_t>> wc(W);
    std::vector<std::vector<double>> wv(W);
    std::vector<std::vector<int32_t>> groups;
    std::vector<int64_t> load, rounds;
    std::vector<int32_t> order, gorder;
    auto len = [&](int32_t r) { return static_cast<int64_t>(q.meta[4 * r + 2] - q.meta[4 * r + 1]); };
    for (int32_t s = 0; s < nsteps; ++s) {
        order.resize(q.step[s + 1] - q.step[s]);
        std::iota(order.begin(), order.end(), q.step[s]);
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return len(a) > len(b); });
        // group width: the fewest rounds for the step (ties: the narrower group)
        int lg = 0;
        int64_t best = -1;
        for (int g = 0; g <= 6; ++g) {
            rounds.resize(order.size());
            for (size_t k = 0; k < order.size(); ++k) rounds[k] = (len(order[k]) + (1 << g) - 1) / (1 << g) + 1;
            const int64_t m = deal(order, rounds, NL >> g, nullptr, nullptr);
            if (best < 0 || m < best) {
                best = m;
                lg = g;
            }
        }
        const int G = 1 << lg, ng = NL >> lg, gpw = 64 >> lg;  // groups per wave
        for (size_t k = 0; k < order.size(); ++k) rounds[k] = (len(order[k]) + G - 1) / G + 1;
        deal(order, rounds, ng, &groups, &load);
        gorder.resize(ng);
        std::iota(gorder.begin(), gorder.end(), 0);
        std::stable_sort(gorder.begin(), gorder.end(), [&](int32_t a, int32_t b) { return load[a] > load[b]; });
        const uint32_t tag = static_cast<uint32_t>(lg) << kSparseGroupShift;
        for (int w = 0; w < W; ++w) {
            int64_t U = 0;
            for (int i = 0; i < gpw; ++i) U = std::max(U, load[gorder[gpw * w + i]]);
            const size_t base = wc[w].size();
            wc[w].resize(base + static_cast<size_t>(U + 1) * 64, 0);
            wv[w].resize(base + static_cast<size_t>(U + 1) * 64, 0.0);
            for (int i = 0; i < gpw; ++i) {
                int64_t u = 0;  // next round of this group
                for (int32_t r : groups[gorder[gpw * w + i]]) {
                    const int32_t e0 = q.meta[4 * r + 1], e1 = q.meta[4 * r + 2];
                    for (int32_t e = e0; e < e1; ++e) {
                        const size_t at = base + static_cast<size_t>(u + (e - e0) / G) * 64 + i * G + (e - e0) % G;
                        wc[w][at] = static_cast<uint16_t>(q.col[e]);
                        wv[w][at] = q.val[e];
                    }
                    u += (e1 - e0 + G - 1) / G;
                    // terminator: the destination and the group width in the value's low 32 bits
                    const uint64_t pay = static_cast<uint32_t>(q.meta[4 * r]) | tag;
                    double pv;
                    std::memcpy(&pv, &pay, sizeof pv);
                    for (int l = 0; l < G; ++l) {
                        wc[w][base + static_cast<size_t>(u) * 64 + i * G + l] = static_cast<uint16_t>(kSparseTerm);
                        wv[w][base + static_cast<size_t>(u) * 64 + i * G + l] = pv;
                    }
                    ++u;
                }
            }
            for (int l = 0; l < 64; ++l) wc[w][base + static_cast<size_t>(U) * 64 + l] = static_cast<uint16_t>(kSparseMark);
        }
    }
    // a round count per wave that is a multiple of the device's load lead (an even
    // number: the columns of two rounds share a word; the kernel then needs no
    // bound check inside a group of rounds); the padding rounds follow the last
    // marker and add nothing
    for (int w = 0; w < W; ++w) {
        const size_t r = wc[w].size() / 64, rp = (r + kSparseLead - 1) / kSparseLead * kSparseLead;
        wc[w].resize(rp * 64, 0);
        wv[w].resize(rp * 64, 0.0);
    }
    out->wave.assign(2 * W, 0);
    out->col.clear();
    out->val.clear();
    for (int w = 0; w < W; ++w) {
        out->wave[2 * w] = static_cast<int32_t>(out->col.size() / 64);
        out->wave[2 * w + 1] = static_cast<int32_t>(wc[w].size() / 64);
        out->col.insert(out->col.end(), wc[w].begin(), wc[w].end());
        out->val.insert(out->val.end(), wv[w].begin(), wv[w].end());
    }
}

// The block threshold of one subdomain: the fewest steps over both passes whose
// block slots fit beside the vector in LDS (ties: the larger threshold, fewer
// inverse entries).
int32_t choose_min_block(const SparseFactor& F, const std::vector<int32_t>& runs, int64_t slots_avail) {
    int32_t best = 0;
    int64_t best_steps = -1;
    std::vector<int32_t> ready, bstep;
    for (int32_t mb : {0, 64, 32, 16, 8, 4, 2}) {
        const PassShape f = schedule_steps(F, runs, mb, true, ready, bstep);
        const PassShape b = schedule_steps(F, runs, mb, false, ready, bstep);
        if (std::max(f.slots, b.slots) > slots_avail) continue;
        const int64_t steps = static_cast<int64_t>(f.nsteps) + b.nsteps;
        if (best_steps < 0 || steps < best_steps) {
            best_steps = steps;
            best = mb;
        }
    }
    return best;
}

void sparse_factor_local(Plan& plan, size_t lds_bytes, size_t value_bytes) {
    parallel_for(plan.P, [&](int64_t p, int) {
        Subdomain& sd = plan.subs[p];
        sparse_factor_one(plan, sd, static_cast<int32_t>(p));
        const std::vector<int32_t> runs = dense_runs(sd.sf);
        // slots fit in LDS beside the vector, and in the items' 16-bit columns
        const int64_t avail = std::min<int64_t>(static_cast<int64_t>(lds_bytes / value_bytes), kSparseMaxSlots) -
                              static_cast<int64_t>(sd.omega.size());
        sd.min_block = choose_min_block(sd.sf, runs, avail);
        sparse_schedule(sd.sf, runs, sd.min_block, true, &sd.sched[0]);
        sparse_schedule(sd.sf, runs, sd.min_block, false, &sd.sched[1]);
        for (int k = 0; k < 2; ++k) pack_schedule(sd.sched[k], &sd.lanes[k]);
    });
}

}  // namespace ras
