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
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

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
    static constexpr size_t kLeaf = 48;

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

void sparse_factor_local(Plan& plan) {
    parallel_for(plan.P, [&](int64_t p, int) { sparse_factor_one(plan, plan.subs[p], static_cast<int32_t>(p)); });
}

}  // namespace ras
