// Chordal extension of an aggregate sparsity pattern and its maximal cliques
// (paper: Sec. II-A, Definition 1 and the remark that a minimum-fill chordal
// extension is NP-complete to find, so a fill-reducing heuristic is used; the
// "chordal decomposition" part of the Setup step of Algorithms 1 and 2).
//
// Host code, integer work only:
//  1. The graph of the pattern: vertices that occur in some entry, edges the
//     off-diagonal entries.
//  2. Maximum cardinality search (Tarjan & Yannakakis 1984).  If its order is
//     a perfect elimination ordering the graph is already chordal and nothing
//     is added.
//  3. Otherwise a minimum-degree elimination on the explicit elimination
//     graph: the vertex of smallest current degree (smallest label on ties) is
//     eliminated and its remaining neighbours are joined into a clique; the
//     edges that adds are the fill.  The elimination order is a perfect
//     elimination ordering of the filled (chordal) graph.
//  4. Maximal cliques from the perfect elimination ordering: with N+(v) the
//     neighbours of v eliminated after it and parent(v) the first of them,
//     C_v = {v} + N+(v) is a clique of the filled graph, and it is maximal
//     unless a vertex u with parent(u) = v has |N+(u)| = |N+(v)| + 1 (then
//     C_v is a subset of C_u).  Cliques come out in elimination order, each
//     with its vertices sorted.
#include <algorithm>
#include <iterator>
#include <set>
#include <string>
#include <unordered_set>
#include <vector>

#include "cdcs_internal.h"

namespace cdcs {

namespace {

inline uint64_t key_of(int32_t i, int32_t j) {
    const uint32_t hi = (uint32_t)std::max(i, j), lo = (uint32_t)std::min(i, j);
    return ((uint64_t)hi << 32) | lo;
}

// Maximum cardinality search: returns the elimination order (the reverse of
// the visiting order) and whether it is a perfect elimination ordering.
bool mcs_peo(int32_t n, const std::vector<std::vector<int32_t>> &adj, const std::vector<char> &used,
             std::vector<int32_t> &order) {
    std::vector<int32_t> weight((size_t)n, 0), visit;
    std::vector<char> done((size_t)n, 0);
    // buckets of unvisited vertices by weight (doubly linked lists)
    std::vector<int32_t> head((size_t)n + 1, -1), next((size_t)n, -1), prev((size_t)n, -1);
    auto push = [&](int32_t v) {
        const int32_t w = weight[(size_t)v];
        prev[(size_t)v] = -1;
        next[(size_t)v] = head[(size_t)w];
        if (head[(size_t)w] >= 0) prev[(size_t)head[(size_t)w]] = v;
        head[(size_t)w] = v;
    };
    auto pop = [&](int32_t v) {
        const int32_t w = weight[(size_t)v];
        if (prev[(size_t)v] >= 0) next[(size_t)prev[(size_t)v]] = next[(size_t)v];
        else head[(size_t)w] = next[(size_t)v];
        if (next[(size_t)v] >= 0) prev[(size_t)next[(size_t)v]] = prev[(size_t)v];
    };
    int32_t nv = 0;
    for (int32_t v = n - 1; v >= 0; --v)
        if (used[(size_t)v]) {
            push(v);
            ++nv;
        }
    int32_t wmax = 0;
    visit.reserve((size_t)nv);
    for (int32_t t = 0; t < nv; ++t) {
        while (wmax > 0 && head[(size_t)wmax] < 0) --wmax;
        const int32_t v = head[(size_t)wmax];
        pop(v);
        done[(size_t)v] = 1;
        visit.push_back(v);
        for (int32_t u : adj[(size_t)v])
            if (!done[(size_t)u]) {
                pop(u);
                ++weight[(size_t)u];
                push(u);
                wmax = std::max(wmax, weight[(size_t)u]);
            }
    }
    order.assign(visit.rbegin(), visit.rend());
    // perfect elimination test: for each v, its later neighbours minus the
    // first of them must be neighbours of that first one
    std::vector<int32_t> pos((size_t)n, -1);
    for (int32_t t = 0; t < nv; ++t) pos[(size_t)order[(size_t)t]] = t;
    std::vector<int32_t> mark((size_t)n, -1);
    for (int32_t t = 0; t < nv; ++t) {
        const int32_t v = order[(size_t)t];
        int32_t par = -1;
        for (int32_t u : adj[(size_t)v])
            if (pos[(size_t)u] > t && (par < 0 || pos[(size_t)u] < pos[(size_t)par])) par = u;
        if (par < 0) continue;
        for (int32_t u : adj[(size_t)par]) mark[(size_t)u] = par;
        for (int32_t u : adj[(size_t)v])
            if (pos[(size_t)u] > t && u != par && mark[(size_t)u] != par) return false;
    }
    return true;
}

}  // namespace

bool elimination_order(int32_t n, const std::vector<std::vector<int32_t>> &adj, const std::vector<char> &used,
                       std::vector<int32_t> &order, std::vector<std::vector<int32_t>> &later) {
    later.assign((size_t)n, {});
    const bool chordal = mcs_peo(n, adj, used, order);
    if (chordal) {
        std::vector<int32_t> pos((size_t)n, -1);
        for (size_t t = 0; t < order.size(); ++t) pos[(size_t)order[t]] = (int32_t)t;
        for (int32_t v : order)
            for (int32_t u : adj[(size_t)v])
                if (pos[(size_t)u] > pos[(size_t)v]) later[(size_t)v].push_back(u);
        return true;
    }
    // minimum degree on the elimination graph (sorted adjacency vectors)
    std::vector<std::vector<int32_t>> g((size_t)n);
    for (int32_t v = 0; v < n; ++v) {
        g[(size_t)v] = adj[(size_t)v];
        std::sort(g[(size_t)v].begin(), g[(size_t)v].end());
    }
    // (degree, vertex) pairs of the vertices not yet eliminated, ordered
    std::set<std::pair<int32_t, int32_t>> queue;
    for (int32_t v = 0; v < n; ++v)
        if (used[(size_t)v]) queue.insert({(int32_t)g[(size_t)v].size(), v});
    order.clear();
    order.reserve(queue.size());
    std::vector<int32_t> merged;
    while (!queue.empty()) {
        const int32_t v = queue.begin()->second;
        queue.erase(queue.begin());
        order.push_back(v);
        const std::vector<int32_t> nb = g[(size_t)v];
        later[(size_t)v] = nb;
        // join the neighbours into a clique, drop v from their lists
        for (int32_t a : nb) {
            std::vector<int32_t> &ga = g[(size_t)a];
            queue.erase({(int32_t)ga.size(), a});
            merged.clear();
            std::set_union(ga.begin(), ga.end(), nb.begin(), nb.end(), std::back_inserter(merged));
            ga.clear();
            for (int32_t u : merged)
                if (u != a && u != v) ga.push_back(u);
            queue.insert({(int32_t)ga.size(), a});
        }
        g[(size_t)v].clear();
    }
    return false;
}

cdcs_status chordal_extension(int32_t n, int64_t nnz, const int32_t *ei, const int32_t *ej, ChordalExt &out,
                              std::string &err) {
    out = ChordalExt();
    if (n < 1 || nnz < 1 || !ei || !ej) {
        err = "empty or NULL pattern";
        return CDCS_E_ARG;
    }
    std::vector<char> used((size_t)n, 0);
    std::unordered_set<uint64_t> entries;
    entries.reserve((size_t)nnz * 2);
    std::vector<std::vector<int32_t>> adj((size_t)n);
    for (int64_t e = 0; e < nnz; ++e) {
        const int32_t i = ei[e], j = ej[e];
        if (j < 0 || i < j || i >= n) {
            err = "pattern entry " + std::to_string(e) + " not lower triangular / out of range";
            return CDCS_E_PATTERN;
        }
        used[(size_t)i] = used[(size_t)j] = 1;
        if (!entries.insert(key_of(i, j)).second) {
            err = "duplicate pattern entry";
            return CDCS_E_PATTERN;
        }
        if (i != j) {
            adj[(size_t)i].push_back(j);
            adj[(size_t)j].push_back(i);
        }
    }
    std::vector<int32_t> order;
    std::vector<std::vector<int32_t>> later;  // N+(v) in the filled graph
    out.chordal_input = elimination_order(n, adj, used, order, later);
    // maximal cliques from the elimination order
    const size_t nv = order.size();
    std::vector<int32_t> pos((size_t)n, -1);
    for (size_t t = 0; t < nv; ++t) pos[(size_t)order[t]] = (int32_t)t;
    std::vector<char> maximal((size_t)n, 1);
    for (int32_t v : order) {
        int32_t par = -1;
        for (int32_t u : later[(size_t)v])
            if (par < 0 || pos[(size_t)u] < pos[(size_t)par]) par = u;
        if (par >= 0 && later[(size_t)v].size() == later[(size_t)par].size() + 1) maximal[(size_t)par] = 0;
    }
    out.ptr.assign(1, 0);
    std::vector<int32_t> cl;
    std::unordered_set<uint64_t> fill;
    for (int32_t v : order) {
        if (!maximal[(size_t)v]) continue;
        cl.assign(1, v);
        cl.insert(cl.end(), later[(size_t)v].begin(), later[(size_t)v].end());
        std::sort(cl.begin(), cl.end());
        out.vert.insert(out.vert.end(), cl.begin(), cl.end());
        out.ptr.push_back((int64_t)out.vert.size());
        for (size_t a = 0; a < cl.size(); ++a)
            for (size_t b = 0; b <= a; ++b) {
                const uint64_t k = key_of(cl[a], cl[b]);
                if (!entries.count(k) && fill.insert(k).second) {
                    out.fill_i.push_back(cl[a]);
                    out.fill_j.push_back(cl[b]);
                }
            }
    }
    return CDCS_OK;
}

}  // namespace cdcs
