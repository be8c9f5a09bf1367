// Locality relabelling of a graph for the edge pass: reverse Cuthill-McKee (RCM) order.
//
// The edge pass gathers one neighbour row per edge; its speed is set by where those rows sit.  A
// triangulation of random points (the paper's test matrices) numbered in point order has
// neighbours spread over the whole block, so every gather misses the caches.  RCM numbers the nodes
// breadth first, so that neighbours receive nearby ids: a mesh-like graph then gathers mostly rows
// it has just used.  The order is computed once on the host (it is a property of the graph, not
// of U) and applied by the caller to the graph and to U once per solve; the kernels are unchanged.
//
// Cuthill-McKee: per connected component, breadth-first search from a pseudo-peripheral node
// (George and Liu's iteration: from a minimum-degree node, repeatedly restart at a minimum-degree
// node of the last BFS level while the eccentricity grows), visiting the unvisited neighbours of
// each node in increasing (degree, id).  Components are taken in increasing (degree, id) of their
// lowest-degree node, and the whole sequence is reversed.  Deterministic: no ties are left open.
#include <algorithm>
#include <vector>

#include "common.hpp"

namespace pspec {
namespace {

struct Bfs {
    int64_t n;
    const int64_t *rowptr;
    const int32_t *col;
    std::vector<int64_t> level;  // BFS level per node of the current search, -1 unreached
    std::vector<int64_t> touched;

    // Levels from `root` over its component; returns the eccentricity and a minimum-(degree, id)
    // node of the last level.
    std::pair<int64_t, int64_t> run(int64_t root) {
        for (int64_t v : touched) level[v] = -1;
        touched.clear();
        level[root] = 0;
        touched.push_back(root);
        for (size_t h = 0; h < touched.size(); ++h) {
            const int64_t v = touched[h];
            for (int64_t e = rowptr[v]; e < rowptr[v + 1]; ++e) {
                const int64_t u = col[e];
                if (level[u] < 0) {
                    level[u] = level[v] + 1;
                    touched.push_back(u);
                }
            }
        }
        const int64_t ecc = level[touched.back()];
        int64_t best = -1;
        for (size_t h = touched.size(); h-- > 0;) {
            const int64_t v = touched[h];
            if (level[v] != ecc) break;
            if (best < 0 || deg(v) < deg(best) || (deg(v) == deg(best) && v < best)) best = v;
        }
        return {ecc, best};
    }
    int64_t deg(int64_t v) const { return rowptr[v + 1] - rowptr[v]; }
};

}  // namespace
}  // namespace pspec

using namespace pspec;

extern "C" pspec_status pspec_rcm_order(int64_t n, const int64_t *rowptr, const int32_t *col, int64_t *perm) {
    clear_error();
    PSPEC_ARG(n >= 0, "rcm_order: n = %lld < 0", (long long)n);
    PSPEC_ARG(n <= INT32_MAX, "rcm_order: n = %lld does not fit 32-bit column ids", (long long)n);
    if (n == 0) return PSPEC_OK;
    PSPEC_ARG(rowptr != nullptr && perm != nullptr, "rcm_order: rowptr or perm is NULL");
    PSPEC_ARG(rowptr[0] == 0, "rcm_order: rowptr[0] = %lld != 0", (long long)rowptr[0]);
    for (int64_t i = 0; i < n; ++i)
        PSPEC_ARG(rowptr[i + 1] >= rowptr[i], "rcm_order: rowptr decreases at row %lld", (long long)i);
    PSPEC_ARG(rowptr[n] == 0 || col != nullptr, "rcm_order: col is NULL");
    for (int64_t e = 0; e < rowptr[n]; ++e)
        PSPEC_ARG(col[e] >= 0 && col[e] < n, "rcm_order: column id %d out of range at entry %lld", col[e],
                  (long long)e);

    Bfs bfs{n, rowptr, col, std::vector<int64_t>(n, -1), {}};
    auto before = [&](int64_t a, int64_t b) {
        const int64_t da = bfs.deg(a), db = bfs.deg(b);
        return da < db || (da == db && a < b);
    };
    std::vector<int64_t> by_degree(n);
    for (int64_t i = 0; i < n; ++i) by_degree[i] = i;
    std::stable_sort(by_degree.begin(), by_degree.end(), before);

    std::vector<char> seen(n, 0);
    std::vector<int64_t> order;
    order.reserve(n);
    std::vector<int64_t> nbr;
    for (int64_t s : by_degree) {
        if (seen[s]) continue;
        // pseudo-peripheral start of s's component
        int64_t root = s;
        auto [ecc, cand] = bfs.run(root);
        while (cand != root) {
            auto [ecc2, cand2] = bfs.run(cand);
            if (ecc2 <= ecc) break;
            root = cand;
            ecc = ecc2;
            cand = cand2;
        }
        // Cuthill-McKee sweep of the component
        size_t head = order.size();
        order.push_back(root);
        seen[root] = 1;
        for (; head < order.size(); ++head) {
            const int64_t v = order[head];
            nbr.clear();
            for (int64_t e = rowptr[v]; e < rowptr[v + 1]; ++e) {
                const int64_t u = col[e];
                if (!seen[u]) {
                    seen[u] = 1;
                    nbr.push_back(u);
                }
            }
            std::sort(nbr.begin(), nbr.end(), before);
            order.insert(order.end(), nbr.begin(), nbr.end());
        }
    }
    // reverse: node order[h] gets id n - 1 - h
    for (int64_t h = 0; h < n; ++h) perm[order[h]] = n - 1 - h;
    return PSPEC_OK;
}
