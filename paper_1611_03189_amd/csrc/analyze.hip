// Host symbolic analysis: clustering, footprint adjacency, simulated elimination
// (block fill, neighbour / well-separated sets, colour order) for every level.
//
// Paper anchors: §2.1 (graph of A, block partition, block graph), §3 (2^L red nodes by
// recursive bisection, pairwise merge into super nodes), §3.1 (adjacency by the original
// graph, unchanged during elimination; well separated = not a neighbour), §3.2 (fill-in
// created by eliminating a super node couples all pairs of its neighbours; the new red
// node inherits the neighbours of its super node and takes over its well-separated
// blocks).
//
// Rules for what the paper leaves open (the CPU checker follows the same rules in its own
// code; both are listed with the design notes):
//  * depth L = integer nearest log2(n/leaf), decided exactly as the smallest L >= 0 with
//    n^2 < leaf^2 2^(2L+1), capped at floor(log2 n);
//  * bisection along the axis of largest extent (ties: lowest axis), median split after
//    sorting by (coordinate, index), left child = first ceil(size/2); leaves keep their
//    unknowns in ascending index;
//  * a red node is empty exactly when its super node had no well-separated block; empty
//    nodes carry no blocks;
//  * elimination order inside a level: colour by colour; each colour is a greedy pass over
//    the remaining nodes (in index order, or most partners still waiting first with ties by
//    index, opt.order), a node joining only if it has no block to a node already in the
//    colour; a colour is eliminated in index order.
#include <algorithm>
#include <cmath>
#include <limits>
#include <numeric>

#include <string>

#include "hs_internal.h"

namespace hs {

static int depth_for(int64_t n, int64_t leaf) {
    if (n <= 1) return 0;
    int L = 0;
    for (;;) {
        unsigned __int128 lhs = (unsigned __int128)n * (unsigned __int128)n;
        unsigned __int128 rhs = ((unsigned __int128)leaf * (unsigned __int128)leaf) << (2 * L + 1);
        if (lhs < rhs) break;
        ++L;
        if (L > 40) break;
    }
    int cap = 0;
    while ((int64_t(1) << (cap + 1)) <= n) ++cap;
    return std::min(L, cap);
}

static void sorted_insert(std::vector<int>& v, int x) {
    auto it = std::lower_bound(v.begin(), v.end(), x);
    if (it == v.end() || *it != x) v.insert(it, x);
}

static void sorted_erase(std::vector<int>& v, int x) {
    auto it = std::lower_bound(v.begin(), v.end(), x);
    if (it != v.end() && *it == x) v.erase(it);
}

static void validate_pattern(const Plan& P) {
    const int n = P.n;
    if (P.row_ptr[0] != 0) throw Error{HSOLVE_ERR_INVALID, "row_ptr[0] != 0"};
    for (int i = 0; i < n; ++i) {
        if (P.row_ptr[i + 1] < P.row_ptr[i]) throw Error{HSOLVE_ERR_INVALID, "row_ptr decreasing"};
        for (int64_t t = P.row_ptr[i]; t < P.row_ptr[i + 1]; ++t) {
            int c = P.col_idx[t];
            if (c < 0 || c >= n) throw Error{HSOLVE_ERR_INVALID, "column index out of range"};
            if (t > P.row_ptr[i] && P.col_idx[t - 1] >= c)
                throw Error{HSOLVE_ERR_INVALID, "columns not strictly ascending"};
        }
    }
    for (int i = 0; i < n; ++i) {
        for (int64_t t = P.row_ptr[i]; t < P.row_ptr[i + 1]; ++t) {
            int c = P.col_idx[t];
            const int32_t* b = P.col_idx.data() + P.row_ptr[c];
            const int32_t* e = P.col_idx.data() + P.row_ptr[c + 1];
            if (!std::binary_search(b, e, i))
                throw Error{HSOLVE_ERR_NOT_SYMMETRIC, "pattern not symmetric"};
        }
    }
}

// Recursive bisection into 2^L leaves (leaf order perm, leaf offsets).
static void bisect(Plan& P) {
    const int n = P.n, L = P.L;
    const int dim = (P.opt.coords && P.opt.dim > 0) ? P.opt.dim : 0;
    auto coord = [&](int u, int t) -> double {
        return dim ? P.coords[size_t(u) * dim + t] : double(u);
    };
    const int nd = dim ? dim : 1;
    std::vector<int32_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::vector<std::pair<int, int>> ranges{{0, n}}, next;
    for (int lev = 0; lev < L; ++lev) {
        next.clear();
        for (auto [b, e] : ranges) {
            int axis = 0;
            double best = -1.0;
            for (int t = 0; t < nd; ++t) {
                double lo = coord(order[b], t), hi = lo;
                for (int q = b + 1; q < e; ++q) {
                    double x = coord(order[q], t);
                    lo = std::min(lo, x);
                    hi = std::max(hi, x);
                }
                if (hi - lo > best) { best = hi - lo; axis = t; }
            }
            std::sort(order.begin() + b, order.begin() + e, [&](int u, int v) {
                double cu = coord(u, axis), cv = coord(v, axis);
                return cu < cv || (cu == cv && u < v);
            });
            int half = (e - b + 1) / 2;
            next.push_back({b, b + half});
            next.push_back({b + half, e});
        }
        ranges.swap(next);
    }
    P.leaf_off.assign(ranges.size() + 1, 0);
    for (size_t i = 0; i < ranges.size(); ++i) {
        std::sort(order.begin() + ranges[i].first, order.begin() + ranges[i].second);
        P.leaf_off[i] = ranges[i].first;
    }
    P.leaf_off[ranges.size()] = n;
    P.perm = order;
    P.iperm.assign(n, 0);
    for (int p = 0; p < n; ++p) P.iperm[P.perm[p]] = p;
}

void analyze(Plan& P) {
    validate_pattern(P);
    const int n = P.n;
    P.L = depth_for(n, std::max(1, P.opt.leaf_size));
    bisect(P);
    const int L = P.L;
    // the first super nodes are sibling pairs of leaves (the whole matrix when L = 0); larger
    // ones appear later only when ranks grow, which the factorization checks
    for (int s = 0; s < (L > 0 ? (1 << (L - 1)) : 1); ++s) {
        const int m = (L > 0) ? P.leaf_off[2 * s + 2] - P.leaf_off[2 * s] : n;
        if (m > P.opt.max_super)
            throw Error{HSOLVE_ERR_INVALID, "leaf pairs larger than max_super = " +
                                                std::to_string(P.opt.max_super) + " unknowns (reduce leaf_size)"};
    }

    // leaf of every unknown, and the unique leaf-level block pairs
    std::vector<int> leaf_of(n);
    for (int i = 0; i < (1 << L); ++i)
        for (int p = P.leaf_off[i]; p < P.leaf_off[i + 1]; ++p) leaf_of[P.perm[p]] = i;
    std::vector<uint64_t> pairs;
    pairs.reserve(size_t(P.nnz));
    for (int u = 0; u < n; ++u)
        for (int64_t t = P.row_ptr[u]; t < P.row_ptr[u + 1]; ++t) {
            int a = leaf_of[u], b = leaf_of[P.col_idx[t]];
            if (a != b) pairs.push_back(bkey(a, b));
        }
    std::sort(pairs.begin(), pairs.end());
    pairs.erase(std::unique(pairs.begin(), pairs.end()), pairs.end());

    P.total_colours = 0;
    if (L == 0) {      // a single leaf: one super node, eliminated exactly
        P.sym.assign(1, LevelSym{});
        LevelSym& S = P.sym[0];
        S.d = 0;
        S.colours = {{0}};
        S.colour_of = {0};
        S.N.assign(1, {});
        S.W.assign(1, {});
        S.Nred.assign(1, {});
        S.Wred.assign(1, {});
        S.super_nonempty = {1};
        S.red_nonempty = {0};
        S.init_partners.assign(1, {});
        P.total_colours = 1;
        return;
    }
    P.sym.assign(L, LevelSym{});

    // footprint adjacency of depth d, as sorted neighbour lists
    auto adjacency = [&](int d) {
        std::vector<std::vector<int>> adj(size_t(1) << d);
        int sh = L - d;
        for (uint64_t k : pairs) {
            int a = int(k >> 32) >> sh, b = int(k & 0xffffffffu) >> sh;
            if (a != b) adj[a].push_back(b);
        }
        for (auto& v : adj) {
            std::sort(v.begin(), v.end());
            v.erase(std::unique(v.begin(), v.end()), v.end());
        }
        return adj;
    };

    // Geometric neighbours (opt.neighbours = HSOLVE_NEIGHBOURS_GEOMETRIC, the rule of §7's
    // experiments): every unknown is a unit cell at its coordinates (its index when there are
    // none), a cluster the box [min, max + 1) of its cells, its size the box's largest side;
    // clusters are well separated when the Euclidean gap between their boxes exceeds the larger
    // size. Boxes of depth d are unions of the boxes of depth d + 1.
    const bool geometric = P.opt.neighbours == HSOLVE_NEIGHBOURS_GEOMETRIC;
    const int dim = (P.coords.empty() || P.opt.dim < 1) ? 1 : P.opt.dim;
    std::vector<std::vector<double>> box_lo, box_hi;   // [depth][cluster * dim + t]
    if (geometric) {
        box_lo.assign(L + 1, {});
        box_hi.assign(L + 1, {});
        box_lo[L].assign(size_t(1 << L) * dim, std::numeric_limits<double>::infinity());
        box_hi[L].assign(size_t(1 << L) * dim, -std::numeric_limits<double>::infinity());
        for (int i = 0; i < (1 << L); ++i)
            for (int q = P.leaf_off[i]; q < P.leaf_off[i + 1]; ++q)
                for (int t = 0; t < dim; ++t) {
                    const double x = P.coords.empty() ? double(P.perm[q]) : P.coords[size_t(P.perm[q]) * dim + t];
                    box_lo[L][size_t(i) * dim + t] = std::min(box_lo[L][size_t(i) * dim + t], x);
                    box_hi[L][size_t(i) * dim + t] = std::max(box_hi[L][size_t(i) * dim + t], x + 1.0);
                }
        for (int d = L - 1; d >= 0; --d) {
            box_lo[d].resize(size_t(1 << d) * dim);
            box_hi[d].resize(size_t(1 << d) * dim);
            for (int c = 0; c < (1 << d); ++c)
                for (int t = 0; t < dim; ++t) {
                    box_lo[d][size_t(c) * dim + t] =
                        std::min(box_lo[d + 1][size_t(2 * c) * dim + t], box_lo[d + 1][size_t(2 * c + 1) * dim + t]);
                    box_hi[d][size_t(c) * dim + t] =
                        std::max(box_hi[d + 1][size_t(2 * c) * dim + t], box_hi[d + 1][size_t(2 * c + 1) * dim + t]);
                }
        }
    }
    auto geo_near = [&](int d, int i, int j) {
        const double* li = &box_lo[d][size_t(i) * dim];
        const double* hi_ = &box_hi[d][size_t(i) * dim];
        const double* lj = &box_lo[d][size_t(j) * dim];
        const double* hj = &box_hi[d][size_t(j) * dim];
        double g2 = 0.0, si = 0.0, sj = 0.0;
        for (int t = 0; t < dim; ++t) {
            const double g = std::max(0.0, std::max(lj[t] - hi_[t], li[t] - hj[t]));
            g2 += g * g;
            si = std::max(si, hi_[t] - li[t]);
            sj = std::max(sj, hj[t] - lj[t]);
        }
        return std::sqrt(g2) <= std::max(si, sj);
    };

    // pattern of the first level = footprint adjacency of depth L-1 (all nodes non-empty)
    std::vector<std::vector<int>> partners = adjacency(L - 1);
    std::vector<uint8_t> nonempty(size_t(1) << (L - 1), 1);

    for (int d = L - 1; d >= 0; --d) {
        const int nd = 1 << d;
        LevelSym& S = P.sym[d];
        S.d = d;
        S.colour_of.assign(nd, -1);
        S.N.assign(nd, {});
        S.W.assign(nd, {});
        S.Nred.assign(nd, {});
        S.Wred.assign(nd, {});
        S.super_nonempty = nonempty;
        S.red_nonempty.assign(nd, 0);
        S.init_partners = partners;
        std::vector<std::vector<int>> adj;
        if (!geometric) adj = adjacency(d);
        std::vector<uint8_t> is_red(nd, 0);
        std::vector<int> remaining;
        for (int s = 0; s < nd; ++s)
            if (nonempty[s]) remaining.push_back(s);
        std::vector<int> mark(nd, -1);
        while (!remaining.empty()) {
            const int cid = int(S.colours.size());
            // the greedy pass: in index order, or (HSOLVE_ORDER_WAITING) the nodes with the most
            // partners still waiting at this level first, ties by index; either way the colour
            // itself is eliminated in index order
            std::vector<int> order(remaining.size());
            std::iota(order.begin(), order.end(), 0);
            if (P.opt.order == HSOLVE_ORDER_WAITING) {
                std::vector<int> waiting(remaining.size(), 0);
                for (size_t q = 0; q < remaining.size(); ++q)
                    for (int j : partners[remaining[q]]) waiting[q] += S.colour_of[j] < 0;
                std::stable_sort(order.begin(), order.end(),
                                 [&](int a, int b) { return waiting[a] > waiting[b]; });
            }
            std::vector<int> colour;
            for (int q : order) {
                const int s = remaining[q];
                bool ok = true;
                for (int j : partners[s])
                    if (mark[j] == cid) { ok = false; break; }
                if (ok) { colour.push_back(s); mark[s] = cid; }
            }
            std::sort(colour.begin(), colour.end());
            for (int s : colour) {
                S.colour_of[s] = cid;
                std::vector<int>& Ns = S.N[s];
                std::vector<int>& Ws = S.W[s];
                for (int j : partners[s]) {
                    const bool nb = geometric ? geo_near(d, s, j)
                                              : std::binary_search(adj[s].begin(), adj[s].end(), j);
                    (nb ? Ns : Ws).push_back(j);
                    (nb ? S.Nred[s] : S.Wred[s]).push_back(is_red[j]);
                }
                // fill: every pair of neighbours becomes coupled
                for (size_t a = 0; a < Ns.size(); ++a)
                    for (size_t b = a + 1; b < Ns.size(); ++b) {
                        sorted_insert(partners[Ns[a]], Ns[b]);
                        sorted_insert(partners[Ns[b]], Ns[a]);
                    }
                is_red[s] = 1;
                if (Ws.empty()) {            // empty red node: leaves the pattern
                    for (int j : partners[s]) sorted_erase(partners[j], s);
                    partners[s].clear();
                } else {
                    S.red_nonempty[s] = 1;
                }
            }
            std::vector<int> rest;
            for (int s : remaining)
                if (S.colour_of[s] < 0) rest.push_back(s);
            remaining.swap(rest);
            S.colours.push_back(std::move(colour));
        }
        P.total_colours += int(S.colours.size());
        if (d == 0) break;
        // merge sibling red nodes into the super nodes of depth d-1
        std::vector<std::vector<int>> up(size_t(nd) / 2);
        std::vector<uint8_t> up_nonempty(size_t(nd) / 2, 0);
        for (int s = 0; s < nd; ++s)
            if (S.red_nonempty[s]) up_nonempty[s >> 1] = 1;
        for (int s = 0; s < nd; ++s)
            for (int j : partners[s])
                if ((s >> 1) != (j >> 1)) up[s >> 1].push_back(j >> 1);
        for (auto& v : up) {
            std::sort(v.begin(), v.end());
            v.erase(std::unique(v.begin(), v.end()), v.end());
        }
        partners.swap(up);
        nonempty.swap(up_nonempty);
    }
}

}  // namespace hs
