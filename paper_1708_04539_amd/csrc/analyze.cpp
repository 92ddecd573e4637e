// analyze.cpp -- symbolic analysis for supernodal selected inversion.
//
// Two forms (paper, section 2: the method itself needs no structural
// symmetrization, R_L(K) and R_U(K) may differ).
//
// Symmetrized form (all on the host, O(|L|) time):
//   1. validate the CSC pattern and the ordering;
//   2. adjacency of At + At^T (At = P A P^T);
//   3. elimination tree by Liu's path-compressed ancestor walk;
//   4. postorder of that tree (children in increasing order) folded into
//      the ordering, so that every subtree is a contiguous column range;
//   5. column counts of L from row subtrees;
//   6. supernode partition (paper, section 2: relaxed supernodes of nearly
//      identical columns, capped at a maximal width): maximal subtrees of at
//      most `relax` columns; chains (parent(j-1) = j, j has one child) whose
//      padding estimate stays within `pad_pct` percent; cuts every
//      `max_super` columns;
//   7. supernodal symbolic factorisation: R(K) = adjacency of K's columns
//      beyond K, merged with R(C) of every child supernode C;  R_L = R_U = R.
//
// Exact form (no symmetrization, ordering kept as given):
//   2'. lower and upper parts of the pattern of At;
//   3'. the exact structure of the unpivoted L and U, condensed on the fly
//       into fundamental supernodes of L, with symmetric pruning;
//   6'. those supernodes cut every `max_super` columns;
//   7'. R_L(K), R_U(K) from At and the block fill R_L(K') x R_U(K') of the
//       earlier supernodes K' (blockwise pruned the same way).
//
// Both forms then:
//   8. levels of the supernodal dependency graph (root at level 0: Algorithm
//      1 walks K = N..1, and every supernode on one level depends only on
//      shallower ones -- section on inter-supernode parallelism);
//   9. storage offsets, relative-index maps of the gather (Theorem 1: every
//      entry of A^{-T}(R_L(K), R_U(K)) lies in an ancestor's block), storage
//      location of every entry of A, and the flop / byte accounting.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "plan.hpp"

namespace selinv {

int64_t Plan::locate(int32_t r, int32_t c) const {
    int32_t I = supof[r], J = supof[c];
    if (I == J) {
        int32_t f = xsup[I], s = width(I);
        return (LOC_DIAG << LOC_SHIFT) | (off_d[I] + (r - f) + int64_t(c - f) * s);
    }
    if (I > J) {
        const int32_t *b = rl.data() + rl_ptr[J], *e = rl.data() + rl_ptr[J + 1];
        const int32_t *it = std::lower_bound(b, e, r);
        if (it == e || *it != r) return -1;
        return (LOC_L << LOC_SHIFT) | (off_l[J] + (it - b) + int64_t(c - xsup[J]) * cl(J));
    }
    const int32_t *b = ru.data() + ru_ptr[I], *e = ru.data() + ru_ptr[I + 1];
    const int32_t *it = std::lower_bound(b, e, c);
    if (it == e || *it != c) return -1;
    return (LOC_U << LOC_SHIFT) | (off_u[I] + (it - b) + int64_t(r - xsup[I]) * cu(I));
}

namespace {

// adjacency of the symmetric pattern, both triangles, diagonal removed
void symmetric_adjacency(int64_t n, const int64_t *colptr, const int32_t *rowind,
                         const std::vector<int32_t> &q, std::vector<int64_t> &ptr,
                         std::vector<int32_t> &adj) {
    std::vector<int64_t> cnt(n + 1, 0);
    for (int64_t j = 0; j < n; j++)
        for (int64_t k = colptr[j]; k < colptr[j + 1]; k++) {
            int32_t a = q[rowind[k]], b = q[j];
            if (a == b) continue;
            cnt[a + 1]++;
            cnt[b + 1]++;
        }
    for (int64_t i = 0; i < n; i++) cnt[i + 1] += cnt[i];
    std::vector<int32_t> tmp(cnt[n]);
    std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
    for (int64_t j = 0; j < n; j++)
        for (int64_t k = colptr[j]; k < colptr[j + 1]; k++) {
            int32_t a = q[rowind[k]], b = q[j];
            if (a == b) continue;
            tmp[pos[a]++] = b;
            tmp[pos[b]++] = a;
        }
    ptr.assign(n + 1, 0);
    adj.clear();
    adj.reserve(tmp.size());
    for (int64_t i = 0; i < n; i++) {
        int32_t *b = tmp.data() + cnt[i], *e = tmp.data() + cnt[i + 1];
        std::sort(b, e);
        e = std::unique(b, e);
        adj.insert(adj.end(), b, e);
        ptr[i + 1] = adj.size();
    }
}

// Liu's algorithm: for each column k, every i < k adjacent to k is walked up
// (with path compression) to its current root r, which gets parent k.
void etree(int64_t n, const std::vector<int64_t> &ptr, const std::vector<int32_t> &adj,
           std::vector<int32_t> &parent) {
    parent.assign(n, -1);
    std::vector<int32_t> anc(n, -1);
    for (int64_t k = 0; k < n; k++) {
        for (int64_t t = ptr[k]; t < ptr[k + 1]; t++) {
            int32_t i = adj[t];
            if (i >= k) continue;
            while (i != -1 && i != k) {
                int32_t next = anc[i];
                anc[i] = (int32_t)k;
                if (next == -1) parent[i] = (int32_t)k;
                i = next;
            }
        }
    }
}

// Postorder of an elimination forest (parent[j] > j, or -1 at a root),
// children taken in increasing order.  In that order every subtree occupies
// a contiguous block of positions: the blocks of the node's children, in
// increasing order, then the node itself.  A pass from the leaves up sizes
// every block and places each child's block inside its parent's (children
// are met in increasing order, so they are placed in that order); a pass from
// the roots down turns the relative places into absolute positions.
void tree_postorder(int64_t n, const std::vector<int32_t> &parent, std::vector<int32_t> &post) {
    std::vector<int64_t> size(n, 1), used(n, 0), place(n, 0);
    int64_t roots_used = 0;
    for (int64_t j = 0; j < n; j++) {
        const int32_t p = parent[j];
        if (p < 0) {
            place[j] = roots_used;
            roots_used += size[j];
        } else {
            place[j] = used[p];
            used[p] += size[j];
            size[p] += size[j];
        }
    }
    post.assign(n, 0);
    for (int64_t v = n - 1; v >= 0; v--) {
        if (parent[v] >= 0) place[v] += place[parent[v]];
        post[place[v] + size[v] - 1] = (int32_t)v;
    }
}

// number of off-diagonal entries in each column of L, from row subtrees
void column_counts(int64_t n, const std::vector<int64_t> &ptr, const std::vector<int32_t> &adj,
                   const std::vector<int32_t> &parent, std::vector<int64_t> &count) {
    count.assign(n, 0);
    std::vector<int32_t> mark(n, -1);
    for (int64_t i = 0; i < n; i++) {
        mark[i] = (int32_t)i;
        for (int64_t t = ptr[i]; t < ptr[i + 1]; t++) {
            int32_t k = adj[t];
            if (k >= i) continue;
            while (k != -1 && mark[k] != i) {
                count[k]++;
                mark[k] = (int32_t)i;
                k = parent[k];
            }
        }
    }
}

// Lower and upper parts of the permuted pattern: the rows r > k of column k
// of At and the columns c > k of row k, each list sorted.
void split_pattern(int64_t n, const int64_t *colptr, const int32_t *rowind, const std::vector<int32_t> &q,
                   std::vector<int64_t> &lptr, std::vector<int32_t> &lidx, std::vector<int64_t> &uptr,
                   std::vector<int32_t> &uidx) {
    lptr.assign(n + 1, 0);
    uptr.assign(n + 1, 0);
    for (int64_t j = 0; j < n; j++)
        for (int64_t k = colptr[j]; k < colptr[j + 1]; k++) {
            const int32_t r = q[rowind[k]], c = q[j];
            if (r > c) lptr[c + 1]++;
            if (r < c) uptr[r + 1]++;
        }
    for (int64_t i = 0; i < n; i++) {
        lptr[i + 1] += lptr[i];
        uptr[i + 1] += uptr[i];
    }
    lidx.resize(lptr[n]);
    uidx.resize(uptr[n]);
    std::vector<int64_t> lpos(lptr.begin(), lptr.end() - 1), upos(uptr.begin(), uptr.end() - 1);
    for (int64_t j = 0; j < n; j++)
        for (int64_t k = colptr[j]; k < colptr[j + 1]; k++) {
            const int32_t r = q[rowind[k]], c = q[j];
            if (r > c) lidx[lpos[c]++] = r;
            if (r < c) uidx[upos[r]++] = c;
        }
    for (int64_t i = 0; i < n; i++) {
        std::sort(lidx.begin() + lptr[i], lidx.begin() + lptr[i + 1]);
        std::sort(uidx.begin() + uptr[i], uidx.begin() + uptr[i + 1]);
    }
}

// One singly linked list of ids per slot (a column, a row or a supernode).
struct SlotLists {
    std::vector<int64_t> head, next;
    std::vector<int32_t> val;
    void init(int64_t slots) {
        head.assign(slots, -1);
        next.clear();
        val.clear();
    }
    void push(int64_t slot, int32_t v) {
        next.push_back(head[slot]);
        val.push_back(v);
        head[slot] = (int64_t)val.size() - 1;
    }
};

// First value present in both sorted lists (key() maps an entry to the value
// compared), or `none`.
template <typename Key>
int32_t first_common(const int32_t *a, int64_t na, const int32_t *b, int64_t nb, Key key, int32_t none) {
    for (int64_t x = 0, y = 0; x < na && y < nb;) {
        const int32_t ka = key(a[x]), kb = key(b[y]);
        if (ka == kb) return ka;
        if (ka < kb) x++; else y++;
    }
    return none;
}

// Starts of the fundamental supernodes of L for the exact (unsymmetrized)
// pattern: column j joins column j-1 when L(j, j-1) != 0 and both columns
// have the same rows below j.
//
// Gaussian elimination without pivoting gives (the fill rule):
//   rows of L(:, k) below k    = At(k+1:, k)  u  U L(k+1:, j) over the pivots
//                                j < k with U(j, k) != 0,
//   columns of U(k, :) past k  = At(k, k+1:)  u  U U(j, k+1:) over the pivots
//                                j < k with L(k, j) != 0.
// Columns are processed in order and kept condensed: inside a run of
// columns that joined, every column has the same rows FL below the run and,
// since L(i, i-1) != 0 there, row i of U covers row i-1 of U past i.  So the
// pivots of a finished run J act on later columns exactly as its last pivot
// does: column m in FU(J) (the columns of U past the run, last row) receives
// FL(J) beyond m, row m in FL(J) receives FU(J) beyond m.  The run still
// open acts on the next column through its last pivot k-1 alone.  Symmetric
// pruning: once m lies in both FL(J) and FU(J), pivot m has received all of
// FL(J) and FU(J) beyond it and carries them on to every later column and
// row that J would reach, so the pushes of J stop at that m.
void fundamental_starts(int64_t n, const std::vector<int64_t> &lptr, const std::vector<int32_t> &lidx,
                        const std::vector<int64_t> &uptr, const std::vector<int32_t> &uidx,
                        std::vector<int32_t> &starts, std::vector<int64_t> &cntL, std::vector<int64_t> &cntU) {
    cntL.assign(n, 0);
    cntU.assign(n, 0);
    std::vector<int64_t> fl_ptr(1, 0), fu_ptr(1, 0);
    std::vector<int32_t> fl, fu;
    SlotLists toL, toU;  // finished runs whose FL a column (FU a row) receives
    toL.init(n);
    toU.init(n);
    std::vector<int32_t> markL(n, -1), markU(n, -1), prevL, prevU, curL, curU;
    starts.clear();
    int32_t nruns = 0;
    auto finish = [&](int64_t l) {  // the run ending at column l; prevL/prevU are its FL/FU
        const int32_t J = nruns++;
        fl.insert(fl.end(), prevL.begin(), prevL.end());
        fu.insert(fu.end(), prevU.begin(), prevU.end());
        fl_ptr.push_back((int64_t)fl.size());
        fu_ptr.push_back((int64_t)fu.size());
        const int32_t stop = first_common(prevL.data(), (int64_t)prevL.size(), prevU.data(),
                                          (int64_t)prevU.size(), [](int32_t x) { return x; }, INT32_MAX);
        // column and row l + 1 have taken pivot l already (as the open run)
        for (int32_t m : prevU) {
            if (m > stop) break;
            if (m > l + 1) toL.push(m, J);
        }
        for (int32_t m : prevL) {
            if (m > stop) break;
            if (m > l + 1) toU.push(m, J);
        }
    };
    for (int64_t k = 0; k < n; k++) {
        const int32_t k32 = (int32_t)k;
        curL.clear();
        curU.clear();
        auto addL = [&](int32_t r) {
            if (markL[r] != k32) {
                markL[r] = k32;
                curL.push_back(r);
            }
        };
        auto addU = [&](int32_t c) {
            if (markU[c] != k32) {
                markU[c] = k32;
                curU.push_back(c);
            }
        };
        for (int64_t t = lptr[k]; t < lptr[k + 1]; t++) addL(lidx[t]);
        for (int64_t t = uptr[k]; t < uptr[k + 1]; t++) addU(uidx[t]);
        for (int64_t e = toL.head[k]; e >= 0; e = toL.next[e]) {
            const int32_t J = toL.val[e];
            const int32_t *b = fl.data() + fl_ptr[J], *en = fl.data() + fl_ptr[J + 1];
            for (const int32_t *it = std::upper_bound(b, en, k32); it < en; it++) addL(*it);
        }
        for (int64_t e = toU.head[k]; e >= 0; e = toU.next[e]) {
            const int32_t J = toU.val[e];
            const int32_t *b = fu.data() + fu_ptr[J], *en = fu.data() + fu_ptr[J + 1];
            for (const int32_t *it = std::upper_bound(b, en, k32); it < en; it++) addU(*it);
        }
        // pivot k - 1 of the open run
        const bool l_sub = k > 0 && std::binary_search(prevL.begin(), prevL.end(), k32);  // L(k, k-1) != 0
        const bool u_sub = k > 0 && std::binary_search(prevU.begin(), prevU.end(), k32);  // U(k-1, k) != 0
        const auto pl = std::upper_bound(prevL.begin(), prevL.end(), k32);
        const auto pu = std::upper_bound(prevU.begin(), prevU.end(), k32);
        if (u_sub)
            for (auto it = pl; it != prevL.end(); ++it) addL(*it);
        if (l_sub)
            for (auto it = pu; it != prevU.end(); ++it) addU(*it);
        std::sort(curL.begin(), curL.end());
        std::sort(curU.begin(), curU.end());
        cntL[k] = (int64_t)curL.size();
        cntU[k] = (int64_t)curU.size();
        const bool join = l_sub && (size_t)(prevL.end() - pl) == curL.size() && std::equal(pl, prevL.end(), curL.begin());
        if (!join) {
            if (k > 0) finish(k - 1);
            starts.push_back(k32);
        }
        std::swap(prevL, curL);
        std::swap(prevU, curU);
    }
}

// Relaxation of the exact form (section 2: relaxed supernodes of nearly
// identical columns).  Any partition into column ranges is valid, since the
// block sets are closed under the block fill whatever the partition; merged
// columns store explicit zeros.  On the elimination tree of At + At^T (in the
// given order):
//   * every maximal subtree with at most `relax` columns that occupies a
//     contiguous column range becomes one supernode;
//   * elsewhere column j stays joined to j-1 where the fundamental rule
//     joined it, and also joins the run [f, j-1] when j-1 is the only child
//     of j and the padding estimate of the exact counts (cntL: rows of L
//     below the diagonal, cntU: columns of U past it), with s = j-f+1,
//       Z = s cntL(j) - sum_t cntL(t) + s cntU(j) - sum_t cntU(t) + s(s-1),
//     stays at most pad_pct percent of s (cntL(j) + cntU(j) + 2 s).
void relax_exact(int64_t n, const int64_t *colptr, const int32_t *rowind, const std::vector<int32_t> &q,
                 int32_t relax, int32_t pad_pct, const std::vector<int64_t> &cntL,
                 const std::vector<int64_t> &cntU, std::vector<int32_t> &starts) {
    std::vector<int64_t> aptr;
    std::vector<int32_t> adj, parent;
    symmetric_adjacency(n, colptr, rowind, q, aptr, adj);
    etree(n, aptr, adj, parent);
    std::vector<int64_t> size(n, 1);
    std::vector<int32_t> lo(n), nkids(n, 0);  // lo: smallest column of the subtree
    for (int64_t j = 0; j < n; j++) lo[j] = (int32_t)j;
    for (int64_t j = 0; j < n; j++)
        if (parent[j] >= 0) {
            size[parent[j]] += size[j];
            lo[parent[j]] = std::min(lo[parent[j]], lo[j]);
            nkids[parent[j]]++;
        }
    auto ok = [&](int64_t v) { return size[v] <= relax && v - lo[v] + 1 == size[v]; };
    std::vector<int32_t> root(n, -1);
    for (int64_t v = 0; v < n; v++)
        if (ok(v) && (parent[v] < 0 || !ok(parent[v])))
            for (int64_t u = lo[v]; u <= v; u++) root[u] = (int32_t)v;
    std::vector<char> fund_start(n + 1, 0);
    for (int32_t j : starts) fund_start[j] = 1;
    std::vector<int32_t> out;
    int64_t first = 0, sumL = 0, sumU = 0;
    for (int64_t j = 0; j < n; j++) {
        bool join = false;
        if (j > 0) {
            if (root[j] >= 0 || root[j - 1] >= 0) {
                join = root[j] >= 0 && root[j] == root[j - 1];
            } else if (!fund_start[j]) {
                join = true;
            } else if (parent[j - 1] == j && nkids[j] == 1) {
                const int64_t sz = j - first + 1;
                const int64_t Z = sz * cntL[j] - (sumL + cntL[j]) + sz * cntU[j] - (sumU + cntU[j]) + sz * (sz - 1);
                join = 100 * Z <= int64_t(pad_pct) * sz * (cntL[j] + cntU[j] + 2 * sz);
            }
        }
        if (!join) {
            out.push_back((int32_t)j);
            first = j;
            sumL = sumU = 0;
        }
        sumL += cntL[j];
        sumU += cntU[j];
    }
    starts.swap(out);
}

// R_L(K) and R_U(K) of the exact form for the partition in P.xsup: the rows
// of At below K in the columns of K and the columns of At right of K in the
// rows of K, plus the block fill of every earlier supernode K': the entries
// R_L(K') x R_U(K') put the rows of R_L(K') beyond J into R_L(J) for every
// supernode J that R_U(K') meets, and the columns of R_U(K') beyond I into
// R_U(I) for every I that R_L(K') meets.  Every entry of L+U that elimination
// by blocks touches is then in the pattern (the closure the gather relies
// on).  Blockwise symmetric pruning: the first supernode S met by both
// R_L(K') and R_U(K') receives both sets beyond it, and its own fill carries
// them on to every later supernode, so K' pushes to supernodes up to S only.
void exact_block_sets(Plan &P, const std::vector<int64_t> &lptr, const std::vector<int32_t> &lidx,
                      const std::vector<int64_t> &uptr, const std::vector<int32_t> &uidx) {
    const int32_t ns = P.ns;
    SlotLists toL, toU;
    toL.init(ns);
    toU.init(ns);
    P.rl_ptr.assign(ns + 1, 0);
    P.ru_ptr.assign(ns + 1, 0);
    P.rl.clear();
    P.ru.clear();
    std::vector<int32_t> markL(P.n, -1), markU(P.n, -1), RL, RU;
    for (int32_t K = 0; K < ns; K++) {
        const int32_t f = P.xsup[K], l = P.xsup[K + 1] - 1;
        RL.clear();
        RU.clear();
        auto addL = [&](int32_t r) {
            if (markL[r] != K) {
                markL[r] = K;
                RL.push_back(r);
            }
        };
        auto addU = [&](int32_t c) {
            if (markU[c] != K) {
                markU[c] = K;
                RU.push_back(c);
            }
        };
        for (int32_t j = f; j <= l; j++) {
            for (int64_t t = lptr[j]; t < lptr[j + 1]; t++)
                if (lidx[t] > l) addL(lidx[t]);
            for (int64_t t = uptr[j]; t < uptr[j + 1]; t++)
                if (uidx[t] > l) addU(uidx[t]);
        }
        for (int64_t e = toL.head[K]; e >= 0; e = toL.next[e]) {
            const int32_t Q = toL.val[e];
            const int32_t *b = P.rl.data() + P.rl_ptr[Q], *en = P.rl.data() + P.rl_ptr[Q + 1];
            for (const int32_t *it = std::upper_bound(b, en, l); it < en; it++) addL(*it);
        }
        for (int64_t e = toU.head[K]; e >= 0; e = toU.next[e]) {
            const int32_t Q = toU.val[e];
            const int32_t *b = P.ru.data() + P.ru_ptr[Q], *en = P.ru.data() + P.ru_ptr[Q + 1];
            for (const int32_t *it = std::upper_bound(b, en, l); it < en; it++) addU(*it);
        }
        std::sort(RL.begin(), RL.end());
        std::sort(RU.begin(), RU.end());
        P.rl.insert(P.rl.end(), RL.begin(), RL.end());
        P.ru.insert(P.ru.end(), RU.begin(), RU.end());
        P.rl_ptr[K + 1] = (int64_t)P.rl.size();
        P.ru_ptr[K + 1] = (int64_t)P.ru.size();
        const int32_t *sup = P.supof.data();
        const int32_t stop = first_common(RL.data(), (int64_t)RL.size(), RU.data(), (int64_t)RU.size(),
                                          [sup](int32_t x) { return sup[x]; }, INT32_MAX);
        int32_t last = -1;
        for (int32_t c : RU) {
            const int32_t J = sup[c];
            if (J > stop) break;
            if (J != last) toL.push(J, K);
            last = J;
        }
        last = -1;
        for (int32_t r : RL) {
            const int32_t I = sup[r];
            if (I > stop) break;
            if (I != last) toU.push(I, K);
            last = I;
        }
    }
}

// xsup from the starts of the unsplit supernodes (ending with n): each is cut
// into pieces of max_super columns from its first column on.
void cut_partition(Plan &P, const std::vector<int32_t> &starts, int32_t max_super) {
    P.xsup.clear();
    for (size_t t = 0; t + 1 < starts.size(); t++) {
        const int32_t f = starts[t], e = starts[t + 1];
        const int32_t step = max_super > 0 ? max_super : (e - f);
        for (int32_t c = f; c < e; c += step) P.xsup.push_back(c);
    }
    P.xsup.push_back((int32_t)P.n);
    P.ns = (int32_t)P.xsup.size() - 1;
    P.supof.resize(P.n);
    for (int32_t K = 0; K < P.ns; K++)
        for (int32_t c = P.xsup[K]; c < P.xsup[K + 1]; c++) P.supof[c] = K;
}

// Levels of the supernodal dependency graph, processed from the last
// supernode: level(K) = 0 if R_L(K) u R_U(K) is empty, else 1 + the deepest
// level among the supernodes it meets (all later than K).  The blocks of
// A^{-T} that the gather of K reads belong to those supernodes, and the
// left-looking factorisation of K reads exactly the supernodes whose sets
// meet K, so both run level by level.  sparent(K) is the first supernode met
// on level(K) - 1; one_top(K) tells whether it is the only one.
void dependency_levels(Plan &P) {
    const int32_t ns = P.ns;
    P.level.assign(ns, 0);
    P.sparent.assign(ns, -1);
    P.one_top.assign(ns, 1);
    std::vector<int32_t> blk;
    for (int32_t K = ns - 1; K >= 0; K--) {
        blk.clear();
        for (int64_t a = P.rl_ptr[K]; a < P.rl_ptr[K + 1]; a++) {
            const int32_t J = P.supof[P.rl[a]];
            if (blk.empty() || blk.back() != J) blk.push_back(J);
        }
        for (int64_t b = P.ru_ptr[K]; b < P.ru_ptr[K + 1]; b++) {
            const int32_t J = P.supof[P.ru[b]];
            if (blk.empty() || blk.back() != J) blk.push_back(J);
        }
        std::sort(blk.begin(), blk.end());
        blk.erase(std::unique(blk.begin(), blk.end()), blk.end());
        int32_t lev = 0;
        for (int32_t J : blk) lev = std::max(lev, P.level[J] + 1);
        P.level[K] = lev;
        int top = 0;
        for (int32_t J : blk)
            if (P.level[J] == lev - 1 && top++ == 0) P.sparent[K] = J;
        P.one_top[K] = top <= 1;
    }
    P.nlevels = 0;
    for (int32_t K = 0; K < ns; K++) P.nlevels = std::max(P.nlevels, P.level[K] + 1);
    P.levels.assign(P.nlevels, {});
    for (int32_t K = 0; K < ns; K++) P.levels[P.level[K]].push_back(K);
}

// Symmetrized form: pattern of At + At^T, postordered elimination tree,
// relaxed and capped supernodes, R_L = R_U.
void symmetrized_sets(Plan &P, int64_t n, const int64_t *colptr, const int32_t *rowind, int32_t max_super,
                      int32_t relax, int32_t pad_pct) {
    std::vector<int64_t> aptr;
    std::vector<int32_t> adj, parent, post;
    symmetric_adjacency(n, colptr, rowind, P.q, aptr, adj);
    etree(n, aptr, adj, parent);
    tree_postorder(n, parent, post);
    bool ident = true;
    for (int64_t k = 0; k < n; k++) ident &= post[k] == k;
    if (!ident) {
        std::vector<int32_t> np(n);
        for (int64_t k = 0; k < n; k++) np[k] = P.p[post[k]];
        P.p = np;
        for (int64_t k = 0; k < n; k++) P.q[P.p[k]] = (int32_t)k;
        symmetric_adjacency(n, colptr, rowind, P.q, aptr, adj);
        etree(n, aptr, adj, parent);
    }

    // ---- partition -------------------------------------------------------
    // Columns are in postorder, so the subtree of v is the column range
    // [v - size(v) + 1, v].  (i) Every maximal subtree of at most `relax`
    // columns is one supernode.  (ii) Elsewhere a supernode starts at a column
    // and takes in the next column j while j is the parent of the last column
    // taken and has no other child (a chain), and the padding estimate of the
    // extended run [f, j],
    //     Z = s cnt(j) - (cnt(f) + ... + cnt(j)) + s(s-1)/2,   s = j - f + 1,
    // stays within pad_pct percent of the s (cnt(j) + s) entries it stores
    // (Z counts the explicit zeros a run of nested column structures would
    // hold; 0 for identical structures).  (iii) Cut at max_super.
    std::vector<int64_t> cnt;
    column_counts(n, aptr, adj, parent, cnt);
    std::vector<int64_t> size(n, 1), pre(n + 1, 0);
    std::vector<int32_t> nchild(n, 0);
    for (int64_t j = 0; j < n; j++) {
        pre[j + 1] = pre[j] + cnt[j];
        if (parent[j] >= 0) {
            size[parent[j]] += size[j];
            nchild[parent[j]]++;
        }
    }
    std::vector<int32_t> relaxed_last(n, -1);  // at the first column of a relaxed subtree: its last
    for (int64_t v = 0; v < n; v++) {
        const bool top = parent[v] < 0 || size[parent[v]] > relax;
        if (size[v] <= relax && top) relaxed_last[v - size[v] + 1] = (int32_t)v;
    }
    auto extends = [&](int64_t f, int64_t j) {  // may column j join the run [f, j-1]?
        if (relaxed_last[j] >= 0 || parent[j - 1] != j || nchild[j] != 1) return false;
        const int64_t s = j - f + 1;
        const int64_t Z = s * cnt[j] - (pre[j + 1] - pre[f]) + s * (s - 1) / 2;
        return 100 * Z <= int64_t(pad_pct) * s * (cnt[j] + s);
    };
    std::vector<int32_t> starts;
    for (int64_t j = 0; j < n;) {
        starts.push_back((int32_t)j);
        if (relaxed_last[j] >= 0) {
            j = relaxed_last[j] + 1;
            continue;
        }
        const int64_t f = j;
        while (j + 1 < n && extends(f, j + 1)) j++;
        j++;
    }
    starts.push_back((int32_t)n);
    cut_partition(P, starts, max_super);

    // ---- supernodal symbolic ------------------------------------------
    const int32_t ns = P.ns;
    P.rl_ptr.assign(ns + 1, 0);
    P.rl.clear();
    std::vector<std::vector<int32_t>> kids(ns);
    std::vector<int32_t> mark(n, -1), R;
    for (int32_t K = 0; K < ns; K++) {
        int32_t f = P.xsup[K], l = P.xsup[K + 1] - 1;
        R.clear();
        for (int32_t j = f; j <= l; j++)
            for (int64_t t = aptr[j]; t < aptr[j + 1]; t++) {
                int32_t i = adj[t];
                if (i > l && mark[i] != K) {
                    mark[i] = K;
                    R.push_back(i);
                }
            }
        for (int32_t C : kids[K])
            for (int64_t t = P.rl_ptr[C]; t < P.rl_ptr[C + 1]; t++) {
                int32_t i = P.rl[t];
                if (i > l && mark[i] != K) {
                    mark[i] = K;
                    R.push_back(i);
                }
            }
        std::sort(R.begin(), R.end());
        P.rl.insert(P.rl.end(), R.begin(), R.end());
        P.rl_ptr[K + 1] = P.rl.size();
        if (!R.empty()) kids[P.supof[R[0]]].push_back(K);
    }
    P.ru_ptr = P.rl_ptr;
    P.ru = P.rl;
}

// Storage offsets, accounting, gather maps and the location of every entry
// of A, for the sets and levels in P.
selinv_status finish_plan(Plan &P, int64_t n, const int64_t *colptr, const int32_t *rowind, std::string &err) {
    const int32_t ns = P.ns;
    // ---- storage and accounting -----------------------------------------
    P.off_d.assign(ns + 1, 0);
    P.off_l.assign(ns + 1, 0);
    P.off_u.assign(ns + 1, 0);
    P.flops = P.flops_gemm = P.bytes64 = P.bytes32 = P.max_gemm_flops = 0;
    P.max_s = P.max_c = 0;
    for (int32_t K = 0; K < ns; K++) {
        double s = P.width(K), cl = (double)P.cl(K), cu = (double)P.cu(K);
        P.off_d[K + 1] = P.off_d[K] + int64_t(s * s);
        P.off_l[K + 1] = P.off_l[K] + int64_t(cl * s);
        P.off_u[K + 1] = P.off_u[K] + int64_t(cu * s);
        double g = 4 * s * cl * cu + 2 * s * s * cu;
        P.flops_gemm += g;
        P.flops += g + s * s * (cl + cu) + 4.0 / 3.0 * s * s * s;
        double in_out = 8 * s * s + 8 * s * (cl + cu) + 8 * s * s;
        P.bytes64 += in_out + 8 * s * (cl + cu) + 8 * cl * cu;
        P.bytes32 += in_out + 4 * s * (cl + cu) + 4 * cl * cu;
        double big = 2 * s * cl * cu;
        if (big > P.max_gemm_flops) {
            P.max_gemm_flops = big;
            P.max_gemm_m = (int32_t)cl;
            P.max_gemm_n = (int32_t)s;
            P.max_gemm_k = (int32_t)cu;
        }
        P.max_s = std::max<int32_t>(P.max_s, (int32_t)s);
        P.max_c = std::max<int32_t>(P.max_c, (int32_t)std::max(cl, cu));
    }
    P.tot_d = P.off_d[ns];
    P.tot_l = P.off_l[ns];
    P.tot_u = P.off_u[ns];

    // ---- gather maps ------------------------------------------------------
    P.l_coloff.assign(P.ru.size(), -1);
    P.u_rowoff.assign(P.rl.size(), -1);
    P.mapL.clear();
    P.mapU.clear();
    for (int32_t K = 0; K < ns; K++) {
        const int32_t *RL = P.rl.data() + P.rl_ptr[K], *RU = P.ru.data() + P.ru_ptr[K];
        int64_t cl = P.cl(K), cu = P.cu(K);
        // L side: for each block J of R_U(K)
        for (int64_t b = 0; b < cu;) {
            int32_t J = P.supof[RU[b]];
            int64_t be = b;
            while (be < cu && P.supof[RU[be]] == J) be++;
            int32_t lastJ = P.xsup[J + 1] - 1;
            int64_t a0 = std::upper_bound(RL, RL + cl, lastJ) - RL;
            int64_t seg = (int64_t)P.mapL.size();
            const int32_t *RJ = P.rl.data() + P.rl_ptr[J];
            int64_t clJ = P.cl(J), t = 0;
            for (int64_t a = a0; a < cl; a++) {
                while (t < clJ && RJ[t] < RL[a]) t++;
                if (t == clJ || RJ[t] != RL[a]) {
                    err = "closure violated (L side)";
                    return SELINV_E_BAD_PATTERN;
                }
                P.mapL.push_back((int32_t)t);
            }
            for (int64_t x = b; x < be; x++) P.l_coloff[P.ru_ptr[K] + x] = seg - a0;
            b = be;
        }
        // U side: for each block I of R_L(K)
        for (int64_t a = 0; a < cl;) {
            int32_t I = P.supof[RL[a]];
            int64_t ae = a;
            while (ae < cl && P.supof[RL[ae]] == I) ae++;
            int32_t lastI = P.xsup[I + 1] - 1;
            int64_t b0 = std::upper_bound(RU, RU + cu, lastI) - RU;
            int64_t seg = (int64_t)P.mapU.size();
            const int32_t *RI = P.ru.data() + P.ru_ptr[I];
            int64_t cuI = P.cu(I), t = 0;
            for (int64_t b = b0; b < cu; b++) {
                while (t < cuI && RI[t] < RU[b]) t++;
                if (t == cuI || RI[t] != RU[b]) {
                    err = "closure violated (U side)";
                    return SELINV_E_BAD_PATTERN;
                }
                P.mapU.push_back((int32_t)t);
            }
            for (int64_t x = a; x < ae; x++) P.u_rowoff[P.rl_ptr[K] + x] = seg - b0;
            a = ae;
        }
    }

    // ---- where the entries of A live --------------------------------------
    P.a_loc.resize(P.nnz_a);
    for (int64_t j = 0; j < n; j++)
        for (int64_t k = colptr[j]; k < colptr[j + 1]; k++) {
            int64_t loc = P.locate(P.q[rowind[k]], P.q[j]);
            if (loc < 0) {
                err = "entry of A outside the symbolic pattern";
                return SELINV_E_BAD_PATTERN;
            }
            P.a_loc[k] = loc;
        }
    return SELINV_OK;
}

}  // namespace

selinv_status analyze(Plan &P, int64_t n, const int64_t *colptr, const int32_t *rowind,
                      const int32_t *perm, int32_t max_super, int32_t relax, int32_t pad_pct,
                      int32_t symbolic, std::string &err) {
    if (n < 1 || !colptr || !rowind) {
        err = "n must be >= 1 and colptr/rowind non-null";
        return SELINV_E_INVALID_ARG;
    }
    if (n >= (int64_t(1) << 31) - 1) {
        err = "n exceeds the int32 index range";
        return SELINV_E_INVALID_ARG;
    }
    if (colptr[0] != 0) {
        err = "colptr[0] != 0";
        return SELINV_E_BAD_PATTERN;
    }
    for (int64_t j = 0; j < n; j++) {
        if (colptr[j + 1] < colptr[j]) {
            err = "colptr decreases";
            return SELINV_E_BAD_PATTERN;
        }
        bool diag = false;
        for (int64_t k = colptr[j]; k < colptr[j + 1]; k++) {
            int32_t r = rowind[k];
            if (r < 0 || r >= n || (k > colptr[j] && rowind[k - 1] >= r)) {
                err = "row indices out of range, unsorted or duplicated in column " + std::to_string(j);
                return SELINV_E_BAD_PATTERN;
            }
            diag |= r == j;
        }
        if (!diag) {
            err = "missing diagonal entry in column " + std::to_string(j);
            return SELINV_E_BAD_PATTERN;
        }
    }
    P.n = n;
    P.nnz_a = colptr[n];
    P.a_colptr.assign(colptr, colptr + n + 1);
    P.a_rowind.assign(rowind, rowind + P.nnz_a);
    P.p.resize(n);
    P.q.assign(n, -1);
    for (int64_t i = 0; i < n; i++) {
        int32_t v = perm ? perm[i] : (int32_t)i;
        if (v < 0 || v >= n || P.q[v] >= 0) {
            err = "perm is not a permutation";
            return SELINV_E_BAD_PERM;
        }
        P.p[i] = v;
        P.q[v] = (int32_t)i;
    }
    P.symbolic = symbolic;
    if (symbolic == SELINV_SYMBOLIC_EXACT) {
        std::vector<int64_t> lptr, uptr;
        std::vector<int32_t> lidx, uidx, starts;
        std::vector<int64_t> cntL, cntU;
        split_pattern(n, colptr, rowind, P.q, lptr, lidx, uptr, uidx);
        fundamental_starts(n, lptr, lidx, uptr, uidx, starts, cntL, cntU);
        if (relax > 0 || pad_pct > 0) relax_exact(n, colptr, rowind, P.q, relax, pad_pct, cntL, cntU, starts);
        starts.push_back((int32_t)n);
        cut_partition(P, starts, max_super);
        exact_block_sets(P, lptr, lidx, uptr, uidx);
    } else {
        symmetrized_sets(P, n, colptr, rowind, max_super, relax, pad_pct);
    }
    dependency_levels(P);
    return finish_plan(P, n, colptr, rowind, err);
}

// Recompute every source index of the gather exactly as the kernel does (from
// the relative-index maps) and compare it with an independent binary-search
// location of the same entry.  Also checks that every location is inside its
// array.  Returns the number of mismatches (0 = consistent).
int64_t check_gather_maps(const Plan &P, std::string &err) {
    int64_t bad = 0;
    for (int32_t K = 0; K < P.ns; K++) {
        const int64_t cl = P.cl(K), cu = P.cu(K);
        const int32_t *RL = P.rl.data() + P.rl_ptr[K], *RU = P.ru.data() + P.ru_ptr[K];
        for (int64_t b = 0; b < cu; b++) {
            const int32_t c = RU[b], J = P.supof[c];
            for (int64_t a = 0; a < cl; a++) {
                const int32_t r = RL[a], I = P.supof[r];
                int64_t kind, off;
                if (I == J) {
                    kind = LOC_DIAG;
                    off = P.off_d[J] + int64_t(c - P.xsup[J]) * P.width(J) - P.xsup[J] + r;
                } else if (I > J) {
                    const int64_t m = P.l_coloff[P.ru_ptr[K] + b] + a;
                    if (m < 0 || m >= (int64_t)P.mapL.size()) {
                        bad++;
                        continue;
                    }
                    kind = LOC_L;
                    off = P.off_l[J] + int64_t(c - P.xsup[J]) * P.cl(J) + P.mapL[m];
                } else {
                    const int64_t m = P.u_rowoff[P.rl_ptr[K] + a] + b;
                    if (m < 0 || m >= (int64_t)P.mapU.size()) {
                        bad++;
                        continue;
                    }
                    kind = LOC_U;
                    off = P.off_u[I] + int64_t(r - P.xsup[I]) * P.cu(I) + P.mapU[m];
                }
                const int64_t limit = kind == LOC_DIAG ? P.tot_d : kind == LOC_L ? P.tot_l : P.tot_u;
                const int64_t want = P.locate(r, c);
                if (off < 0 || off >= limit || want != ((kind << LOC_SHIFT) | off)) bad++;
            }
        }
    }
    for (int64_t k = 0; k < P.nnz_a; k++) {
        const int64_t kind = P.a_loc[k] >> LOC_SHIFT, off = P.a_loc[k] & LOC_MASK;
        const int64_t limit = kind == LOC_DIAG ? P.tot_d : kind == LOC_L ? P.tot_l : P.tot_u;
        if (off < 0 || off >= limit) bad++;
    }
    if (bad) err = std::to_string(bad) + " inconsistent gather or extraction indices";
    return bad;
}

}  // namespace selinv
