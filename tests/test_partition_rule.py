"""The supernode partition rule (section 2, paragraph on supernodes: relaxed
supernodes of nearly identical columns, with a maximal width), pinned by
partitions derived by hand from the rule, for the library's analysis and the
oracle's alike.

Reading of the rule (the paper gives no parameters): on the postordered
elimination tree of At + At^T,
  (i)   every maximal subtree of at most `relax` columns is one supernode;
  (ii)  elsewhere column j joins the run [f, j-1] when j-1 is its only child
        and the padding estimate Z = s cnt(j) - sum_{t=f..j} cnt(t) + s(s-1)/2
        (s = j-f+1, cnt = off-diagonal entries of a column of L) is at most
        pad_pct percent of s (cnt(j) + s);
  (iii) every supernode is cut into pieces of max_super columns.

Fixture "path" (tridiagonal pattern, n = 12, natural order): the tree is a
chain, cnt(j) = 1 for j < 11 and cnt(11) = 0.  For j < 11 a run of s columns
has Z = s(s-1)/2, so (ii) joins while 50 (s-1) <= pad_pct (s+1): pad 20 allows
s <= 2, pad 34 allows s <= 5, pad 0 nothing.  At the last column
Z = (s-1)(s-2)/2: 0 for s = 2, 1 for s = 3.

Fixture "forks" (n = 12): paths 0-1-2 and 3-4-5 both attached to 6, and a
clique on 6..11.  Tree: 0->1->2->6, 3->4->5->6, 6->7->...->11; node 6 has two
children; cnt = 1 on 0..5, cnt(6..11) = 5, 4, 3, 2, 1, 0 (nested clique
columns, Z = 0 along 6..11); subtree sizes 3 (node 2, node 5), 7 (node 6),
8..12 (nodes 7..11).
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import Oracle


def csc_from_edges(n, edges):
    rows = [i for i in range(n)] + [a for a, b in edges] + [b for a, b in edges]
    cols = [i for i in range(n)] + [b for a, b in edges] + [a for a, b in edges]
    m = sp.csc_matrix((np.ones(len(rows)), (rows, cols)), shape=(n, n))
    m.sum_duplicates()
    m.sort_indices()
    return m.indptr.astype(np.int64), m.indices.astype(np.int32)


PATH = [(j, j + 1) for j in range(11)]
FORKS = [(0, 1), (1, 2), (2, 6), (3, 4), (4, 5), (5, 6)] + [(a, b) for a in range(6, 12) for b in range(a + 1, 12)]

# (fixture, relax, pad_pct, max_super, hand-derived xsup)
CASES = [
    # pad 0, no relaxation: fundamental supernodes; only {10, 11} have nested structures
    ("path", 0, 0, 0, [0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 12]),
    # pad 20: pairs (s = 3 gives 100 > 80); the last pair has Z = 0
    ("path", 0, 20, 0, [0, 2, 4, 6, 8, 10, 12]),
    # pad 34: runs of 5 (s = 6 gives 250 > 238), then {10, 11}
    ("path", 0, 34, 0, [0, 5, 10, 12]),
    # relax 3: subtree of node 2 = {0, 1, 2}; pairs from 3 on; {9, 10, 11} joins
    # at the last column (Z = 1, 100 <= 20 * 3 * 3 = 180)
    ("path", 3, 20, 0, [0, 3, 5, 7, 9, 12]),
    # the same cut at 2 columns
    ("path", 3, 20, 2, [0, 2, 3, 5, 7, 9, 11, 12]),
    # relax 3: {0, 1, 2}, {3, 4, 5}; column 6 cannot join 5 (relaxed boundary),
    # 7..11 join 6 (Z = 0)
    ("forks", 3, 0, 0, [0, 3, 6, 12]),
    # no relaxation: the paths stay singletons (Z = 1 > 0), 6 has two
    # children, 6..11 is one fundamental supernode
    ("forks", 0, 0, 0, [0, 1, 2, 3, 4, 5, 6, 12]),
    # relax 7: the subtree of node 6 (7 columns), then 7..11; cut at 3
    ("forks", 7, 0, 3, [0, 3, 6, 7, 10, 12]),
    # relax 2: subtrees of node 1 and node 4; 2 and 5 alone (the next column
    # starts a relaxed subtree / has two children); 6..11 together
    ("forks", 2, 50, 0, [0, 2, 3, 5, 6, 12]),
]


@pytest.fixture(scope="module")
def si():
    from paper_1708_04539_amd import selinv
    return selinv


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}_r{c[1]}_p{c[2]}_cap{c[3]}" for c in CASES])
def test_partition_matches_hand_derivation(si, oracle_mod, case):
    name, relax, pad, cap, want = case
    cp, ri = csc_from_edges(12, PATH if name == "path" else FORKS)
    s = si.SelInv(12, cp, ri, None, cap, relax, pad)
    st = s.structure()
    assert np.array_equal(st["perm"], np.arange(12)), "natural order is already a postorder"
    assert st["xsup"].tolist() == want
    o = Oracle(12, cp, ri, None, cap, relax, 0, pad)
    ost = o.structure()
    assert np.array_equal(ost["perm"], np.arange(12))
    assert ost["xsup"].tolist() == want


def test_postorder_of_a_shuffled_tree(si, oracle_mod):
    """The symmetrized analysis replaces the ordering by a postorder of the
    elimination tree (children in increasing order).  A path 0-1-...-7 given
    in the order [3, 1, 6, 0, 7, 2, 5, 4]: its tree, hand-derived from the
    elimination, is recomputed here by brute force and its postorder by a
    recursive walk; both analyses must return that order."""
    n = 8
    cp, ri = csc_from_edges(n, [(j, j + 1) for j in range(n - 1)])
    perm = np.array([3, 1, 6, 0, 7, 2, 5, 4], np.int32)
    A = sp.csc_matrix((np.ones(len(ri)), ri, cp), shape=(n, n)).toarray() != 0
    At = A[np.ix_(perm, perm)]
    # dense boolean elimination for the tree of At + At^T
    S = At | At.T
    parent = [-1] * n
    for k in range(n):
        below = [i for i in range(k + 1, n) if S[i, k]]
        if below:
            parent[k] = below[0]
            for i in below:
                for j in below:
                    S[i, j] = True
    kids = [[] for _ in range(n)]
    for v in range(n):
        if parent[v] >= 0:
            kids[parent[v]].append(v)
    post = []

    def walk(v):
        for c in kids[v]:
            walk(c)
        post.append(v)

    for r in range(n):
        if parent[r] < 0:
            walk(r)
    want = perm[np.array(post)].tolist()
    assert want != perm.tolist(), "the fixture must need a reordering"
    s = si.SelInv(n, cp, ri, perm, 0, 0, 0)
    assert s.structure()["perm"].tolist() == want
    o = Oracle(n, cp, ri, perm, 0, 0, 0, 0)
    assert o.structure()["perm"].tolist() == want
