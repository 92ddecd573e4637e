"""Pins of the FP64 oracle against facts fixed outside it.

Each test checks the oracle against something it does not share code with:
LAPACK's dense inverse (numpy.linalg.inv), closed forms (the 2x2 block
formula of the paper, the inverse of tridiag(-1, 2, -1), the Usmani formula for
a general tridiagonal matrix), the triangular special case, the identities
(A A^{-1})_ii = (A^{-1} A)_jj = 1 evaluated on selected entries only, ordering
invariance, the other step-4 formula, and the block structure of the paper's
Fig. 2 (b).
"""
import json
import os

import numpy as np
import pytest

from oracle import Oracle, OracleError
from workloads import config_c0, nested_dissection, random_sparse, tridiag_csc

from fig2b import fig2b_factors as _fig2b_factors

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def superset_err(o, dense_inv):
    r, c, v = o.export()
    return np.abs(v - dense_inv[r, c]).max() / np.abs(dense_inv).max()


def run(n, cp, ri, v, perm=None, max_super=0, relax=0, mode=0):
    return Oracle(n, cp, ri, perm, max_super, relax, mode).factor(v).selinv()


# --------------------------------------------------------------------------
# dense inverse (brute force) on small inputs
# --------------------------------------------------------------------------
@pytest.mark.parametrize("seed", [0, 1, 2, 3])
@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("cap,relax", [(1, 0), (3, 0), (4, 6), (64, 16)])
def test_random_unsymmetric_vs_dense_inverse(seed, mode, cap, relax):
    n = 70
    cp, ri, v, dense = random_sparse(n, 0.04, seed)
    perm = np.random.default_rng(100 + seed).permutation(n).astype(np.int32)
    o = run(n, cp, ri, v, perm, cap, relax, mode)
    assert superset_err(o, np.linalg.inv(dense)) < 1e-13


def test_exact_mode_has_unequal_block_rows_and_columns():
    """The non-symmetric case (C_L != C_U) really occurs in the exact mode."""
    n = 70
    cp, ri, v, dense = random_sparse(n, 0.04, 5)
    o = run(n, cp, ri, v, None, 4, 0, 1)
    st = o.structure()
    ns = len(st["xsup"]) - 1
    differ = sum(
        not np.array_equal(st["rl"][st["rl_ptr"][K]:st["rl_ptr"][K + 1]],
                           st["ru"][st["ru_ptr"][K]:st["ru_ptr"][K + 1]]) for K in range(ns))
    assert differ > ns // 4
    assert superset_err(o, np.linalg.inv(dense)) < 1e-13


def test_c0_whole_superset_vs_dense_inverse():
    w = config_c0()
    o = run(w.n, w.colptr, w.rowind, w.values, w.perm, w.max_super, w.relax)
    inv = np.linalg.inv(w.to_scipy().toarray())
    assert superset_err(o, inv) < 1e-13
    r, c, v = o.export()
    d = r == c
    assert d.sum() == w.n
    assert np.abs(v[d] / inv[r[d], c[d]] - 1).max() < 1e-13


def test_single_supernode_is_dense_inverse():
    n = 24
    cp, ri, v, dense = random_sparse(n, 0.3, 7)
    o = run(n, cp, ri, v, None, n, n)
    r, c, val = o.export()
    assert len(val) == n * n
    assert np.abs(val - np.linalg.inv(dense)[r, c]).max() < 1e-14


# --------------------------------------------------------------------------
# closed forms
# --------------------------------------------------------------------------
def _laplace_inv(n, i, j):
    """tridiag(-1, 2, -1)^{-1}(i, j) = min(i,j) (n + 1 - max(i,j)) / (n + 1), 1-based."""
    i1, j1 = i + 1, j + 1
    return np.minimum(i1, j1) * (n + 1 - np.maximum(i1, j1)) / (n + 1)


@pytest.mark.parametrize("order", ["natural", "bisection"])
@pytest.mark.parametrize("cap,relax", [(1, 0), (8, 0), (16, 8)])
def test_tridiag_laplacian_closed_form(order, cap, relax):
    n = 150
    cp, ri, v = tridiag_csc(-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1))
    perm = None if order == "natural" else nested_dissection((n,), 3)
    o = run(n, cp, ri, v, perm, cap, relax)
    r, c, val = o.export()
    ref = _laplace_inv(n, r, c)
    assert np.abs(val - ref).max() / np.abs(ref).max() < 1e-12


def _usmani_inv(a, b, c):
    """Inverse of the tridiagonal matrix with diagonal a, super-diagonal b and
    sub-diagonal c via the leading (theta) and trailing (phi) principal minors."""
    n = len(a)
    th = np.zeros(n + 1)
    th[0], th[1] = 1.0, a[0]
    for i in range(2, n + 1):
        th[i] = a[i - 1] * th[i - 1] - b[i - 2] * c[i - 2] * th[i - 2]
    ph = np.zeros(n + 2)
    ph[n + 1], ph[n] = 1.0, a[n - 1]
    for i in range(n - 1, 0, -1):
        ph[i] = a[i - 1] * ph[i + 1] - b[i - 1] * c[i - 1] * ph[i + 2]
    inv = np.zeros((n, n))
    for i in range(1, n + 1):
        for j in range(1, n + 1):
            if i < j:
                inv[i - 1, j - 1] = (-1) ** (i + j) * np.prod(b[i - 1:j - 1]) * th[i - 1] * ph[j + 1] / th[n]
            elif i == j:
                inv[i - 1, j - 1] = th[i - 1] * ph[i + 1] / th[n]
            else:
                inv[i - 1, j - 1] = (-1) ** (i + j) * np.prod(c[j - 1:i - 1]) * th[j - 1] * ph[i + 1] / th[n]
    return inv


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("order", ["natural", "bisection"])
def test_unsymmetric_tridiagonal_closed_form(mode, order):
    n = 40
    rng = np.random.default_rng(11)
    a = rng.uniform(3, 4, n)
    b = rng.uniform(-1, 1, n - 1)
    c = rng.uniform(-1, 1, n - 1)
    cp, ri, v = tridiag_csc(c, a, b)
    perm = None if order == "natural" else nested_dissection((n,), 2)
    o = run(n, cp, ri, v, perm, 4, 0, mode)
    r, cc, val = o.export()
    ref = _usmani_inv(a, b, c)
    assert np.abs(val - ref[r, cc]).max() / np.abs(ref).max() < 1e-14


@pytest.mark.parametrize("cap", [1, 2])
def test_two_by_two_block_formula(cap):
    """eq. Ainv2by2 with scalar blocks: L11 = 1, U11 = a, S = d - c b / a."""
    a, b, c, d = 3.0, -1.25, 0.5, 2.0
    dense = np.array([[a, b], [c, d]])
    cp = np.array([0, 2, 4], np.int64)
    ri = np.array([0, 1, 0, 1], np.int32)
    v = np.array([a, c, b, d])
    o = run(2, cp, ri, v, None, cap, 0)
    S = d - c * b / a
    L21, U12 = c / a, b
    ref = np.array([[1 / a + (1 / a) * U12 * (1 / S) * L21, -(1 / a) * U12 * (1 / S)],
                    [-(1 / S) * L21, 1 / S]])
    got = np.array([[o.get(i, j) for j in range(2)] for i in range(2)])
    assert np.abs(got - ref).max() < 1e-15
    adj = np.array([[d, -b], [-c, a]]) / (a * d - b * c)
    assert np.abs(got - adj).max() < 1e-15
    assert np.abs(got - np.linalg.inv(dense)).max() < 1e-15


@pytest.mark.parametrize("lower", [True, False])
def test_triangular_selected_entries(lower):
    """For triangular A the only nonzero selected entries are 1 / A_ii."""
    n = 60
    cp, ri, v, dense = random_sparse(n, 0.06, 3, lower_only=lower, upper_only=not lower)
    o = run(n, cp, ri, v, None, 5, 0, 1)
    sel = o.get_selected()
    cols = np.repeat(np.arange(n), np.diff(cp))
    diag = ri == cols
    assert np.abs(sel[diag] * v[diag] - 1).max() < 1e-15
    assert np.all(sel[~diag] == 0.0)


# --------------------------------------------------------------------------
# identities on the selected set
# --------------------------------------------------------------------------
def _row_col_checks(n, cp, ri, v, sel):
    cols = np.repeat(np.arange(n), np.diff(cp))
    prod = v * sel  # A(i, j) * A^{-1}(j, i)
    row = np.bincount(ri, weights=prod, minlength=n)   # (A A^{-1})_ii
    col = np.bincount(cols, weights=prod, minlength=n)  # (A^{-1} A)_jj
    return row, col


def test_identities_on_selected_entries_c0():
    w = config_c0()
    o = run(w.n, w.colptr, w.rowind, w.values, w.perm, w.max_super, w.relax)
    sel = o.get_selected()
    row, col = _row_col_checks(w.n, w.colptr, w.rowind, w.values, sel)
    assert np.abs(row - 1).max() < 1e-13
    assert np.abs(col - 1).max() < 1e-13
    assert abs(row.sum() - w.n) < 1e-10


def test_identities_on_selected_entries_random():
    n = 300
    cp, ri, v, _ = random_sparse(n, 0.01, 9)
    perm = np.random.default_rng(9).permutation(n).astype(np.int32)
    o = run(n, cp, ri, v, perm, 8, 4)
    row, col = _row_col_checks(n, cp, ri, v, o.get_selected())
    assert np.abs(row - 1).max() < 1e-13
    assert np.abs(col - 1).max() < 1e-13


def test_ordering_invariance():
    n = 120
    cp, ri, v, _ = random_sparse(n, 0.03, 4)
    ref = run(n, cp, ri, v, None, 6, 0).get_selected()
    for s in range(3):
        perm = np.random.default_rng(s).permutation(n).astype(np.int32)
        got = run(n, cp, ri, v, perm, 6, 3).get_selected()
        assert np.abs(got - ref).max() / np.abs(ref).max() < 1e-13


def test_other_diagonal_formula_agrees():
    w = config_c0()
    o = run(w.n, w.colptr, w.rowind, w.values, w.perm, w.max_super, w.relax)
    diff, mx = o.diag_alt()
    assert diff <= 1e-13 * mx


# --------------------------------------------------------------------------
# structure
# --------------------------------------------------------------------------
def test_partition_rules_c0():
    w = config_c0()
    o = Oracle(w.n, w.colptr, w.rowind, w.perm, w.max_super, w.relax)
    st = o.structure()
    xs = st["xsup"]
    assert xs[0] == 0 and xs[-1] == w.n
    assert np.all(np.diff(xs) >= 1) and np.all(np.diff(xs) <= w.max_super)
    assert sorted(st["perm"].tolist()) == list(range(w.n))
    for K in range(len(xs) - 1):
        R = st["rl"][st["rl_ptr"][K]:st["rl_ptr"][K + 1]]
        assert np.all(np.diff(R) > 0)
        assert R.size == 0 or R[0] >= xs[K + 1]
    # the top separator (32 nodes) is the last supernode and has no block rows
    assert xs[-1] - xs[-2] == 32 and st["rl_ptr"][-1] == st["rl_ptr"][-2]


def test_fig2b_block_structure():
    spec, xs, rl_ptr, rl, ru_ptr, ru, L, U = _fig2b_factors()
    n = int(xs[-1])
    sup = np.searchsorted(xs, np.arange(n), side="right") - 1

    def blocks(ptr, idx, K):
        return sorted({int(sup[i]) + 1 for i in idx[ptr[K]:ptr[K + 1]]})

    for K, want in spec["expect"]["C_L"].items():
        assert blocks(rl_ptr, rl, int(K) - 1) == want
    for K, want in spec["expect"]["C_U"].items():
        assert blocks(ru_ptr, ru, int(K) - 1) == want
    o = Oracle.from_factors(n, xs, rl_ptr, rl, ru_ptr, ru, L, U).selinv()
    A = L @ U
    inv = np.linalg.inv(A)
    r, c, v = o.export()
    assert np.abs(v - inv[r, c]).max() / np.abs(inv).max() < 1e-13
    # A^{-T}(9, 5) is exactly zero: supernode 5 has no U block beyond its diagonal
    zb = spec["expect"]["zero_block_of_Ainv_T"]
    I, J = zb["I"] - 1, zb["J"] - 1
    for rr in range(xs[I], xs[I + 1]):
        for cc in range(xs[J], xs[J + 1]):
            assert o.get(cc, rr) == 0.0  # A^{-1}(cc, rr) = A^{-T}(rr, cc)
    # only part of A^{-T}(10, 10) lies in the columns gathered for supernode 6
    K6 = 5
    R_U6 = ru[ru_ptr[K6]:ru_ptr[K6 + 1]]
    assert len([x for x in R_U6 if sup[x] == 9]) == 3 < spec["widths"][9]


# --------------------------------------------------------------------------
# error paths
# --------------------------------------------------------------------------
def test_error_paths():
    cp = np.array([0, 2, 4], np.int64)
    with pytest.raises(OracleError) as e:
        Oracle(2, cp, np.array([1, 0, 0, 1], np.int32))  # unsorted rows
    assert e.value.status == "BAD_PATTERN"
    with pytest.raises(OracleError) as e:
        Oracle(2, np.array([0, 1, 2], np.int64), np.array([1, 0], np.int32))  # no diagonal
    assert e.value.status == "BAD_PATTERN"
    with pytest.raises(OracleError) as e:
        Oracle(2, cp, np.array([0, 1, 0, 1], np.int32), np.array([0, 0], np.int32))
    assert e.value.status == "BAD_PERM"
    o = Oracle(2, cp, np.array([0, 1, 0, 1], np.int32), None, 2, 0)
    with pytest.raises(OracleError) as e:
        o.factor(np.array([0.0, 1.0, 1.0, 0.0]))  # zero pivot without pivoting
    assert e.value.status == "ZERO_PIVOT"
    with pytest.raises(OracleError) as e:
        o.selinv()
    assert e.value.status == "STATE"
    # get outside the computed set
    n = 3
    cp3, ri3, v3 = tridiag_csc(np.zeros(2) + 0.5, np.ones(3) * 2, np.zeros(2) + 0.5)
    # drop the (0, 2)-pair by construction: tridiagonal, natural order, cap 1
    o3 = run(n, cp3, ri3, v3, None, 1, 0)
    with pytest.raises(OracleError) as e:
        o3.get(0, 2)
    assert e.value.status == "NOT_SELECTED"


# --------------------------------------------------------------------------
# complex selected entries from their definition (oracle/complex_ref.py)
# --------------------------------------------------------------------------
def test_complex_oracle_diagonal_and_2x2_closed_forms():
    from oracle.complex_ref import selected_dense
    d = np.array([2 + 1j, -1 + 3j, 0.5 - 0.25j])
    cp = np.arange(4, dtype=np.int64)
    ri = np.arange(3, dtype=np.int32)
    assert np.allclose(selected_dense(3, cp, ri, d), 1 / d, rtol=1e-15, atol=0)
    # [[a, b], [c, e]]^{-1} = [[e, -b], [-c, a]] / (a e - b c)
    a, b, c, e = 3 + 1j, -1 + 0.5j, 0.25 - 2j, 4 - 1j
    cp = np.array([0, 2, 4], np.int64)
    ri = np.array([0, 1, 0, 1], np.int32)
    vals = np.array([a, c, b, e])  # CSC: column 0 = (a, c), column 1 = (b, e)
    det = a * e - b * c
    inv = np.array([[e, -b], [-c, a]]) / det
    # out[p] = A^{-1}(j, i) for entry p at (i, j)
    want = np.array([inv[0, 0], inv[0, 1], inv[1, 0], inv[1, 1]])
    assert np.allclose(selected_dense(2, cp, ri, vals), want, rtol=1e-14, atol=0)


def test_complex_oracle_sparse_columns_match_dense():
    """The two routes of the complex oracle (LAPACK dense inverse, SuperLU
    solves) agree, and the dense one satisfies A X = I."""
    from oracle.complex_ref import selected_dense, solve_columns, to_dense
    from workloads import stencil_csc_complex
    cp, ri, v = stencil_csc_complex((12, 10), "box", 0.05, seed=4)
    n = 120
    A = to_dense(n, cp, ri, v)
    inv = np.linalg.inv(A)
    assert np.abs(A @ inv - np.eye(n)).max() < 1e-12
    xs = solve_columns(n, cp, ri, v, [0, 57, 119])
    for j, x in zip([0, 57, 119], xs):
        assert np.abs(x - inv[:, j]).max() < 1e-13 * np.abs(inv).max()
    sel = selected_dense(n, cp, ri, v)
    cols = np.repeat(np.arange(n), np.diff(cp))
    assert np.array_equal(sel, inv[cols, ri])


# --------------------------------------------------------------------------
# sampled exact columns (oracle.sampled): the reference at full size
# --------------------------------------------------------------------------
@pytest.mark.parametrize("which", ["c0", "grid3d_27pt"])
def test_sampled_columns_match_dense_inverse(which):
    """solve_column against LAPACK's dense inverse, on C0 and on a 13x13x12
    27-point stencil of the C4 recipe (n = 2028): every entry of each solved
    column to 1e-13, and the returned bound (Varah's bound on ||A^{-1}||_inf
    times the extended-precision residual) holds and is small."""
    from oracle.sampled import solve_column, solve_columns, varah_bound
    from workloads import config_grid
    if which == "c0":
        w = config_c0()
    else:
        w = config_grid("g", (13, 13, 12), "box", "sym_perturbed", 0.1, 0, 512, 64, delta=0.15)
    A = w.to_scipy()
    inv = np.linalg.inv(A.toarray())
    js = [0, w.n - 1, int(w.perm[-1])] + [int(j) for j in np.random.default_rng(5).integers(0, w.n, 3)]
    for j in js[:3]:
        x, bound = solve_column(A, j)
        err = np.abs(x - inv[:, j]).max()
        assert err <= 1e-13, (j, err)
        assert bound <= 1e-13, (j, bound)
        assert err <= bound + 1e-14, (j, err, bound)
    # the pool gives the same columns
    for j, (x, bound) in zip(js, solve_columns(A, js, workers=2)):
        assert np.abs(x - inv[:, j]).max() <= 1e-13 and bound <= 1e-13


def test_varah_bound_is_the_margin():
    """The stencil recipe makes every row dominant by exactly its margin, so
    the bound is 1 / margin, and it bounds ||A^{-1}||_inf."""
    from oracle.sampled import varah_bound
    w = config_c0()  # margin 0.1
    A = w.to_scipy()
    b = varah_bound(A)
    assert abs(b - 10.0) < 1e-9
    assert np.abs(np.linalg.inv(A.toarray())).sum(axis=1).max() <= b
