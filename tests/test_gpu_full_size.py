"""Full-size parity of the mixed-precision and the largest configurations.

C2 (3D 48^3 7-point convection-diffusion, n = 110,592, supernodes <= 256):
every computed entry (1.0e8 of them) against the supernodal FP64 oracle, in
all three forms.  The oracle's setup and Algorithm 1 run as tests of their
own, so that no single step runs for minutes without a result line.

C4 (3D 64^3 27-point, n = 262,144, supernodes <= 512): every computed entry
of 41 columns of A^{-1} (every 32nd column of the root supernode and its
last column, 512 columns wide, and on every level of the supernodal tree the
first column of the supernode with the largest |R_L|; 5.2e5 entries) against
the columns A^{-1} e_j solved from the definition (oracle.sampled, with
certified error bounds), and the identities (A A^{-1})_ii = (A^{-1} A)_jj = 1
over all rows.  The computed entries of a column come from the block pattern:
with r = q[j], row r of At^{-T} is computed at the columns of sup(r), at
R_U(sup(r)), and at the columns of every supernode J with r in R_L(J)
(A^{-1}(i, j) = At^{-T}(q[j], q[i]), Theorem 2).

Bars (R-9 reading of the accuracy table): max(err_norm, err_diag) <= 1e-11
(FP64) and <= 1e-5 (mixed).  The identity residuals follow from the entry bar:
|sum_j A_ij (X_ji - R_ji)| <= ||A||_inf max|X - R| <= ||A||_inf * bar * max|R|,
so they are held to bar * ||A||_inf * max|X| * (1 + bar).
"""
import sys

import numpy as np
import pytest

from oracle import Oracle
from records import record
from workloads import config_c2, config_c4

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-11, "mixed_fp32": 1e-5, "mixed_bf16x3": 1e-5}
PRECS = ["fp64", "mixed_fp32", "mixed_bf16x3"]


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def si():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1708_04539_amd import selinv
    return selinv


def errs(X, R, diag):
    err_norm = float(np.abs(X - R).max() / np.abs(R).max())
    err_diag = float((np.abs(X[diag] - R[diag]) / np.abs(R[diag])).max()) if diag.any() else 0.0
    return err_norm, err_diag


def identity_residuals(w, sel):
    cols = np.repeat(np.arange(w.n), np.diff(w.colptr))
    prod = w.values * sel
    row = np.bincount(w.rowind, weights=prod, minlength=w.n)
    col = np.bincount(cols, weights=prod, minlength=w.n)
    return float(np.abs(row - 1).max()), float(np.abs(col - 1).max())


def identity_tol(w, sel, bar):
    A = w.to_scipy()
    norm_inf = float(np.abs(A).sum(axis=1).max())
    norm_1 = float(np.abs(A).sum(axis=0).max())
    return bar * max(norm_inf, norm_1) * float(np.abs(sel).max()) * (1 + bar)


# --------------------------------------------------------------------------
# C2: whole computed set against the supernodal oracle
# --------------------------------------------------------------------------
_C2 = {}


def test_c2_oracle_analyze_and_factor():
    w = config_c2()
    say("c2 oracle analyze + factor")
    o = Oracle(w.n, w.colptr, w.rowind, w.perm, w.max_super, w.relax, 0, w.pad_pct).factor(w.values)
    _C2.update(w=w, o=o)


def test_c2_oracle_selinv():
    if "o" not in _C2:
        pytest.skip("the oracle setup did not run")
    say("c2 oracle selinv")
    _C2["o"].selinv()


def test_c2_index_sets_match(si):
    if "o" not in _C2:
        pytest.skip("the oracle did not run")
    w, o = _C2["w"], _C2["o"]
    say("c2 export + library setup")
    r, c, v = o.export()  # sorted by (column, row)
    o.close()
    del _C2["o"]
    s = si.SelInv(w.n, w.colptr, w.rowind, w.perm, w.max_super, w.relax, w.pad_pct).factor(w.values)
    s.run("fp64")
    rs, cs, _ = s.export(sort=False)
    key = cs.astype(np.int64) * w.n + rs
    order = np.argsort(key)
    assert np.array_equal(key[order], c.astype(np.int64) * w.n + r)  # the same computed set, bit for bit
    ref = np.empty_like(v)
    ref[order] = v  # the oracle's values in the library's storage order
    _C2.update(s=s, ref=ref, diag=rs == cs)


@pytest.mark.parametrize("prec", PRECS)
def test_c2_whole_superset(si, prec):
    if "ref" not in _C2:
        pytest.skip("the oracle did not run")
    w, s, ref, diag = _C2["w"], _C2["s"], _C2["ref"], _C2["diag"]
    say("c2 whole set", prec)
    s.run(prec)
    v = s.export(sort=False)[2]
    en, ed = errs(v, ref, diag)
    sel = s.get_selected()
    rr, cr = identity_residuals(w, sel)
    tol_id = identity_tol(w, sel, TOL[prec])
    record("c2 whole computed set", prec, f"entries={len(v)}", "err_norm", en, "err_diag", ed,
           "identity", max(rr, cr), "bound", tol_id)
    assert max(en, ed) <= TOL[prec], (en, ed)
    assert max(rr, cr) <= tol_id, (rr, cr, tol_id)


# --------------------------------------------------------------------------
# C4: every computed entry of 41 columns against the definition
# --------------------------------------------------------------------------
def column_entries(st, r):
    """Columns c of the computed entries At^{-T}(r, c) in row r of the block pattern."""
    xsup, rlp, rl, rup, ru = st["xsup"], st["rl_ptr"], st["rl"], st["ru_ptr"], st["ru"]
    K = int(np.searchsorted(xsup, r, side="right") - 1)
    parts = [np.arange(xsup[K], xsup[K + 1]), ru[rup[K]:rup[K + 1]]]
    for J in np.searchsorted(rlp, np.nonzero(rl == r)[0], side="right") - 1:
        parts.append(np.arange(xsup[J], xsup[J + 1]))
    return np.concatenate(parts).astype(np.int64)


@pytest.fixture(scope="module")
def c4(si):
    from oracle.sampled import solve_columns
    w = config_c4()
    say("c4 setup")
    s = si.SelInv(w.n, w.colptr, w.rowind, w.perm, w.max_super, w.relax, w.pad_pct).factor(w.values)
    st = s.structure()
    xsup, lev, cl = st["xsup"], st["level"], np.diff(st["rl_ptr"])
    ns = len(xsup) - 1
    rows = list(range(int(xsup[ns - 1]), int(xsup[ns]), 32)) + [int(xsup[ns]) - 1]
    for d in range(int(lev.max()) + 1):
        ks = np.nonzero(lev == d)[0]
        rows.append(int(xsup[ks[np.argmax(cl[ks])]]))
    rows = sorted(set(rows))
    perm = st["perm"].astype(np.int64)
    js = [int(perm[r]) for r in rows]
    say("c4 solving", len(js), "columns")
    sols = solve_columns(w.to_scipy(), js)
    cols = []
    for r, j, (x, bound) in zip(rows, js, sols):
        assert bound < 1e-13, (j, bound)
        i = perm[column_entries(st, r)]
        cols.append((j, i, x[i]))
    return w, s, cols


@pytest.mark.parametrize("prec", PRECS)
def test_c4_columns_every_computed_entry(si, c4, prec):
    w, s, cols = c4
    say("c4 columns", prec)
    s.run(prec)
    X, R, D = [], [], []
    for j, i, ref in cols:
        X.append(s.get_many(i, np.full(len(i), j)))
        R.append(ref)
        D.append(i == j)
    X, R, D = np.concatenate(X), np.concatenate(R), np.concatenate(D)
    en, ed = errs(X, R, D)
    sel = s.get_selected()
    rr, cr = identity_residuals(w, sel)
    tol_id = identity_tol(w, sel, TOL[prec])
    record("c4 41 columns", prec, f"entries={len(X)}", "err_norm", en, "err_diag", ed,
           "identity", max(rr, cr), "bound", tol_id)
    assert len(X) > 100000
    assert max(en, ed) <= TOL[prec], (en, ed)
    assert max(rr, cr) <= tol_id, (rr, cr, tol_id)


@pytest.mark.parametrize("prec", ["fp64", "mixed_bf16x3"])
def test_c4_gather_in_products_and_tuned(si, c4, prec):
    """At full size: every level's G_K read inside the products gives the
    stored-G results bit for bit on the sampled columns' entries, and the
    tuner's mix of both forms keeps them within the bar."""
    w, s, cols = c4
    say("c4 G in products", prec)
    idx_i = np.concatenate([i for _, i, _ in cols])
    idx_j = np.concatenate([np.full(len(i), j) for j, i, _ in cols])
    R = np.concatenate([ref for _, _, ref in cols])
    D = idx_i == idx_j
    out = {}
    for form in ("stored", "in_products"):
        s.set_sweep_mode("levels")
        s.set_gather_form(form)
        s.run(prec)
        assert (form == "stored") == all(s.level_stats(d)["gather_fused"] != 2 for d in range(s.info["nlevels"]))
        out[form] = s.get_many(idx_i, idx_j)
    assert np.array_equal(out["stored"], out["in_products"])
    s.set_gather_form("auto")
    s.set_sweep_mode("auto")
    s.tune(prec, reps=1)
    s.run(prec, graph=True)
    X = s.get_many(idx_i, idx_j)
    en, ed = errs(X, R, D)
    record("c4 41 columns, tuned (G stored or in the products per level)", prec, "err_norm", en, "err_diag", ed)
    assert max(en, ed) <= TOL[prec], (en, ed)
    s.set_tuning([], prec)
