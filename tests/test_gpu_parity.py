"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bar (R-9 reading of the paper's accuracy table): over the compared entries X
(library) and R (oracle),
    err_norm = max |X - R| / max |R|,   err_diag = max_i |X_ii - R_ii| / |R_ii|,
    max(err_norm, err_diag) <= 1e-11 for the FP64 form and <= 1e-5 for the
    mixed forms.
Index sets (which entries are computed) must match the oracle's bit for bit.
Full-size cases are compared on sampled columns solved from the definition
(oracle.sampled) and on identities that hold at any size.
"""
import sys

import numpy as np
import pytest

from oracle import Oracle
from records import record
from workloads import config_c0, config_c1, config_c3, random_sparse, tridiag_csc

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-11, "mixed_fp32": 1e-5, "mixed_bf16x3": 1e-5}


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


def errs(X, R, rows, cols):
    err_norm = np.abs(X - R).max() / np.abs(R).max()
    d = rows == cols
    err_diag = (np.abs(X[d] - R[d]) / np.abs(R[d])).max() if d.any() else 0.0
    return err_norm, err_diag


def compare_superset(s, o, tol):
    r1, c1, v1 = s.export()
    r2, c2, v2 = o.export()
    assert np.array_equal(r1, r2) and np.array_equal(c1, c2)
    en, ed = errs(v1, v2, r2, c2)
    assert max(en, ed) <= tol, (en, ed)
    return en, ed


def lib_and_oracle(si, n, cp, ri, v, perm, cap, relax, pad):
    s = si.SelInv(n, cp, ri, perm, cap, relax, pad)
    assert s.check_plan() == 0
    s.factor(v)
    o = Oracle(n, cp, ri, perm, cap, relax, 0, pad).factor(v).selinv()
    return s, o


# --------------------------------------------------------------------------
# small and ragged cases, whole computed superset
# --------------------------------------------------------------------------
@pytest.mark.parametrize("prec", ["fp64", "mixed_fp32", "mixed_bf16x3"])
def test_c0_whole_superset(si, prec):
    w = config_c0()
    say("c0", prec)
    s, o = lib_and_oracle(si, w.n, w.colptr, w.rowind, w.values, w.perm, w.max_super, w.relax, w.pad_pct)
    s.run(prec)
    compare_superset(s, o, TOL[prec])
    if prec == "fp64":
        inv = np.linalg.inv(w.to_scipy().toarray())
        r, c, v = s.export()
        assert np.abs(v - inv[r, c]).max() / np.abs(inv).max() < 1e-11


CASES = [  # n, density, seed, cap, relax, pad
    (1, 0.0, 0, 1, 0, 0),
    (2, 0.5, 1, 1, 0, 0),
    (37, 0.08, 2, 5, 0, 0),
    (150, 0.03, 3, 16, 4, 5),
    (400, 0.01, 4, 70, 10, 20),
    (300, 0.6, 5, 300, 0, 0),     # one dense supernode of 300 columns
    (700, 0.004, 6, 3, 0, 100),
]


@pytest.mark.parametrize("case", CASES, ids=[f"n{c[0]}_cap{c[3]}" for c in CASES])
@pytest.mark.parametrize("prec", ["fp64", "mixed_fp32"])
def test_random_ragged(si, case, prec):
    n, dens, seed, cap, relax, pad = case
    say("random", case, prec)
    cp, ri, v, _ = random_sparse(n, dens, seed, symmetric_pattern=seed % 2 == 0)
    perm = np.random.default_rng(seed).permutation(n).astype(np.int32)
    s, o = lib_and_oracle(si, n, cp, ri, v, perm, cap, relax, pad)
    s.run(prec)
    compare_superset(s, o, TOL[prec])


def test_widest_supernode_1024(si):
    """Diagonal blocks of the maximal width the inversion kernel takes."""
    n = 1100
    say("wide 1024")
    cp, ri, v, dense = random_sparse(n, 0.01, 8, symmetric_pattern=True)
    s, o = lib_and_oracle(si, n, cp, ri, v, None, 1024, n, 0)
    assert s.info["max_s"] == 1024
    s.run("fp64")
    compare_superset(s, o, TOL["fp64"])


def test_tridiagonal_closed_form(si):
    n = 500
    say("tridiag")
    cp, ri, v = tridiag_csc(-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1))
    s = si.SelInv(n, cp, ri, None, 7, 0, 0).factor(v).run("fp64")
    r, c, val = s.export()
    ref = np.minimum(r + 1, c + 1) * (n + 1 - np.maximum(r + 1, c + 1)) / (n + 1)
    assert np.abs(val - ref).max() / ref.max() < 1e-11


# --------------------------------------------------------------------------
# C1 at full size: whole superset against the oracle
# --------------------------------------------------------------------------
@pytest.fixture(scope="module")
def c1_pair(si):
    w = config_c1()
    say("c1 setup")
    s, o = lib_and_oracle(si, w.n, w.colptr, w.rowind, w.values, w.perm, w.max_super, w.relax, w.pad_pct)
    return w, s, o


@pytest.mark.parametrize("prec", ["fp64", "mixed_fp32", "mixed_bf16x3"])
def test_c1_whole_superset(si, c1_pair, prec):
    w, s, o = c1_pair
    say("c1", prec)
    s.run(prec)
    en, ed = compare_superset(s, o, TOL[prec])
    record("c1 whole computed set", prec, "err_norm", en, "err_diag", ed)


def test_c1_graph_replay_and_determinism(si, c1_pair):
    import torch
    w, s, o = c1_pair
    say("c1 graph")
    s.run("fp64")
    ref = s.get_selected()
    s.run("fp64")
    assert np.array_equal(s.get_selected(), ref)  # bitwise deterministic
    st = torch.cuda.Stream()
    for rep in range(3):
        s.run("fp64", stream=st, graph=True)
        got = s.get_selected()
        assert np.array_equal(got, ref), rep
        torch.cuda.synchronize()
        s.run("fp64")  # eager work between replays
        assert np.array_equal(s.get_selected(), ref)


def test_c1_get_and_extraction(si, c1_pair):
    import torch
    w, s, o = c1_pair
    say("c1 get")
    s.run("fp64")
    sel = s.get_selected()
    ref = o.get_selected()
    assert np.abs(sel - ref).max() / np.abs(ref).max() < 1e-11
    dev = torch.empty(w.nnz, dtype=torch.float64, device="cuda")
    s.get_selected_device(dev)
    torch.cuda.synchronize()
    assert np.array_equal(dev.cpu().numpy(), sel)
    rng = np.random.default_rng(0)
    cols = np.repeat(np.arange(w.n), np.diff(w.colptr))
    for p in rng.integers(0, w.nnz, 50):
        i, j = int(w.rowind[p]), int(cols[p])
        assert s.get(j, i) == sel[p]  # out[p] = A^{-1}(j, i)
    with pytest.raises(si.SelinvError) as e:
        s.get(0, w.n - 1)
    assert e.value.status == "NOT_SELECTED"


# --------------------------------------------------------------------------
# batches (C3): one sweep over all 32 matrices
# --------------------------------------------------------------------------
@pytest.fixture(scope="module")
def c3_all(si):
    ws = config_c3()
    say("c3 setup", len(ws), "matrices, n", min(w.n for w in ws), "..", max(w.n for w in ws))
    mats = [si.SelInv(w.n, w.colptr, w.rowind, w.perm, w.max_super, w.relax, w.pad_pct).factor(w.values)
            for w in ws]
    single = {}
    for prec in ["fp64", "mixed_fp32", "mixed_bf16x3"]:
        single[prec] = []
        for m in mats:
            m.run(prec)
            single[prec].append(m.get_selected())
    return ws, mats, single


@pytest.mark.parametrize("prec", ["fp64", "mixed_fp32", "mixed_bf16x3"])
def test_c3_batch_of_32_equals_single_runs(si, c3_all, prec):
    """Every launch of the batch covers one level of all 32 matrices; each
    matrix's results equal its single run bit for bit (every output entry is
    formed by the same products in the same order), eagerly and from the
    batch's HIP graph, with eager single runs between the replays."""
    import torch
    ws, mats, single = c3_all
    say("c3 batch", prec)
    b = si.Batch(mats)
    assert b.info["count"] == 32
    b.run(prec)
    for k, m in enumerate(mats):
        assert np.array_equal(m.get_selected(), single[prec][k]), k
    st = torch.cuda.Stream()
    for rep in range(3):
        b.run(prec, stream=st, graph=True)
        for k, m in enumerate(mats):
            assert np.array_equal(m.get_selected(), single[prec][k]), (rep, k)
        torch.cuda.synchronize()
        mats[rep].run(prec)  # eager work between replays
        assert np.array_equal(mats[rep].get_selected(), single[prec][rep])
    b.close()


def test_c3_batch_against_the_oracle(si, c3_all):
    """Four matrices of the batch (the smallest, the largest and two between)
    over their whole computed set, in all three forms, after batch runs."""
    ws, mats, _ = c3_all
    order = np.argsort([w.n for w in ws])
    pick = [int(order[0]), int(order[len(order) // 3]), int(order[2 * len(order) // 3]), int(order[-1])]
    say("c3 oracle", [ws[k].n for k in pick])
    b = si.Batch(mats)
    for k in pick:
        w = ws[k]
        o = Oracle(w.n, w.colptr, w.rowind, w.perm, w.max_super, w.relax, 0, w.pad_pct).factor(w.values).selinv()
        for prec in ["fp64", "mixed_fp32", "mixed_bf16x3"]:
            b.run(prec)
            en, ed = compare_superset(mats[k], o, TOL[prec])
            record(f"c3 matrix {k} (n={w.n}) whole set, batch", prec, "err_norm", en, "err_diag", ed)
    b.close()


def test_c3_batch_tuned_and_profiled(si, c3_all):
    """The batch's own tuning table changes launch shapes only: FP64 results
    stay equal to the single runs bit for bit; its profiled run reports the
    work of every aligned level."""
    ws, mats, single = c3_all
    say("c3 batch tune")
    b = si.Batch(mats)
    ms_pol, ms_tun = b.tune("fp64", reps=2)
    table = b.get_tuning("fp64")
    assert ms_tun <= ms_pol and len(table) == 8 + 4 * b.info["nlevels"]
    b.run("fp64", graph=True)
    for k, m in enumerate(mats):
        assert np.array_equal(m.get_selected(), single["fp64"][k]), k
    b.set_profiling(True)
    b.run("fp64")
    t = b.timings()
    assert t.shape == (3 + 4 * b.info["nlevels"],) and (t >= 0).all()
    work = sum(b.level_stats(d)["flops35"] + b.level_stats(d)["flops4"] + b.level_stats(d)["small_flops"]
               for d in range(b.info["nlevels"]))
    assert work > 0
    b.set_tuning([], "fp64")
    b.close()


def identity_residuals(w, sel):
    """max_i |(A A^{-1})_ii - 1| and max_j |(A^{-1} A)_jj - 1| from the selected entries."""
    cols = np.repeat(np.arange(w.n), np.diff(w.colptr))
    prod = w.values * sel
    row = np.bincount(w.rowind, weights=prod, minlength=w.n)
    col = np.bincount(cols, weights=prod, minlength=w.n)
    return np.abs(row - 1).max(), np.abs(col - 1).max()


def identity_tol(w, sel, bar):
    """Bound on the identity residuals implied by the entry bar:
    |sum_j A_ij (X_ji - R_ji)| <= ||A|| max|X - R| <= ||A|| bar max|R|."""
    A = w.to_scipy()
    norm = max(float(np.abs(A).sum(axis=1).max()), float(np.abs(A).sum(axis=0).max()))
    return bar * norm * float(np.abs(sel).max()) * (1 + bar)


# --------------------------------------------------------------------------
# persistent, dependency-driven sweep vs per-level launches
# --------------------------------------------------------------------------
@pytest.mark.parametrize("prec", ["fp64", "mixed_fp32", "mixed_bf16x3"])
def test_persistent_sweep_matches_level_sweep_c1(si, c1_pair, prec):
    import torch
    w, s, o = c1_pair
    say("c1 persistent", prec)
    s.set_sweep_mode("levels")
    s.run(prec)
    ref = s.get_selected()
    s.set_sweep_mode("persistent")
    s.run(prec)
    assert s.sweep_is_persistent(prec) == 1
    # FP64 and FP32: the same products in the same k order, bitwise equal.
    # Split-BF16: the fused small-supernode launches of the level sweep run
    # their products in FP32, the persistent sweep in split-BF16.
    same = (lambda x: np.array_equal(x, ref)) if prec != "mixed_bf16x3" else \
        (lambda x: np.abs(x - ref).max() <= TOL[prec] * np.abs(ref).max())
    assert same(s.get_selected())
    st = torch.cuda.Stream()
    for rep in range(3):
        s.run(prec, stream=st, graph=True)
        assert same(s.get_selected()), rep
    s.set_sweep_mode("auto")


@pytest.mark.parametrize("case", CASES, ids=[f"n{c[0]}_cap{c[3]}" for c in CASES])
def test_persistent_sweep_random(si, case):
    n, dens, seed, cap, relax, pad = case
    say("persistent random", case)
    cp, ri, v, _ = random_sparse(n, dens, seed, symmetric_pattern=seed % 2 == 0)
    perm = np.random.default_rng(seed).permutation(n).astype(np.int32)
    s, o = lib_and_oracle(si, n, cp, ri, v, perm, cap, relax, pad)
    s.set_sweep_mode("persistent").run("fp64")
    compare_superset(s, o, TOL["fp64"])


def test_persistent_sweep_batch(si):
    ws = config_c3(count=3)
    say("persistent batch", [w.n for w in ws])
    mats = [si.SelInv(w.n, w.colptr, w.rowind, w.perm, w.max_super, w.relax, w.pad_pct).factor(w.values)
            for w in ws]
    refs = []
    for m in mats:
        m.set_sweep_mode("levels").run("fp64")
        refs.append(m.get_selected())
    b = si.Batch(mats).set_sweep_mode("persistent")
    b.run("fp64")
    for m, ref in zip(mats, refs):
        assert np.array_equal(m.get_selected(), ref)
    b.close()


# --------------------------------------------------------------------------
# profiled run: per-phase events and per-level work accounting
# --------------------------------------------------------------------------
def test_c1_profiled_run_and_level_work(si, c1_pair):
    w, s, o = c1_pair
    say("c1 profiled")
    s.set_sweep_mode("levels")
    s.set_profiling(True)
    s.run("fp64")
    t = s.timings()
    s.set_profiling(False)
    L = s.info["nlevels"]
    assert t.shape == (3 + 4 * L,) and np.all(np.isfinite(t)) and np.all(t >= 0)
    # the profiled run computes the same result
    assert np.abs(s.get_selected() - o.get_selected()).max() / np.abs(o.get_selected()).max() < 1e-11
    lev = [s.level_stats(d) for d in range(L)]
    st = s.structure()
    assert sum(l["nsup"] for l in lev) == len(st["xsup"]) - 1
    # every supernode's steps 3-5 are counted once, in the fused launch or in
    # the large-supernode launches: total flops = sum_K 4 s c_L c_U + 2 s^2 c_U
    rl = np.diff(st["rl_ptr"]).astype(np.float64)
    ru = np.diff(st["ru_ptr"]).astype(np.float64)
    s_ = np.diff(st["xsup"]).astype(np.float64)
    want = float(np.sum(4 * s_ * rl * ru + 2 * s_ * s_ * ru * (ru > 0)))
    got = sum(l["flops35"] + l["flops4"] + l["small_flops"] for l in lev)
    assert abs(got - want) <= 1e-9 * want
    assert sum(l["small_count"] for l in lev) > 0
    s.set_sweep_mode("auto")


# --------------------------------------------------------------------------
# exact (unsymmetrized) analysis: C_L != C_U
# --------------------------------------------------------------------------
def lib_and_oracle_exact(si, n, cp, ri, v, perm, cap):
    """Library with the exact analysis against the oracle's exact mode: the
    same partition and block sets, so the computed supersets must agree."""
    s = si.SelInv(n, cp, ri, perm, cap, 0, 0, symbolic="exact")
    assert s.check_plan() == 0
    s.factor(v)
    o = Oracle(n, cp, ri, perm, cap, 0, 1, 0).factor(v).selinv()
    return s, o


EXACT_CASES = [  # n, density, seed, cap, triangle
    (1, 0.0, 0, 1, None),
    (2, 0.5, 1, 1, None),
    (37, 0.08, 2, 5, None),
    (300, 0.01, 3, 16, None),
    (400, 0.02, 4, 70, "lower"),   # U(K, R_U) empty everywhere
    (400, 0.02, 5, 64, "upper"),   # L(R_L, K) empty everywhere
    (300, 0.3, 6, 300, None),
    (700, 0.004, 7, 3, None),
]


@pytest.mark.parametrize("case", EXACT_CASES, ids=[f"n{c[0]}_cap{c[3]}_{c[4]}" for c in EXACT_CASES])
@pytest.mark.parametrize("prec", ["fp64", "mixed_fp32"])
def test_exact_random_ragged(si, case, prec):
    n, dens, seed, cap, tri = case
    say("exact random", case, prec)
    cp, ri, v, _ = random_sparse(n, dens, seed, lower_only=tri == "lower", upper_only=tri == "upper")
    perm = None if tri else np.random.default_rng(seed).permutation(n).astype(np.int32)
    s, o = lib_and_oracle_exact(si, n, cp, ri, v, perm, cap)
    s.run(prec)
    compare_superset(s, o, TOL[prec])


@pytest.fixture(scope="module", params=[0.0, 0.25])
def upwind_pair(si, request):
    from workloads import config_upwind
    w = config_upwind((64, 64), "box", request.param, 3, 64, 32)
    say("upwind 64x64 setup keep", request.param)
    s, o = lib_and_oracle_exact(si, w.n, w.colptr, w.rowind, w.values, w.perm, w.max_super)
    return w, s, o


@pytest.mark.parametrize("prec", ["fp64", "mixed_fp32", "mixed_bf16x3"])
def test_exact_upwind_whole_superset(si, upwind_pair, prec):
    w, s, o = upwind_pair
    say("upwind 64x64", prec)
    s.run(prec)
    en, ed = compare_superset(s, o, TOL[prec])
    say("upwind 64x64", prec, "err_norm", en, "err_diag", ed)


def test_exact_fig2b_factors_dense_inverse(si):
    """A = L U with the factor pattern of the paper's Fig. 2 (b), natural
    order: every computed entry equals the dense inverse."""
    import scipy.sparse as sp
    from fig2b import fig2b_factors
    say("fig2b")
    _, _, _, _, _, _, L, U = fig2b_factors()
    A = L @ U
    n = A.shape[0]
    m = sp.csc_matrix(A)
    m.sort_indices()
    cp, ri = m.indptr.astype(np.int64), m.indices.astype(np.int32)
    s, o = lib_and_oracle_exact(si, n, cp, ri, m.data.astype(np.float64), None, 4)
    s.run("fp64")
    compare_superset(s, o, TOL["fp64"])
    r, c, v = s.export()
    inv = np.linalg.inv(A)
    assert np.abs(v - inv[r, c]).max() / np.abs(inv).max() < 1e-11


@pytest.fixture(scope="module")
def u1_pair(si):
    """Full-size upwind grid (n = 65536): the library's exact analysis against
    the oracle's symmetrized one.  Both compute exact entries of A^{-1}, so the
    selected entries and every entry of the two supersets' intersection must
    agree."""
    from workloads import config_u1
    w = config_u1()
    say("u1 setup")
    s = si.SelInv(w.n, w.colptr, w.rowind, w.perm, w.max_super, w.relax, w.pad_pct, symbolic="exact")
    assert s.check_plan() == 0
    s.factor(w.values)
    o = Oracle(w.n, w.colptr, w.rowind, w.perm, w.max_super, w.relax, 0, w.pad_pct).factor(w.values).selinv()
    return w, s, o


@pytest.mark.parametrize("prec", ["fp64", "mixed_fp32", "mixed_bf16x3"])
def test_u1_exact_vs_symmetrized_oracle(si, u1_pair, prec):
    w, s, o = u1_pair
    say("u1", prec)
    s.run(prec)
    sel, ref = s.get_selected(), o.get_selected()
    cols = np.repeat(np.arange(w.n), np.diff(w.colptr))
    en, ed = errs(sel, ref, w.rowind, cols)
    r1, c1, v1 = s.export()
    r2, c2, v2 = o.export()
    k1 = r1.astype(np.int64) * w.n + c1
    k2 = r2.astype(np.int64) * w.n + c2
    common, i1, i2 = np.intersect1d(k1, k2, assume_unique=True, return_indices=True)
    assert common.size > 0.9 * k1.size
    en2, ed2 = errs(v1[i1], v2[i2], r1[i1], c1[i1])
    rr, cr = identity_residuals(w, sel)
    record("u1 exact (selected and common entries)", prec, "err_norm", max(en, en2), "err_diag", max(ed, ed2),
           "identity", max(rr, cr))
    assert max(en, ed, en2, ed2) <= TOL[prec]
    assert max(rr, cr) <= identity_tol(w, sel, TOL[prec])


def test_u1_exact_graph_replay_and_sweep_forms(si, u1_pair):
    import torch
    w, s, o = u1_pair
    say("u1 graph")
    s.run("fp64")
    ref = s.get_selected()
    assert s.sweep_is_persistent("fp64") == 0  # auto: level sweep for exact plans
    st = torch.cuda.Stream()
    for rep in range(3):
        s.run("fp64", stream=st, graph=True)
        assert np.array_equal(s.get_selected(), ref), rep
        torch.cuda.synchronize()
        s.run("fp64")
        assert np.array_equal(s.get_selected(), ref)
    s.set_sweep_mode("levels")
    s.run("fp64")
    lev = s.get_selected()
    # the dependency-driven sweep waits on every supernode that R_L u R_U meets
    s.set_sweep_mode("persistent")
    s.run("fp64")
    assert s.sweep_is_persistent("fp64") == 1
    assert np.array_equal(s.get_selected(), lev)
    s.set_sweep_mode("auto")
    s.run("fp64")
    assert np.array_equal(s.get_selected(), ref)


@pytest.mark.parametrize("case", EXACT_CASES, ids=[f"n{c[0]}_cap{c[3]}_{c[4]}" for c in EXACT_CASES])
def test_exact_persistent_sweep(si, case):
    n, dens, seed, cap, tri = case
    say("exact persistent", case)
    cp, ri, v, _ = random_sparse(n, dens, seed, lower_only=tri == "lower", upper_only=tri == "upper")
    perm = None if tri else np.random.default_rng(seed).permutation(n).astype(np.int32)
    s, o = lib_and_oracle_exact(si, n, cp, ri, v, perm, cap)
    s.set_sweep_mode("persistent").run("fp64")
    compare_superset(s, o, TOL["fp64"])


def test_exact_batch_matches_single_runs(si):
    from workloads import config_upwind
    ws = [config_upwind((48, 48), "box", 0.25, 10 + m, 64, 32) for m in range(3)]
    say("exact batch")
    mats = [si.SelInv(w.n, w.colptr, w.rowind, w.perm, w.max_super, w.relax, w.pad_pct,
                      symbolic="exact").factor(w.values) for w in ws]
    refs = []
    for m in mats:
        m.run("fp64")
        refs.append(m.get_selected())
    b = si.Batch(mats)
    b.run("fp64")
    for m, ref in zip(mats, refs):
        assert np.array_equal(m.get_selected(), ref)
    b.close()


# --------------------------------------------------------------------------
# autotuner: measured launch choices keep the results
# --------------------------------------------------------------------------
@pytest.mark.parametrize("prec", ["fp64", "mixed_bf16x3"])
def test_tune_c1_keeps_parity(si, c1_pair, prec):
    w, s, o = c1_pair
    say("c1 tune", prec)
    ms_pol, ms_tun = s.tune(prec, reps=3)
    table = s.get_tuning(prec)
    say("c1 tune", prec, "policy ms", ms_pol, "tuned ms", ms_tun, "table", table)
    assert ms_tun <= ms_pol and len(table) == 8 + 4 * s.info["nlevels"]
    s.run(prec)
    compare_superset(s, o, TOL[prec])
    s.run(prec, graph=True)
    compare_superset(s, o, TOL[prec])
    s.set_tuning([], prec)


@pytest.mark.parametrize("prec", ["fp64", "mixed_fp32", "mixed_bf16x3"])
def test_forced_tables_keep_parity(si, prec):
    """Every tile edge on every launch class, the per-phase launches on the
    levels of small supernodes, and G_K read by the products give the same
    results."""
    w = config_c0()
    say("c0 forced tables", prec)
    s, o = lib_and_oracle(si, w.n, w.colptr, w.rowind, w.values, w.perm, w.max_super, w.relax, w.pad_pct)
    L = s.info["nlevels"]
    for edge in (32, 64, 128):
        for per_phase in (0, 1):
            s.set_tuning([2, L, 1, edge, edge, edge, per_phase] + [edge, edge, per_phase] * L, prec)
            s.run(prec)
            compare_superset(s, o, TOL[prec])
            # G_K read by the products on every level that allows it
            s.set_tuning([4, L, 1, edge, edge, edge, per_phase, 0] + [edge, edge, per_phase, 1] * L, prec)
            s.run(prec)
            compare_superset(s, o, TOL[prec])


def test_side_inversion_chunks_bitwise_c1(si, c1_pair):
    """The side stream's tile inversions cut into chunks (ragged last chunk
    included) give bitwise the same results as one launch, eager and from the
    HIP graph: every item writes only its own outputs."""
    w, s, o = c1_pair
    L = s.info["nlevels"]
    say("c1 side chunks")
    s.set_tuning([3, L, 1, 0, 0, 0, 0, 0] + [0, 0, 0] * L, "fp64")
    s.run("fp64")
    ref = s.export()[2]
    for chunk in (37, 300, 1 << 20):
        s.set_tuning([3, L, 1, 0, 0, 0, 0, chunk] + [0, 0, 0] * L, "fp64")
        s.run("fp64")
        assert np.array_equal(s.export()[2], ref)
        s.run("fp64", graph=True)
        assert np.array_equal(s.export()[2], ref)
    s.set_tuning([], "fp64")


@pytest.mark.parametrize("prec", ["fp64", "mixed_bf16x3"])
def test_prologue_part_per_level_bitwise(si, c1_pair, split_pair, prec):
    """One side-stream prologue part per upper level, each joined before its
    level, gives bitwise the results of the prologue before the sweep,
    eager and from the HIP graph (each part writes only its own supernodes'
    blocks)."""
    for w, s, o in (c1_pair, split_pair):
        L = s.info["nlevels"]
        say("prologue parts", w.name, prec)
        s.set_tuning([4, L, 1, 0, 0, 0, 1, 0] + [0, 0, 0, 0] * L, prec)
        s.run(prec)
        ref = s.export()[2]
        s.set_tuning([4, L, 1, 0, 0, 0, 2, 0] + [0, 0, 0, 0] * L, prec)
        s.run(prec)
        assert np.array_equal(s.export()[2], ref)
        for _ in range(3):
            s.run(prec, graph=True)
            assert np.array_equal(s.export()[2], ref)
        s.set_tuning([4, L, 1, 0, 0, 0, 2, 37] + [0, 0, 0, 1] * L, prec)  # chunks, G in products
        s.run(prec, graph=True)
        assert np.array_equal(s.export()[2], ref)
        s.set_tuning([], prec)


def test_tune_exact_upwind_and_cache(si, tmp_path):
    from paper_1708_04539_amd.autotune import tuned
    from workloads import config_upwind
    w = config_upwind((64, 64), "box", 0.25, 3, 64, 32)
    say("tune exact upwind + cache")
    s, o = lib_and_oracle_exact(si, w.n, w.colptr, w.rowind, w.values, w.perm, w.max_super)
    path = str(tmp_path / "tuning.json")
    r1 = tuned(s, "fp64", path, reps=2)
    assert not r1["cached"] and r1["table"] and r1["table"][2] != 2  # never the persistent form here
    s.run("fp64")
    compare_superset(s, o, TOL["fp64"])
    s2 = si.SelInv(w.n, w.colptr, w.rowind, w.perm, w.max_super, 0, 0, symbolic="exact").factor(w.values)
    r2 = tuned(s2, "fp64", path)
    assert r2["cached"] and r2["table"] == r1["table"] and s2.get_tuning("fp64") == r1["table"]
    s2.run("fp64")
    compare_superset(s2, o, TOL["fp64"])


# --------------------------------------------------------------------------
# complex matrices (real form), against the complex oracle (the definition)
# --------------------------------------------------------------------------
def random_complex(n, dens, seed):
    """Random complex matrix on random_sparse's pattern: off-diagonals
    v (1 + 0.3 i u), diagonal 1.35 Re + 0.2 i |.|, u ~ U[-1, 1]."""
    cp, ri, v, _ = random_sparse(n, dens, seed)
    rng = np.random.default_rng(seed + 1000)
    cols = np.repeat(np.arange(n), np.diff(cp))
    z = v * (1 + 0.3j * rng.uniform(-1, 1, v.size))
    d = ri == cols
    z[d] = 1.35 * v[d] + 0.2j * np.abs(v[d])
    return cp, ri, z


def complex_errs(X, R, rows, cols):
    err_norm = np.abs(X - R).max() / np.abs(R).max()
    dg = rows == cols
    err_diag = (np.abs(X[dg] - R[dg]) / np.abs(R[dg])).max() if dg.any() else 0.0
    return err_norm, err_diag


COMPLEX_CASES = [  # n, density, seed, cap (real-form columns), symbolic
    (1, 0.0, 0, 2, "symmetrized"),
    (2, 0.5, 1, 2, "symmetrized"),
    (37, 0.08, 2, 6, "symmetrized"),
    (150, 0.03, 3, 32, "exact"),
    (300, 0.01, 4, 64, "symmetrized"),
    (300, 0.02, 5, 16, "exact"),
]


@pytest.mark.parametrize("case", COMPLEX_CASES, ids=[f"n{c[0]}_{c[4]}" for c in COMPLEX_CASES])
@pytest.mark.parametrize("prec", ["fp64", "mixed_fp32"])
def test_complex_random_selected(si, case, prec):
    from oracle.complex_ref import selected_dense
    n, dens, seed, cap, sym = case
    say("complex random", case, prec)
    cp, ri, z = random_complex(n, dens, seed)
    perm = np.random.default_rng(seed).permutation(n).astype(np.int32)
    s = si.SelInv(n, cp, ri, perm, cap, 0, 0, symbolic=sym, complex_values=True)
    assert s.check_plan() == 0
    s.factor(z).run(prec)
    got, ref = s.get_selected(), selected_dense(n, cp, ri, z)
    cols = np.repeat(np.arange(n), np.diff(cp))
    en, ed = complex_errs(got, ref, ri, cols)
    assert max(en, ed) <= TOL[prec], (en, ed)
    for p in np.random.default_rng(seed).integers(0, len(ri), 5):
        assert s.get(int(cols[p]), int(ri[p])) == got[p]  # out[p] = A^{-1}(j, i)


@pytest.fixture(scope="module")
def z48(si):
    from oracle.complex_ref import selected_dense
    from workloads import config_complex
    w = config_complex((48, 48), "box", 2, 32, 32)
    say("complex 48x48 setup")
    s = si.SelInv(w.n, w.colptr, w.rowind, w.perm, w.max_super, w.relax, w.pad_pct, complex_values=True)
    s.factor(w.values)
    return w, s, selected_dense(w.n, w.colptr, w.rowind, w.values)


@pytest.mark.parametrize("prec", ["fp64", "mixed_fp32", "mixed_bf16x3"])
def test_complex_stencil_selected(si, z48, prec):
    import torch
    w, s, ref = z48
    say("complex 48x48", prec)
    s.run(prec)
    got = s.get_selected()
    cols = np.repeat(np.arange(w.n), np.diff(w.colptr))
    en, ed = complex_errs(got, ref, w.rowind, cols)
    say("complex 48x48", prec, "err_norm", en, "err_diag", ed)
    assert max(en, ed) <= TOL[prec]
    dev = torch.empty(w.nnz, dtype=torch.complex128, device="cuda")
    s.get_selected_device(dev)
    torch.cuda.synchronize()
    assert np.array_equal(dev.cpu().numpy(), got)


@pytest.mark.parametrize("prec", ["fp64", "mixed_fp32"])
def test_complex_z1_full_size(si, prec):
    """n = 65536 complex (131072 real-form columns): sampled exact columns and
    the identities sum_j A(i,j) A^{-1}(j,i) = 1 = sum_i A(i,j) A^{-1}(j,i)."""
    from oracle.complex_ref import solve_columns
    from workloads import config_z1
    w = getattr(test_complex_z1_full_size, "_w", None) or config_z1()
    test_complex_z1_full_size._w = w
    say("z1", prec)
    s = getattr(test_complex_z1_full_size, "_s", None)
    if s is None:
        s = si.SelInv(w.n, w.colptr, w.rowind, w.perm, w.max_super, w.relax, w.pad_pct,
                      complex_values=True).factor(w.values)
        test_complex_z1_full_size._s = s
    s.run(prec)
    sel = s.get_selected()
    cols = np.repeat(np.arange(w.n), np.diff(w.colptr))
    prod = w.values * sel
    rr = np.abs(np.bincount(w.rowind, prod.real, w.n) + 1j * np.bincount(w.rowind, prod.imag, w.n) - 1).max()
    cr = np.abs(np.bincount(cols, prod.real, w.n) + 1j * np.bincount(cols, prod.imag, w.n) - 1).max()
    js = [int(j) for j in np.random.default_rng(7).integers(0, w.n, 2)] + [int(w.perm[-1])]
    xs = solve_columns(w.n, w.colptr, w.rowind, w.values, js)
    A = w.to_scipy().tocsr()
    en = ed = 0.0
    for j, x in zip(js, xs):
        rows = A.indices[A.indptr[j]:A.indptr[j + 1]]  # A(j, i) != 0 -> A^{-1}(i, j) selected
        got = np.array([s.get(int(i), j) for i in rows])
        en = max(en, np.abs(got - x[rows]).max() / np.abs(x[rows]).max())
        ed = max(ed, abs(s.get(j, j) - x[j]) / abs(x[j]))
    record("z1 complex sampled columns", prec, "err_norm", en, "err_diag", ed, "identity", max(rr, cr))
    assert max(rr, cr) <= identity_tol(w, sel, TOL[prec])
    assert max(en, ed) <= TOL[prec]


# --------------------------------------------------------------------------
# split-K of the step-4 products, over the whole computed set
# --------------------------------------------------------------------------
@pytest.fixture(scope="module")
def split_pair(si):
    """3D 32^3 27-point stencil, supernodes <= 256: levels 4-6 have one or two
    supernodes with c_U >= 1024, so their step-4 products are split in k."""
    from workloads import config_grid
    w = config_grid("split", (32, 32, 32), "box", "sym_perturbed", 0.1, 5, 256, 64, delta=0.15)
    say("split-K setup")
    s, o = lib_and_oracle(si, w.n, w.colptr, w.rowind, w.values, w.perm, w.max_super, w.relax, w.pad_pct)
    st = s.structure()
    wd, cl, cu, lev = (np.diff(st["xsup"]), np.diff(st["rl_ptr"]), np.diff(st["ru_ptr"]), st["level"])
    split = []
    for d in range(lev.max() + 1):
        m = (lev == d) & (cu > 0) & ~((wd <= 64) & (cl <= 64) & (cu <= 64))
        t64 = (np.ceil(wd[m] / 64) ** 2).sum()
        if 0 < t64 < 512 and (cu[m] // 512 >= 2).any():
            split.append(d)
    assert split  # the case exercises the split products and their reduction
    return w, s, o


@pytest.mark.parametrize("prec", ["fp64", "mixed_fp32", "mixed_bf16x3"])
def test_split_k_whole_superset(si, split_pair, prec):
    w, s, o = split_pair
    say("split-K", prec)
    s.run(prec)
    en, ed = compare_superset(s, o, TOL[prec])
    record("split-K 32^3 whole computed set", prec, "err_norm", en, "err_diag", ed)
    s.run(prec, graph=True)
    compare_superset(s, o, TOL[prec])


# --------------------------------------------------------------------------
# gather through the relative-index maps (source codes off), both sweep forms
# --------------------------------------------------------------------------
@pytest.fixture(scope="module")
def c1_maps(si, c1_pair):
    w, _, o = c1_pair
    say("c1 maps setup")
    s = si.SelInv(w.n, w.colptr, w.rowind, w.perm, w.max_super, w.relax, w.pad_pct)
    s.set_gather_code_budget(0)
    assert s.check_plan() == 0
    s.factor(w.values)
    return w, s, o


@pytest.mark.parametrize("sweep", ["levels", "persistent"])
@pytest.mark.parametrize("prec", ["fp64", "mixed_fp32", "mixed_bf16x3"])
def test_map_gather_c1_whole_superset(si, c1_maps, prec, sweep):
    """Every gather reads its sources through the maps of Theorem 1 (the
    branch the wide supernodes of C2 and C4 take), at C1 over the whole set."""
    w, s, o = c1_maps
    say("c1 maps", prec, sweep)
    s.set_sweep_mode(sweep)
    s.run(prec)
    assert s.sweep_is_persistent(prec) == (sweep == "persistent")
    en, ed = compare_superset(s, o, TOL[prec])
    record("c1 map gather", sweep, prec, "err_norm", en, "err_diag", ed)


@pytest.mark.parametrize("sweep", ["levels", "persistent"])
@pytest.mark.parametrize("prec", ["fp64", "mixed_fp32", "mixed_bf16x3"])
def test_map_gather_split_k_whole_superset(si, split_pair, prec, sweep):
    w, _, o = split_pair
    say("split-K maps", prec, sweep)
    s = getattr(test_map_gather_split_k_whole_superset, "_s", None)
    if s is None:
        s = si.SelInv(w.n, w.colptr, w.rowind, w.perm, w.max_super, w.relax, w.pad_pct)
        s.set_gather_code_budget(0)
        s.factor(w.values)
        test_map_gather_split_k_whole_superset._s = s
    s.set_sweep_mode(sweep)
    s.run(prec)
    en, ed = compare_superset(s, o, TOL[prec])
    record("split-K 32^3 map gather", sweep, prec, "err_norm", en, "err_diag", ed)


# --------------------------------------------------------------------------
# device memory from the allocator hook; many entries at once
# --------------------------------------------------------------------------
# --------------------------------------------------------------------------
# G_K read from its sources inside the step-3/5 products (no stored G)
# --------------------------------------------------------------------------
def in_product_levels(s):
    """Levels of the last run whose steps 3/5 read G_K from its sources."""
    return [d for d in range(s.info["nlevels"]) if s.level_stats(d)["gather_fused"] == 2]


def stored_and_in_products(s, prec, graph=False):
    """Results with a stored G and with G_K read by the products (level sweep)."""
    s.set_sweep_mode("levels")
    s.set_gather_form("stored")
    s.run(prec, graph=graph)
    assert in_product_levels(s) == [] or graph
    ref = s.export()
    s.set_gather_form("in_products")
    s.run(prec, graph=graph)
    got = s.export()
    s.set_gather_form("auto")
    s.set_sweep_mode("auto")
    return ref, got


@pytest.mark.parametrize("prec", ["fp64", "mixed_fp32", "mixed_bf16x3"])
def test_gather_in_products_c1(si, c1_pair, prec):
    """The products take every entry of G_K from the block that holds it: the
    values staged are those the gather stores, so the results equal the
    stored-G results bit for bit, and the oracle's to the bar."""
    w, s, o = c1_pair
    say("c1 G in products", prec)
    ref, got = stored_and_in_products(s, prec)
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)
    s.set_sweep_mode("levels")
    s.set_gather_form("in_products")
    s.run(prec)
    lv = in_product_levels(s)
    assert lv and all(s.level_stats(d)["gather_tiles"] == 0 for d in lv)
    en, ed = compare_superset(s, o, TOL[prec])
    record("c1 G in products", prec, "err_norm", en, "err_diag", ed)
    s.set_gather_form("auto")
    s.set_sweep_mode("auto")


@pytest.mark.parametrize("prec", ["fp64", "mixed_fp32", "mixed_bf16x3"])
def test_gather_in_products_split_k(si, split_pair, prec):
    """Wide levels with split step-4 products (whose reductions then push
    nothing): bitwise equal to the stored G, and the oracle's to the bar."""
    w, s, o = split_pair
    say("split-K G in products", prec)
    ref, got = stored_and_in_products(s, prec)
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)
    s.set_sweep_mode("levels")
    s.set_gather_form("in_products")
    s.run(prec)
    assert len(in_product_levels(s)) >= 3
    en, ed = compare_superset(s, o, TOL[prec])
    record("split-K 32^3 G in products", prec, "err_norm", en, "err_diag", ed)
    s.set_gather_form("auto")
    s.set_sweep_mode("auto")


def test_gather_in_products_graph_replay(si, c1_pair):
    import torch
    w, s, o = c1_pair
    say("c1 G in products, graph")
    ref, _ = stored_and_in_products(s, "fp64")
    s.set_sweep_mode("levels")
    s.set_gather_form("in_products")
    st = torch.cuda.Stream()
    for rep in range(3):
        s.run("fp64", stream=st, graph=True)
        assert np.array_equal(s.export()[2], ref[2]), rep
        torch.cuda.synchronize()
        s.run("fp64")
        assert np.array_equal(s.export()[2], ref[2]), rep
    s.set_gather_form("auto")
    s.set_sweep_mode("auto")


@pytest.mark.parametrize("prec", ["fp64", "mixed_bf16x3"])
def test_gather_in_products_batch(si, c3_all, prec):
    """A batch of the 8 largest C3 matrices (one code array per matrix)."""
    ws, mats, single = c3_all
    order = np.argsort([w.n for w in ws])[-8:]
    say("c3 G in products", prec, [ws[k].n for k in order])
    b = si.Batch([mats[k] for k in order]).set_sweep_mode("levels").set_gather_form("in_products")
    b.run(prec)
    assert any(b.level_stats(d)["gather_fused"] == 2 for d in range(b.info["nlevels"]))
    for k in order:
        assert np.array_equal(mats[k].get_selected(), single[prec][k]), k
    b.run(prec, graph=True)
    for k in order:
        assert np.array_equal(mats[k].get_selected(), single[prec][k]), k
    b.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed_fp32"])
def test_gather_in_products_complex(si, z48, prec):
    """Complex blocks (products forming the even columns only)."""
    w, s, ref = z48
    say("complex 48x48 G in products", prec)
    a, b = stored_and_in_products(s, prec)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_gather_in_products_exact_sets(si, upwind_pair):
    """Exact (unsymmetrized) block sets: G_K meets several ancestors."""
    w, s, o = upwind_pair
    say("upwind G in products")
    for prec in ("fp64", "mixed_bf16x3"):
        a, b = stored_and_in_products(s, prec)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


def test_allocator_hook_nomem_and_torch_memory(si):
    import torch
    w = config_c0()
    say("allocator hook")
    si.set_allocator("custom", alloc=lambda nbytes: None, free=lambda ptr: None)
    try:
        s = si.SelInv(w.n, w.colptr, w.rowind, w.perm, w.max_super, w.relax, w.pad_pct)
        with pytest.raises(si.SelinvError) as e:
            s.factor(w.values)
        assert e.value.status == "NOMEM"
        s.close()
    finally:
        si.set_allocator("torch")
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    s, o = lib_and_oracle(si, w.n, w.colptr, w.rowind, w.values, w.perm, w.max_super, w.relax, w.pad_pct)
    factored = torch.cuda.memory_allocated()
    assert factored - before >= 8 * s.info["nnz_lu"]  # the factors live in torch's pool
    s.run("mixed_fp32")
    assert torch.cuda.memory_allocated() > factored
    compare_superset(s, o, TOL["mixed_fp32"])
    s.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before  # every allocation went back
    # handles made under hipMalloc keep working beside torch's pool
    si.set_allocator("hip")
    try:
        s2, _ = lib_and_oracle(si, w.n, w.colptr, w.rowind, w.values, w.perm, w.max_super, w.relax, w.pad_pct)
        assert torch.cuda.memory_allocated() == before
        s2.run("fp64")
        compare_superset(s2, o, TOL["fp64"])
        s2.close()
    finally:
        si.set_allocator("torch")


def test_get_many_matches_get(si, c1_pair):
    w, s, o = c1_pair
    say("c1 get_many")
    s.run("mixed_fp32")
    rng = np.random.default_rng(3)
    cols = np.repeat(np.arange(w.n), np.diff(w.colptr))
    p = rng.integers(0, w.nnz, 2000)
    i, j = cols[p], w.rowind[p].astype(np.int64)  # A(j, i) != 0: A^{-1}(i, j) is selected
    got = s.get_many(i, j)
    assert np.array_equal(got, s.get_selected()[p])
    assert all(got[k] == s.get(int(i[k]), int(j[k])) for k in range(0, 2000, 97))
