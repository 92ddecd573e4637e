"""CPU checks of the C ABI library: it loads, exports every declared entry
point, and its host analysis reproduces the oracle's partition and block sets
exactly.  No compute call here needs a GPU."""
import ctypes as C
import os
import re

import numpy as np
import scipy.sparse as sp
import pytest

from oracle import Oracle
from workloads import config_c0, config_c1, config_c3, random_sparse

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def si():
    from paper_1708_04539_amd import selinv
    return selinv


def declared_functions():
    text = open(os.path.join(ROOT, "include", "selinv.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(selinv_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol(si):
    names = declared_functions()
    assert len(names) >= 18
    lib = C.CDLL(si.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(si.EXPORTED)


def _same_structure(w_or_args, si):
    n, cp, ri, perm, cap, relax, pad = w_or_args
    s = si.SelInv(n, cp, ri, perm, cap, relax, pad)
    o = Oracle(n, cp, ri, perm, cap, relax, 0, pad)
    a, b = s.structure(), o.structure()
    for k in ["perm", "xsup", "rl_ptr", "rl", "ru_ptr", "ru"]:
        assert np.array_equal(a[k], b[k]), k
    return s


@pytest.mark.parametrize("name", ["c0", "c1"])
def test_partition_matches_oracle_configs(si, name):
    w = config_c0() if name == "c0" else config_c1()
    s = _same_structure((w.n, w.colptr, w.rowind, w.perm, w.max_super, w.relax, w.pad_pct), si)
    info = s.info
    assert info["nsuper"] == (63 if name == "c0" else 2048)
    assert info["nlevels"] == (6 if name == "c0" else 12)


def test_partition_matches_oracle_c3_member(si):
    w = config_c3(count=3)[2]
    _same_structure((w.n, w.colptr, w.rowind, w.perm, w.max_super, w.relax, w.pad_pct), si)


@pytest.mark.parametrize("seed,cap,relax,pad", [(0, 1, 0, 0), (1, 4, 3, 0), (2, 8, 8, 5), (3, 64, 20, 30),
                                                (4, 3, 0, 100)])
def test_partition_matches_oracle_random(si, seed, cap, relax, pad):
    n = 300
    cp, ri, _, _ = random_sparse(n, 0.012, seed)
    perm = np.random.default_rng(seed).permutation(n).astype(np.int32)
    _same_structure((n, cp, ri, perm, cap, relax, pad), si)


def test_levels_respect_dependencies(si):
    w = config_c1()
    s = si.SelInv(w.n, w.colptr, w.rowind, w.perm, w.max_super, w.relax, w.pad_pct)
    st = s.structure()
    xs, lev = st["xsup"], st["level"]
    sup = np.searchsorted(xs, np.arange(w.n), side="right") - 1
    for K in range(len(xs) - 1):
        R = st["rl"][st["rl_ptr"][K]:st["rl_ptr"][K + 1]]
        # every block row of K belongs to a strictly shallower level
        assert np.all(lev[sup[R]] < lev[K])


def test_flop_count_convention(si):
    """F_K = 4 s cL cU + 2 s^2 cU + s^2 (cL + cU) + 4/3 s^3, summed over K."""
    w = config_c0()
    s = si.SelInv(w.n, w.colptr, w.rowind, w.perm, w.max_super, w.relax, w.pad_pct)
    st = s.structure()
    s_ = np.diff(st["xsup"]).astype(float)
    cl = np.diff(st["rl_ptr"]).astype(float)
    cu = np.diff(st["ru_ptr"]).astype(float)
    F = (4 * s_ * cl * cu + 2 * s_ ** 2 * cu + s_ ** 2 * (cl + cu) + 4.0 / 3.0 * s_ ** 3).sum()
    assert abs(s.info["flops"] - F) <= 1e-9 * F
    assert s.info["nnz_lu"] == int((s_ * s_ + s_ * cl + s_ * cu).sum())


def test_error_paths(si):
    cp = np.array([0, 2, 4], np.int64)
    with pytest.raises(si.SelinvError) as e:
        si.SelInv(2, cp, np.array([1, 0, 0, 1], np.int32))
    assert e.value.status == "BAD_PATTERN"
    with pytest.raises(si.SelinvError) as e:
        si.SelInv(2, np.array([0, 1, 2], np.int64), np.array([1, 0], np.int32))
    assert e.value.status == "BAD_PATTERN"
    with pytest.raises(si.SelinvError) as e:
        si.SelInv(2, cp, np.array([0, 1, 0, 1], np.int32), np.array([1, 1], np.int32))
    assert e.value.status == "BAD_PERM"
    s = si.SelInv(2, cp, np.array([0, 1, 0, 1], np.int32))
    with pytest.raises(si.SelinvError) as e:
        s.run("fp64")
    assert e.value.status == "STATE"
    with pytest.raises(si.SelinvError) as e:
        s.get(0, 0)
    assert e.value.status == "STATE"
    with pytest.raises(si.SelinvError) as e:
        s.run(7)
    assert e.value.status == "INVALID_ARG"


@pytest.mark.parametrize("name", ["c0", "c1", "c3", "random", "tridiag"])
def test_plan_and_push_maps_consistent(si, name):
    """Gather maps, extraction locations and the maps that let a parent's
    step-4 product write its diagonal block into its children's G all agree
    with R_L / R_U (host-side check, no device needed)."""
    from workloads import tridiag_csc
    if name == "c0":
        w = config_c0()
        args = (w.n, w.colptr, w.rowind, w.perm, w.max_super, w.relax, w.pad_pct)
    elif name == "c1":
        w = config_c1()
        args = (w.n, w.colptr, w.rowind, w.perm, w.max_super, w.relax, w.pad_pct)
    elif name == "c3":
        w = config_c3(count=2)[1]
        args = (w.n, w.colptr, w.rowind, w.perm, w.max_super, w.relax, w.pad_pct)
    elif name == "random":
        cp, ri, v, _ = random_sparse(300, 0.02, 5, symmetric_pattern=False)
        args = (300, cp, ri, np.random.default_rng(5).permutation(300).astype(np.int32), 7, 3, 5)
    else:
        n = 200
        cp, ri, v = tridiag_csc(-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1))
        args = (n, cp, ri, None, 16, 0, 0)
    s = si.SelInv(*args)
    assert s.check_plan() == 0
    s.close()


# --------------------------------------------------------------------------
# exact (unsymmetrized) analysis: C_L != C_U
# --------------------------------------------------------------------------
STRUCT_KEYS = ["perm", "xsup", "rl_ptr", "rl", "ru_ptr", "ru"]


def _exact_same_as_oracle(si, n, cp, ri, perm, cap):
    """Partition and block sets of the library's exact analysis equal the
    oracle's exact mode (dense boolean elimination), bit for bit."""
    s = si.SelInv(n, cp, ri, perm, cap, 0, 0, symbolic="exact")
    o = Oracle(n, cp, ri, perm, cap, 0, 1, 0)
    a, b = s.structure(), o.structure()
    for k in STRUCT_KEYS:
        assert np.array_equal(a[k], b[k]), k
    assert s.info["symbolic"] == 1
    assert s.check_plan() == 0
    return s, a


def _unequal_sets(st):
    ns = len(st["xsup"]) - 1
    return sum(not np.array_equal(st["rl"][st["rl_ptr"][K]:st["rl_ptr"][K + 1]],
                                  st["ru"][st["ru_ptr"][K]:st["ru_ptr"][K + 1]]) for K in range(ns))


@pytest.mark.parametrize("seed,n,dens,cap", [(0, 300, 0.01, 8), (1, 300, 0.02, 4), (2, 300, 0.005, 64),
                                             (3, 250, 0.03, 1), (4, 300, 0.01, 1024), (5, 1, 0.0, 3),
                                             (6, 2, 0.5, 1), (7, 600, 0.004, 5)])
def test_exact_analysis_matches_oracle_random(si, seed, n, dens, cap):
    cp, ri, _, _ = random_sparse(n, dens, seed)
    perm = np.random.default_rng(seed).permutation(n).astype(np.int32)
    s, st = _exact_same_as_oracle(si, n, cp, ri, perm, cap)
    if n >= 100:
        assert _unequal_sets(st) > 0  # R_L(K) != R_U(K) really occurs
        sym = si.SelInv(n, cp, ri, perm, cap, 0, 0)
        assert s.info["nnz_lu"] < sym.info["nnz_lu"]


@pytest.mark.parametrize("lower", [True, False])
def test_exact_analysis_triangular(si, lower):
    """The paper's extreme case: a triangular A has L = I (or U diagonal), so
    one of the two block-set families is empty, while symmetrizing the
    pattern fills both."""
    n = 400
    cp, ri, _, _ = random_sparse(n, 0.02, 11, lower_only=lower, upper_only=not lower)
    s, st = _exact_same_as_oracle(si, n, cp, ri, None, 16)
    assert s.info["nnz_u" if lower else "nnz_l"] == 0
    assert s.info["nnz_l" if lower else "nnz_u"] > 0
    sym = si.SelInv(n, cp, ri, None, 16, 0, 0)
    assert sym.info["nnz_lu"] > 5 * s.info["nnz_lu"]


@pytest.mark.parametrize("keep", [0.0, 0.25, 1.0])
def test_exact_analysis_upwind_grid(si, keep):
    from workloads import config_upwind
    w = config_upwind((40, 40), "box", keep, 3, 32, 16)
    s, st = _exact_same_as_oracle(si, w.n, w.colptr, w.rowind, w.perm, w.max_super)
    if keep < 1.0:
        assert _unequal_sets(st) > 0
    else:  # every coupling kept: a structurally symmetric pattern
        assert _unequal_sets(st) == 0


def test_exact_analysis_symmetric_pattern_equal_sets(si):
    """On a structurally symmetric pattern the exact L and U^T share their
    structure, so R_L(K) = R_U(K) for every supernode."""
    w = config_c0()
    s, st = _exact_same_as_oracle(si, w.n, w.colptr, w.rowind, w.perm, w.max_super)
    assert _unequal_sets(st) == 0


def test_exact_analysis_covers_fig2b_factors(si):
    """A = L U for factors with the block pattern of the paper's Fig. 2 (b):
    the exact analysis of A (natural order) must hold every nonzero of L and
    U in its block pattern (unpivoted LU of A reproduces exactly these
    factors), and matches the oracle's exact mode."""
    from fig2b import fig2b_factors
    _, _, _, _, _, _, L, U = fig2b_factors()
    A = L @ U
    n = A.shape[0]
    m = sp.csc_matrix(np.where(np.abs(A) > 0, A, 0.0))
    m.sort_indices()
    cp, ri = m.indptr.astype(np.int64), m.indices.astype(np.int32)
    s, st = _exact_same_as_oracle(si, n, cp, ri, None, 8)
    xs = st["xsup"]
    sup = np.searchsorted(xs, np.arange(n), side="right") - 1
    for r, c in zip(*np.nonzero(L + U)):
        I, J = sup[r], sup[c]
        if I == J:
            continue
        if I > J:
            assert r in st["rl"][st["rl_ptr"][J]:st["rl_ptr"][J + 1]]
        else:
            assert c in st["ru"][st["ru_ptr"][I]:st["ru_ptr"][I + 1]]


def test_exact_analysis_levels_and_fusion_flags(si):
    """Every supernode met by R_L(K) u R_U(K) lies on a shallower level
    (host check of the plan, including the parent / push maps)."""
    from workloads import config_upwind
    w = config_upwind((96, 96), "box", 0.25, 1, 64, 32)
    s = si.SelInv(w.n, w.colptr, w.rowind, w.perm, w.max_super, w.relax, w.pad_pct, symbolic="exact")
    assert s.check_plan() == 0
    st = s.structure()
    xs, lev = st["xsup"], st["level"]
    sup = np.searchsorted(xs, np.arange(w.n), side="right") - 1
    for K in range(len(xs) - 1):
        R = np.concatenate([st["rl"][st["rl_ptr"][K]:st["rl_ptr"][K + 1]],
                            st["ru"][st["ru_ptr"][K]:st["ru_ptr"][K + 1]]])
        if R.size:
            assert lev[K] == lev[sup[R]].max() + 1
        else:
            assert lev[K] == 0


def test_exact_option_errors(si):
    cp = np.array([0, 2, 4], np.int64)
    with pytest.raises(si.SelinvError) as e:
        si.SelInv(2, cp, np.array([0, 1, 0, 1], np.int32), symbolic=2)
    assert e.value.status == "INVALID_ARG"


def test_exact_relaxed_partition(si):
    """Relaxation of the exact form (leaf subtrees, padded chains): any
    column-range partition is closed by the block fill, so the plan stays
    consistent; the relaxed form has far fewer supernodes and levels than the
    fundamental one and still stores less than the symmetrized form."""
    from workloads import config_upwind
    w = config_upwind((96, 96), "box", 0.25, 2, 64, 32)
    fund = si.SelInv(w.n, w.colptr, w.rowind, w.perm, w.max_super, 0, 0, symbolic="exact")
    rel = si.SelInv(w.n, w.colptr, w.rowind, w.perm, w.max_super, w.relax, w.pad_pct, symbolic="exact")
    sym = si.SelInv(w.n, w.colptr, w.rowind, w.perm, w.max_super, w.relax, 5)
    assert rel.check_plan() == 0
    assert rel.info["nsuper"] < fund.info["nsuper"] // 4
    assert rel.info["nlevels"] < fund.info["nlevels"] // 2
    assert fund.info["nnz_lu"] <= rel.info["nnz_lu"] < sym.info["nnz_lu"]
    st = rel.structure()
    assert np.array_equal(st["perm"], w.perm)  # the exact form keeps the ordering
    assert _unequal_sets(st) > 0


# --------------------------------------------------------------------------
# tuning tables (host side; selinv_tune itself needs the device)
# --------------------------------------------------------------------------
def test_tuning_table_set_get_and_validation(si):
    w = config_c0()
    s = si.SelInv(w.n, w.colptr, w.rowind, w.perm, w.max_super, w.relax, w.pad_pct)
    L = s.info["nlevels"]
    assert s.get_tuning("fp64") == []
    table = [4, L, 1, 64, 32, 0, 0, 448]
    for d in range(L):
        table += [32 if d % 2 else 64, 128, d % 2, (d // 2) % 2]
    s.set_tuning(table, "mixed_fp32")
    assert s.get_tuning("mixed_fp32") == table
    assert s.get_tuning("fp64") == []
    # the earlier layouts are still accepted, with a stored G on every level:
    # three values per level; without the side chunk (one side launch); and
    # without the prologue flag as well (side stream kept)
    per3 = [v for d in range(L) for v in table[8 + 4 * d: 11 + 4 * d]]
    stored = [v for d in range(L) for v in table[8 + 4 * d: 11 + 4 * d] + [0]]
    v3 = [3] + table[1:8] + per3
    s.set_tuning(v3, "fp64")
    assert s.get_tuning("fp64") == table[:8] + stored
    v2 = [2] + table[1:7] + per3
    s.set_tuning(v2, "fp64")
    assert s.get_tuning("fp64") == table[:7] + [0] + stored
    v1 = [1] + table[1:6] + per3
    s.set_tuning(v1, "mixed_bf16x3")
    assert s.get_tuning("mixed_bf16x3") == table[:6] + [0, 0] + stored
    bad = [table[:-1], [5] + table[1:], table[:1] + [L + 1] + table[2:], table[:3] + [48] + table[4:],
           table[:10] + [2] + table[11:], table[:11] + [2] + table[12:], table[:2] + [3] + table[3:],
           table[:6] + [3] + table[7:], table[:7] + [-1] + table[8:], table[:7] + [(1 << 20) + 1] + table[8:],
           v2[:-1], v3 + [0], v3[:6] + [2] + v3[7:]]
    for b in bad:
        with pytest.raises(si.SelinvError) as e:
            s.set_tuning(b, "mixed_fp32")
        assert e.value.status == "INVALID_ARG"
    assert s.get_tuning("mixed_fp32") == table  # unchanged by the rejected tables
    per_level = table[:6] + [2] + table[7:]  # one prologue part per upper level
    s.set_tuning(per_level, "mixed_fp32")
    assert s.get_tuning("mixed_fp32") == per_level
    s.set_tuning([], "mixed_fp32")
    assert s.get_tuning("mixed_fp32") == []
    # both sweep forms for an exact analysis too
    x = si.SelInv(w.n, w.colptr, w.rowind, w.perm, w.max_super, w.relax, w.pad_pct, symbolic="exact")
    Lx = x.info["nlevels"]
    x.set_tuning([3, Lx, 2, 0, 0, 0, 0, 0] + [0, 0, 0] * Lx)
    x.set_tuning([4, Lx, 1, 0, 0, 0, 1, 0] + [0, 0, 0, 1] * Lx)


def test_autotune_describe():
    from paper_1708_04539_amd.autotune import describe
    assert describe([]) == {"tuned": False}
    d = describe([1, 2, 1, 64, 32, 32, 32, 64, 0, 128, 128, 1])
    assert d["steps35_tiles"] == [32, 128] and d["step4_tiles"] == [64, 128]
    assert d["small_per_phase_levels"] == [1] and d["sweep"] == "levels"
    d = describe([2, 2, 1, 64, 32, 32, 1, 32, 64, 0, 128, 128, 1])
    assert d["steps35_tiles"] == [32, 128] and not d["prologue_side_stream"]
    d = describe([3, 2, 1, 64, 32, 32, 0, 512, 32, 64, 0, 128, 128, 1])
    assert d["steps35_tiles"] == [32, 128] and d["prologue_side_stream"] and d["side_inversion_chunk"] == 512
    assert d["gather_in_products_levels"] == []
    d = describe([4, 2, 1, 64, 32, 32, 0, 512, 32, 64, 0, 1, 128, 128, 1, 0])
    assert d["steps35_tiles"] == [32, 128] and d["step4_tiles"] == [64, 128]
    assert d["small_per_phase_levels"] == [1] and d["gather_in_products_levels"] == [0]
    assert not d["prologue_part_per_level"]
    assert describe([4, 1, 1, 0, 0, 0, 2, 0, 0, 0, 0, 0])["prologue_part_per_level"]


def test_gather_form_argument(si):
    """selinv_set_gather_form takes 0..2 (host side; the runs need the device)."""
    w = config_c0()
    s = si.SelInv(w.n, w.colptr, w.rowind, w.perm, w.max_super, w.relax, w.pad_pct)
    for f in ("auto", "stored", "in_products", 0, 2):
        s.set_gather_form(f)
    for f in (-1, 3):
        with pytest.raises(si.SelinvError) as e:
            s.set_gather_form(f)
        assert e.value.status == "INVALID_ARG"


# --------------------------------------------------------------------------
# complex matrices (real form of order 2n), host side
# --------------------------------------------------------------------------
def test_complex_handle_is_the_real_form(si):
    """A complex handle analyses M (entry a -> [[Re a, -Im a], [Im a, Re a]],
    node rows and columns interleaved): its plan equals the plan of a real
    handle built on that pattern and ordering."""
    from workloads import config_complex
    w = config_complex((24, 20), "box", 1, 16, 16)
    z = si.SelInv(w.n, w.colptr, w.rowind, w.perm, w.max_super, w.relax, w.pad_pct, complex_values=True)
    assert z.info["complex_values"] == 1 and z.info["n"] == 2 * w.n and z.info["nnz_a"] == 4 * w.nnz
    assert z.check_plan() == 0
    cols = np.repeat(np.arange(w.n), np.diff(w.colptr))
    r2, c2 = [], []
    for i, j in zip(w.rowind, cols):
        for a in range(2):
            for b in range(2):
                r2.append(2 * i + a)
                c2.append(2 * j + b)
    m = sp.csc_matrix((np.ones(len(r2)), (r2, c2)), shape=(2 * w.n, 2 * w.n))
    m.sort_indices()
    perm2 = np.stack([2 * w.perm, 2 * w.perm + 1], 1).ravel().astype(np.int32)
    r = si.SelInv(2 * w.n, m.indptr.astype(np.int64), m.indices.astype(np.int32), perm2, w.max_super, w.relax,
                  w.pad_pct)
    a, b = z.structure(), r.structure()
    for k in STRUCT_KEYS:
        assert np.array_equal(a[k], b[k]), k
    x = si.SelInv(w.n, w.colptr, w.rowind, w.perm, w.max_super, 0, 0, symbolic="exact", complex_values=True)
    assert x.check_plan() == 0 and x.info["symbolic"] == 1


def test_complex_error_paths(si):
    cp = np.array([0, 2, 4], np.int64)
    with pytest.raises(si.SelinvError) as e:
        si.SelInv(2, cp, np.array([0, 1, 0, 1], np.int32), np.array([1, 1], np.int32), complex_values=True)
    assert e.value.status == "BAD_PERM"
    with pytest.raises(si.SelinvError) as e:
        si.SelInv(2, cp, np.array([0, 2, 0, 1], np.int32), complex_values=True)
    assert e.value.status == "BAD_PATTERN"
    with pytest.raises(si.SelinvError) as e:
        si.SelInv(2, cp, np.array([1, 0, 0, 1], np.int32), complex_values=True)
    assert e.value.status == "BAD_PATTERN"


def test_allocator_hook_arguments(si):
    """selinv_set_allocator: both hooks or neither (NULL, NULL restores
    hipMalloc); the binding installs torch's caching allocator by default."""
    lib = si.lib()
    alloc, free = si._hooks["torch"]
    assert lib.selinv_set_allocator(si.ALLOC_FN(), free, None) == 1
    assert lib.selinv_set_allocator(alloc, si.FREE_FN(), None) == 1
    assert lib.selinv_set_allocator(si.ALLOC_FN(), si.FREE_FN(), None) == 0
    si.set_allocator("torch")


def test_get_many_host_checks(si):
    """Positions are checked on the host before any device work: outside the
    matrix -> INVALID_ARG, outside the computed set -> NOT_SELECTED, and a
    valid list without a completed run -> STATE."""
    w = config_c0()
    s = si.SelInv(w.n, w.colptr, w.rowind, w.perm, w.max_super, w.relax, w.pad_pct)
    with pytest.raises(si.SelinvError) as e:
        s.get_many([0, w.n], [0, 0])
    assert e.value.status == "INVALID_ARG"
    # the first and last nodes of the 32x32 grid are far apart in the
    # nested-dissection tree: (0, n-1) is outside the computed set
    st = s.structure()
    q = np.empty(w.n, np.int64)
    q[st["perm"]] = np.arange(w.n)
    r, c = int(st["perm"][0]), int(st["perm"][1])  # two leaf-box neighbours: inside
    with pytest.raises(si.SelinvError) as e:
        s.get_many([r, 0], [c, w.n - 1])
    assert e.value.status == "NOT_SELECTED"
    with pytest.raises(si.SelinvError) as e:
        s.get_many([r], [c])
    assert e.value.status == "STATE"
    assert s.get_many([], []).size == 0


def test_gather_code_budget(si):
    """The gather's source codes can be limited or switched off before the
    first factor; the plan stays consistent either way."""
    w = config_c1()
    for budget in (0, 4096, -1):
        s = si.SelInv(w.n, w.colptr, w.rowind, w.perm, w.max_super, w.relax, w.pad_pct)
        s.set_gather_code_budget(budget)
        assert s.check_plan() == 0
    with pytest.raises(si.SelinvError) as e:
        s._check(si.lib().selinv_set_gather_code_budget(None, 0), "x")
    assert e.value.status == "INVALID_ARG"


def test_level_stats_and_timings_without_a_run(si):
    """Introspection before any run reports STATE instead of reading a sweep
    that does not exist."""
    w = config_c0()
    s = si.SelInv(w.n, w.colptr, w.rowind, w.perm, w.max_super, w.relax, w.pad_pct)
    with pytest.raises(si.SelinvError) as e:
        s.level_stats(0)
    assert e.value.status == "STATE"
    s.set_profiling(True)
    with pytest.raises(si.SelinvError) as e:
        s.timings()
    assert e.value.status == "STATE"
