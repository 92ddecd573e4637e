"""CPU checks of the C ABI library: it loads, exports every declared entry
point, and its host analysis reproduces the oracle's partition and block sets
exactly.  No compute call here needs a GPU."""
import ctypes as C
import os
import re

import numpy as np
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
