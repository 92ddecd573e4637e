"""The LU factorisation on the GPU (selinv_factor_device), checked through
the selected inversion it feeds: the computed superset after the device LU
against the oracle (whose LU is its own host code), and against the same
handle factored by the host LU.  Marked gpu."""
import ctypes as C
import sys

import numpy as np
import pytest

from oracle import Oracle
from workloads import config_c1, random_sparse

pytestmark = pytest.mark.gpu

TOL = 1e-11


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


def on_device(values):
    import torch
    return torch.from_numpy(np.ascontiguousarray(values)).to("cuda")


def rel_err(s, o):
    r1, c1, v1 = s.export()
    r2, c2, v2 = o.export()
    assert np.array_equal(r1, r2) and np.array_equal(c1, c2)
    en = np.abs(v1 - v2).max() / np.abs(v2).max()
    d = r2 == c2
    ed = (np.abs(v1[d] - v2[d]) / np.abs(v2[d])).max() if d.any() else 0.0
    return max(en, ed)


CASES = [  # n, density, seed, cap, relax, pad, symbolic
    (1, 0.0, 0, 1, 0, 0, "symmetrized"),
    (37, 0.08, 2, 5, 0, 0, "symmetrized"),
    (150, 0.03, 3, 16, 4, 5, "symmetrized"),
    (400, 0.01, 4, 70, 10, 20, "symmetrized"),   # two 64-column steps in the widest blocks
    (300, 0.6, 5, 300, 0, 0, "symmetrized"),     # one dense supernode: 5 steps, ragged last
    (300, 0.01, 3, 16, 0, 0, "exact"),
    (300, 0.3, 6, 300, 0, 0, "exact"),
    (700, 0.004, 7, 3, 0, 0, "exact"),
]


@pytest.mark.parametrize("case", CASES, ids=[f"n{c[0]}_cap{c[3]}_{c[6]}" for c in CASES])
def test_device_lu_random(si, case):
    n, dens, seed, cap, relax, pad, sym = case
    say("device LU random", case)
    cp, ri, v, _ = random_sparse(n, dens, seed, symmetric_pattern=(sym == "symmetrized" and seed % 2 == 0))
    perm = np.random.default_rng(seed).permutation(n).astype(np.int32)
    s = si.SelInv(n, cp, ri, perm, cap, relax, pad, symbolic=sym)
    s.factor_device(on_device(v)).run("fp64")
    o = Oracle(n, cp, ri, perm, cap, relax, 1 if sym == "exact" else 0, pad).factor(v).selinv()
    e = rel_err(s, o)
    say("device LU random", case, "err", e)
    assert e <= TOL


@pytest.mark.parametrize("tri", ["lower", "upper"])
def test_device_lu_triangular_patterns(si, tri):
    """Exact analysis with L(R_L, K) or U(K, R_U) empty everywhere: no Schur
    complement products at all."""
    n, seed = 400, 4
    say("device LU triangular", tri)
    cp, ri, v, _ = random_sparse(n, 0.02, seed, lower_only=tri == "lower", upper_only=tri == "upper")
    s = si.SelInv(n, cp, ri, None, 64, 0, 0, symbolic="exact")
    s.factor_device(on_device(v)).run("fp64")
    o = Oracle(n, cp, ri, None, 64, 0, 1, 0).factor(v).selinv()
    assert rel_err(s, o) <= TOL


def test_device_lu_widest_supernode_1024(si):
    n = 1100
    say("device LU wide 1024")
    cp, ri, v, _ = random_sparse(n, 0.01, 8, symmetric_pattern=True)
    s = si.SelInv(n, cp, ri, None, 1024, n, 0)
    assert s.info["max_s"] == 1024
    s.factor_device(on_device(v)).run("fp64")
    o = Oracle(n, cp, ri, None, 1024, n, 0, 0).factor(v).selinv()
    assert rel_err(s, o) <= TOL


def test_device_lu_c1_matches_host_lu(si):
    """2D 256^2 9-point stencil at full size: the run after the device LU
    against the run after the host LU of the same handle, over the whole
    computed superset, then a host LU again (the handle switches back)."""
    w = config_c1()
    say("device LU c1")
    s = si.SelInv(w.n, w.colptr, w.rowind, w.perm, w.max_super, w.relax, w.pad_pct)
    s.factor(w.values).run("fp64")
    r0, c0, v0 = s.export()
    s.factor_device(on_device(w.values)).run("fp64")
    r1, c1, v1 = s.export()
    assert np.array_equal(r0, r1) and np.array_equal(c0, c1)
    e = np.abs(v1 - v0).max() / np.abs(v0).max()
    d = r0 == c0
    ed = (np.abs(v1[d] - v0[d]) / np.abs(v0[d])).max()
    say("device LU c1", "err", e, ed)
    assert max(e, ed) <= TOL
    s.factor(w.values).run("fp64")
    assert np.array_equal(s.export()[2], v0)


@pytest.mark.parametrize("sym", ["symmetrized", "exact"])
def test_device_lu_complex(si, sym):
    import torch
    from oracle.complex_ref import selected_dense
    n, seed = 300, 5
    say("device LU complex", sym)
    cp, ri, v, _ = random_sparse(n, 0.02, seed)
    rng = np.random.default_rng(seed + 1000)
    cols = np.repeat(np.arange(n), np.diff(cp))
    z = v * (1 + 0.3j * rng.uniform(-1, 1, v.size))
    d = ri == cols
    z[d] = 1.35 * v[d] + 0.2j * np.abs(v[d])
    perm = np.random.default_rng(seed).permutation(n).astype(np.int32)
    s = si.SelInv(n, cp, ri, perm, 32, 0, 0, symbolic=sym, complex_values=True)
    s.factor_device(torch.from_numpy(z).to("cuda")).run("fp64")
    got, ref = s.get_selected(), selected_dense(n, cp, ri, z)
    e = np.abs(got - ref).max() / np.abs(ref).max()
    say("device LU complex", sym, "err", e)
    assert e <= TOL


def test_device_lu_zero_pivot_and_recovery(si):
    """An exact zero pivot is reported at the same column as the host LU
    reports it; the handle is then unfactored, and a good factorisation after
    it works.  Row and column 0 hold only zeros, so the pivot of column 0 is
    exactly zero in any elimination order (nothing updates it)."""
    n = 40
    cp, ri, v, _ = random_sparse(n, 0.1, 11, symmetric_pattern=True)
    cols = np.repeat(np.arange(n), np.diff(cp))
    bad = v.copy()
    bad[(ri == 0) | (cols == 0)] = 0.0
    s = si.SelInv(n, cp, ri, None, 8, 0, 0)
    with pytest.raises(si.SelinvError) as host:
        s.factor(bad)
    with pytest.raises(si.SelinvError) as dev:
        s.factor_device(on_device(bad))
    assert host.value.status == dev.value.status == "ZERO_PIVOT"
    mh, md = str(host.value), str(dev.value)
    assert "(original column 0)" in mh and mh.split("factor")[-1] == md.split("factor_device")[-1], (mh, md)
    with pytest.raises(si.SelinvError) as st:
        s.run("fp64")
    assert st.value.status == "STATE"
    s.factor_device(on_device(v)).run("fp64")
    o = Oracle(n, cp, ri, None, 8, 0, 0, 0).factor(v).selinv()
    assert rel_err(s, o) <= TOL


def test_device_lu_rejects_host_pointer(si):
    n = 10
    cp, ri, v, _ = random_sparse(n, 0.2, 3)
    s = si.SelInv(n, cp, ri, None, 4, 0, 0)
    rc = si.lib().selinv_factor_device(s._h, C.c_void_p(v.ctypes.data), None)
    assert si.STATUS[rc] == "INVALID_ARG"
    with pytest.raises(ValueError):
        s.factor_device(on_device(v.astype(np.float32)))


@pytest.mark.parametrize("name", ["u1", "z1"])
def test_device_lu_full_size_matches_host_lu(si, name):
    """Full-size exact-analysis (2D 256^2 upwind, n = 65536) and complex
    (2D 256^2, n = 65536 complex, real form of order 131072) workloads: the
    selected entries after the device LU against those after the host LU,
    and the identity sum_i A(i,j) A^{-1}(j,i) = 1 over every column j for the
    device-LU result (a property independent of either LU)."""
    import torch
    from workloads import get_config
    w = get_config(name)
    cplx = name == "z1"
    say("device LU full size", name)
    s = si.SelInv(w.n, w.colptr, w.rowind, w.perm, w.max_super, w.relax, w.pad_pct,
                  symbolic="exact" if name == "u1" else "symmetrized", complex_values=cplx)
    s.factor(w.values).run("fp64")
    ref = s.get_selected()
    s.factor_device(torch.from_numpy(np.ascontiguousarray(w.values)).to("cuda")).run("fp64")
    got = s.get_selected()
    e = np.abs(got - ref).max() / np.abs(ref).max()
    cols = np.repeat(np.arange(w.n), np.diff(w.colptr))
    prod = w.values * got
    colsum = np.bincount(cols, prod.real, w.n) + (1j * np.bincount(cols, prod.imag, w.n) if cplx else 0)
    idr = np.abs(colsum - 1).max()
    say("device LU full size", name, "diff vs host LU", e, "identity", idr)
    assert e <= TOL and idr <= 1e-10
