"""The allocation-free extraction (selinv_get_selected_noalloc) against
selinv_get_selected, through the C ABI: two calls in a row, the second on a
smaller matrix, bit for bit."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def si():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1708_04539_amd import selinv
    return selinv


def noalloc(si, s, count):
    out = np.full(count, np.nan)
    rc = si.lib().selinv_get_selected_noalloc(s.handle, out.ctypes.data_as(C.POINTER(C.c_double)))
    assert rc == 0, si.lib().selinv_last_error(s.handle)
    return out


def test_get_selected_noalloc_matches_get_selected(si):
    import torch
    from workloads import config_c0, config_grid
    # 400x400 9-point: 1.44e6 selected entries, more than one chunk of the
    # 2^20-entry staging array; then the 32x32 5-point C0 (5e3 entries)
    big = config_grid("g400", (400, 400), "box", "sym_perturbed", 0.05, 3, 128, 64, delta=0.2)
    small = config_c0()
    assert big.nnz > (1 << 20) > small.nnz
    for w, prec in ((big, "fp64"), (small, "mixed_fp32"), (small, "fp64")):
        s = si.SelInv(w.n, w.colptr, w.rowind, w.perm, w.max_super, w.relax, w.pad_pct).factor(w.values)
        s.run(prec)
        ref = s.get_selected()
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        got = noalloc(si, s, w.nnz)
        assert torch.cuda.memory_allocated() == before  # nothing taken from the allocator
        assert np.array_equal(got, ref), (w.name, prec)
        s.close()
