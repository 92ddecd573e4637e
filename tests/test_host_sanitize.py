"""Host analysis and LU under AddressSanitizer and UndefinedBehaviorSanitizer.

Builds tests/host_sanitize/driver.cpp with the library's analyze.cpp and
factor.cpp (g++, host code only, no GPU) and runs the symbolic analysis in
both forms, the host check of every gather / extraction index and the LU on
random, triangular, upwind and stencil patterns.  Any sanitizer report fails
the test."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from workloads import config_c0, config_upwind, random_sparse

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1708_04539_amd", "csrc")


def _dump(path, n, cp, ri, perm, v, cap, relax, pad):
    with open(path, "wb") as f:
        np.array([n, cp[-1]], np.int64).tofile(f)
        np.asarray(cp, np.int64).tofile(f)
        np.asarray(ri, np.int32).tofile(f)
        np.asarray(perm, np.int32).tofile(f)
        np.asarray(v, np.float64).tofile(f)
        np.array([cap, relax, pad], np.int32).tofile(f)


@pytest.mark.slow
def test_analysis_and_lu_are_sanitizer_clean(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    exe = str(tmp_path / "driver")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fopenmp", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-fno-sanitize-recover=undefined", "-I", CSRC, os.path.join(ROOT, "tests", "host_sanitize", "driver.cpp"),
           os.path.join(CSRC, "analyze.cpp"), os.path.join(CSRC, "factor.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in r.stderr.lower():
        pytest.skip("sanitizer runtime not available: " + r.stderr[-200:])
    assert r.returncode == 0, r.stderr[-2000:]
    cases = []
    for seed, n, dens, cap, relax, pad in [(0, 300, 0.01, 8, 0, 0), (1, 250, 0.03, 1, 4, 10), (2, 1, 0.0, 3, 0, 0),
                                           (3, 2, 0.5, 1, 2, 50), (4, 600, 0.004, 64, 10, 30)]:
        cp, ri, v, _ = random_sparse(n, dens, seed)
        cases.append((n, cp, ri, np.random.default_rng(seed).permutation(n), v, cap, relax, pad))
    for lower in (True, False):
        cp, ri, v, _ = random_sparse(200, 0.02, 9, lower_only=lower, upper_only=not lower)
        cases.append((200, cp, ri, np.arange(200), v, 16, 8, 50))
    for w in (config_upwind((40, 40), "box", 0.25, 3, 32, 16), config_c0()):
        cases.append((w.n, w.colptr, w.rowind, w.perm, w.values, w.max_super, w.relax, w.pad_pct))
    env = dict(os.environ, OMP_NUM_THREADS="4", ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    for k, c in enumerate(cases):
        path = str(tmp_path / f"case{k}.bin")
        _dump(path, *c)
        r = subprocess.run([exe, path], capture_output=True, text=True, env=env, timeout=120)
        assert r.returncode == 0 and "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, \
            (k, r.stdout[-500:], r.stderr[-3000:])
