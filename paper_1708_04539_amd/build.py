"""Build the gfx950 selected-inversion library in-tree.

Host analysis and LU (C++17, OpenMP) are compiled with g++; the kernels and the
C ABI runtime with hipcc for gfx950.  The result is
``paper_1708_04539_amd/libselinv.so``.  Every call recompiles.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libselinv.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")

HOST_SOURCES = ["analyze.cpp", "factor.cpp"]
HIP_SOURCES = ["kernels.hip", "gemm.hip", "persist.hip", "lu_device.hip", "runtime.hip"]

HOST_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-fopenmp", "-march=x86-64-v3", "-Wall", "-Wextra",
              "-Wno-unused-parameter"]
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-mcode-object-version=5",
             # keep packed FP32 instructions out of every kernel
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             # MFMA accumulators in ordinary VGPRs: keeps the loop-carried
             # accumulators from being copied between register files
             "-mllvm", "-amdgpu-mfma-vgpr-form=1",
             "-Wall", "-Wno-unused-parameter"]


def _run(cmd, log):
    log.write(" ".join(cmd) + "\n")
    log.flush()
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if out.strip():
        log.write(out + "\n")
    if r.returncode != 0:
        raise RuntimeError(f"build step failed ({r.returncode}): {' '.join(cmd)}\n{out}")


def build(verbose: bool = False) -> str:
    if not os.path.exists(HIPCC):
        raise RuntimeError(f"hipcc not found at {HIPCC}")
    log = sys.stdout if verbose else open(os.devnull, "w")
    tmp = tempfile.mkdtemp(prefix="selinv_build_")
    try:
        objs = []
        jobs = []
        for s in HOST_SOURCES:
            o = os.path.join(tmp, s + ".o")
            jobs.append((["g++", *HOST_FLAGS, "-c", os.path.join(CSRC, s), "-o", o], o))
        for s in HIP_SOURCES:
            o = os.path.join(tmp, s + ".o")
            jobs.append(([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, s), "-o", o], o))
        procs = []
        for cmd, o in jobs:
            log.write(" ".join(cmd) + "\n")
            procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                                                text=True)))
            objs.append(o)
        for cmd, p in procs:
            out, _ = p.communicate()
            out = "\n".join(l for l in out.splitlines() if "packed-fp32-ops" not in l)
            if out.strip():
                log.write(out + "\n")
            if p.returncode != 0:
                raise RuntimeError(f"build step failed: {' '.join(cmd)}\n{out}")
        tmp_lib = os.path.join(tmp, "libselinv.so")
        _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp_lib, "-lgomp",
              "-Wl,-z,defs", "-lamdhip64"], log)
        shutil.copyfile(tmp_lib, LIB + ".tmp")
        os.replace(LIB + ".tmp", LIB)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
        if log is not sys.stdout:
            log.close()
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
