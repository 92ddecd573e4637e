"""Single entries of A^{-1} straight from the definition, for sizes where the
supernodal oracle is too slow.

TEST INFRASTRUCTURE ONLY (see the package docstring).

A^{-1}(i, j) is entry i of the solution x of A x = e_j.  The solve uses
restarted GMRES (scipy) with a Jacobi preconditioner as the inner solver and
iterative refinement whose residual b - A x is accumulated in extended
precision (numpy.longdouble), until the residual stops decreasing.  For the
strictly row-diagonally-dominant stencil matrices, ||A^{-1}||_inf is at most
1 / (min_i |a_ii| - sum_{j != i} |a_ij|) (Varah's bound), so the error of every
entry is at most that bound times the final residual; ``solve_column``
returns the bound with the column.

This path shares nothing with the factor-based oracle or with the HIP library:
it never forms L or U.
"""
from __future__ import annotations

import os

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def varah_bound(A: sp.spmatrix) -> float:
    A = sp.csr_matrix(A)
    d = np.abs(A.diagonal())
    off = np.asarray(abs(A).sum(axis=1)).ravel() - d
    margin = (d - off).min()
    return float("inf") if margin <= 0 else 1.0 / margin


def solve_column(A: sp.spmatrix, j: int, max_refine: int = 6):
    """Returns (x, err_bound) with x = A^{-1} e_j."""
    A = sp.csr_matrix(A)
    n = A.shape[0]
    d = A.diagonal()
    M = spla.LinearOperator((n, n), matvec=lambda v: v / d, dtype=np.float64)
    A_ld = A.astype(np.longdouble)
    b = np.zeros(n, dtype=np.longdouble)
    b[j] = 1
    x = np.zeros(n)
    last = np.inf
    res = 1.0
    for _ in range(max_refine):
        r = b - A_ld @ x.astype(np.longdouble)
        res = float(np.abs(r).max())
        if res > 0.5 * last or res == 0.0:
            break
        last = res
        dx, _ = spla.gmres(A, r.astype(np.float64), M=M, rtol=1e-12, restart=80, maxiter=4000)
        x = x + dx
    r = b - A_ld @ x.astype(np.longdouble)
    res = float(np.abs(r).max())
    return x, varah_bound(A) * res


_A = None


def _init_worker(A):
    global _A
    _A = A


def _solve_one(j):
    return solve_column(_A, j)


def solve_columns(A: sp.spmatrix, js, workers: int = 0):
    """solve_column for every column in js, in a pool of worker processes
    (spawned, one BLAS thread each; workers = 0: one per available core, at
    most 16).  Returns a list of (x, err_bound) in the order of js."""
    import multiprocessing as mp
    js = [int(j) for j in js]
    if workers <= 0:
        workers = min(16, len(os.sched_getaffinity(0)))
    workers = max(1, min(workers, len(js)))
    A = sp.csr_matrix(A)
    if workers == 1:
        return [solve_column(A, j) for j in js]
    keep = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in keep:
        os.environ[k] = "1"
    try:
        with mp.get_context("spawn").Pool(workers, initializer=_init_worker, initargs=(A,)) as pool:
            return pool.map(_solve_one, js, chunksize=1)
    finally:
        for k, v in keep.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
