"""Complex selected entries from their definition -- test infrastructure.

The paper's experiments invert complex matrices (shifted Hamiltonians
H - zS).  The selected entries of a complex A are A^{-1}(j, i) for every
stored entry A(i, j) (the selected set of the paper's introduction, reached
by Theorem 2).  This module computes them straight from that definition and
shares nothing with the library:

  selected_dense(n, colptr, rowind, values)
      the whole inverse in complex128 from LAPACK (numpy), then the selected
      entries, in CSC entry order (out[p] = A^{-1}(j, i) for entry p at
      (i, j)); small n only;
  solve_columns(n, colptr, rowind, values, js)
      exact columns x = A^{-1} e_j for a few j, from a sparse complex LU
      (SuperLU through scipy) with iterative refinement, for full-size
      matrices.

Only the tests, smoke() and bench.py's CPU baseline may use it.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def to_dense(n, colptr, rowind, values) -> np.ndarray:
    return sp.csc_matrix((np.asarray(values, np.complex128), rowind, colptr), shape=(n, n)).toarray()


def selected_dense(n, colptr, rowind, values) -> np.ndarray:
    """out[p] = A^{-1}(j, i) for the p-th stored entry (i, j) of A."""
    inv = np.linalg.inv(to_dense(n, colptr, rowind, values))
    cols = np.repeat(np.arange(n), np.diff(colptr))
    return inv[cols, np.asarray(rowind)]


def solve_columns(n, colptr, rowind, values, js, refine: int = 3):
    """Columns x_j = A^{-1} e_j (complex128), sparse LU + iterative refinement."""
    A = sp.csc_matrix((np.asarray(values, np.complex128), rowind, colptr), shape=(n, n))
    lu = spla.splu(A, permc_spec="COLAMD")
    out = []
    for j in js:
        e = np.zeros(n, np.complex128)
        e[j] = 1.0
        x = lu.solve(e)
        for _ in range(refine):
            x = x + lu.solve(e - A @ x)
        out.append(x)
    return out
