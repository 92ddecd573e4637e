"""Factors with the block structure of the paper's Fig. 2 (b) (non-symmetric
PMatrix layout), built from the golden fixture tests/golden/fig2b_block_structure.json.

fig2b_factors(seed) returns (spec, xsup, rl_ptr, rl, ru_ptr, ru, L, U): the
supernode partition of the figure, the block row set R_L(K) and column set
R_U(K) read from its L and U blocks, and dense unit-lower L / upper U with
seeded U[-0.5, 0.5] entries on exactly that pattern (diagonal of U in [2, 3]).
"""
import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def fig2b_factors(seed=0):
    spec = json.load(open(os.path.join(GOLDEN, "fig2b_block_structure.json")))
    wd = spec["widths"]
    xs = np.concatenate([[0], np.cumsum(wd)]).astype(np.int32)
    n = int(xs[-1])
    ns = len(wd)
    rows = {K: set() for K in range(ns)}
    cols = {K: set() for K in range(ns)}
    for blk in spec["L_blocks"]:
        I, J = blk["I"] - 1, blk["J"] - 1
        loc = blk.get("rows_local", range(wd[I]))
        rows[J] |= {int(xs[I] + t) for t in loc}
    for blk in spec["U_blocks"]:
        I, J = blk["I"] - 1, blk["J"] - 1
        loc = blk.get("cols_local", range(wd[J]))
        cols[I] |= {int(xs[J] + t) for t in loc}
    rl_ptr = np.zeros(ns + 1, np.int64)
    ru_ptr = np.zeros(ns + 1, np.int64)
    rl, ru = [], []
    for K in range(ns):
        rl += sorted(rows[K])
        ru += sorted(cols[K])
        rl_ptr[K + 1] = len(rl)
        ru_ptr[K + 1] = len(ru)
    rng = np.random.default_rng(seed)
    L = np.eye(n)
    U = np.zeros((n, n))
    for K in range(ns):
        f, l = xs[K], xs[K + 1]
        for c in range(f, l):
            for r in range(c + 1, l):
                L[r, c] = rng.uniform(-0.5, 0.5)
            for r in rows[K]:
                L[r, c] = rng.uniform(-0.5, 0.5)
            for r in range(f, c):
                U[r, c] = rng.uniform(-0.5, 0.5)
            U[c, c] = rng.uniform(2, 3)
        for r in range(f, l):
            for c in cols[K]:
                U[r, c] = rng.uniform(-0.5, 0.5)
    return spec, xs, rl_ptr, np.array(rl, np.int32), ru_ptr, np.array(ru, np.int32), L, U
