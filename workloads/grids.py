"""Stencil matrices on 2D/3D grids and a geometric nested-dissection ordering.

The paper's experiments use matrices from electronic-structure codes and a
public sparse-matrix collection (Table "test problems"); none of them is
available here.  These seeded synthetic matrices stand in for them: 2D and 3D
grid stencils whose nested-dissection elimination trees have the same
"1D/2D/3D system" shape the paper's cost discussion relies on (section on weak
scaling: the largest separator dominates the cost).

Conventions
-----------
* Grid node id = x + nx*(y + ny*z), x fastest.
* Matrices are returned in CSC form: ``colptr`` (int64, n+1), ``rowind``
  (int32, sorted and unique within a column), ``values`` (float64).
* ``perm`` is the fill-reducing ordering, perm[new] = old, so that the
  permuted matrix is At[a, b] = A[perm[a], perm[b]].
* All generators are deterministic; random values come from
  ``numpy.random.default_rng(seed)`` (PCG64), drawn in a fixed order.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp


@dataclass
class Workload:
    name: str
    n: int
    colptr: np.ndarray
    rowind: np.ndarray
    values: np.ndarray
    perm: np.ndarray
    max_super: int
    relax: int
    dims: tuple = ()
    pad_pct: int = 5
    desc: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.colptr[-1])

    def to_scipy(self) -> sp.csc_matrix:
        return sp.csc_matrix((self.values, self.rowind, self.colptr), shape=(self.n, self.n))


# ----------------------------------------------------------------------------
# ordering
# ----------------------------------------------------------------------------

def _box_ids(lo, hi, dims3):
    nx, ny, _ = dims3
    xs = np.arange(lo[0], hi[0], dtype=np.int64)
    ys = np.arange(lo[1], hi[1], dtype=np.int64)
    zs = np.arange(lo[2], hi[2], dtype=np.int64)
    ids = (zs[:, None, None] * ny + ys[None, :, None]) * nx + xs[None, None, :]
    return ids.ravel()


def nested_dissection(dims, leaf: int) -> np.ndarray:
    """Geometric nested dissection of a box grid; returns perm[new] = old.

    A box with at most ``leaf`` nodes is ordered lexicographically (x fastest).
    A larger box is split across its longest axis (ties go to the lower axis,
    x before y before z) at mid = lo + (hi - lo) // 2: the plane at ``mid`` is
    the separator, and the order is left box, right box, separator.  One grid
    plane separates 5/7/9/27-point stencils because no stencil couples nodes
    two planes apart.
    """
    dims3 = tuple(int(d) for d in dims) + (1,) * (3 - len(dims))
    out = []

    def rec(lo, hi):
        ext = [h - l for l, h in zip(lo, hi)]
        size = ext[0] * ext[1] * ext[2]
        if size <= 0:
            return
        if size <= leaf:
            out.append(_box_ids(lo, hi, dims3))
            return
        ax = max(range(3), key=lambda a: (ext[a], -a))
        mid = lo[ax] + ext[ax] // 2
        lhi = list(hi)
        lhi[ax] = mid
        rlo = list(lo)
        rlo[ax] = mid + 1
        slo = list(lo)
        slo[ax] = mid
        shi = list(hi)
        shi[ax] = mid + 1
        rec(list(lo), lhi)
        rec(rlo, list(hi))
        out.append(_box_ids(slo, shi, dims3))

    rec([0, 0, 0], list(dims3))
    perm = np.concatenate(out).astype(np.int32)
    assert perm.size == dims3[0] * dims3[1] * dims3[2]
    return perm


# ----------------------------------------------------------------------------
# matrix assembly
# ----------------------------------------------------------------------------

def _offsets(ndim: int, kind: str):
    """Neighbour offsets (dx, dy, dz).  kind: 'star' (5/7-point) or 'box' (9/27-point)."""
    offs = []
    rng = [-1, 0, 1]
    for dz in (rng if ndim == 3 else [0]):
        for dy in rng:
            for dx in rng:
                if dx == dy == dz == 0:
                    continue
                if kind == "star" and abs(dx) + abs(dy) + abs(dz) != 1:
                    continue
                offs.append((dx, dy, dz))
    return offs


def _pairs(dims3, off):
    """All (i, j) with j = i + off inside the grid, i in increasing id order."""
    nx, ny, nz = dims3
    dx, dy, dz = off
    xs = np.arange(max(0, -dx), min(nx, nx - dx), dtype=np.int64)
    ys = np.arange(max(0, -dy), min(ny, ny - dy), dtype=np.int64)
    zs = np.arange(max(0, -dz), min(nz, nz - dz), dtype=np.int64)
    i = ((zs[:, None, None] * ny + ys[None, :, None]) * nx + xs[None, None, :]).ravel()
    j = i + dx + nx * (dy + ny * dz)
    return i, j


def _assemble(n, rows, cols, vals, margin):
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    diag = np.zeros(n)
    np.add.at(diag, rows, np.abs(vals))
    diag += margin
    rows = np.concatenate([rows, np.arange(n)])
    cols = np.concatenate([cols, np.arange(n)])
    vals = np.concatenate([vals, diag])
    m = sp.csc_matrix((vals, (rows, cols)), shape=(n, n))
    m.sum_duplicates()
    m.sort_indices()
    return m.indptr.astype(np.int64), m.indices.astype(np.int32), m.data.astype(np.float64)


def stencil_csc(dims, kind: str, value_mode: str, margin: float, seed=None,
                asym: float = 0.3, delta: float = 0.0, jitter: float = 0.0,
                keep: float = 0.0):
    """Assemble a grid stencil matrix.

    value_mode:
      'convection': entry (i, i+d) = -1 + asym*s, s = +1 if d points to +x/+y/+z
                    and -1 otherwise, plus a seeded U[-jitter, jitter] per entry.
      'sym_perturbed': per unordered neighbour pair a symmetric weight
                    w ~ U[-1, 0], plus an independent eps ~ U[-delta, delta]
                    for each of the two ordered entries.
      'upwind':     one-sided (first-order upwind) convection along the flow
                    b = (1, 1/2, 1/4): row i couples to every upstream
                    neighbour i+d (d.b < 0) with -(1 + asym) + U[-jitter,
                    jitter], and to a downstream neighbour (d.b > 0) only with
                    probability ``keep`` (seeded Bernoulli per entry), value
                    -(1 - asym) + U[-jitter, jitter].  The pattern is not
                    symmetric: keep = 0 gives a permuted triangular matrix.
    The diagonal is the row sum of |off-diagonals| plus ``margin`` (strict row
    diagonal dominance, so an unpivoted LU exists and is stable).
    """
    dims3 = tuple(int(d) for d in dims) + (1,) * (3 - len(dims))
    ndim = len(dims)
    n = dims3[0] * dims3[1] * dims3[2]
    rng = np.random.default_rng(seed)
    rows, cols, vals = [], [], []
    if value_mode == "convection":
        for off in _offsets(ndim, kind):
            i, j = _pairs(dims3, off)
            s = 1.0 if sum(off) > 0 else -1.0
            v = np.full(i.size, -1.0 + asym * s)
            if jitter:
                v = v + rng.uniform(-jitter, jitter, size=i.size)
            rows.append(i)
            cols.append(j)
            vals.append(v)
    elif value_mode == "sym_perturbed":
        for off in _offsets(ndim, kind):
            if (off[2], off[1], off[0]) <= (0, 0, 0):
                continue  # positive half: each unordered pair once
            i, j = _pairs(dims3, off)
            w = rng.uniform(-1.0, 0.0, size=i.size)
            e_ij = rng.uniform(-delta, delta, size=i.size)
            e_ji = rng.uniform(-delta, delta, size=i.size)
            rows += [i, j]
            cols += [j, i]
            vals += [w + e_ij, w + e_ji]
    elif value_mode == "upwind":
        flow = (1.0, 0.5, 0.25)
        for off in _offsets(ndim, kind):
            i, j = _pairs(dims3, off)
            down = sum(o * b for o, b in zip(off, flow)) > 0
            if down:
                take = rng.random(i.size) < keep
                i, j = i[take], j[take]
            v = np.full(i.size, -(1.0 - asym) if down else -(1.0 + asym))
            if jitter:
                v = v + rng.uniform(-jitter, jitter, size=i.size)
            rows.append(i)
            cols.append(j)
            vals.append(v)
    else:
        raise ValueError(value_mode)
    return _assemble(n, rows, cols, vals, margin)


# ----------------------------------------------------------------------------
# the five stencil workloads
# ----------------------------------------------------------------------------

def _grid_workload(name, dims, kind, value_mode, margin, seed, max_super, leaf,
                   desc, **kw):
    colptr, rowind, values = stencil_csc(dims, kind, value_mode, margin, seed=seed, **kw)
    n = int(np.prod(dims))
    perm = nested_dissection(dims, leaf)
    return Workload(name=name, n=n, colptr=colptr, rowind=rowind, values=values,
                    perm=perm, max_super=max_super, relax=leaf, dims=tuple(dims),
                    desc=desc)


def config_c0() -> Workload:
    """2D 32x32 5-point convection-diffusion, n=1024, supernodes <= 32."""
    return _grid_workload("c0", (32, 32), "star", "convection", 0.1, None, 32, 32,
                          "2D 32x32 5-point asymmetric convection-diffusion, n=1024, cap 32")


def config_c1() -> Workload:
    """2D 256x256 9-point, symmetric U[-1,0] weights + U[-0.2,0.2] asymmetry."""
    return _grid_workload("c1", (256, 256), "box", "sym_perturbed", 0.05, 0, 128, 64,
                          "2D 256x256 9-point asymmetric stencil, n=65536, cap 128",
                          delta=0.2)


def config_c2() -> Workload:
    """3D 48^3 7-point convection-diffusion, asymmetry 0.3, margin 0.1."""
    return _grid_workload("c2", (48, 48, 48), "star", "convection", 0.1, None, 256, 64,
                          "3D 48^3 7-point asymmetric convection-diffusion, n=110592, cap 256")


def config_c3(count: int = 32, side_lo: int = 64, side_hi: int = 256):
    """Batch of 2D 5-point matrices; matrix m draws its side from rng(seed=m)."""
    out = []
    for m in range(count):
        rng = np.random.default_rng(m)
        side = int(rng.integers(side_lo, side_hi + 1))
        w = _grid_workload(f"c3_{m}", (side, side), "star", "convection", 0.1, 1000 + m,
                           128, 64,
                           f"2D {side}x{side} 5-point asymmetric, n={side * side}, cap 128",
                           jitter=0.05)
        out.append(w)
    return out


def config_c4() -> Workload:
    """3D 64^3 27-point, symmetric U[-1,0] weights + U[-0.15,0.15] asymmetry."""
    return _grid_workload("c4", (64, 64, 64), "box", "sym_perturbed", 0.1, 0, 512, 64,
                          "3D 64^3 27-point asymmetric stencil, n=262144, cap 512",
                          delta=0.15)


def config_grid(name, dims, kind, value_mode, margin, seed, max_super, leaf, **kw) -> Workload:
    """A stencil workload of any grid (stencil_csc arguments), nested-dissection order."""
    pts = {("star", 2): 5, ("box", 2): 9, ("star", 3): 7, ("box", 3): 27}[(kind, len(dims))]
    return _grid_workload(name, tuple(dims), kind, value_mode, margin, seed, max_super, leaf,
                          f"{len(dims)}D {'x'.join(str(d) for d in dims)} {pts}-point {value_mode}, "
                          f"n={int(np.prod(dims))}, cap {max_super}", **kw)


def config_upwind(dims=(64, 64), kind: str = "box", keep: float = 0.25, seed: int = 0,
                  max_super: int = 128, leaf: int = 64) -> Workload:
    """Structurally non-symmetric grid stencil (one-sided upwind couplings,
    downstream ones kept with probability ``keep``), nested-dissection order."""
    name = "u" + "x".join(str(d) for d in dims)
    pts = {("star", 2): 5, ("box", 2): 9, ("star", 3): 7, ("box", 3): 27}[(kind, len(dims))]
    w = _grid_workload(name, tuple(dims), kind, "upwind", 0.1, seed, max_super, leaf,
                       f"{len(dims)}D {'x'.join(str(d) for d in dims)} {pts}-point upwind "
                       f"(downstream kept with p={keep}), n={int(np.prod(dims))}, cap {max_super}",
                       keep=keep, jitter=0.05)
    # the exact L and U columns of a separator differ more from one another
    # than those of a symmetric pattern: a looser padding bound keeps the
    # separator chains whole
    w.pad_pct = 50
    return w


def config_u1() -> Workload:
    """2D 256x256 9-point upwind stencil, downstream couplings kept with p = 0.25:
    the C1 grid and ordering with a structurally non-symmetric pattern."""
    return config_upwind((256, 256), "box", 0.25, 0, 128, 64)


def config_u4() -> Workload:
    """3D 64^3 27-point upwind stencil, downstream couplings kept with p = 0.25:
    the C4 grid and ordering with a structurally non-symmetric pattern."""
    return config_upwind((64, 64, 64), "box", 0.25, 0, 512, 64)


def stencil_csc_complex(dims, kind: str, margin: float, seed=None, delta: float = 0.2, eta: float = 0.5):
    """Complex grid stencil shaped like a shifted Hamiltonian H - zS.

    Per unordered neighbour pair a symmetric weight w ~ U[-1, 0]; each ordered
    entry is w (1 + i eps), eps ~ U[-delta, delta] drawn independently.  The
    diagonal is the row sum of |off-diagonals| plus ``margin``, plus i*eta, so
    its real part dominates the row (an unpivoted LU exists and is stable).
    Returns (colptr, rowind, values complex128).
    """
    dims3 = tuple(int(d) for d in dims) + (1,) * (3 - len(dims))
    ndim = len(dims)
    n = dims3[0] * dims3[1] * dims3[2]
    rng = np.random.default_rng(seed)
    rows, cols, vals = [], [], []
    for off in _offsets(ndim, kind):
        if (off[2], off[1], off[0]) <= (0, 0, 0):
            continue
        i, j = _pairs(dims3, off)
        w = rng.uniform(-1.0, 0.0, size=i.size)
        e_ij = rng.uniform(-delta, delta, size=i.size)
        e_ji = rng.uniform(-delta, delta, size=i.size)
        rows += [i, j]
        cols += [j, i]
        vals += [w * (1 + 1j * e_ij), w * (1 + 1j * e_ji)]
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    diag = np.zeros(n)
    np.add.at(diag, rows, np.abs(vals))
    dvals = diag + margin + 1j * eta
    m = sp.csc_matrix((np.concatenate([vals, dvals]), (np.concatenate([rows, np.arange(n)]),
                                                       np.concatenate([cols, np.arange(n)]))), shape=(n, n))
    m.sum_duplicates()
    m.sort_indices()
    return m.indptr.astype(np.int64), m.indices.astype(np.int32), m.data.astype(np.complex128)


def config_complex(dims=(64, 64), kind: str = "box", seed: int = 0, max_nodes: int = 64,
                   leaf: int = 64) -> Workload:
    """Complex stencil (stencil_csc_complex), nested-dissection order.  The
    library holds a complex matrix in its real form of order 2n, so the
    supernode sizes (max_super, relax) count 2 real columns per node."""
    colptr, rowind, values = stencil_csc_complex(dims, kind, 0.05, seed)
    n = int(np.prod(dims))
    pts = {("star", 2): 5, ("box", 2): 9, ("star", 3): 7, ("box", 3): 27}[(kind, len(dims))]
    return Workload(name="z" + "x".join(str(d) for d in dims), n=n, colptr=colptr, rowind=rowind,
                    values=values, perm=nested_dissection(dims, leaf), max_super=2 * max_nodes,
                    relax=2 * leaf, dims=tuple(dims),
                    desc=f"complex {len(dims)}D {'x'.join(str(d) for d in dims)} {pts}-point shifted stencil, "
                         f"n={n}, supernodes <= {max_nodes} nodes",
                    extra={"complex": True})


def config_z1() -> Workload:
    """Complex counterpart of C1: 2D 256x256 9-point stencil, n = 65536,
    supernodes of at most 128 nodes (256 columns of the real form)."""
    return config_complex((256, 256), "box", 0, 128, 64)


CONFIG_NAMES = ("c0", "c1", "c2", "c3", "c4")


def get_config(name: str):
    return {"c0": config_c0, "c1": config_c1, "c2": config_c2, "c3": config_c3,
            "c4": config_c4, "u1": config_u1, "u4": config_u4, "z1": config_z1}[name]()


# ----------------------------------------------------------------------------
# small test matrices
# ----------------------------------------------------------------------------

def random_sparse(n: int, density: float, seed: int, margin: float = 1.0,
                  symmetric_pattern: bool = False, lower_only: bool = False,
                  upper_only: bool = False):
    """Random sparse matrix with a structurally full diagonal (CSC arrays).

    Off-diagonals are N(0,1) at a Bernoulli(density) pattern; the diagonal is
    the row sum of |off-diagonals| plus ``margin`` times a U[0.5, 1.5] factor.
    """
    rng = np.random.default_rng(seed)
    mask = rng.random((n, n)) < density
    if symmetric_pattern:
        mask = mask | mask.T
    if lower_only:
        mask = np.tril(mask)
    if upper_only:
        mask = np.triu(mask)
    np.fill_diagonal(mask, False)
    dense = np.where(mask, rng.standard_normal((n, n)), 0.0)
    d = np.abs(dense).sum(axis=1) + margin * rng.uniform(0.5, 1.5, size=n)
    dense[np.arange(n), np.arange(n)] = d * np.where(rng.random(n) < 0.5, -1.0, 1.0)
    m = sp.csc_matrix(dense)
    m.sort_indices()
    return (m.indptr.astype(np.int64), m.indices.astype(np.int32),
            m.data.astype(np.float64), dense)


def tridiag_csc(sub, diag, sup):
    """CSC of the tridiagonal matrix with the given sub-, main and super-diagonals."""
    n = len(diag)
    m = sp.diags([np.asarray(sub, float), np.asarray(diag, float), np.asarray(sup, float)],
                 [-1, 0, 1], shape=(n, n), format="csc")
    m.sort_indices()
    return m.indptr.astype(np.int64), m.indices.astype(np.int32), m.data.astype(np.float64)
