"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This package holds no arithmetic of the selected-inversion method: it only
builds sparse matrices (CSC) with the shapes, stencils and value
distributions of the stencil workloads, plus a geometric nested-dissection
ordering.  Both the oracle and the HIP library consume its output; neither
is imported here.
"""
from .grids import (  # noqa: F401
    Workload,
    nested_dissection,
    stencil_csc,
    config_c0,
    config_c1,
    config_c2,
    config_c3,
    config_c4,
    config_grid,
    config_upwind,
    config_u1,
    config_u4,
    config_complex,
    config_z1,
    stencil_csc_complex,
    get_config,
    random_sparse,
    tridiag_csc,
    CONFIG_NAMES,
)
