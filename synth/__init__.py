"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This package only builds inputs (matrices, right-hand sides, random blocks).
It contains no step of the solver: no factorization, no triangular solve, no
Krylov iteration.
"""

from .elasticity import (  # noqa: F401
    WORKLOADS,
    ElasticityProblem,
    build_workload,
    q1_elasticity,
    q1_unit_stiffness,
    body_load,
    traction_loads,
    rigid_body_modes,
    expected_sizes,
    node_blocks,
)
from .small import (  # noqa: F401
    tridiagonal_spd,
    dense_spd,
    dense_to_csr,
    kershaw4,
    laplacian7,
    spectrum_spd,
    banded_spd,
)
