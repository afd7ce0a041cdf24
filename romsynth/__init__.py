"""Seeded synthetic inputs for the Galerkin ROM hot path.

This package only draws random numbers and lays them out as the operators of a
reduced model (stiffness A, advection tensor C or its CP factors, initial
coefficients u0).  It holds none of the time-stepping or contraction
arithmetic; both the FP64 oracle and the HIP path consume what it returns.
"""
from .inputs import (  # noqa: F401
    Problem,
    skew_cp_factors,
    dense_from_skew_cp,
    dense_rough,
    stiffness_diag,
    stiffness_spd,
    stiffness_graded,
    mass_spd,
    zeroth_terms,
    initial_u,
    integer_dense,
    integer_cp_factors,
    integer_u,
    make_config,
    make_problem,
    truncate_cp,
    CONFIGS,
)
