"""FP64 CPU oracle for the Galerkin ROM hot path (test infrastructure only).

Only tests, the smoke check and the benchmark's CPU-baseline leg import this package.
The product library never calls it.  See rom_oracle.c for the definitions and citations.
"""
from .oracle import (  # noqa: F401
    build,
    lib_path,
    nonlinear_dense,
    nonlinear_dense_rows,
    nonlinear_cp,
    nonlinear_cp_skew,
    nonlinear_svd,
    reconstruct,
    cholesky,
    chol_solve,
    energy,
    explicit_full,
    run,
    round_f32,
    round_bf16,
    split_bf16x3,
    set_threads,
    get_threads,
    threads,
)
from . import als  # noqa: F401,E402
