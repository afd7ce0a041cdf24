"""Shared test utilities: error measures and the tolerances of each number format."""
import numpy as np

# Relative-error bars of each contraction format against the FP64 oracle.
#  fp64   : 1e-12 (evaluations and trajectories)
#  fp32   : 1e-5
#  bf16x3 : 1e-5 (split products recover FP32-class accuracy)
#  bf16   : 1e-3 on trajectories against the exact operator; single evaluations are
#           checked against the oracle on BF16-rounded operands (FP32 accumulation only,
#           1e-5) and against the exact operator with the rounding bound of bf16_bound()
TRAJ_TOL = {"fp64": 1e-12, "fp32": 1e-5, "bf16x3": 1e-5, "bf16": 1e-3}
EVAL_TOL = {"fp64": 1e-12, "fp32": 1e-5, "bf16x3": 1e-5, "bf16": 1e-5}


def rel(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def traj_rel(U, Uref) -> float:
    """max over levels of |u^n - u_ref^n| / |u_ref^n| (rows = levels)."""
    U = np.asarray(U).reshape(len(U), -1)
    Uref = np.asarray(Uref).reshape(len(Uref), -1)
    num = np.linalg.norm(U - Uref, axis=1)
    den = np.linalg.norm(Uref, axis=1)
    return float(np.max(num / np.where(den > 0, den, 1.0)))


def bf16_bound(C, u) -> np.ndarray:
    """Elementwise bound on |y_bf16 - y| for a dense tensor: each product
    C_ijk u_j u_k carries three BF16 roundings (relative 2^-9 each) and the FP32
    sum of N^2 terms adds at most N^2 * 2^-24 relative to sum |C_ijk u_j u_k|."""
    N = C.shape[0]
    au = np.abs(u)
    s = np.einsum("ijk,j,k->i", np.abs(C), au, au)
    g = (1 + 2.0 ** -8) ** 3 - 1 + N * N * 2.0 ** -24
    return g * s
