"""Shared test utilities: error measures and the tolerances of each number format."""
import numpy as np

# Relative-error bars of each contraction format against the FP64 oracle.
#  trajectories (max over levels of |u - u_ref| / |u_ref| and of the energy):
#    fp64 1e-12, fp32 1e-5, bf16x3 1e-5, bf16 1e-3 (all against the exact operator)
#  single evaluations y = C(u)u: |y - y_ref| <= max(EVAL_TOL |y_ref|, derived bound),
#    the bound being the rounding analysis of eval_bound_dense / eval_bound_cp; bf16 is
#    compared with the oracle on BF16-rounded operands (its products are exact, so only
#    the FP32 accumulation remains), the other formats with the exact operator.
TRAJ_TOL = {"fp64": 1e-12, "fp32": 1e-5, "bf16x3": 1e-5, "bf16": 1e-3}
EVAL_TOL = {"fp64": 1e-12, "fp32": 1e-5, "bf16x3": 1e-5, "bf16": 1e-5}

U32 = 2.0 ** -24
U64 = 2.0 ** -53
# relative perturbation of one product c*u_j*u_k by the operand formats (worst case):
#  fp32: three FP32 roundings; bf16x3: the split x = hi + lo + O(2^-18 x) of each
#  operand and the dropped lo*lo term (2^-18), plus the FP32 roundings; bf16 against
#  BF16-rounded operands: none; fp64: none.
EPS_OP = {"fp64": 0.0, "fp32": 3 * U32, "bf16": 0.0, "bf16x3": 3 * 2.0 ** -18 + 3 * U32}
U_ACC = {"fp64": U64, "fp32": U32, "bf16": U32, "bf16x3": U32}


def eval_bound_dense(dt, C, u):
    """Norm-wise bound on |y - y_ref| for the dense contraction: operand error EPS_OP
    plus the probabilistic accumulation bound 4 sqrt(n) u (n = N^2 terms per output,
    Higham's lambda = 4), both relative to |C|(|u| (x) |u|)."""
    N = C.shape[0]
    au = np.abs(u)
    yabs = np.einsum("ijk,j,k->i", np.abs(C), au, au)
    return float(np.linalg.norm(yabs) * (EPS_OP[dt] + 4.0 * N * U_ACC[dt]))


def eval_bound_cp(dt, lam, Af, Bf, Cf, u):
    """Same for the CP contraction: s and t carry the operand and accumulation errors of
    N-term sums, w = lam s t doubles them, the scatter adds an R-term sum."""
    N, R = Af.shape
    au = np.abs(u)
    sa = np.abs(Bf).T @ au
    ta = np.abs(Cf).T @ au
    yabs = np.abs(Af) @ (np.abs(lam) * sa * ta)
    acc = 4.0 * (2.0 * np.sqrt(N) + np.sqrt(R)) * U_ACC[dt]
    return float(np.linalg.norm(yabs) * (3.0 * EPS_OP[dt] + acc))


def check_eval(dt, y, y_ref, bound):
    err = float(np.linalg.norm(np.asarray(y) - np.asarray(y_ref)))
    lim = max(EVAL_TOL[dt] * float(np.linalg.norm(y_ref)), bound)
    assert err <= lim, (dt, err, lim, err / max(float(np.linalg.norm(y_ref)), 1e-300))


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
