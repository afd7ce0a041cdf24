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
# The energy E = |u|^2 / 2 has the relative error dE/E = 2 u.du / |u|^2 <= 2 |du| / |u| to
# first order, so a trajectory within TRAJ_TOL of the oracle has its energies within twice it.
ENERGY_TOL = {k: 2.0 * v for k, v in TRAJ_TOL.items()}
EVAL_TOL = {"fp64": 1e-12, "fp32": 1e-5, "bf16x3": 1e-5, "bf16": 1e-5}

U32 = 2.0 ** -24
U64 = 2.0 ** -53
# relative perturbation of one product c*u_j*u_k by the operand formats (worst case):
#  fp32: three FP32 roundings; bf16x3: the split x = hi + lo + O(2^-16 x) of each
#  operand and the dropped lo*lo term (2^-16), plus the FP32 roundings; bf16 against
#  BF16-rounded operands: none; fp64: none.
EPS_OP = {"fp64": 0.0, "fp32": 3 * U32, "bf16": 0.0, "bf16x3": 3 * 2.0 ** -16 + 3 * U32}
U_ACC = {"fp64": U64, "fp32": U32, "bf16": U32, "bf16x3": U32}


def cond_traj_bar(cond_h: float, level: int) -> float:
    """Relative bar for FP64 level `level` of a trajectory whose Helmholtz matrix has
    condition number cond_h: each backward-stable FP64 solve carries a forward error of
    order cond_h * u64, and the errors of the levels add along a decaying trajectory, so
    level m may differ from another FP64 solver's by up to m * cond_h * u64 (a rounding-
    level perturbation of the stiffness alone moves the oracle by about a fifth of that)."""
    return max(TRAJ_TOL["fp64"], level * cond_h * 2.0 ** -53)


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


# ----------------------------------------------------------------------------- per-row bounds
#
# Elementwise bounds |y_i - y_ref_i| <= g * Y_i, Y_i the sum of the magnitudes of the terms
# of row i (dense: sum_jk |C_ijk| |u_j| |u_k|; CP: sum_r |A_ir| |lam_r| S_r T_r with
# S = |B|^T |u|, T = |C|^T |u|).  g counts, worst case, every rounding a term passes through
# in the kernels' arithmetic (conversions of operands into the format, products, the
# BF16X3 split residual and dropped lo*lo product), plus the probabilistic accumulation
# bound LAM sqrt(n) u of Higham and Mary (SIAM J. Sci. Comput. 41, 2019) for each n-term
# sum.  Unit roundoffs: FP64 2^-53, FP32 2^-24, BF16 2^-8 (8-bit significand); the
# BF16X3 residual x - hi - lo of an FP32 value is at most 2^-16 |x|.
LAM = 4.0
U_BF16 = 2.0 ** -8
U_SPLIT = 2.0 ** -16


def _acc(dt, n):
    return LAM * np.sqrt(float(n)) * U_ACC[dt]


def g_dense(dt, N, rounded=False):
    """Relative per-row bound of the dense contraction y_i = sum_j u_j sum_k C_ijk u_k
    against the exact operator (rounded=True, BF16 only: against the oracle evaluated on
    BF16-rounded C and u, where the products are exact)."""
    acc = _acc(dt, N * N)
    if dt == "fp64":
        return 2 * U64 + acc
    if dt == "fp32":
        return 5 * U32 + acc                      # C, u_j, u_k to FP32; two products
    if dt == "bf16":
        if rounded:
            return 2 * U32 + acc                  # the u_j weight product, the dot accumulation
        return (1 + U_BF16 + U32) ** 3 - 1 + 2 * U32 + acc
    return 3 * U_SPLIT + 5 * U32 + acc            # bf16x3: two residuals, lo*lo, FP32 steps


def _cp_eps(dt, N, R, rounded=False):
    """(e_s, e_w, e_y): relative error of one projection against its magnitude S (or T),
    of w = lam s t beyond the projections, and of the scatter against |A| |w|."""
    aN, aR = _acc(dt, N), _acc(dt, R)
    if dt == "fp64":
        return U64 + aN, 2 * U64, U64 + aR
    if dt == "fp32":
        return 3 * U32 + aN, 3 * U32, 2 * U32 + aR            # B, u to FP32 + product; lam + 2 products; A + product
    if dt == "bf16":
        if rounded:
            return aN, 2 * U32, U32 + aR                        # exact products of the rounded operands
        ub = U_BF16 + U32                                       # FP64 -> FP32 -> BF16
        return 2 * ub + aN, ub + 2 * U32, ub + U32 + aR
    return 3 * U_SPLIT + 2 * U32 + aN, 3 * U32, U_SPLIT + 3 * U32 + aR   # bf16x3


def bound_cp(dt, lam, Af, Bf, Cf, u, S=None, T=None, rounded=False):
    """Per-row bound of the CP contraction y = A (lam . s . t), s = B^T u, t = C^T u:
    each projection is off by at most e_s S (S = |B|^T |u| unless given, e.g. |M_k| |rhs|
    for projections formed from the right-hand side), so
      |dw_r| <= |lam_r| (e_s S_r |t_r| + e_s |s_r| T_r + e_s^2 S_r T_r) + e_w |lam_r s_r t_r|,
      |dy_i| <= sum_r |A_ir| |dw_r| + e_y sum_r |A_ir| |w_r|,
    with the exact s, t, w in FP64."""
    N, R = Af.shape
    s = Bf.T @ u
    t = Cf.T @ u
    au = np.abs(u)
    S = np.abs(Bf).T @ au if S is None else S
    T = np.abs(Cf).T @ au if T is None else T
    es, ew, ey = _cp_eps(dt, N, R, rounded)
    al = np.abs(lam)
    w = al * np.abs(s * t)
    dw = al * (es * S * np.abs(t) + es * np.abs(s) * T + es * es * S * T) + ew * w
    aA = np.abs(Af)
    return aA @ dw + ey * (aA @ w)


def bound_dense(dt, C, u, rounded=False):
    """g_dense times the row magnitudes sum_jk |C_ijk| |u_j| |u_k|."""
    return g_dense(dt, C.shape[0], rounded) * mag_dense(C, u)


def mag_dense(C, u):
    au = np.abs(u)
    return np.einsum("ijk,j,k->i", np.abs(C), au, au)


def elem_violations(y, y_ref, bound):
    """Indices of rows outside the bound (an empty array means the check passes)."""
    d = np.abs(np.asarray(y, dtype=np.float64) - np.asarray(y_ref, dtype=np.float64))
    return np.nonzero(~(d <= bound))[0]


def check_elem(y, y_ref, bound, what=""):
    bad = elem_violations(y, y_ref, bound)
    if bad.size:
        d = np.abs(np.asarray(y) - np.asarray(y_ref))
        q = bad[np.argmax(d[bad] / np.maximum(bound[bad], 1e-300))]
        raise AssertionError(f"{what}: {bad.size} rows outside the elementwise bound; worst row {q}: "
                             f"|dy| = {d[q]:.3e}, bound {bound[q]:.3e}")
