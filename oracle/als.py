"""CP-ALS for a dense third-order tensor (Sec. 2.3, eqs. cp_nls and cp_als): plain FP64
numpy, test infrastructure only (only the tests and the benchmark's CPU leg use it).

Each sweep solves the three linear least-squares subproblems of eq. cp_als in the
paper's order, each through its normal equations: for the first factor
    A1 (A2^T A2 * A3^T A3) = X_(1) (A3 kr A2),   (X_(1) (A3 kr A2))[i][r] = sum_jk X_ijk A2_jr A3_kr,
and likewise for the second and third factors with the other two fixed (* is the
elementwise product).  No weights or column normalisation: the paper fits
[[A1, A2, A3]] directly, so the CP weights are ones.  The initial factors are the
caller's (the paper does not fix an initialisation).

Parity status: pinned (tests/test_oracle_pins.py: each update equals numpy's lstsq of
the unfolded subproblem, exact factors are a fixed point, the residual never grows).
"""
import numpy as np


def mttkrp(X, F, mode):
    """The right-hand side of subproblem `mode` (0, 1, 2): X contracted with the two
    other factors over their indices, [N][R]."""
    A1, A2, A3 = F
    if mode == 0:
        return np.einsum("ijk,jr,kr->ir", X, A2, A3)
    if mode == 1:
        return np.einsum("ijk,ir,kr->jr", X, A1, A3)
    return np.einsum("ijk,ir,jr->kr", X, A1, A2)


def normal_matrix(F, mode):
    """(F_a^T F_a) * (F_b^T F_b) over the two factors other than `mode`."""
    others = [F[m] for m in range(3) if m != mode]
    return (others[0].T @ others[0]) * (others[1].T @ others[1])


def residual(X, F):
    """||X - [[A1, A2, A3]]||_F / ||X||_F (eq. cp_nls, relative)."""
    K = np.einsum("ir,jr,kr->ijk", *F)
    return float(np.linalg.norm((X - K).ravel()) / np.linalg.norm(np.asarray(X).ravel()))


def cp_als(X, A1, A2, A3, sweeps):
    """`sweeps` ALS sweeps from the given factors; returns ([A1, A2, A3], residuals after
    each sweep)."""
    X = np.asarray(X, dtype=np.float64)
    F = [np.array(A, dtype=np.float64) for A in (A1, A2, A3)]
    res = []
    for _ in range(sweeps):
        for mode in range(3):
            V = normal_matrix(F, mode)
            M = mttkrp(X, F, mode)
            F[mode] = np.linalg.solve(V, M.T).T
        res.append(residual(X, F))
    return F, res
