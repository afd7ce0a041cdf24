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


def skew_factors(A11, A12, B1):
    """The three factor matrices of the skew-symmetry preserving CP structure (Sec. 3.3,
    eq. skew_abc_struct): A1 = [A11 A12], A2 = [B1 B1], A3 = [A12 -A11] ([N][2P] each)."""
    return [np.hstack([A11, A12]), np.hstack([B1, B1]), np.hstack([A12, -A11])]


def als_skew(X, A11, A12, B1, sweeps, subiters, momentum=0.5):
    """ALS-skew (Sec. 3.3, eq. cp_als_quad): `sweeps` sweeps from the given blocks
    (A11, A12, B1 [N][P]); returns ((A11, A12, B1), residuals after each sweep).

    Each sweep
      1. updates the second factor as ALS does (Sec. 2.3, eq. cp_als), as the least-squares
         solution with its two halves tied, A2 = [B1 B1] = B1 S with S = [I; I]: through
         the normal equations B1 (S^T V2 S) = X_(2)(A3 kr A1) S, V2 = (A1^T A1) * (A3^T A3)
         (for a tensor skew in positions 1 and 3 the untied solution has equal halves, so
         the two coincide);
      2. runs `subiters` subiterations on the first factor: the least-squares solution
         with the third factor held fixed (eq. cp_als_quad),
             A1_next = X_(1)(A3 kr A2) V1^{-1},  V1 = (A2^T A2) * (A3^T A3),
         then the momentum update A1 <- momentum A1 + (1 - momentum) A1_next, and the third
         factor tied to it again, A3 = [A12 -A11].
    The paper fixes neither the momentum nor the number of subiterations; both are
    arguments (momentum 1/2 averages the iterate and the new solution, as the Babylonian
    square-root iteration the paper likens the scheme to does)."""
    X = np.asarray(X, dtype=np.float64)
    A11 = np.array(A11, dtype=np.float64)
    A12 = np.array(A12, dtype=np.float64)
    B1 = np.array(B1, dtype=np.float64)
    P = A11.shape[1]
    S = np.vstack([np.eye(P), np.eye(P)])
    res = []
    for _ in range(sweeps):
        F = skew_factors(A11, A12, B1)
        V2 = normal_matrix(F, 1)
        M2 = mttkrp(X, F, 1)
        B1 = np.linalg.solve(S.T @ V2 @ S, (M2 @ S).T).T
        for _ in range(subiters):
            F = skew_factors(A11, A12, B1)
            V1 = normal_matrix(F, 0)
            M1 = mttkrp(X, F, 0)
            A1n = np.linalg.solve(V1, M1.T).T
            A1 = momentum * F[0] + (1.0 - momentum) * A1n
            A11, A12 = A1[:, :P].copy(), A1[:, P:].copy()
        res.append(residual(X, skew_factors(A11, A12, B1)))
    return (A11, A12, B1), res
