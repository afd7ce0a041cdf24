// als.h -- CP-ALS launchers (k_als.hip) and the SPD inverse they use (k_bdf.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "rom_dev.h"

namespace rom {

// Unfolding of C [N][N][N] into U [N^2][np] (zero padding past column N): layout 0 rows
// (i, j) and columns k, layout 1 rows (i, k) and columns j.
void launch_als_unfold(int N, int np, int layout, const double* C, double* U, hipStream_t s);
// Ft [R][np] = F^T for F [N][R], zero padding.
void launch_als_transpose(int N, int R, int np, const double* F, double* Ft, hipStream_t s);
// T [Bn][R] = U Ft^T in FP64 for U [Bn][np] and Ft [R][np] (np a multiple of 8, Ft with at
// least 8 readable elements past its end): the plan stages 32 (else 16) rows of U per block
// in at most lds_cap bytes of LDS; ok is false when neither fits or the allowance is refused.
struct AlsProductPlan {
    int kc, kcp, nbt;
    size_t lds;
    bool ok;
};
AlsProductPlan als_product_plan(int np, int lds_cap);
void launch_als_product(const AlsProductPlan& pl, int R, int np, long long Bn, const double* U, const double* Ft,
                        double* T, hipStream_t s);
// M[p][r] (pitch ldm) = sum_q T[row][r] F[q][r] with row = p N + q (keep_first) or q N + p.
void launch_als_reduce(int N, int R, int keep_first, const double* T, const double* F, double* M, int ldm,
                       hipStream_t s);
// V[r][s] = (Fa^T Fa)[r][s] * (Fb^T Fb)[r][s], [R][R], factors [N][R].
void launch_gram_hadamard(int N, int R, const double* Fa, const double* Fb, double* V, hipStream_t s);
// ALS-skew (Sec. 3.3): A1 = [A11 A12], A2 = [B1 B1], A3 = [A12 -A11] ([N][2P]) from the
// blocks [N][P]; the tied normal equations Vt = S^T V S [P][P], Mt = M S (S = [I; I]; a
// NULL V or M skips that part); B1
// and A2 from the tied solve Y; the momentum update of A1 from the subiteration's solution
// Y, with the blocks and A3 tied again.
void launch_skew_assemble(int N, int P, const double* A11, const double* A12, const double* B1, double* A1,
                          double* A2, double* A3, hipStream_t s);
void launch_skew_tie(int N, int P, const double* V, double* Vt, const double* M, int ldm, double* Mt, int ldt,
                     hipStream_t s);
void launch_skew_set_b(int N, int P, const double* Y, int ldy, double* B1, double* A2, hipStream_t s);
void launch_skew_momentum(int N, int P, double mom, const double* Y, int ldy, double* A1, double* A3, double* A11,
                          double* A12, hipStream_t s);
// launch_gemm_f64 (Y[b][m] = sum_k A[m][k] X[b][k]) storing only the first `rows` of the
// Bpad rows b of Y, so that Y can be an unpadded [rows][M] array (the ALS factor updates).
void launch_gemm_f64_rows(const GemmPlan& pl, const double* A, long long lda, const double* X, long long ldx,
                          double* Y, int M, int K, int Bpad, int rows, hipStream_t s);
// Hinv [n][np] = H^{-1} for SPD H [n][n] by blocked Gauss-Jordan sweeps, one kernel per
// 32-column panel, with L and X as the two buffers the panels alternate between (each
// n x n); columns past n of Hinv are left as they are.  *info becomes 1 if a pivot is not
// positive.
void spd_inverse_gj(int n, int np, const double* H, double* L, double* X, double* Hinv, int* info, hipStream_t s);

}  // namespace rom
