// als.h -- CP-ALS launchers (k_als.hip) and the SPD inverse they use (k_bdf.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace rom {

// Unfolding of C [N][N][N] into U [N^2][np] (zero padding past column N): layout 0 rows
// (i, j) and columns k, layout 1 rows (i, k) and columns j.
void launch_als_unfold(int N, int np, int layout, const double* C, double* U, hipStream_t s);
// Ft [R][np] = F^T for F [N][R], zero padding.
void launch_als_transpose(int N, int R, int np, const double* F, double* Ft, hipStream_t s);
// M[p][r] (pitch ldm) = sum_q T[row][r] F[q][r] with row = p N + q (keep_first) or q N + p.
void launch_als_reduce(int N, int R, int keep_first, const double* T, const double* F, double* M, int ldm,
                       hipStream_t s);
// V[r][s] = (Fa^T Fa)[r][s] * (Fb^T Fb)[r][s], [R][R], factors [N][R].
void launch_gram_hadamard(int N, int R, const double* Fa, const double* Fb, double* V, hipStream_t s);
// Hinv [n][np] = H^{-1} for SPD H [n][n] by Cholesky (L), the inverse factor (X) and its
// Gram product; columns past n of Hinv are left as they are.  *info becomes 1 if a pivot
// is not positive.
void spd_inverse(int n, int np, const double* H, double* L, double* X, double* Hinv, int* info, hipStream_t s);

}  // namespace rom
