// als.h -- CP-ALS launchers (k_als.hip) and the SPD inverse they use (k_bdf.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace rom {

// M[p][r] (row pitch ldm) = sum_{q,t} X(p, q, t) Fq[q][r] Ft[t][r], the right-hand side of
// subproblem `mode` (0, 1, 2) of eq. cp_als, for the dense tensor C [N][N][N] (C[i][j][k])
// and factors F0, F1, F2 [N][R]: mode 0 contracts j and k with F1, F2; mode 1 contracts
// i and k with F0, F2; mode 2 contracts i and j with F0, F1.
void launch_mttkrp(int mode, int N, int R, const double* C, const double* F0, const double* F1, const double* F2,
                   double* M, int ldm, hipStream_t s);
// V[r][s] = (Fa^T Fa)[r][s] * (Fb^T Fb)[r][s], [R][R], factors [N][R].
void launch_gram_hadamard(int N, int R, const double* Fa, const double* Fb, double* V, hipStream_t s);
// Hinv [n][np] = H^{-1} for SPD H [n][n] by Cholesky (L), the inverse factor (X) and its
// Gram product; columns past n of Hinv are left as they are.  *info becomes 1 if a pivot
// is not positive.
void spd_inverse(int n, int np, const double* H, double* L, double* X, double* Hinv, int* info, hipStream_t s);

}  // namespace rom
