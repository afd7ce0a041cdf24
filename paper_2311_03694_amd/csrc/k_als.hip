// k_als.hip -- CP-ALS on the GPU (Sec. 2.3, eqs. cp_nls and cp_als), FP64: the
// right-hand sides of the three least-squares subproblems (matricized tensor times
// Khatri-Rao product, as an FP64 MFMA product with one factor followed by an elementwise
// reduction with the other) and their normal matrices (elementwise products of factor
// Grams).  The normal equations are solved by the SPD inverse of k_bdf.hip and an FP64
// MFMA product (k_gemm.hip).
#include "als.h"
#include "kcommon.h"

namespace rom {

// The right-hand sides go through two unfoldings of the tensor, each a padded copy
// [N^2 (rows, padded to bpad)][np] with zero padding:
//   layout 0: row (i, j), column k = C[i][j][k];   layout 1: row (i, k), column j = C[i][j][k].
// A product with one factor (FP64 MFMA, k_gemm.hip) then gives T[(a, b)][r], and an
// elementwise reduction with a second factor the right-hand side.
__global__ __launch_bounds__(256) void k_als_unfold(int N, int np, int layout, const double* __restrict__ C,
                                                    double* __restrict__ U, long long total) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total) return;
    const long long row = q / np;
    const int c = (int)(q % np);
    double v = 0.0;
    if (c < N) {
        const long long a = row / N, b = row % N;
        v = layout == 0 ? C[row * N + c] : C[(a * N + c) * N + b];
    }
    U[q] = v;
}

void launch_als_unfold(int N, int np, int layout, const double* C, double* U, hipStream_t s) {
    const long long total = (long long)N * N * np;
    hipLaunchKernelGGL(k_als_unfold, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, N, np, layout, C, U,
                       total);
}

// Ft [R][np] = F^T with zero padding (the product's operand rows).
__global__ __launch_bounds__(256) void k_als_transpose(int N, int R, int np, const double* __restrict__ F,
                                                       double* __restrict__ Ft) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (long long)R * np) return;
    const int m = (int)(q / np), k = (int)(q % np);
    Ft[q] = k < N ? F[(size_t)k * R + m] : 0.0;
}

void launch_als_transpose(int N, int R, int np, const double* F, double* Ft, hipStream_t s) {
    const long long total = (long long)R * np;
    hipLaunchKernelGGL(k_als_transpose, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, N, R, np, F, Ft);
}

// M[p][r] (pitch ldm) = sum_q T[row(p, q)][r] F[q][r], row = p N + q (first index
// kept) or q N + p (second index kept); thread r, block row p.
__global__ __launch_bounds__(256) void k_als_reduce(int N, int R, int keep_first, const double* __restrict__ T,
                                                    const double* __restrict__ F, double* __restrict__ M, int ldm) {
    const int p = blockIdx.y, r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    double a0 = 0.0, a1 = 0.0;
    int q = 0;
    for (; q + 1 < N; q += 2) {
        const size_t r0 = keep_first ? (size_t)p * N + q : (size_t)q * N + p;
        const size_t r1 = keep_first ? (size_t)p * N + q + 1 : (size_t)(q + 1) * N + p;
        a0 += T[r0 * R + r] * F[(size_t)q * R + r];
        a1 += T[r1 * R + r] * F[(size_t)(q + 1) * R + r];
    }
    if (q < N) {
        const size_t r0 = keep_first ? (size_t)p * N + q : (size_t)q * N + p;
        a0 += T[r0 * R + r] * F[(size_t)q * R + r];
    }
    M[(size_t)p * ldm + r] = a0 + a1;
}

void launch_als_reduce(int N, int R, int keep_first, const double* T, const double* F, double* M, int ldm,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_als_reduce, dim3((R + 255) / 256, N), dim3(256), 0, s, N, R, keep_first, T, F, M, ldm);
}

// Block row r, thread column s: both Gram entries over the N factor rows.
__global__ __launch_bounds__(256) void k_gram_hadamard(int N, int R, const double* __restrict__ Fa,
                                                       const double* __restrict__ Fb, double* __restrict__ V) {
    const int r = blockIdx.y, c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= R) return;
    double ga = 0.0, gb = 0.0;
    for (int i = 0; i < N; ++i) {
        const size_t o = (size_t)i * R;
        ga += Fa[o + r] * Fa[o + c];
        gb += Fb[o + r] * Fb[o + c];
    }
    V[(size_t)r * R + c] = ga * gb;
}

void launch_gram_hadamard(int N, int R, const double* Fa, const double* Fb, double* V, hipStream_t s) {
    hipLaunchKernelGGL(k_gram_hadamard, dim3((R + 255) / 256, R), dim3(256), 0, s, N, R, Fa, Fb, V);
}

}  // namespace rom
