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
// kept) or q N + p (second index kept); thread r, block row p.  T is streamed once (N^2 R
// values): eight rows are loaded before they are used, into eight partial sums added in a
// fixed order.
__global__ __launch_bounds__(256) void k_als_reduce(int N, int R, int keep_first, const double* __restrict__ T,
                                                    const double* __restrict__ F, double* __restrict__ M, int ldm) {
    const int p = blockIdx.y, r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    auto row = [&](int q) { return keep_first ? (size_t)p * N + q : (size_t)q * N + p; };
    double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int q = 0;
    for (; q + 8 <= N; q += 8) {
        double t[8], f[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            t[e] = T[row(q + e) * R + r];
            f[e] = F[(size_t)(q + e) * R + r];
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) acc[e] += t[e] * f[e];
    }
    for (; q < N; ++q) acc[0] += T[row(q) * R + r] * F[(size_t)q * R + r];
    M[(size_t)p * ldm + r] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
}

void launch_als_reduce(int N, int R, int keep_first, const double* T, const double* F, double* M, int ldm,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_als_reduce, dim3((R + 255) / 256, N), dim3(256), 0, s, N, R, keep_first, T, F, M, ldm);
}

// V = (Fa^T Fa) .* (Fb^T Fb) [R][R] on FP64 MFMA: a block per 32 x 32 tile of V, eight
// waves: wave w forms quarter w % 4 (rows r0, columns c0) over the factor rows of issues
// s = w / 4, w / 4 + 2, ... (two halves of the contracted range, added in LDS).  Lane l
// feeds row / column l % 16 and factor row k = 4 s + l / 16 of issue s, its operands read
// straight from the factors (16 consecutive values of one factor row per 16 lanes); rows
// past N give zeros and columns past R are clamped for the loads and not stored.
__global__ __launch_bounds__(512) void k_gram_hadamard(int N, int R, const double* __restrict__ Fa,
                                                       const double* __restrict__ Fb, double* __restrict__ V) {
    __shared__ f64x4 part[4][kWave][2];
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave, qd = w % 4, half = w / 4;
    const int r0 = blockIdx.y * 32 + (qd / 2) * 16, c0 = blockIdx.x * 32 + (qd % 2) * 16;
    const int rr = min(r0 + lane % 16, R - 1), cc = min(c0 + lane % 16, R - 1);
    f64x4 ga = {0.0, 0.0, 0.0, 0.0}, gb = {0.0, 0.0, 0.0, 0.0};
    const int steps = (N + 3) / 4;
#pragma unroll 8
    for (int st = half; st < steps; st += 2) {
        const int k = 4 * st + lane / 16;
        const bool in = k < N;
        const size_t o = (size_t)(in ? k : 0) * R;
        const double ar = in ? Fa[o + rr] : 0.0, ac = in ? Fa[o + cc] : 0.0;
        const double br = in ? Fb[o + rr] : 0.0, bc = in ? Fb[o + cc] : 0.0;
        ga = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, ac, ga, 0, 0, 0);
        gb = __builtin_amdgcn_mfma_f64_16x16x4f64(br, bc, gb, 0, 0, 0);
    }
    if (half == 1) {
        part[qd][lane][0] = ga;
        part[qd][lane][1] = gb;
    }
    __syncthreads();
    if (half == 1) return;
    ga += part[qd][lane][0];
    gb += part[qd][lane][1];
    // accumulator element v of lane l: row l / 16 + 4 v, column l % 16
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int r = r0 + lane / 16 + 4 * v, c = c0 + lane % 16;
        if (r < R && c < R) V[(size_t)r * R + c] = ga[v] * gb[v];
    }
}

void launch_gram_hadamard(int N, int R, const double* Fa, const double* Fb, double* V, hipStream_t s) {
    const unsigned t = (unsigned)((R + 31) / 32);
    hipLaunchKernelGGL(k_gram_hadamard, dim3(t, t), dim3(512), 0, s, N, R, Fa, Fb, V);
}

// ---------------------------------------------------------------- ALS-skew (Sec. 3.3)
//
// Factors of the skew-symmetry preserving structure (eq. skew_abc_struct) with P column
// pairs, R = 2P: A1 = [A11 A12], A2 = [B1 B1], A3 = [A12 -A11], each [N][R].

// The three full factors from the blocks A11, A12, B1 [N][P].
__global__ void k_skew_assemble(int N, int P, const double* __restrict__ A11, const double* __restrict__ A12,
                                const double* __restrict__ B1, double* __restrict__ A1, double* __restrict__ A2,
                                double* __restrict__ A3) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (long long)N * P) return;
    const int i = (int)(q / P), p = (int)(q % P);
    const size_t o = (size_t)i * 2 * P;
    const double a = A11[q], c = A12[q], b = B1[q];
    A1[o + p] = a;
    A1[o + P + p] = c;
    A2[o + p] = b;
    A2[o + P + p] = b;
    A3[o + p] = c;
    A3[o + P + p] = -a;
}

void launch_skew_assemble(int N, int P, const double* A11, const double* A12, const double* B1, double* A1,
                          double* A2, double* A3, hipStream_t s) {
    const long long n = (long long)N * P;
    hipLaunchKernelGGL(k_skew_assemble, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, N, P, A11, A12, B1, A1,
                       A2, A3);
}

// The normal equations of the tied second factor A2 = B1 S, S = [I; I]:
// Vt = S^T V S [P][P] from V [R][R], and Mt = M S [npad][ldt] from M [N][ldm].
__global__ void k_skew_tie(int N, int P, const double* __restrict__ V, double* __restrict__ Vt,
                           const double* __restrict__ M, int ldm, double* __restrict__ Mt, int ldt) {
    const int row = blockIdx.y, p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const int R = 2 * P;
    if (row < P) {
        const double* v0 = V + (size_t)row * R;
        const double* v1 = V + (size_t)(P + row) * R;
        Vt[(size_t)row * P + p] = (v0[p] + v0[P + p]) + (v1[p] + v1[P + p]);
    }
    if (row < N) Mt[(size_t)row * ldt + p] = M[(size_t)row * ldm + p] + M[(size_t)row * ldm + P + p];
}

void launch_skew_tie(int N, int P, const double* V, double* Vt, const double* M, int ldm, double* Mt, int ldt,
                     hipStream_t s) {
    const int rows = N > P ? N : P;
    hipLaunchKernelGGL(k_skew_tie, dim3((P + 255) / 256, rows), dim3(256), 0, s, N, P, V, Vt, M, ldm, Mt, ldt);
}

// B1 from the tied solve Y [..][ldy] (first P columns), and A2 = [B1 B1].
__global__ void k_skew_set_b(int N, int P, const double* __restrict__ Y, int ldy, double* __restrict__ B1,
                             double* __restrict__ A2) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (long long)N * P) return;
    const int i = (int)(q / P), p = (int)(q % P);
    const double b = Y[(size_t)i * ldy + p];
    B1[q] = b;
    A2[(size_t)i * 2 * P + p] = b;
    A2[(size_t)i * 2 * P + P + p] = b;
}

void launch_skew_set_b(int N, int P, const double* Y, int ldy, double* B1, double* A2, hipStream_t s) {
    const long long n = (long long)N * P;
    hipLaunchKernelGGL(k_skew_set_b, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, N, P, Y, ldy, B1, A2);
}

// Momentum update of the first factor from the subiteration's solution Y [..][ldy]:
// A1 <- mom A1 + (1 - mom) Y, the blocks A11, A12 written out, and A3 = [A12 -A11].
__global__ void k_skew_momentum(int N, int P, double mom, const double* __restrict__ Y, int ldy,
                                double* __restrict__ A1, double* __restrict__ A3, double* __restrict__ A11,
                                double* __restrict__ A12) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (long long)N * P) return;
    const int i = (int)(q / P), p = (int)(q % P);
    const size_t o = (size_t)i * 2 * P;
    const double a = mom * A1[o + p] + (1.0 - mom) * Y[(size_t)i * ldy + p];
    const double c = mom * A1[o + P + p] + (1.0 - mom) * Y[(size_t)i * ldy + P + p];
    A1[o + p] = a;
    A1[o + P + p] = c;
    A3[o + p] = c;
    A3[o + P + p] = -a;
    A11[q] = a;
    A12[q] = c;
}

void launch_skew_momentum(int N, int P, double mom, const double* Y, int ldy, double* A1, double* A3, double* A11,
                          double* A12, hipStream_t s) {
    const long long n = (long long)N * P;
    hipLaunchKernelGGL(k_skew_momentum, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, N, P, mom, Y, ldy, A1, A3,
                       A11, A12);
}

}  // namespace rom
