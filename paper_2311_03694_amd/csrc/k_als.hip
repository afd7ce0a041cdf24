// k_als.hip -- CP-ALS on the GPU (Sec. 2.3, eqs. cp_nls and cp_als), FP64: the
// right-hand sides of the three least-squares subproblems (matricized tensor times
// Khatri-Rao product) and their normal matrices (elementwise products of factor Grams).
// The normal equations are solved by the SPD inverse of k_bdf.hip and an FP64 MFMA
// product (k_gemm.hip).
#include "als.h"
#include "kcommon.h"

namespace rom {

// One block per (output row p, 256 columns r): thread r walks q and t; the tensor entry
// is the same for the whole block (a broadcast load), the factor rows are coalesced
// along r.  2 N^2 flops per output entry.
__global__ __launch_bounds__(256) void k_mttkrp(int mode, int N, int R, const double* __restrict__ C,
                                                const double* __restrict__ Fq, const double* __restrict__ Ft,
                                                double* __restrict__ M, int ldm) {
    const int p = blockIdx.y, r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    const size_t NN = (size_t)N * N;
    // X(p, q, t) = C[base + q sq + t st]
    size_t base, sq, st;
    if (mode == 0) {
        base = (size_t)p * NN; sq = N; st = 1;           // C[p][q][t]
    } else if (mode == 1) {
        base = (size_t)p * N; sq = NN; st = 1;           // C[q][p][t]
    } else {
        base = (size_t)p; sq = NN; st = N;               // C[q][t][p]
    }
    double acc = 0.0;
    for (int q = 0; q < N; ++q) {
        const double* x = C + base + (size_t)q * sq;
        double s0 = 0.0, s1 = 0.0;
        int t = 0;
        for (; t + 1 < N; t += 2) {
            s0 += x[(size_t)t * st] * Ft[(size_t)t * R + r];
            s1 += x[(size_t)(t + 1) * st] * Ft[(size_t)(t + 1) * R + r];
        }
        if (t < N) s0 += x[(size_t)t * st] * Ft[(size_t)t * R + r];
        acc += Fq[(size_t)q * R + r] * (s0 + s1);
    }
    M[(size_t)p * ldm + r] = acc;
}

void launch_mttkrp(int mode, int N, int R, const double* C, const double* F0, const double* F1, const double* F2,
                   double* M, int ldm, hipStream_t s) {
    const double* Fq = mode == 0 ? F1 : F0;
    const double* Ft = mode == 2 ? F1 : F2;
    hipLaunchKernelGGL(k_mttkrp, dim3((R + 255) / 256, N), dim3(256), 0, s, mode, N, R, C, Fq, Ft, M, ldm);
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
