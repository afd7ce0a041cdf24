// k_als.hip -- CP-ALS on the GPU (Sec. 2.3, eqs. cp_nls and cp_als), FP64: the
// right-hand sides of the three least-squares subproblems (matricized tensor times
// Khatri-Rao product, as an FP64 MFMA product with one factor followed by an elementwise
// reduction with the other) and their normal matrices (elementwise products of factor
// Grams).  The normal equations are solved by the SPD inverse of k_bdf.hip and an FP64
// MFMA product (k_gemm.hip).
#include <algorithm>

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

// T[b][m] = sum_k U[b][k] Ft[m][k] in FP64: the unfolding times one factor, T [Bn][R].
// A block stages 16 NBT rows of U [Bn][np] in LDS (zeros past np, up to kc = np rounded up
// to 16, and past Bn; an odd number of 16-byte units per row, so the fragment reads meet
// no bank conflicts) and forms those rows of T for every m: its four wavefronts take the
// 16 x 16 tiles (b-tile t % NBT, m-tile t / NBT) for t = w, w + 4, ..., up to four at a
// time.  A wavefront's U fragment of a step is shared by its tiles; the factor fragments
// stream from global memory (the factor stays in L2) two steps ahead.  Lane l feeds row
// l % 16 and the k group l / 16 of a 16-k step, two consecutive k per half-step in both
// operands; accumulator element v of lane l is row b = l / 16 + 4 v and column
// m = l % 16.  Rows of Ft past R are clamped for the loads and not stored; k in
// [np, kc) meets the LDS zeros (the factor rows are finite and the last one has
// zeroed slack past its end).
template <int G>
__device__ __forceinline__ void als_product_round(const double* xs, int kcp, int nsteps, const double* __restrict__ Ft,
                                                  int np, int R, int mt0, int dm, int bt, long long b0, long long Bn,
                                                  double* __restrict__ T) {
    const int lane = threadIdx.x % kWave, g = lane >> 4, c16 = lane & 15;
    size_t off[G];
#pragma unroll
    for (int i = 0; i < G; ++i) {
        const int m = min((mt0 + i * dm) * 16 + c16, R - 1);
        off[i] = (size_t)m * np + 4 * g;
    }
    const double* xrow = xs + (size_t)(bt * 16 + c16) * kcp + 4 * g;
    f64x4 acc[G];
#pragma unroll
    for (int i = 0; i < G; ++i) acc[i] = f64x4{0.0, 0.0, 0.0, 0.0};
    // two-step ring of factor fragments; loads past the last step reload it
    double2 ring[2][G][2];
    auto issue = [&](int slot, int st) {
        st = min(st, nsteps - 1);
#pragma unroll
        for (int i = 0; i < G; ++i)
#pragma unroll
            for (int h = 0; h < 2; ++h) ring[slot][i][h] = *reinterpret_cast<const double2*>(Ft + off[i] + 16 * st + 2 * h);
    };
    auto consume = [&](int slot, int st) {
        double2 a[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) a[h] = *reinterpret_cast<const double2*>(xrow + 16 * st + 2 * h);
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int i = 0; i < G; ++i) {
                acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[h].x, ring[slot][i][h].x, acc[i], 0, 0, 0);
                acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[h].y, ring[slot][i][h].y, acc[i], 0, 0, 0);
            }
    };
    issue(0, 0);
    issue(1, 1);
    int st = 0;
    for (; st + 2 <= nsteps; st += 2) {
        consume(0, st);
        issue(0, st + 2);
        consume(1, st + 1);
        issue(1, st + 3);
    }
    if (st < nsteps) consume(0, st);
#pragma unroll
    for (int i = 0; i < G; ++i) {
        const int m = (mt0 + i * dm) * 16 + c16;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const long long b = b0 + bt * 16 + g + 4 * v;
            if (b < Bn && m < R) T[b * R + m] = acc[i][v];
        }
    }
}

template <int NBT>
__global__ __launch_bounds__(256) void k_als_product(int R, int np, int kc, int kcp, long long Bn,
                                                     const double* __restrict__ U, const double* __restrict__ Ft,
                                                     double* __restrict__ T) {
    extern __shared__ __attribute__((aligned(16))) char smem[];
    double* xs = reinterpret_cast<double*>(smem);
    const long long b0 = (long long)blockIdx.x * (16 * NBT);
    const int vr = kc / 2;      // 16-byte vectors per staged row
    staged_copy<4, double2>(
        16 * NBT * vr,
        [&](int q) {
            const int r = q / vr, k = (q - r * vr) * 2;
            double2 v = {0.0, 0.0};
            if (b0 + r < Bn && k < np) v = *reinterpret_cast<const double2*>(U + (size_t)(b0 + r) * np + k);
            return v;
        },
        [&](int q, const double2& v) {
            const int r = q / vr, k = (q - r * vr) * 2;
            *reinterpret_cast<double2*>(xs + (size_t)r * kcp + k) = v;
        });
    __syncthreads();
    const int w = threadIdx.x / kWave, nmt = (R + 15) / 16, bt = w % NBT, dm = 4 / NBT;
    const int nsteps = kc / 16;
    int mt0 = w / NBT;
    int left = mt0 < nmt ? (nmt - mt0 + dm - 1) / dm : 0;
    // rounds of at most four tiles, as even as possible (13 tiles as 4, 3, 3, 3), so no
    // round is left with a single accumulator chain
    for (int rounds = (left + 3) / 4; rounds > 0; --rounds) {
        const int gsz = (left + rounds - 1) / rounds;
        if (gsz == 4) als_product_round<4>(xs, kcp, nsteps, Ft, np, R, mt0, dm, bt, b0, Bn, T);
        else if (gsz == 3) als_product_round<3>(xs, kcp, nsteps, Ft, np, R, mt0, dm, bt, b0, Bn, T);
        else if (gsz == 2) als_product_round<2>(xs, kcp, nsteps, Ft, np, R, mt0, dm, bt, b0, Bn, T);
        else als_product_round<1>(xs, kcp, nsteps, Ft, np, R, mt0, dm, bt, b0, Bn, T);
        left -= gsz;
        mt0 += gsz * dm;
    }
}

// Each block reserves at least kProductLdsFloor bytes of LDS: two blocks then fill at most
// 128 KB of a compute unit's 160 KB, which leaves room for a block of the SPD inverse
// (k_gj_step, 35 KB) that runs beside the product on a side stream; at three blocks per
// compute unit the inverse's panels wait for product blocks to retire (measured at
// N = 200, R = 400: 4-7% slower sweeps, and the product itself no faster).
constexpr size_t kProductLdsFloor = 57344;

AlsProductPlan als_product_plan(int np, int lds_cap) {
    AlsProductPlan pl{};
    pl.kc = (np + 15) / 16 * 16;
    int units = pl.kc / 2;                  // 16-byte units of a staged row
    if (units % 2 == 0) units += 1;
    pl.kcp = units * 2;
    for (int nbt = 2; nbt >= 1; --nbt) {
        const size_t lds = (size_t)nbt * 16 * pl.kcp * sizeof(double);
        if (lds <= (size_t)lds_cap) {
            pl.nbt = nbt;
            pl.lds = std::max(lds, std::min(kProductLdsFloor, (size_t)lds_cap));
            break;
        }
    }
    if (pl.nbt == 2)
        pl.ok = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_als_product<2>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)pl.lds) == hipSuccess;
    else if (pl.nbt == 1)
        pl.ok = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_als_product<1>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)pl.lds) == hipSuccess;
    if (!pl.ok) (void)hipGetLastError();    // a refused allowance is not the caller's error
    return pl;
}

void launch_als_product(const AlsProductPlan& pl, int R, int np, long long Bn, const double* U, const double* Ft,
                        double* T, hipStream_t s) {
    const unsigned blocks = (unsigned)((Bn + 16 * pl.nbt - 1) / (16 * pl.nbt));
    if (pl.nbt == 2)
        hipLaunchKernelGGL(k_als_product<2>, dim3(blocks), dim3(256), pl.lds, s, R, np, pl.kc, pl.kcp, Bn, U, Ft, T);
    else
        hipLaunchKernelGGL(k_als_product<1>, dim3(blocks), dim3(256), pl.lds, s, R, np, pl.kc, pl.kcp, Bn, U, Ft, T);
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

// V = (Fa^T Fa) .* (Fb^T Fb) [R][R] on FP64 MFMA: a block per 32 x 32 tile of V, sixteen
// waves: wave w forms quarter w % 4 (rows r0, columns c0) over the factor rows of issues
// s = w / 4, w / 4 + 4, ... (four parts of the contracted range, added in LDS in a fixed
// order).  Lane l feeds row / column l % 16 and factor row k = 4 s + l / 16 of issue s, its
// operands read straight from the factors (16 consecutive values of one factor row per 16
// lanes); rows past N give zeros and columns past R are clamped for the loads and not
// stored.
constexpr int kGramParts = 4;
__global__ __launch_bounds__(256 * kGramParts) void k_gram_hadamard(int N, int R, const double* __restrict__ Fa,
                                                                   const double* __restrict__ Fb,
                                                                   double* __restrict__ V) {
    __shared__ f64x4 part[kGramParts - 1][4][kWave][2];
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave, qd = w % 4, kp = w / 4;
    const int r0 = blockIdx.y * 32 + (qd / 2) * 16, c0 = blockIdx.x * 32 + (qd % 2) * 16;
    const int rr = min(r0 + lane % 16, R - 1), cc = min(c0 + lane % 16, R - 1);
    f64x4 ga = {0.0, 0.0, 0.0, 0.0}, gb = {0.0, 0.0, 0.0, 0.0};
    const int steps = (N + 3) / 4;
#pragma unroll 4
    for (int st = kp; st < steps; st += kGramParts) {
        const int k = 4 * st + lane / 16;
        const bool in = k < N;
        const size_t o = (size_t)(in ? k : 0) * R;
        const double ar = in ? Fa[o + rr] : 0.0, ac = in ? Fa[o + cc] : 0.0;
        const double br = in ? Fb[o + rr] : 0.0, bc = in ? Fb[o + cc] : 0.0;
        ga = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, ac, ga, 0, 0, 0);
        gb = __builtin_amdgcn_mfma_f64_16x16x4f64(br, bc, gb, 0, 0, 0);
    }
    if (kp > 0) {
        part[kp - 1][qd][lane][0] = ga;
        part[kp - 1][qd][lane][1] = gb;
    }
    __syncthreads();
    if (kp > 0) return;
#pragma unroll
    for (int q = 0; q < kGramParts - 1; ++q) {
        ga += part[q][qd][lane][0];
        gb += part[q][qd][lane][1];
    }
    // accumulator element v of lane l: row l / 16 + 4 v, column l % 16
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int r = r0 + lane / 16 + 4 * v, c = c0 + lane % 16;
        if (r < R && c < R) V[(size_t)r * R + c] = ga[v] * gb[v];
    }
}

void launch_gram_hadamard(int N, int R, const double* Fa, const double* Fb, double* V, hipStream_t s) {
    const unsigned t = (unsigned)((R + 31) / 32);
    hipLaunchKernelGGL(k_gram_hadamard, dim3(t, t), dim3(256 * kGramParts), 0, s, N, R, Fa, Fb, V);
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
// Vt = S^T V S [P][P] from V [R][R], and Mt = M S [npad][ldt] from M [N][ldm]; a NULL V
// or M skips its part (the inverse of Vt can then start before M exists).
__global__ void k_skew_tie(int N, int P, const double* __restrict__ V, double* __restrict__ Vt,
                           const double* __restrict__ M, int ldm, double* __restrict__ Mt, int ldt) {
    const int row = blockIdx.y, p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const int R = 2 * P;
    if (row < P && V) {
        const double* v0 = V + (size_t)row * R;
        const double* v1 = V + (size_t)(P + row) * R;
        Vt[(size_t)row * P + p] = (v0[p] + v0[P + p]) + (v1[p] + v1[P + p]);
    }
    if (row < N && M) Mt[(size_t)row * ldt + p] = M[(size_t)row * ldm + p] + M[(size_t)row * ldm + P + p];
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
