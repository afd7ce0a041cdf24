// k_bdf.hip -- FP64 parts of the time step and their one-time setup:
//   * the semi-implicit BDFk/EXTk right-hand side and update (eq. nse_d1, identity
//     mass matrix), the energy E = |u|^2/2 per trajectory and level (eq. ene_fluc)
//     and the non-finite health flag;
//   * the Helmholtz operators (beta0_k/dt) I + nu A for k = 1, 2, 3: reciprocals of
//     the diagonal, or for a dense stiffness a Cholesky factorisation, the inverse of
//     the factor by triangular solves, and the explicit SPD inverse;
//   * storage conversions of the operators (round to nearest even).
#include <climits>

#include "als.h"
#include "kbody.h"

namespace rom {

// ============================================================== update kernels

// Grid (nbx, B) for the right-hand side; with DIAG (the update kernel) one more row
// whose block 0 closes the previous level and advances the counter (the rest of that
// row exits at once).
template <class ACC, bool DIAG>
__global__ __launch_bounds__(256) void k_bdf_partials(StepArgs a, const ACC* __restrict__ part,
                                                      int nchunk, int pbstride) {
    if constexpr (DIAG) {
        if ((int)blockIdx.y == a.B) {
            if (blockIdx.x == 0) close_and_advance(a, *a.step, (int)gridDim.x);
            return;
        }
        bdf_partials_body<ACC, true>(a, *a.step, part, nchunk, pbstride, blockIdx.x, blockIdx.y, gridDim.x);
    } else {
        bdf_partials_body<ACC, false>(a, *a.step, part, nchunk, pbstride, blockIdx.x, blockIdx.y, gridDim.x);
    }
}

// ceil(N/4) row blocks plus a last block that closes the previous level and advances
// the counter.
template <bool EVEN>
__global__ __launch_bounds__(256) void k_helm_gemv(StepArgs a) {
    if (blockIdx.x == gridDim.x - 1) {
        close_and_advance(a, *a.step, (int)gridDim.x - 1);
        return;
    }
    helm_gemv_body<EVEN>(a, *a.step, blockIdx.x);
}

// Sums the energy of the newest level if it is still pending (the last level of a
// sequence of steps; the update kernels close every earlier one).  One block per state.
__device__ __forceinline__ void close_body(const StepArgs& a) {
    close_level(a, *a.step);
    __syncthreads();                      // every thread has read closep
    if (threadIdx.x == 0) *a.closep = 0;
}

__global__ __launch_bounds__(256) void k_close(StepArgs a) { close_body(a); }

__global__ __launch_bounds__(256) void k_close_group(const FinJob* __restrict__ jobs) {
    close_body(jobs[blockIdx.x].a);
}

// Batched coefficient copies of u [B][N] (state creation / restart, batched
// rom_nonlinear), padding included: trajectories b >= B and indices i >= N are written
// as zeros, so the copies never depend on what their memory held before (the
// contractions multiply the zero padding of the operators by these entries).
// Grid (ceil(Np/256), Bpad).
__global__ void k_prep_ucv(StepArgs a, const double* __restrict__ u) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x, b = blockIdx.y;
    if (i < a.Np) write_ucv(a, b, i, (b < a.B && i < a.N) ? u[(size_t)b * a.N + i] : 0.0);
}

template <class ACC>
__global__ void k_sum_partials(const ACC* __restrict__ part, int nchunk, int B, int N,
                               double* __restrict__ y, int pbstride) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x, b = blockIdx.y;
    if (i >= N) return;
    double s = 0.0;
    const size_t cs = (size_t)pbstride * N;
    const ACC* pp = part + (size_t)b * N + i;
    int q = 0;
    for (; q + 8 <= nchunk; q += 8) {
        ACC v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = pp[(size_t)(q + e) * cs];
#pragma unroll
        for (int e = 0; e < 8; ++e) s += (double)v[e];
    }
    for (; q < nchunk; ++q) s += (double)pp[(size_t)q * cs];
    y[(size_t)b * N + i] = s;
}

// ============================================================== launchers

void launch_bdf_from_partials(const StepArgs& a, int acc_f64, const void* part, int nchunk,
                              int pb, int diag, hipStream_t s) {
    dim3 grid((a.N + 255) / 256, a.B + (diag ? 1 : 0));
    if (acc_f64) {
        if (diag) hipLaunchKernelGGL((k_bdf_partials<double, true>), grid, dim3(256), 0, s, a, (const double*)part, nchunk, pb);
        else hipLaunchKernelGGL((k_bdf_partials<double, false>), grid, dim3(256), 0, s, a, (const double*)part, nchunk, pb);
    } else {
        if (diag) hipLaunchKernelGGL((k_bdf_partials<float, true>), grid, dim3(256), 0, s, a, (const float*)part, nchunk, pb);
        else hipLaunchKernelGGL((k_bdf_partials<float, false>), grid, dim3(256), 0, s, a, (const float*)part, nchunk, pb);
    }
}

void launch_close(const StepArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_close, dim3(1), dim3(256), 0, s, a);
}

void launch_close_group(const FinJob* jobs_dev, int njobs, hipStream_t s) {
    if (njobs > 0) hipLaunchKernelGGL(k_close_group, dim3((unsigned)njobs), dim3(256), 0, s, jobs_dev);
}


void launch_helm_apply(const StepArgs& a, hipStream_t s) {
    const size_t lds = sizeof(double) * a.N;
    const unsigned blocks = (unsigned)((a.N + 3) / 4 + 1);
    if (a.N % 2 == 0) hipLaunchKernelGGL(k_helm_gemv<true>, dim3(blocks), dim3(256), lds, s, a);
    else hipLaunchKernelGGL(k_helm_gemv<false>, dim3(blocks), dim3(256), lds, s, a);
}

void launch_prep_ucv(const StepArgs& a, const double* u_src, hipStream_t s) {
    hipLaunchKernelGGL(k_prep_ucv, dim3((a.Np + 255) / 256, a.Bpad), dim3(256), 0, s, a, u_src);
}

void launch_sum_partials(int acc_f64, const void* part, int nchunk, int pb, int B, int N,
                         double* y, hipStream_t s) {
    dim3 grid((N + 255) / 256, B);
    if (acc_f64) hipLaunchKernelGGL(k_sum_partials<double>, grid, dim3(256), 0, s, (const double*)part, nchunk, B, N, y, pb);
    else hipLaunchKernelGGL(k_sum_partials<float>, grid, dim3(256), 0, s, (const float*)part, nchunk, B, N, y, pb);
}

// ============================================================== Helmholtz setup

// H = nu A + (beta0/dt) M, M the mass matrix (NULL: the identity).
__global__ void k_build_h(int N, double nu, double diag, const double* __restrict__ A,
                          const double* __restrict__ M, double* __restrict__ H) {
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (size_t)N * N) return;
    const int i = (int)(q / N), m = (int)(q % N);
    H[q] = nu * A[q] + diag * (M ? M[q] : (i == m ? 1.0 : 0.0));
}

// Blocked right-looking Cholesky of an SPD matrix in place: L starts as (the lower
// triangle of) H and ends as its factor, H = L L^T.  Panel after panel of kCholNb
// columns: k_chol_panel factors the panel's diagonal block (already updated by the panels
// before) in LDS and solves the rows below it, L21 = A21 L11^{-T}; k_chol_update subtracts
// L21 L21^T from the trailing lower triangle.  Only the lower triangle is read or written.
constexpr int kCholNb = 32;
constexpr int kCholRows = 256;          // panel rows solved per block (one per thread)

__global__ void k_tril_copy(int n, const double* __restrict__ H, double* __restrict__ L) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (long long)n * n) return;
    const int i = (int)(q / n), m = (int)(q % n);
    if (m <= i) L[q] = H[q];
}

// Load the diagonal block of panel j0 (b x b, already updated by the panels before) into
// D and factor it there (whole block); `report` raises *info on a non-positive pivot.
__device__ void chol_diag_block(int n, int j0, int b, const double* __restrict__ L, double (*D)[kCholNb + 1],
                                int* info, bool report) {
    const int t = threadIdx.x;
    for (int q = t; q < b * b; q += blockDim.x) {
        const int r = q / b, c = q % b;
        D[r][c] = c <= r ? L[(size_t)(j0 + r) * n + j0 + c] : 0.0;
    }
    __syncthreads();
    // column c, then the rank-1 update of the columns after it
    for (int c = 0; c < b; ++c) {
        const double piv = D[c][c];
        __syncthreads();
        const double dcc = sqrt(piv);
        if (t == 0 && report && !(piv > 0.0)) atomicMax(info, 1);
        for (int r = c + 1 + t; r < b; r += blockDim.x) D[r][c] /= dcc;
        __syncthreads();
        if (t == 0) D[c][c] = dcc;
        for (int q = t; q < b * b; q += blockDim.x) {
            const int r = q / b, s2 = q % b;
            if (s2 > c && s2 <= r) D[r][s2] -= D[r][c] * D[s2][c];
        }
        __syncthreads();
    }
}

__device__ void chol_store_diag(int n, int j0, int b, double* __restrict__ L, const double (*D)[kCholNb + 1]) {
    for (int q = threadIdx.x; q < b * b; q += blockDim.x) {
        const int r = q / b, c = q % b;
        if (c <= r) L[(size_t)(j0 + r) * n + j0 + c] = D[r][c];
    }
}

// Panel j0: every block factors the diagonal block for itself (none writes it: other
// blocks may still be reading it) and solves its rows below it, x L11^T = a, by forward
// substitution, one row per thread.  With no rows below (one block) it stores the factor.
__global__ __launch_bounds__(256) void k_chol_panel(int n, int j0, double* __restrict__ L, int* info) {
    __shared__ double D[kCholNb][kCholNb + 1];
    const int b = n - j0 < kCholNb ? n - j0 : kCholNb;
    const int t = threadIdx.x;
    chol_diag_block(n, j0, b, L, D, info, blockIdx.x == 0);
    if (n - j0 - b == 0) {
        chol_store_diag(n, j0, b, L, D);
        return;
    }
    const int i = j0 + b + blockIdx.x * kCholRows + t;
    if (t < kCholRows && i < n) {
        double x[kCholNb];
        double* row = L + (size_t)i * n + j0;
#pragma unroll
        for (int c = 0; c < kCholNb; ++c)
            if (c < b) x[c] = row[c];
#pragma unroll
        for (int c = 0; c < kCholNb; ++c) {
            if (c < b) {
                double v = x[c];
#pragma unroll
                for (int m = 0; m < kCholNb; ++m)
                    if (m < c) v -= x[m] * D[c][m];
                x[c] = v / D[c][c];
            }
        }
#pragma unroll
        for (int c = 0; c < kCholNb; ++c)
            if (c < b) row[c] = x[c];
    }
}

// Trailing update of the lower triangle: L[i][k] -= sum_{m < b} L[i][j0 + m] L[k][j0 + m]
// for j0 + b <= k <= i < n, one 16 x 16 tile per block (tiles on or below the diagonal);
// one more block factors panel j0's diagonal block again and stores it (the panel kernel,
// whose blocks all read it, has finished).
__global__ __launch_bounds__(256) void k_chol_update(int n, int j0, int b, int ntiles, double* __restrict__ L) {
    __shared__ double Pi[16][kCholNb + 1], Pk[16][kCholNb + 1];
    const int q = blockIdx.x;
    if (q == ntiles) {
        __shared__ double D[kCholNb][kCholNb + 1];
        chol_diag_block(n, j0, b, L, D, nullptr, false);
        chol_store_diag(n, j0, b, L, D);
        return;
    }
    // tile (ti, tk), tk <= ti, from the linear block index q = ti (ti + 1) / 2 + tk
    int ti = (int)((sqrt(8.0 * q + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= q) ++ti;
    while (ti * (ti + 1) / 2 > q) --ti;
    const int tk = q - ti * (ti + 1) / 2;
    const int base = j0 + b;
    const int i0 = base + ti * 16, k0 = base + tk * 16;
    const int t = threadIdx.x;
    for (int e = t; e < 16 * kCholNb; e += blockDim.x) {
        const int r = e / kCholNb, m = e % kCholNb;
        Pi[r][m] = (i0 + r < n && m < b) ? L[(size_t)(i0 + r) * n + j0 + m] : 0.0;
        Pk[r][m] = (k0 + r < n && m < b) ? L[(size_t)(k0 + r) * n + j0 + m] : 0.0;
    }
    __syncthreads();
    const int r = t / 16, c = t % 16;
    const int i = i0 + r, k = k0 + c;
    if (i < n && k <= i) {
        double s = 0.0;
#pragma unroll
        for (int m = 0; m < kCholNb; ++m) s += Pi[r][m] * Pk[c][m];
        L[(size_t)i * n + k] -= s;
    }
}

void chol_blocked(int n, const double* H, double* L, int* info, hipStream_t s) {
    const long long nn = (long long)n * n;
    hipLaunchKernelGGL(k_tril_copy, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, n, H, L);
    for (int j0 = 0; j0 < n; j0 += kCholNb) {
        const int b = n - j0 < kCholNb ? n - j0 : kCholNb;
        const int below = n - j0 - b;
        hipLaunchKernelGGL(k_chol_panel, dim3(below > 0 ? (below + kCholRows - 1) / kCholRows : 1), dim3(256), 0, s,
                           n, j0, L, info);
        if (below > 0) {
            const int tiles = (below + 15) / 16, ntiles = tiles * (tiles + 1) / 2;
            hipLaunchKernelGGL(k_chol_update, dim3(ntiles + 1), dim3(256), 0, s, n, j0, b, ntiles, L);
        }
    }
}

// X = L^{-1} column by column (one wavefront per column c, values kept in LDS):
//   X_cc = 1/L_cc,  X_rc = -(sum_{c<=m<r} L_rm X_mc) / L_rr  for r > c.
__global__ __launch_bounds__(64) void k_trinv_col(int N, const double* __restrict__ L,
                                                  double* __restrict__ X) {
    extern __shared__ double x[];
    const int c = blockIdx.x, lane = threadIdx.x;
    for (int r = lane; r < N; r += kWave) x[r] = 0.0;
    __syncthreads();
    for (int r = c; r < N; ++r) {
        const double* Lr = L + (size_t)r * N;
        double s = 0.0;
        for (int m = c + lane; m < r; m += kWave) s += Lr[m] * x[m];
        s = wave_sum(s);
        const double v = ((r == c ? 1.0 : 0.0) - s) / Lr[r];
        __syncthreads();
        if (lane == 0) x[r] = v;
        __syncthreads();
    }
    for (int r = lane; r < N; r += kWave) X[(size_t)r * N + c] = x[r];
}

// Hinv = X^T X (X lower triangular): Hinv_im = sum_{r >= max(i,m)} X_ri X_rm, stored
// with row pitch Np (padding columns stay zero).
__global__ void k_gram(int N, int Np, const double* __restrict__ X, double* __restrict__ Hinv) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x, i = blockIdx.y;
    if (m >= N) return;
    double s = 0.0;
    for (int r = (i > m ? i : m); r < N; ++r) s += X[(size_t)r * N + i] * X[(size_t)r * N + m];
    Hinv[(size_t)i * Np + m] = s;
}

__global__ void k_hdiag(int N, double nu, double inv_dt, const double* __restrict__ A,
                        const double* __restrict__ M, double* __restrict__ hd) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double b0[3] = {1.0, 1.5, 11.0 / 6.0};
    const double mi = M ? M[(size_t)i * N + i] : 1.0;
    for (int k = 0; k < 3; ++k) hd[(size_t)k * N + i] = 1.0 / (b0[k] * inv_dt * mi + nu * A[(size_t)i * N + i]);
}

int helm_setup_dense(int N, int Np, double nu, double dt, const double* A_dev, const double* M_dev,
                     double* hinv_dev, double* work_dev, int* info_dev, hipStream_t s) {
    // work_dev: 3 N^2 doubles (H, L, X)
    double* H = work_dev;
    double* L = work_dev + (size_t)N * N;
    double* X = work_dev + 2 * (size_t)N * N;
    const double b0[3] = {1.0, 1.5, 11.0 / 6.0};
    const size_t nn = (size_t)N * N;
    for (int k = 0; k < 3; ++k) {
        hipLaunchKernelGGL(k_build_h, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, N, nu, b0[k] / dt, A_dev, M_dev, H);
        hipMemsetAsync(L, 0, nn * sizeof(double), s);
        chol_blocked(N, H, L, info_dev, s);
        hipLaunchKernelGGL(k_trinv_col, dim3(N), dim3(64), sizeof(double) * N, s, N, L, X);
        hipLaunchKernelGGL(k_gram, dim3((N + 255) / 256, N), dim3(256), 0, s, N, Np, X,
                           hinv_dev + (size_t)k * N * Np);
    }
    return 0;
}

// Blocked Gauss-Jordan inverse of an SPD matrix (no pivoting: the pivot blocks of an SPD
// matrix are Schur complements of SPD matrices, so SPD themselves).  Panel K (kGjNb columns
// from k0, b of them) maps the matrix out of place:
//   A'_KK = P^-1,  A'_KJ = P^-1 A_KJ,  A'_IK = -A_IK P^-1,  A'_IJ = A_IJ - A_IK P^-1 A_KJ,
// P = A_KK; after every panel the matrix is A^-1.  One kernel per panel, one block per
// 32 x 32 tile of the result.  Every block inverts P itself, by sweeps of the same
// formulas over its 2 x 2 diagonal blocks in registers (thread t holds column t % 32 of
// rows 4 (t / 32) .. +3; the pivot rows and columns go through LDS, one barrier per
// sweep) while its tile operands are in flight; then the block's four waves form the
// tile's 16 x 16 quarters with FP64 MFMA.  The old matrix is only read, so no block waits
// for another.  The block of tile (K, K) raises *info on a pivot block that is not
// positive definite.
constexpr int kGjNb = 32;

namespace {

// acc += A[ra.., 0..31] B[0..31, cb..] for a 16 x 16 quarter (wave-wide; LDS operands of
// pitch kGjNb + 1).  Lane l feeds row / column l % 16 and k group l / 16.
__device__ __forceinline__ void gj_quarter(f64x4& acc, const double (*A)[kGjNb + 1], int ra,
                                           const double (*B)[kGjNb + 1], int cb, double sa) {
    const int lane = threadIdx.x % kWave;
#pragma unroll
    for (int s = 0; s < kGjNb / 4; ++s) {
        const int k = 4 * s + lane / 16;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(sa * A[ra + lane % 16][k], B[k][cb + lane % 16], acc, 0, 0, 0);
    }
}

// 1 / d for a positive normal d: the hardware reciprocal refined by two Newton steps
// (r <- r + r (1 - d r)), within an ulp; five dependent operations where the IEEE division
// takes eleven, on the pivot chain of the sweeps below.
__device__ __forceinline__ double gj_recip(double d) {
    double r = __builtin_amdgcn_rcp(d);
    double e = __builtin_fma(-d, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-d, r, 1.0);
    return __builtin_fma(r, e, r);
}

}  // namespace

__global__ __launch_bounds__(256) void k_gj_step(int n, int k0, const double* __restrict__ src, int sp,
                                                 double* __restrict__ dst, int dp, int* info) {
    __shared__ double Pi[kGjNb][kGjNb + 1], Aik[kGjNb][kGjNb + 1], Akj[kGjNb][kGjNb + 1], Rkj[kGjNb][kGjNb + 1];
    __shared__ __attribute__((aligned(16))) double rowb[2][2][kGjNb], colb[2][2][kGjNb];
    const int b = n - k0 < kGjNb ? n - k0 : kGjNb;
    const int i0 = blockIdx.y * kGjNb, j0 = blockIdx.x * kGjNb;
    const bool ik = i0 == k0, jk = j0 == k0;          // tiles are aligned with the panels
    const int bi = n - i0 < kGjNb ? n - i0 : kGjNb, bj = n - j0 < kGjNb ? n - j0 : kGjNb;
    const int t = threadIdx.x, cc = t % kGjNb, rg = t / kGjNb;
    const int w = t / kWave, lane = t % kWave;
    const int rq = (w / 2) * 16, cq = (w % 2) * 16;    // this wave's quarter of the tile

    // P, extended by the identity beyond b (pivots of 1 with zero rows and columns: their
    // sweeps change nothing, so every block sweeps all kGjNb of them).  The tile operands
    // (zero beyond the tile) stay in registers until the sweeps are done.  Every load is
    // issued (addresses clamped into the matrix) and its value selected afterwards, so the
    // sweeps wait for P's loads alone.
    const int nm = n - 1;
    auto at = [&](int r, int c) { return src[(size_t)(r < nm ? r : nm) * sp + (c < nm ? c : nm)]; };
    double x[4], aik[4], akj[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) x[e] = at(k0 + 4 * rg + e, k0 + cc);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int q = t + e * 256, r = q / kGjNb, c = q % kGjNb;
        aik[e] = at(i0 + r, k0 + c);
        akj[e] = at(k0 + r, j0 + c);
    }
    f64x4 acc;
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] = at(i0 + rq + lane / 16 + 4 * v, j0 + cq + lane % 16);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int r = 4 * rg + e;
        x[e] = (r < b && cc < b) ? x[e] : (r == cc ? 1.0 : 0.0);
    }

    // P -> P^-1 by the same map with 2 x 2 pivot blocks Q (SPD as principal blocks of the
    // Schur complements), pivots c0 = 2s, c1 = 2s + 1: rows c0, c1 become Q^-1 (rows c0, c1),
    // columns c0, c1 become -(columns c0, c1) Q^-1, the pivot block Q^-1, the rest
    // x - (columns c0, c1) Q^-1 (rows c0, c1).  Rows and columns c0, c1 pass through LDS
    // (double buffered: one barrier per pivot block).
    bool bad = false;
#pragma unroll
    for (int st = 0; st < kGjNb / 2; ++st) {
        const int c0 = 2 * st;
        double (*rb)[kGjNb] = rowb[st & 1];
        double (*cb)[kGjNb] = colb[st & 1];
        if (rg == st / 2) {
            rb[0][cc] = x[2 * (st % 2)];
            rb[1][cc] = x[2 * (st % 2) + 1];
        }
        if ((cc & ~1) == c0) {
#pragma unroll
            for (int e = 0; e < 4; ++e) cb[cc - c0][4 * rg + e] = x[e];
        }
        __syncthreads();
        // every LDS read of the sweep at once (one LDS latency per pivot block)
        const double p00 = rb[0][c0], p01 = rb[0][c0 + 1], p10 = rb[1][c0], p11 = rb[1][c0 + 1];
        const double a0 = rb[0][cc], a1 = rb[1][cc];
        double u0[4], u1[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            u0[e] = cb[0][4 * rg + e];
            u1[e] = cb[1][4 * rg + e];
        }
        __builtin_amdgcn_sched_barrier(0);
        const double det = p00 * p11 - p01 * p10;
        bad |= !(p00 > 0.0) || !(det > 0.0);
        const double id = gj_recip(det);
        const double q00 = p11 * id, q01 = -p01 * id, q10 = -p10 * id, q11 = p00 * id;
        const double g0 = q00 * a0 + q01 * a1, g1 = q10 * a0 + q11 * a1;    // (Q^-1 rows)[., cc]
        const bool incol = (cc & ~1) == c0;
        const double qc0 = (cc & 1) ? q01 : q00, qc1 = (cc & 1) ? q11 : q10;  // column cc - c0 of Q^-1
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            double v = x[e] - (u0[e] * g0 + u1[e] * g1);
            v = incol ? -(u0[e] * qc0 + u1[e] * qc1) : v;
            if (e / 2 == st % 2) {
                // rows c0 + e % 2 of the pivot block's row pair
                const double gr = (e % 2) ? g1 : g0;
                const double qr = (e % 2) ? ((cc & 1) ? q11 : q10) : ((cc & 1) ? q01 : q00);
                v = rg == st / 2 ? (incol ? qr : gr) : v;
            }
            x[e] = v;
        }
    }
    if (ik && jk) {
        if (t == 0 && bad) atomicMax(info, 1);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int r = 4 * rg + e;
            if (r < b && cc < b) dst[(size_t)(k0 + r) * dp + k0 + cc] = x[e];
        }
        return;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int q = t + e * 256, r = q / kGjNb, c = q % kGjNb;
        Pi[4 * rg + e][cc] = x[e];
        Aik[r][c] = (!ik && r < bi && c < b) ? aik[e] : 0.0;
        Akj[r][c] = (!jk && r < b && c < bj) ? akj[e] : 0.0;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int r = rq + lane / 16 + 4 * v, c = cq + lane % 16;
        acc[v] = (!ik && !jk && r < bi && c < bj) ? acc[v] : 0.0;
    }
    __syncthreads();

    if (ik) {
        gj_quarter(acc, Pi, rq, Akj, cq, 1.0);                  // P^-1 A_KJ
    } else if (jk) {
        gj_quarter(acc, Aik, rq, Pi, cq, -1.0);                 // -A_IK P^-1
    } else {
        f64x4 rk = {0.0, 0.0, 0.0, 0.0};
        gj_quarter(rk, Pi, rq, Akj, cq, 1.0);                   // R = P^-1 A_KJ
#pragma unroll
        for (int v = 0; v < 4; ++v) Rkj[rq + lane / 16 + 4 * v][cq + lane % 16] = rk[v];
        __syncthreads();
        gj_quarter(acc, Aik, rq, Rkj, cq, -1.0);                // A_IJ - A_IK R
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int r = rq + lane / 16 + 4 * v, c = cq + lane % 16;
        if (r < bi && c < bj) dst[(size_t)(i0 + r) * dp + j0 + c] = acc[v];
    }
}

void spd_inverse_gj(int n, int np, const double* H, double* L, double* X, double* Hinv, int* info, hipStream_t s) {
    const int nb = (n + kGjNb - 1) / kGjNb;
    const dim3 grid((unsigned)nb, (unsigned)nb);
    const double* src = H;
    int sp = n;
    for (int q = 0; q < nb; ++q) {
        const bool last = q == nb - 1;
        double* dst = last ? Hinv : (q % 2 == 0 ? L : X);
        const int dp = last ? np : n;
        hipLaunchKernelGGL(k_gj_step, grid, dim3(256), 0, s, n, q * kGjNb, src, sp, dst, dp, info);
        src = dst;
        sp = dp;
    }
}

void helm_setup_diag(int N, double nu, double dt, const double* A_dev, const double* M_dev, double* hdiag_dev,
                     hipStream_t s) {
    hipLaunchKernelGGL(k_hdiag, dim3((N + 255) / 256), dim3(256), 0, s, N, nu, 1.0 / dt, A_dev, M_dev, hdiag_dev);
}

// ============================================================== full form (zeroth mode, mass)

// G [N][2 Np] = [L | M - I] with L = (C1 + C2)[:, 1:], zero padding; fz = (C1 + C2)[:, 0]
// - c0 (the constant of the bracket of eq. nse_d1 at ubar_0 = 1); az = nu a0.  C1, C2 are
// [N][N+1]; a NULL operator counts as zero (M: the identity).
__global__ void k_full_setup(int N, int Np, double nu, const double* __restrict__ M, const double* __restrict__ C1,
                             const double* __restrict__ C2, const double* __restrict__ c0,
                             const double* __restrict__ a0, double* __restrict__ G, double* __restrict__ fz,
                             double* __restrict__ az) {
    const int i = blockIdx.y, m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= 2 * Np) return;
    const size_t w = (size_t)N + 1;
    double v = 0.0;
    if (m < N) {
        v = (C1 ? C1[(size_t)i * w + 1 + m] : 0.0) + (C2 ? C2[(size_t)i * w + 1 + m] : 0.0);
    } else if (m >= Np && m - Np < N) {
        const int j = m - Np;
        v = M ? M[(size_t)i * N + j] - (i == j ? 1.0 : 0.0) : 0.0;
    }
    G[(size_t)i * 2 * Np + m] = v;
    if (m == 0) {
        fz[i] = (C1 ? C1[(size_t)i * w] : 0.0) + (C2 ? C2[(size_t)i * w] : 0.0) - (c0 ? c0[i] : 0.0);
        az[i] = a0 ? nu * a0[i] : 0.0;
    }
}

void full_setup(int N, int Np, double nu, const double* M, const double* C1, const double* C2,
                const double* c0, const double* a0, double* G, double* fz, double* az, hipStream_t s) {
    hipLaunchKernelGGL(k_full_setup, dim3((2 * Np + 255) / 256, N), dim3(256), 0, s, N, Np, nu, M, C1, C2, c0, a0,
                       G, fz, az);
}

// One state: grid (ceil(N/8), B), 512 threads.
__global__ __launch_bounds__(512) void k_full_terms(StepArgs a, const double* __restrict__ G) {
    full_terms_body(a, G, (int)blockIdx.x, (int)blockIdx.y);
}

void launch_full_terms(const StepArgs& a, const double* G, hipStream_t s) {
    hipLaunchKernelGGL(k_full_terms, dim3((a.N + kFullRows - 1) / kFullRows, a.B), dim3(kFullRows * kWave),
                       sizeof(double) * 2 * a.Np, s, a, G);
}

// X[b] = [uhat_b | h_b] of level n for b < B (row pitch 2 Np; entries j >= N and rows
// b >= B are never written and stay zero): the operand of the batched zfull = X G^T,
// which reads G once for the whole batch.
__global__ __launch_bounds__(256) void k_full_x(StepArgs a, double* __restrict__ X) {
    const int b = blockIdx.y, j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= a.N) return;
    const long long n = *a.step;
    const int k = bdf_order(n);
    const BdfCoef c = bdf_coef(k);
    const size_t BN = (size_t)a.B * a.N, off = (size_t)b * a.N;
    double uh = 0.0, h = 0.0;
#pragma unroll
    for (int q = 0; q < 3; ++q)
        if (q < k) {
            const double u = a.uring[(size_t)slot_of(n - q) * BN + off + j];
            uh += c.alpha[q] * u;
            h += (c.beta[q + 1] * a.inv_dt) * u;
        }
    double* xr = X + (size_t)b * 2 * a.Np;
    xr[j] = uh;
    xr[a.Np + j] = h;
}

void launch_full_x(const StepArgs& a, double* X, hipStream_t s) {
    hipLaunchKernelGGL(k_full_x, dim3((a.N + 255) / 256, a.B), dim3(256), 0, s, a, X);
}

// ============================================================== storage conversion

__global__ void k_cvt(int dt, const double* __restrict__ src, void* dst, void* dst_lo, long long rows,
                      int cols, int dpitch) {
    const long long n = rows * cols;
    const long long q0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long p = q0; p < n; p += stride) {
        const long long r = p / cols;
        const long long d = r * dpitch + (p - r * cols);
        const double v = src[p];
        if (dt == DT_F64) {
            reinterpret_cast<double*>(dst)[d] = v;
        } else if (dt == DT_F32) {
            reinterpret_cast<float*>(dst)[d] = (float)v;
        } else {
            const float f = (float)v;
            const unsigned short h = bf16_bits(f);
            reinterpret_cast<unsigned short*>(dst)[d] = h;
            if (dt == DT_BF16X3) reinterpret_cast<unsigned short*>(dst_lo)[d] = bf16_bits(f - bf16_f(h));
        }
    }
}

// CP weights: FP64 for DT_F64, BF16-rounded FP32 values for DT_BF16, FP32 otherwise.
__global__ void k_cvt_lambda(int dt, const double* __restrict__ src, void* dst, long long n) {
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    if (dt == DT_F64) reinterpret_cast<double*>(dst)[p] = src[p];
    else if (dt == DT_BF16) reinterpret_cast<float*>(dst)[p] = bf16_f(bf16_bits((float)src[p]));
    else reinterpret_cast<float*>(dst)[p] = (float)src[p];
}

void launch_cvt_f64_to(int dt, const double* src, void* dst, void* dst_lo, long long rows, int cols,
                       int dpitch, hipStream_t s) {
    long long blocks = (rows * cols + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_cvt, dim3((unsigned)blocks), dim3(256), 0, s, dt, src, dst, dst_lo, rows, cols, dpitch);
}

void launch_cvt_lambda(int dt, const double* src, void* dst, long long n, hipStream_t s) {
    hipLaunchKernelGGL(k_cvt_lambda, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dt, src, dst, n);
}

}  // namespace rom
