// k_contract.hip -- CP advection contraction for one trajectory.
//
// CP (Sec. 3.1, eq. tc_ap):  s = Bf^T u, t = Cf^T u (one pass over [Bf | Cf]^T stored
// [2Rp][Np]), then y = Af (lam .* s .* t) with the Hadamard product formed in LDS by
// every block of the scatter kernel, which also applies the BDF update to its rows.
// Np and Rp round N and R up to multiples of 8; padding rows and columns hold zeros
// (and zero weights), so they contribute nothing.
#include "kdot.h"
#include "kstep.h"

namespace rom {

// ============================================================== CP, one trajectory

// Projections: st[r] = sum_k BCt[r][k] u_k for r < 2Rp (rows r < Rp are Bf^T u, rows
// Rp + r are Cf^T u).  One wavefront per row, four per block; each lane issues its U
// row loads before u is staged in LDS.
template <int DT, int V, int U>
__global__ __launch_bounds__(256) void k_cp_proj1(const typename Store<DT>::T* __restrict__ BCt,
                                                  const unsigned short* __restrict__ BCt_lo,
                                                  int N, int Np, int R2, const double* __restrict__ u_base,
                                                  const long long* __restrict__ stepp,
                                                  long long slot_stride,
                                                  typename Store<DT>::Acc* __restrict__ st) {
    typedef typename Store<DT>::T T;
    typedef typename Store<DT>::Acc Acc;
    constexpr int BYTES = V * (int)sizeof(T);
    constexpr bool X3 = (DT == DT_BF16X3);
    typedef typename RawT<BYTES>::T Raw;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    LdsU<DT> L;
    L.bind(smem, Np);
    const int lane = threadIdx.x % kWave;
    const int r = blockIdx.x * 4 + threadIdx.x / kWave;
    const bool live = r < R2;
    const T* row = BCt + (size_t)(live ? r : 0) * Np;
    const unsigned short* rowlo = X3 ? BCt_lo + (size_t)(live ? r : 0) * Np : nullptr;
    Raw rv[U], rl[U];
    int k0 = lane * V;
    auto issue = [&](int kb) {
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int k = kb + q * kWave * V;
            if (live && k < Np) {
                rv[q] = ld_plain<BYTES>(row + k);
                if constexpr (X3) rl[q] = ld_plain<BYTES>(rowlo + k);
            }
        }
    };
    issue(k0);
    L.fill(u_base + (stepp ? (size_t)slot_of(*stepp) * slot_stride : 0), N, Np);
    __syncthreads();
    if (!live) return;
    Acc z = 0;
    while (k0 < Np) {
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int k = k0 + q * kWave * V;
            if (k < Np) z += dot_vec<DT, V>(rv[q], rl[q], L, k);
        }
        k0 += kWave * V * U;
        if (k0 < Np) issue(k0);
    }
    z = wave_sum(z);
    if (lane == 0) st[r] = z;
}

// Hadamard-and-scatter: W_r = lam_r s_r t_r in LDS, then y_i = sum_r Af[i][r] W_r, one
// wavefront per row (row loads issued before W is formed).  MODE 0 writes y (FP64);
// MODE 1 applies the diagonal-stiffness BDF update with energy and finalize; MODE 2
// writes the right-hand side for the dense Helmholtz solve.
template <int DT, int V, int U, int MODE>
__global__ __launch_bounds__(256) void k_cp_scatter1(const typename Store<DT>::T* __restrict__ Af,
                                                     const unsigned short* __restrict__ Af_lo,
                                                     const typename Store<DT>::Acc* __restrict__ lam,
                                                     int N, int R,
                                                     const typename Store<DT>::Acc* __restrict__ st,
                                                     double* __restrict__ y_out, StepArgs a) {
    typedef typename Store<DT>::T T;
    typedef typename Store<DT>::Acc Acc;
    constexpr int BYTES = V * (int)sizeof(T);
    constexpr bool X3 = (DT == DT_BF16X3);
    typedef typename RawT<BYTES>::T Raw;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    Acc* W = reinterpret_cast<Acc*>(smem);
    __shared__ double red[4];
    const int lane = threadIdx.x % kWave;
    const int i = blockIdx.x * 4 + threadIdx.x / kWave;
    const bool live = i < N;
    const T* row = Af + (size_t)(live ? i : 0) * R;
    const unsigned short* rowlo = X3 ? Af_lo + (size_t)(live ? i : 0) * R : nullptr;
    Raw rv[U], rl[U];
    int r0 = lane * V;
    auto issue = [&](int rb) {
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int r = rb + q * kWave * V;
            if (live && r < R) {
                rv[q] = ld_plain<BYTES>(row + r);
                if constexpr (X3) rl[q] = ld_plain<BYTES>(rowlo + r);
            }
        }
    };
    issue(r0);
    for (int r = threadIdx.x; r < R; r += blockDim.x) W[r] = lam[r] * st[r] * st[R + r];   // R = Rp here
    __syncthreads();
    Acc z = 0;
    if (live) {
        while (r0 < R) {
#pragma unroll
            for (int q = 0; q < U; ++q) {
                const int r = r0 + q * kWave * V;
                if (r < R) {
                    Acc cv[V];
                    Decode<DT, V>::run(rv[q], cv);
                    if constexpr (X3) {
                        float cl[V];
                        Decode<DT, V>::run(rl[q], cl);
#pragma unroll
                        for (int v = 0; v < V; ++v) z += (cv[v] + cl[v]) * W[r + v];
                    } else {
#pragma unroll
                        for (int v = 0; v < V; ++v) z += cv[v] * W[r + v];
                    }
                }
            }
            r0 += kWave * V * U;
            if (r0 < R) issue(r0);
        }
        z = wave_sum(z);
    }
    if constexpr (MODE == 0) {
        if (live && lane == 0) y_out[i] = (double)z;
    } else {
        const long long n = *a.step;
        const int k = bdf_order(n);
        const BdfCoef c = bdf_coef(k);
        double e = 0.0;
        if (live && lane == 0) {
            const double rhs = bdf_rhs_point(a, n, c, k, 0, i, (double)z);
            if constexpr (MODE == 1) {
                const double un = rhs * a.hdiag[(size_t)(k - 1) * N + i];
                write_level(a, n + 1, 0, i, un);
                e = un * un;
            } else {
                a.rhs[i] = rhs;
            }
        }
        if constexpr (MODE == 1) {
            const double s = block_sum(e, red);
            if (threadIdx.x == 0) a.epart[blockIdx.x] = s;
            finalize_step(a, n, gridDim.x, gridDim.x);
        }
    }
}

template <int DT>
static void proj1_go(const void* BCt, const void* BCt_lo, int N, int Np, int Rp, const double* u,
                     const long long* st, long long ss, void* out, hipStream_t s) {
    typedef typename Store<DT>::T T;
    typedef typename Store<DT>::Acc Acc;
    constexpr int V = 16 / (int)sizeof(T);
    const size_t lds = LdsU<DT>::bytes(Np);
    hipLaunchKernelGGL((k_cp_proj1<DT, V, 4>), dim3((2 * Rp + 3) / 4), dim3(256), lds, s, (const T*)BCt,
                       (const unsigned short*)BCt_lo, N, Np, 2 * Rp, u, st, ss, (Acc*)out);
}

int launch_cp_proj1(int dt, const void* BCt, const void* BCt_lo, int N, int Np, int Rp,
                    const double* u_base, const long long* stepp, long long slot_stride,
                    void* st, hipStream_t s) {
    switch (dt) {
        case DT_F64: proj1_go<DT_F64>(BCt, BCt_lo, N, Np, Rp, u_base, stepp, slot_stride, st, s); break;
        case DT_F32: proj1_go<DT_F32>(BCt, BCt_lo, N, Np, Rp, u_base, stepp, slot_stride, st, s); break;
        case DT_BF16: proj1_go<DT_BF16>(BCt, BCt_lo, N, Np, Rp, u_base, stepp, slot_stride, st, s); break;
        default: proj1_go<DT_BF16X3>(BCt, BCt_lo, N, Np, Rp, u_base, stepp, slot_stride, st, s); break;
    }
    return 0;
}

template <int DT, int MODE>
static void scat1_go(const void* Af, const void* Af_lo, const void* lam, int N, int Rp,
                     const void* st, double* y, const StepArgs* sa, hipStream_t s) {
    typedef typename Store<DT>::T T;
    typedef typename Store<DT>::Acc Acc;
    constexpr int V = 16 / (int)sizeof(T);
    const size_t lds = sizeof(Acc) * Rp;
    StepArgs a{};
    if (sa) a = *sa;
    hipLaunchKernelGGL((k_cp_scatter1<DT, V, 8, MODE>), dim3((N + 3) / 4), dim3(256), lds, s,
                       (const T*)Af, (const unsigned short*)Af_lo, (const Acc*)lam, N, Rp,
                       (const Acc*)st, y, a);
}

template <int DT>
static void scat1_mode(int mode, const void* Af, const void* Af_lo, const void* lam, int N, int Rp,
                       const void* st, double* y, const StepArgs* sa, hipStream_t s) {
    if (mode == 0) scat1_go<DT, 0>(Af, Af_lo, lam, N, Rp, st, y, sa, s);
    else if (mode == 1) scat1_go<DT, 1>(Af, Af_lo, lam, N, Rp, st, y, sa, s);
    else scat1_go<DT, 2>(Af, Af_lo, lam, N, Rp, st, y, sa, s);
}

int launch_cp_scatter1(int dt, const void* Af, const void* Af_lo, const void* lam, int N,
                       int Rp, const void* st, double* y_out, const StepArgs* sa, int mode,
                       hipStream_t s) {
    switch (dt) {
        case DT_F64: scat1_mode<DT_F64>(mode, Af, Af_lo, lam, N, Rp, st, y_out, sa, s); break;
        case DT_F32: scat1_mode<DT_F32>(mode, Af, Af_lo, lam, N, Rp, st, y_out, sa, s); break;
        case DT_BF16: scat1_mode<DT_BF16>(mode, Af, Af_lo, lam, N, Rp, st, y_out, sa, s); break;
        default: scat1_mode<DT_BF16X3>(mode, Af, Af_lo, lam, N, Rp, st, y_out, sa, s); break;
    }
    return 0;
}

}  // namespace rom
