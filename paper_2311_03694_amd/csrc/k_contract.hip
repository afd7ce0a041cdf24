// k_contract.hip -- single-trajectory advection contractions.
//
// Dense (Sec. 2, eq. Cu; the 2N^3-flop G-ROM term):  y_i = sum_j u_j sum_k C[i][j][k] u_k.
// The tensor is streamed once per step from HBM with 16-byte non-temporal loads; each
// row i of C is the contiguous N^2-vector over (j, k), split into chunks, one block
// per (i, chunk).  The coefficients sit in LDS in the contraction's number format; a
// thread walks the (j, k) plane with an incremental index (no division in the loop)
// and weights each vector of V consecutive k by u_j.  Blocks write FP32 (FP64) partial
// sums that the BDF update adds in a fixed order, so results are deterministic.
//
// CP (Sec. 3.1, eq. tc_ap):  s = Bf^T u, t = Cf^T u (one pass over [Bf | Cf]^T stored
// [2R][N]), then y = Af (lam .* s .* t) with the Hadamard product formed in LDS by
// every block of the scatter kernel, which also applies the BDF update to its rows.
#include "kstep.h"

namespace rom {

// ============================================================== dense, one trajectory

// LDS image of u for the contraction: `uh` holds the values the products use (FP64,
// FP32, BF16-rounded, or BF16X3 high words), `ul` the BF16X3 low words, `us` the FP32
// j-weight of BF16X3.  For the other formats the j-weight is `uh` itself.
template <int DT>
__device__ __forceinline__ void load_u_lds(const double* __restrict__ u, int N,
                                           typename Store<DT>::Acc* uh, float* ul, float* us) {
    for (int q = threadIdx.x; q < N; q += blockDim.x) {
        const double v = u[q];
        if constexpr (DT == DT_F64) {
            uh[q] = v;
        } else if constexpr (DT == DT_F32) {
            uh[q] = (float)v;
        } else if constexpr (DT == DT_BF16) {
            uh[q] = bf16_f(bf16_bits((float)v));
        } else {
            const float f = (float)v;
            const float h = bf16_f(bf16_bits(f));
            uh[q] = h;
            ul[q] = bf16_f(bf16_bits(f - h));
            us[q] = f;
        }
    }
}

template <int DT, int V, int UNR, int NT>
__global__ __launch_bounds__(NT) void k_dense_gemv(const typename Store<DT>::T* __restrict__ C,
                                                   const unsigned short* __restrict__ Clo, int N,
                                                   const double* __restrict__ u_base,
                                                   const long long* __restrict__ stepp,
                                                   long long slot_stride,
                                                   typename Store<DT>::Acc* __restrict__ part,
                                                   int nchunk, long long chunk_len) {
    typedef typename Store<DT>::T T;
    typedef typename Store<DT>::Acc Acc;
    constexpr int BYTES = V * (int)sizeof(T);
    constexpr bool X3 = (DT == DT_BF16X3);
    extern __shared__ __attribute__((aligned(16))) char smem[];
    Acc* uh = reinterpret_cast<Acc*>(smem);
    float* ul = reinterpret_cast<float*>(uh + N);
    float* us = ul + (X3 ? N : 0);
    __shared__ Acc red[NT / kWave];

    const double* u = u_base + (stepp ? (size_t)slot_of(*stepp) * slot_stride : 0);
    load_u_lds<DT>(u, N, uh, ul, us);
    __syncthreads();
    const Acc* uw = X3 ? reinterpret_cast<const Acc*>(us) : uh;   // j-weights

    const int i = blockIdx.x / nchunk;
    const int c = blockIdx.x - i * nchunk;
    const long long NN = (long long)N * N;
    const long long m0 = (long long)c * chunk_len;
    const long long m1 = (m0 + chunk_len < NN) ? m0 + chunk_len : NN;
    const T* row = C + (size_t)i * NN;
    const unsigned short* rowlo = X3 ? Clo + (size_t)i * NN : nullptr;

    constexpr int STEP = NT * V;
    const int dj = STEP / N, dk = STEP - (STEP / N) * N;
    long long m = m0 + (long long)threadIdx.x * V;
    int j = (int)(m / N), k = (int)(m - (long long)j * N);
    Acc acc = 0;
    for (; m < m1; m += (long long)STEP * UNR) {
        typename RawT<BYTES>::T r[UNR], rl[UNR];
        int jj[UNR], kk[UNR];
#pragma unroll
        for (int q = 0; q < UNR; ++q) {
            const long long mq = m + (long long)q * STEP;
            jj[q] = j;
            kk[q] = k;
            if (mq < m1) {
                r[q] = ld_stream<BYTES>(row + mq);
                if constexpr (X3) rl[q] = ld_stream<BYTES>(rowlo + mq);
            }
            k += dk;
            j += dj;
            if (k >= N) { k -= N; ++j; }
        }
#pragma unroll
        for (int q = 0; q < UNR; ++q) {
            if (m + (long long)q * STEP < m1) {
                Acc cv[V];
                Decode<DT, V>::run(r[q], cv);
                Acc z = 0;
                if constexpr (X3) {
                    float cl[V];
                    Decode<DT, V>::run(rl[q], cl);
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        const float uhv = uh[kk[q] + v];
                        z += cv[v] * uhv;
                        z += cv[v] * ul[kk[q] + v];
                        z += cl[v] * uhv;
                    }
                } else {
#pragma unroll
                    for (int v = 0; v < V; ++v) z += cv[v] * uh[kk[q] + v];
                }
                acc += uw[jj[q]] * z;
            }
        }
    }
    const Acc s = block_sum(acc, red);
    if (threadIdx.x == 0) part[(size_t)c * N + i] = s;
}

static const GemvTile kGemvTiles[] = {
    {256, 4, 8192}, {256, 2, 8192}, {256, 8, 4096}, {256, 4, 16384}, {256, 4, 4096}, {256, 2, 16384},
};

int dense_gemv_variants() { return (int)(sizeof(kGemvTiles) / sizeof(kGemvTiles[0])); }
GemvTile dense_gemv_variant(int idx) {
    if (idx < 0 || idx >= dense_gemv_variants()) idx = 0;
    return kGemvTiles[idx];
}

static int gemv_vec(int dt, int N) {
    const int vmax = dt == DT_F64 ? 2 : dt == DT_F32 ? 4 : 8;
    for (int v = vmax; v > 1; v /= 2)
        if (N % v == 0) return v;
    return 1;
}

static long long gemv_chunk_len(int N, GemvTile t, int V) {
    const long long NN = (long long)N * N;
    long long nchunk = (t.chunk_target + N - 1) / N;
    if (nchunk < 1) nchunk = 1;
    const long long step = (long long)t.threads * V;
    long long len = (NN + nchunk - 1) / nchunk;
    len = ((len + step - 1) / step) * step;
    return len;
}

int dense_gemv_nchunk(int N, GemvTile t) {
    // the same for every dtype: chunk lengths are multiples of threads*V for the
    // dtype's V, and the count is derived from the smallest V = 1 bound
    const long long NN = (long long)N * N;
    long long nchunk = (t.chunk_target + N - 1) / N;
    if (nchunk < 1) nchunk = 1;
    if (nchunk > NN) nchunk = NN;
    return (int)nchunk;
}

template <int DT, int V, int UNR>
static void gemv_go(const void* C, const void* Clo, int N, const double* u, const long long* st,
                    long long ss, void* part, int nchunk, long long len, hipStream_t s) {
    typedef typename Store<DT>::T T;
    typedef typename Store<DT>::Acc Acc;
    const size_t lds = sizeof(Acc) * N + (DT == DT_BF16X3 ? 2 * sizeof(float) * N : 0);
    hipLaunchKernelGGL((k_dense_gemv<DT, V, UNR, 256>), dim3((unsigned)N * nchunk), dim3(256), lds, s,
                       (const T*)C, (const unsigned short*)Clo, N, u, st, ss, (Acc*)part, nchunk, len);
}

template <int DT, int V>
static int gemv_unr(int unr, const void* C, const void* Clo, int N, const double* u,
                    const long long* st, long long ss, void* part, int nchunk, long long len,
                    hipStream_t s) {
    if (unr == 2) gemv_go<DT, V, 2>(C, Clo, N, u, st, ss, part, nchunk, len, s);
    else if (unr == 8) gemv_go<DT, V, 8>(C, Clo, N, u, st, ss, part, nchunk, len, s);
    else gemv_go<DT, V, 4>(C, Clo, N, u, st, ss, part, nchunk, len, s);
    return 0;
}

template <int DT>
static int gemv_dt(int V, int unr, const void* C, const void* Clo, int N, const double* u,
                   const long long* st, long long ss, void* part, int nchunk, long long len,
                   hipStream_t s) {
    constexpr int VMAX = DT == DT_F64 ? 2 : DT == DT_F32 ? 4 : 8;
    if (V == VMAX) return gemv_unr<DT, VMAX>(unr, C, Clo, N, u, st, ss, part, nchunk, len, s);
    if constexpr (VMAX >= 4) {
        if (V == VMAX / 2) return gemv_unr<DT, VMAX / 2>(unr, C, Clo, N, u, st, ss, part, nchunk, len, s);
    }
    if constexpr (VMAX >= 8) {
        if (V == 2) return gemv_unr<DT, 2>(unr, C, Clo, N, u, st, ss, part, nchunk, len, s);
    }
    return gemv_unr<DT, 1>(unr, C, Clo, N, u, st, ss, part, nchunk, len, s);
}

int launch_dense_gemv(int dt, const void* C, const void* Clo, int N, const double* u_base,
                      const long long* stepp, long long slot_stride, void* part, int nchunk,
                      GemvTile t, hipStream_t s) {
    const int V = gemv_vec(dt, N);
    const long long NN = (long long)N * N;
    const long long step = (long long)t.threads * V;
    long long len = (NN + nchunk - 1) / nchunk;
    len = ((len + step - 1) / step) * step;
    // every chunk index < nchunk must start inside the row; shrink nchunk accordingly
    // is the caller's job (dense_gemv_nchunk); here the tail chunks may be empty.
    switch (dt) {
        case DT_F64: return gemv_dt<DT_F64>(V, t.unroll, C, Clo, N, u_base, stepp, slot_stride, part, nchunk, len, s);
        case DT_F32: return gemv_dt<DT_F32>(V, t.unroll, C, Clo, N, u_base, stepp, slot_stride, part, nchunk, len, s);
        case DT_BF16: return gemv_dt<DT_BF16>(V, t.unroll, C, Clo, N, u_base, stepp, slot_stride, part, nchunk, len, s);
        default: return gemv_dt<DT_BF16X3>(V, t.unroll, C, Clo, N, u_base, stepp, slot_stride, part, nchunk, len, s);
    }
}

// ============================================================== CP, one trajectory

// Projections: st[r] = sum_k BCt[r][k] u_k for r < 2R (rows r < R are Bf^T u, rows
// R + r are Cf^T u).  One wavefront per row, four per block.
template <int DT, int V>
__global__ __launch_bounds__(256) void k_cp_proj1(const typename Store<DT>::T* __restrict__ BCt,
                                                  const unsigned short* __restrict__ BCt_lo,
                                                  int N, int R2, const double* __restrict__ u_base,
                                                  const long long* __restrict__ stepp,
                                                  long long slot_stride,
                                                  typename Store<DT>::Acc* __restrict__ st) {
    typedef typename Store<DT>::T T;
    typedef typename Store<DT>::Acc Acc;
    constexpr int BYTES = V * (int)sizeof(T);
    constexpr bool X3 = (DT == DT_BF16X3);
    extern __shared__ __attribute__((aligned(16))) char smem[];
    Acc* uh = reinterpret_cast<Acc*>(smem);
    float* ul = reinterpret_cast<float*>(uh + N);
    float* us = ul + (X3 ? N : 0);
    const double* u = u_base + (stepp ? (size_t)slot_of(*stepp) * slot_stride : 0);
    load_u_lds<DT>(u, N, uh, ul, us);
    __syncthreads();
    const int lane = threadIdx.x % kWave;
    const int r = blockIdx.x * 4 + threadIdx.x / kWave;
    if (r >= R2) return;
    const T* row = BCt + (size_t)r * N;
    const unsigned short* rowlo = X3 ? BCt_lo + (size_t)r * N : nullptr;
    Acc z = 0;
    for (int k = lane * V; k < N; k += kWave * V) {
        Acc cv[V];
        Decode<DT, V>::run(ld_plain<BYTES>(row + k), cv);
        if constexpr (X3) {
            float cl[V];
            Decode<DT, V>::run(ld_plain<BYTES>(rowlo + k), cl);
#pragma unroll
            for (int v = 0; v < V; ++v) {
                z += cv[v] * uh[k + v];
                z += cv[v] * ul[k + v];
                z += cl[v] * uh[k + v];
            }
        } else {
#pragma unroll
            for (int v = 0; v < V; ++v) z += cv[v] * uh[k + v];
        }
    }
    z = wave_sum(z);
    if (lane == 0) st[r] = z;
}

// Hadamard-and-scatter: W_r = lam_r s_r t_r in LDS, then y_i = sum_r Af[i][r] W_r, one
// wavefront per row.  MODE 0 writes y (FP64); MODE 1 applies the diagonal-stiffness
// BDF update with energy and finalize; MODE 2 writes the right-hand side for the
// dense Helmholtz solve.
template <int DT, int V, int MODE>
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
    extern __shared__ __attribute__((aligned(16))) char smem[];
    Acc* W = reinterpret_cast<Acc*>(smem);
    __shared__ double red[4];
    for (int r = threadIdx.x; r < R; r += blockDim.x) W[r] = lam[r] * st[r] * st[R + r];
    __syncthreads();
    const int lane = threadIdx.x % kWave;
    const int i = blockIdx.x * 4 + threadIdx.x / kWave;
    Acc z = 0;
    if (i < N) {
        const T* row = Af + (size_t)i * R;
        const unsigned short* rowlo = X3 ? Af_lo + (size_t)i * R : nullptr;
        for (int r = lane * V; r < R; r += kWave * V) {
            Acc cv[V];
            Decode<DT, V>::run(ld_plain<BYTES>(row + r), cv);
            if constexpr (X3) {
                float cl[V];
                Decode<DT, V>::run(ld_plain<BYTES>(rowlo + r), cl);
#pragma unroll
                for (int v = 0; v < V; ++v) z += (cv[v] + cl[v]) * W[r + v];
            } else {
#pragma unroll
                for (int v = 0; v < V; ++v) z += cv[v] * W[r + v];
            }
        }
        z = wave_sum(z);
    }
    if constexpr (MODE == 0) {
        if (i < N && lane == 0) y_out[i] = (double)z;
    } else {
        const long long n = *a.step;
        const int k = bdf_order(n);
        const BdfCoef c = bdf_coef(k);
        double e = 0.0;
        if (i < N && lane == 0) {
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

template <int DT, int V>
static void proj1_go(const void* BCt, const void* BCt_lo, int N, int R, const double* u,
                     const long long* st, long long ss, void* out, hipStream_t s) {
    typedef typename Store<DT>::T T;
    typedef typename Store<DT>::Acc Acc;
    const size_t lds = sizeof(Acc) * N + (DT == DT_BF16X3 ? 2 * sizeof(float) * N : 0);
    hipLaunchKernelGGL((k_cp_proj1<DT, V>), dim3((2 * R + 3) / 4), dim3(256), lds, s, (const T*)BCt,
                       (const unsigned short*)BCt_lo, N, 2 * R, u, st, ss, (Acc*)out);
}

template <int DT>
static int proj1_dt(int V, const void* BCt, const void* BCt_lo, int N, int R, const double* u,
                    const long long* st, long long ss, void* out, hipStream_t s) {
    constexpr int VMAX = DT == DT_F64 ? 2 : DT == DT_F32 ? 4 : 8;
    if (V == VMAX) proj1_go<DT, VMAX>(BCt, BCt_lo, N, R, u, st, ss, out, s);
    else proj1_go<DT, 1>(BCt, BCt_lo, N, R, u, st, ss, out, s);
    return 0;
}

int launch_cp_proj1(int dt, const void* BCt, const void* BCt_lo, int N, int R,
                    const double* u_base, const long long* stepp, long long slot_stride,
                    void* st, hipStream_t s) {
    const int vmax = dt == DT_F64 ? 2 : dt == DT_F32 ? 4 : 8;
    const int V = (N % vmax == 0) ? vmax : 1;
    switch (dt) {
        case DT_F64: return proj1_dt<DT_F64>(V, BCt, BCt_lo, N, R, u_base, stepp, slot_stride, st, s);
        case DT_F32: return proj1_dt<DT_F32>(V, BCt, BCt_lo, N, R, u_base, stepp, slot_stride, st, s);
        case DT_BF16: return proj1_dt<DT_BF16>(V, BCt, BCt_lo, N, R, u_base, stepp, slot_stride, st, s);
        default: return proj1_dt<DT_BF16X3>(V, BCt, BCt_lo, N, R, u_base, stepp, slot_stride, st, s);
    }
}

template <int DT, int V, int MODE>
static void scat1_go(const void* Af, const void* Af_lo, const void* lam, int N, int R,
                     const void* st, double* y, const StepArgs* sa, hipStream_t s) {
    typedef typename Store<DT>::T T;
    typedef typename Store<DT>::Acc Acc;
    const size_t lds = sizeof(Acc) * R;
    StepArgs a{};
    if (sa) a = *sa;
    hipLaunchKernelGGL((k_cp_scatter1<DT, V, MODE>), dim3((N + 3) / 4), dim3(256), lds, s,
                       (const T*)Af, (const unsigned short*)Af_lo, (const Acc*)lam, N, R,
                       (const Acc*)st, y, a);
}

template <int DT, int V>
static int scat1_mode(int mode, const void* Af, const void* Af_lo, const void* lam, int N, int R,
                      const void* st, double* y, const StepArgs* sa, hipStream_t s) {
    if (mode == 0) scat1_go<DT, V, 0>(Af, Af_lo, lam, N, R, st, y, sa, s);
    else if (mode == 1) scat1_go<DT, V, 1>(Af, Af_lo, lam, N, R, st, y, sa, s);
    else scat1_go<DT, V, 2>(Af, Af_lo, lam, N, R, st, y, sa, s);
    return 0;
}

template <int DT>
static int scat1_dt(int V, int mode, const void* Af, const void* Af_lo, const void* lam, int N,
                    int R, const void* st, double* y, const StepArgs* sa, hipStream_t s) {
    constexpr int VMAX = DT == DT_F64 ? 2 : DT == DT_F32 ? 4 : 8;
    if (V == VMAX) return scat1_mode<DT, VMAX>(mode, Af, Af_lo, lam, N, R, st, y, sa, s);
    return scat1_mode<DT, 1>(mode, Af, Af_lo, lam, N, R, st, y, sa, s);
}

int launch_cp_scatter1(int dt, const void* Af, const void* Af_lo, const void* lam, int N,
                       int R, const void* st, double* y_out, const StepArgs* sa, int mode,
                       hipStream_t s) {
    const int vmax = dt == DT_F64 ? 2 : dt == DT_F32 ? 4 : 8;
    const int V = (R % vmax == 0) ? vmax : 1;
    switch (dt) {
        case DT_F64: return scat1_dt<DT_F64>(V, mode, Af, Af_lo, lam, N, R, st, y_out, sa, s);
        case DT_F32: return scat1_dt<DT_F32>(V, mode, Af, Af_lo, lam, N, R, st, y_out, sa, s);
        case DT_BF16: return scat1_dt<DT_BF16>(V, mode, Af, Af_lo, lam, N, R, st, y_out, sa, s);
        default: return scat1_dt<DT_BF16X3>(V, mode, Af, Af_lo, lam, N, R, st, y_out, sa, s);
    }
}

}  // namespace rom
