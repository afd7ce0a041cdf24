// k_dense1.hip -- dense advection contraction for one trajectory (Sec. 2, eq. Cu;
// the 2N^3-flop term of the G-ROM):
//     y_i = sum_j u_j * sum_k C[i][j][k] u_k.
//
// The tensor is stored [N][N][Np] with the k index padded by zeros to Np, a multiple
// of 8.  It is read exactly once per step, so the kernel is a stream over HBM: each row
// i of C is the contiguous (N*Np)-vector over (j, k), split into chunks with one block
// per (i, chunk).  Lanes take 16-byte non-temporal loads V elements apart, UNR
// loads in flight per lane (the first batch is issued before u is staged in LDS, to
// overlap the two latencies).  A thread walks the (j, k) plane with an incremental
// index (no division in the loop) and weights each V-vector's dot product with u by
// u_j.  BF16 pairs use the packed dot2 instruction.  Blocks write one partial sum each
// (FP32, or FP64 for the FP64 format); the BDF update adds them in a fixed order, so
// results are deterministic.
#include "kdot.h"

namespace rom {

template <int DT, int V, int UNR, int NT>
__global__ __launch_bounds__(NT) void k_dense_gemv(const typename Store<DT>::T* __restrict__ C,
                                                   const unsigned short* __restrict__ Clo, int N,
                                                   int Np, const double* __restrict__ u_base,
                                                   const long long* __restrict__ stepp,
                                                   long long slot_stride,
                                                   typename Store<DT>::Acc* __restrict__ part,
                                                   int nchunk, long long chunk_len) {
    typedef typename Store<DT>::T T;
    typedef typename Store<DT>::Acc Acc;
    typedef typename RawT<V * (int)sizeof(T)>::T Raw;
    constexpr int BYTES = V * (int)sizeof(T);
    constexpr bool X3 = (DT == DT_BF16X3);
    extern __shared__ __attribute__((aligned(16))) char smem[];
    __shared__ Acc red[NT / kWave];
    LdsU<DT> L;
    L.bind(smem, Np);

    const int i = blockIdx.x / nchunk;
    const int c = blockIdx.x - i * nchunk;
    const long long NN = (long long)N * Np;
    const long long m0 = (long long)c * chunk_len;
    const long long m1 = (m0 + chunk_len < NN) ? m0 + chunk_len : NN;
    const T* row = C + (size_t)i * NN;
    const unsigned short* rowlo = X3 ? Clo + (size_t)i * NN : nullptr;

    constexpr int STEP = NT * V;
    const int dj = STEP / Np, dk = STEP - (STEP / Np) * Np;
    long long m = m0 + (long long)threadIdx.x * V;
    int j = (int)(m / Np), k = (int)(m - (long long)j * Np);

    Raw r[UNR], rl[UNR];
    int jj[UNR], kk[UNR];
    auto issue = [&](long long mb) {
#pragma unroll
        for (int q = 0; q < UNR; ++q) {
            const long long mq = mb + (long long)q * STEP;
            jj[q] = j;
            kk[q] = k;
            if (mq < m1) {
                r[q] = ld_stream<BYTES>(row + mq);
                if constexpr (X3) rl[q] = ld_stream<BYTES>(rowlo + mq);
            }
            k += dk;
            j += dj;
            if (k >= Np) { k -= Np; ++j; }
        }
    };

    if (m < m1) issue(m);
    L.fill(u_base + (stepp ? (size_t)slot_of(*stepp) * slot_stride : 0), N, Np);
    __syncthreads();

    Acc acc = 0;
    while (m < m1) {
#pragma unroll
        for (int q = 0; q < UNR; ++q) {
            if (m + (long long)q * STEP < m1) acc += L.uw[jj[q]] * dot_vec<DT, V>(r[q], rl[q], L, kk[q]);
        }
        m += (long long)STEP * UNR;
        if (m < m1) issue(m);
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

// Number of chunks per row: about chunk_target blocks in total.
int dense_gemv_nchunk(int N, GemvTile t) {
    long long nchunk = (t.chunk_target + N - 1) / N;
    if (nchunk < 1) nchunk = 1;
    if (nchunk > 4096) nchunk = 4096;
    return (int)nchunk;
}

template <int DT, int UNR>
static void gemv_go(const void* C, const void* Clo, int N, int Np, const double* u, const long long* st,
                    long long ss, void* part, int nchunk, long long len, hipStream_t s) {
    typedef typename Store<DT>::T T;
    typedef typename Store<DT>::Acc Acc;
    constexpr int V = 16 / (int)sizeof(T);
    const size_t lds = LdsU<DT>::bytes(Np);
    hipLaunchKernelGGL((k_dense_gemv<DT, V, UNR, 256>), dim3((unsigned)N * nchunk), dim3(256), lds, s,
                       (const T*)C, (const unsigned short*)Clo, N, Np, u, st, ss, (Acc*)part, nchunk, len);
}

template <int DT>
static int gemv_dt(int unr, const void* C, const void* Clo, int N, int Np, const double* u,
                   const long long* st, long long ss, void* part, int nchunk, long long len,
                   hipStream_t s) {
    if (unr == 2) gemv_go<DT, 2>(C, Clo, N, Np, u, st, ss, part, nchunk, len, s);
    else if (unr == 8) gemv_go<DT, 8>(C, Clo, N, Np, u, st, ss, part, nchunk, len, s);
    else gemv_go<DT, 4>(C, Clo, N, Np, u, st, ss, part, nchunk, len, s);
    return 0;
}

int launch_dense_gemv(int dt, const void* C, const void* Clo, int N, int Np, const double* u_base,
                      const long long* stepp, long long slot_stride, void* part, int nchunk,
                      GemvTile t, hipStream_t s) {
    const int V = dt == DT_F64 ? 2 : dt == DT_F32 ? 4 : 8;
    const long long NN = (long long)N * Np;
    const long long step = (long long)t.threads * V;
    // chunk length: a multiple of threads*V covering the row in nchunk pieces (the
    // last pieces may be empty; their blocks write a zero partial)
    long long len = (NN + nchunk - 1) / nchunk;
    len = ((len + step - 1) / step) * step;
    switch (dt) {
        case DT_F64: return gemv_dt<DT_F64>(t.unroll, C, Clo, N, Np, u_base, stepp, slot_stride, part, nchunk, len, s);
        case DT_F32: return gemv_dt<DT_F32>(t.unroll, C, Clo, N, Np, u_base, stepp, slot_stride, part, nchunk, len, s);
        case DT_BF16: return gemv_dt<DT_BF16>(t.unroll, C, Clo, N, Np, u_base, stepp, slot_stride, part, nchunk, len, s);
        default: return gemv_dt<DT_BF16X3>(t.unroll, C, Clo, N, Np, u_base, stepp, slot_stride, part, nchunk, len, s);
    }
}

}  // namespace rom
