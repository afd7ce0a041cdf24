// k_dense1.hip -- dense advection contraction for one trajectory (Sec. 2.2, eq. Cu;
// the 2N^3-flop term of the G-ROM):
//     y_i = sum_j u_j * sum_k C[i][j][k] u_k,
// and, with J slabs of separate weights w, the second product of the SVD-ROM (Sec. 4.4)
//     y_i = sum_r w_r * sum_k V[i][r][k] u_k   (w_r = sigma_r U[:,r]^T u).
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
#include "kbody.h"

namespace rom {

template <int DT, int V, int UNR, int NT>
__global__ __launch_bounds__(NT) void k_dense_gemv(GemvJob jb) {
    dense_gemv_body<DT, V, UNR, NT>(jb, blockIdx.x);
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

static long long chunk_len_of(int dt, int J, int Np, int nchunk, GemvTile t) {
    const int V = dt == DT_F64 ? 2 : dt == DT_F32 ? 4 : 8;
    const long long NN = (long long)J * Np;
    const long long step = (long long)t.threads * V;
    // a multiple of threads*V covering the row in nchunk pieces (trailing pieces may be
    // empty; their blocks write a zero partial)
    long long len = (NN + nchunk - 1) / nchunk;
    return ((len + step - 1) / step) * step;
}

GemvJob make_gemv_job(int dt, const void* C, const void* Clo, int N, int Np, int J, const void* wj,
                      const double* u_base, const long long* stepp, long long slot_stride, void* part, int nchunk,
                      GemvTile t) {
    GemvJob jb{};
    jb.C = C;
    jb.Clo = (const unsigned short*)Clo;
    jb.N = N;
    jb.Np = Np;
    jb.J = J;
    jb.wj = wj;
    jb.u_base = u_base;
    jb.stepp = stepp;
    jb.slot_stride = slot_stride;
    jb.part = part;
    jb.nchunk = nchunk;
    jb.chunk_len = chunk_len_of(dt, J, Np, nchunk, t);
    jb.blk0 = 0;
    jb.nblk = N * nchunk;
    return jb;
}

template <int DT, int UNR>
static void gemv_go(const GemvJob& jb, hipStream_t s) {
    constexpr int V = 16 / (int)sizeof(typename Store<DT>::T);
    const size_t lds = LdsU<DT>::bytes(jb.Np) + (jb.wj ? sizeof(typename Store<DT>::Acc) * (size_t)jb.J : 0);
    hipLaunchKernelGGL((k_dense_gemv<DT, V, UNR, 256>), dim3((unsigned)jb.nblk), dim3(256), lds, s, jb);
}

template <int DT>
static void gemv_dt(int unr, const GemvJob& jb, hipStream_t s) {
    if (unr == 2) gemv_go<DT, 2>(jb, s);
    else if (unr == 8) gemv_go<DT, 8>(jb, s);
    else gemv_go<DT, 4>(jb, s);
}

static void gemv_dispatch(int dt, int unr, const GemvJob& jb, hipStream_t s) {
    switch (dt) {
        case DT_F64: gemv_dt<DT_F64>(unr, jb, s); break;
        case DT_F32: gemv_dt<DT_F32>(unr, jb, s); break;
        case DT_BF16: gemv_dt<DT_BF16>(unr, jb, s); break;
        default: gemv_dt<DT_BF16X3>(unr, jb, s); break;
    }
}

int launch_dense_gemv(int dt, const void* C, const void* Clo, int N, int Np, int J, const void* wj,
                      const double* u_base, const long long* stepp, long long slot_stride, void* part, int nchunk,
                      GemvTile t, hipStream_t s) {
    const GemvJob jb = make_gemv_job(dt, C, Clo, N, Np, J, wj, u_base, stepp, slot_stride, part, nchunk, t);
    gemv_dispatch(dt, t.unroll, jb, s);
    return 0;
}

}  // namespace rom
