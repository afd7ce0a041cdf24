// k_contract.hip -- CP advection contraction for one trajectory.
//
// CP (Sec. 3.1, eq. tc_ap):  w = lam .* s .* t with s = Bf^T u, t = Cf^T u (one pass
// over [Bf | Cf]^T stored [2Rp][Np]: a wavefront takes rows r and Rp + r and writes w_r;
// factors with skew column pairs, Sec. 3.3, read the pair form instead), then y = Af w,
// with w staged in LDS by every block of the scatter kernel, which also applies the BDF
// update to its rows.  With a dense stiffness the Helmholtz kernel forms the next level's
// w.  The file also holds the first product of the SVD-ROM (Sec. 4.4).
// Np and Rp round N and R up to multiples of 8; padding rows and columns hold zeros
// (and zero weights), so they contribute nothing.
#include "kbody.h"

namespace rom {

// ============================================================== CP, one trajectory

template <int DT, int V, int U>
__global__ __launch_bounds__(256) void k_cp_proj1(Proj1Job jb) {
    cp_proj_any_body<DT, V, U>(jb, blockIdx.x);
}
// MODE 1 (the update kernel) runs one block more than there are row blocks: the last
// one closes the previous level and advances the counter.
template <int DT, int V, int U, int MODE, bool FULL>
__global__ __launch_bounds__(256) void k_cp_scatter1(Scat1Job jb, double* y_out) {
    if constexpr (MODE == 1) {
        if (blockIdx.x == gridDim.x - 1) {
            close_and_advance(jb.a, *jb.a.step, (int)gridDim.x - 1);
            return;
        }
        cp_scatter1_body<DT, V, U, MODE, FULL>(jb, y_out, blockIdx.x, *jb.a.step);
    } else {
        cp_scatter1_body<DT, V, U, MODE, FULL>(jb, y_out, blockIdx.x, MODE == 0 ? 0LL : *jb.a.step);
    }
}
// ============================================================== Helmholtz apply and projections

// One state: nh + np blocks and a last one that closes the previous level and advances
// the counter.
template <int DT, bool EVEN>
__global__ __launch_bounds__(256) void k_helm_proj(HelmJob jb) {
    if (blockIdx.x == gridDim.x - 1) {
        close_and_advance(jb.a, *jb.a.step, jb.nh);
        return;
    }
    helm_proj_body<DT, EVEN>(jb, *jb.a.step, blockIdx.x);
}

// ============================================================== SVD-ROM, one trajectory

// First product of the SVD-ROM, one state (svd_proj_body).
template <int DT, int V, int U>
__global__ __launch_bounds__(256) void k_svd_proj(SvdProj a) {
    svd_proj_body<DT, V, U>(a, (int)blockIdx.x);
}

template <int DT>
static void svd_proj_go(const SvdProj& a, hipStream_t s) {
    constexpr int V = 16 / (int)sizeof(typename Store<DT>::T);
    hipLaunchKernelGGL((k_svd_proj<DT, V, 4>), dim3((unsigned)((a.Rsp + 3) / 4)), dim3(256), LdsU<DT>::bytes(a.Np), s,
                       a);
}

void launch_svd_proj(int dt, const void* Ut, const void* Ut_lo, const void* sigma, int N, int Np, int Rs,
                     const double* u_base, const long long* stepp, long long slot_stride, void* w, hipStream_t s) {
    SvdProj a{};
    a.Ut = Ut;
    a.Ut_lo = (const unsigned short*)Ut_lo;
    a.sigma = sigma;
    a.N = N;
    a.Np = Np;
    a.Rsp = (Rs + 7) / 8 * 8;
    a.u_base = u_base;
    a.stepp = stepp;
    a.slot_stride = slot_stride;
    a.w = w;
    switch (dt) {
        case DT_F64: svd_proj_go<DT_F64>(a, s); break;
        case DT_F32: svd_proj_go<DT_F32>(a, s); break;
        case DT_BF16: svd_proj_go<DT_BF16>(a, s); break;
        default: svd_proj_go<DT_BF16X3>(a, s); break;
    }
}

// ---------------------------------------------------------------- launchers

// LDS of the projection kernels: the image of u, and for the BF16 formats a second one
// of -u (read by the pair form).
template <int DT>
static size_t proj_lds(int Np) {
    return (DT == DT_BF16 || DT == DT_BF16X3 ? 2 : 1) * LdsU<DT>::bytes(Np);
}

template <int DT>
static void proj1_go(const Proj1Job& jb, hipStream_t s) {
    constexpr int V = 16 / (int)sizeof(typename Store<DT>::T);
    hipLaunchKernelGGL((k_cp_proj1<DT, V, 4>), dim3((unsigned)jb.nblk), dim3(256), proj_lds<DT>(jb.Np), s, jb);
}

static void proj1_dispatch(int dt, const Proj1Job& jb, hipStream_t s) {
    switch (dt) {
        case DT_F64: proj1_go<DT_F64>(jb, s); break;
        case DT_F32: proj1_go<DT_F32>(jb, s); break;
        case DT_BF16: proj1_go<DT_BF16>(jb, s); break;
        default: proj1_go<DT_BF16X3>(jb, s); break;
    }
}

// Blocks of the projection kernel: four row pairs of [Bf|Cf]^T, or four column pairs
// of the pair form, per block.
int proj1_blocks(int Rp, SkewPairs sk) { return sk.layout ? (Rp / 2 + 3) / 4 : (Rp + 3) / 4; }

int launch_cp_proj1(int dt, const void* BCt, const void* BCt_lo, const void* lam, int N, int Np, int Rp,
                    SkewPairs sk, const double* u_base, const long long* stepp, long long slot_stride,
                    void* w, hipStream_t s) {
    Proj1Job jb{};
    jb.BCt = BCt;
    jb.BCt_lo = (const unsigned short*)BCt_lo;
    jb.lam = lam;
    jb.N = N;
    jb.Np = Np;
    jb.Rp = Rp;
    jb.layout = sk.layout;
    jb.P = sk.P;
    jb.R = sk.R;
    jb.u_base = u_base;
    jb.stepp = stepp;
    jb.slot_stride = slot_stride;
    jb.w = w;
    jb.nblk = proj1_blocks(Rp, sk);
    proj1_dispatch(dt, jb, s);
    return 0;
}

template <int DT, int MODE>
static void scat1_go(const Scat1Job& jb, double* y, hipStream_t s) {
    typedef typename Store<DT>::Acc Acc;
    constexpr int V = 16 / (int)sizeof(typename Store<DT>::T);
    const dim3 grid((unsigned)jb.nblk + (MODE == 1 ? 1u : 0u));
    const size_t w_lds = sizeof(Acc) * jb.Rp;
    if (MODE != 0 && jb.G) {
        // W, then [uhat; h] (2 Np doubles) 16-byte aligned behind it
        const size_t lds = ((w_lds + 15) & ~(size_t)15) + sizeof(double) * 2 * jb.a.Np;
        hipLaunchKernelGGL((k_cp_scatter1<DT, V, 8, MODE, MODE != 0>), grid, dim3(256), lds, s, jb, y);
    } else {
        hipLaunchKernelGGL((k_cp_scatter1<DT, V, 8, MODE, false>), grid, dim3(256), w_lds, s, jb, y);
    }
}

template <int DT>
static void scat1_mode(int mode, const Scat1Job& jb, double* y, hipStream_t s) {
    if (mode == 0) scat1_go<DT, 0>(jb, y, s);
    else if (mode == 1) scat1_go<DT, 1>(jb, y, s);
    else scat1_go<DT, 2>(jb, y, s);
}

static void scat1_dispatch(int dt, int mode, const Scat1Job& jb, double* y, hipStream_t s) {
    switch (dt) {
        case DT_F64: scat1_mode<DT_F64>(mode, jb, y, s); break;
        case DT_F32: scat1_mode<DT_F32>(mode, jb, y, s); break;
        case DT_BF16: scat1_mode<DT_BF16>(mode, jb, y, s); break;
        default: scat1_mode<DT_BF16X3>(mode, jb, y, s); break;
    }
}

int launch_cp_scatter1(int dt, const void* Af, const void* Af_lo, int N, int Rp, const void* w, double* y_out,
                       const StepArgs* sa, int mode, hipStream_t s, const double* G) {
    Scat1Job jb{};
    jb.G = G;
    jb.Af = Af;
    jb.Af_lo = (const unsigned short*)Af_lo;
    jb.N = N;
    jb.Rp = Rp;
    jb.w = w;
    if (sa) jb.a = *sa;
    jb.nblk = (N + 3) / 4;
    scat1_dispatch(dt, mode, jb, y_out, s);
    return 0;
}

template <int DT>
static size_t helm_proj_lds(int N, int Np, bool proj) {
    // projections: images of u and (BF16 formats, pair form) -u
    const size_t h = sizeof(double) * (size_t)N, q = proj ? proj_lds<DT>(Np) : 0;
    return h > q ? h : q;
}

template <int DT>
static void helm_proj_go(const HelmJob& jb, hipStream_t s) {
    const size_t lds = helm_proj_lds<DT>(jb.a.N, jb.a.Np, jb.np > 0);
    const unsigned blocks = (unsigned)(jb.nh + jb.np + 1);
    if (jb.a.N % 2 == 0) hipLaunchKernelGGL((k_helm_proj<DT, true>), dim3(blocks), dim3(256), lds, s, jb);
    else hipLaunchKernelGGL((k_helm_proj<DT, false>), dim3(blocks), dim3(256), lds, s, jb);
}

void launch_helm_proj(int dt, const HelmJob& jb, hipStream_t s) {
    switch (dt) {
        case DT_F64: helm_proj_go<DT_F64>(jb, s); break;
        case DT_F32: helm_proj_go<DT_F32>(jb, s); break;
        case DT_BF16: helm_proj_go<DT_BF16>(jb, s); break;
        default: helm_proj_go<DT_BF16X3>(jb, s); break;
    }
}

}  // namespace rom
