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
#include "kdot.h"
#include "kstep.h"

namespace rom {

// ============================================================== CP, one trajectory

// Projections and Hadamard product: w[r] = lam_r (sum_k BCt[r][k] u_k)
// (sum_k BCt[Rp + r][k] u_k) for r < Rp (rows r < Rp are Bf^T, rows Rp + r are Cf^T).
// One wavefront per row pair, four per block; each lane issues its row loads before u
// is staged in LDS.  Each projection sums in the same order as a one-row dot product,
// and w = (lam s) t.
template <int DT, int V, int U>
__device__ __forceinline__ void cp_proj1_body(const Proj1Job& jb, int blk) {
    typedef typename Store<DT>::T T;
    typedef typename Store<DT>::Acc Acc;
    constexpr int BYTES = V * (int)sizeof(T);
    constexpr bool X3 = (DT == DT_BF16X3);
    typedef typename RawT<BYTES>::T Raw;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int N = jb.N, Np = jb.Np;
    LdsU<DT> L;
    L.bind(smem, Np);
    const int lane = threadIdx.x % kWave;
    const int r = blk * 4 + threadIdx.x / kWave;
    const bool live = r < jb.Rp;
    const size_t pair = (size_t)jb.Rp * Np;
    const T* row = reinterpret_cast<const T*>(jb.BCt) + (size_t)(live ? r : 0) * Np;
    const unsigned short* rowlo = X3 ? jb.BCt_lo + (size_t)(live ? r : 0) * Np : nullptr;
    Raw rv[2][U], rl[2][U];
    int k0 = lane * V;
    auto issue = [&](int kb) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int q = 0; q < U; ++q) {
                const int k = kb + q * kWave * V;
                if (live && k < Np) {
                    rv[h][q] = ld_plain<BYTES>(row + (h ? pair : 0) + k);
                    if constexpr (X3) rl[h][q] = ld_plain<BYTES>(rowlo + (h ? pair : 0) + k);
                }
            }
    };
    issue(k0);
    L.fill(jb.u_base + (jb.stepp ? (size_t)slot_of(*jb.stepp) * jb.slot_stride : 0), N, Np);
    __syncthreads();
    if (!live) return;
    Acc z[2] = {0, 0};
    while (k0 < Np) {
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int k = k0 + q * kWave * V;
            if (k < Np) {
#pragma unroll
                for (int h = 0; h < 2; ++h) z[h] += dot_vec<DT, V>(rv[h][q], rl[h][q], L, k);
            }
        }
        k0 += kWave * V * U;
        if (k0 < Np) issue(k0);
    }
    z[0] = wave_sum(z[0]);
    z[1] = wave_sum(z[1]);
    if (lane == 0) reinterpret_cast<Acc*>(jb.w)[r] = reinterpret_cast<const Acc*>(jb.lam)[r] * z[0] * z[1];
}

// The same for factors that keep the partial skew-symmetry (Sec. 3.3, eq.
// skew_abc_struct): column pair p = (c0, c1) has Bf[:,c1] = Bf[:,c0], Cf[:,c0] = Af[:,c1]
// and Cf[:,c1] = -Af[:,c0], so with beta = Bf[:,c0]^T u, alpha = Af[:,c0]^T u and
// gamma = Af[:,c1]^T u the pair's products are w[c0] = lam beta gamma and
// w[c1] = lam beta (-alpha).  The operator holds the P distinct columns of Bf and the R
// columns of Af as rows, [P + R][Np]: 1.5 R rows where the general form reads 2 R.  One
// wavefront per pair (three rows); pair slots past P write the zero padding of w.  Each
// dot product is computed as in cp_proj1_body.  In FP64 and FP32 the fused multiply-adds
// round symmetrically, so -alpha is the negated dot product; the packed BF16 dot
// instruction does not always give dot(-a, u) = -dot(a, u) to the bit, so the BF16
// formats form -alpha as Af[:,c0]^T (-u) against a second LDS image of -u, which
// presents it the same signed products as (-a) u.  So w is the general form's to the bit
// in every format.
template <int DT, int V, int U>
__device__ __forceinline__ void cp_proj_skew_body(const Proj1Job& jb, int blk) {
    typedef typename Store<DT>::T T;
    typedef typename Store<DT>::Acc Acc;
    constexpr int BYTES = V * (int)sizeof(T);
    constexpr bool X3 = (DT == DT_BF16X3);
    typedef typename RawT<BYTES>::T Raw;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int N = jb.N, Np = jb.Np, P = jb.P, R = jb.R;
    constexpr bool NEGU = (DT == DT_BF16 || DT == DT_BF16X3);
    LdsU<DT> L, Ln;                                      // u and (BF16 formats) -u
    L.bind(smem, Np);
    Ln.bind(smem + (NEGU ? LdsU<DT>::bytes(Np) : 0), Np);
    const int lane = threadIdx.x % kWave;
    const int q = blk * 4 + threadIdx.x / kWave;
    const bool live = q < P;
    const int c0 = jb.layout == 1 ? 2 * q : q, c1 = jb.layout == 1 ? 2 * q + 1 : P + q;
    const size_t rows[3] = {(size_t)(live ? q : 0), (size_t)(live ? P + c0 : 0), (size_t)(live ? P + c1 : 0)};
    const T* op = reinterpret_cast<const T*>(jb.BCt);
    Raw rv[3][U], rl[3][U];
    int k0 = lane * V;
    auto issue = [&](int kb) {
#pragma unroll
        for (int h = 0; h < 3; ++h)
#pragma unroll
            for (int qq = 0; qq < U; ++qq) {
                const int k = kb + qq * kWave * V;
                if (live && k < Np) {
                    rv[h][qq] = ld_plain<BYTES>(op + rows[h] * Np + k);
                    if constexpr (X3) rl[h][qq] = ld_plain<BYTES>(jb.BCt_lo + rows[h] * Np + k);
                }
            }
    };
    issue(k0);
    const double* ub = jb.u_base + (jb.stepp ? (size_t)slot_of(*jb.stepp) * jb.slot_stride : 0);
    L.fill(ub, N, Np);
    if constexpr (NEGU) Ln.fill(ub, N, Np, -1.0);
    __syncthreads();
    Acc* w = reinterpret_cast<Acc*>(jb.w);
    if (!live) {
        const int e = R + 2 * (q - P);                  // zero padding of w past R
        if (lane == 0 && e < jb.Rp) {
            w[e] = 0;
            if (e + 1 < jb.Rp) w[e + 1] = 0;
        }
        return;
    }
    Acc z[3] = {0, 0, 0};                                // beta, -alpha, gamma
    while (k0 < Np) {
#pragma unroll
        for (int qq = 0; qq < U; ++qq) {
            const int k = k0 + qq * kWave * V;
            if (k < Np) {
                z[0] += dot_vec<DT, V>(rv[0][qq], rl[0][qq], L, k);
                z[1] += dot_vec<DT, V>(rv[1][qq], rl[1][qq], NEGU ? Ln : L, k);
                z[2] += dot_vec<DT, V>(rv[2][qq], rl[2][qq], L, k);
            }
        }
        k0 += kWave * V * U;
        if (k0 < Np) issue(k0);
    }
#pragma unroll
    for (int h = 0; h < 3; ++h) z[h] = wave_sum(z[h]);
    if (lane == 0) {
        const Acc* lam = reinterpret_cast<const Acc*>(jb.lam);
        w[c0] = lam[c0] * z[0] * z[2];
        w[c1] = lam[c1] * z[0] * (NEGU ? z[1] : -z[1]);
    }
}

template <int DT, int V, int U>
__device__ __forceinline__ void cp_proj_any_body(const Proj1Job& jb, int blk) {
    if (jb.layout) cp_proj_skew_body<DT, V, U>(jb, blk);
    else cp_proj1_body<DT, V, U>(jb, blk);
}

template <int DT, int V, int U>
__global__ __launch_bounds__(256) void k_cp_proj1(Proj1Job jb) {
    cp_proj_any_body<DT, V, U>(jb, blockIdx.x);
}
template <int DT, int V, int U>
__global__ __launch_bounds__(256) void k_cp_proj1_group(const Proj1Job* __restrict__ jobs, int njobs) {
    const int p = find_job(jobs, njobs, (int)blockIdx.x);
    cp_proj_any_body<DT, V, U>(jobs[p], (int)blockIdx.x - jobs[p].blk0);
}

// Scatter: W = lam .* s .* t staged in LDS, then y_i = sum_r Af[i][r] W_r, one
// wavefront per row (row loads issued before W is staged).  MODE 0 writes y (FP64,
// to y_out); MODE 1 applies the diagonal-stiffness BDF update with its energy
// partials; MODE 2 writes the right-hand side for the dense Helmholtz solve.  n is the
// state's level (MODE 1 and 2).
template <int DT, int V, int U, int MODE>
__device__ __forceinline__ void cp_scatter1_body(const Scat1Job& jb, double* __restrict__ y_out, int blk,
                                                 long long n) {
    typedef typename Store<DT>::T T;
    typedef typename Store<DT>::Acc Acc;
    constexpr int BYTES = V * (int)sizeof(T);
    constexpr bool X3 = (DT == DT_BF16X3);
    typedef typename RawT<BYTES>::T Raw;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    Acc* W = reinterpret_cast<Acc*>(smem);
    __shared__ double red[4];
    const int N = jb.N, R = jb.Rp;
    const StepArgs& a = jb.a;
    const Acc* __restrict__ win = reinterpret_cast<const Acc*>(jb.w);
    const int lane = threadIdx.x % kWave;
    const int i = blk * 4 + threadIdx.x / kWave;
    const bool live = i < N;
    const T* row = reinterpret_cast<const T*>(jb.Af) + (size_t)(live ? i : 0) * R;
    const unsigned short* rowlo = X3 ? jb.Af_lo + (size_t)(live ? i : 0) * R : nullptr;
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
    // the update's history (and diagonal inverse) behind the row loads
    BdfHist hist{};
    double hd = 0.0;
    int k = 0;
    if constexpr (MODE != 0) {
        k = bdf_order(n);
        if (live && lane == 0) {
            hist = bdf_hist_point(a, n, k, 0, i);
            if constexpr (MODE == 1) hd = a.hdiag[(size_t)(k - 1) * N + i];
        }
    }
    staged_copy<8, Acc>(R, [&](int r) { return win[r]; }, [&](int r, Acc v) { W[r] = v; });
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
        const BdfCoef c = bdf_coef(k);
        double e = 0.0;
        if (live && lane == 0) {
            const double rhs = bdf_rhs_hist(a, n, c, k, 0, i, (double)z, hist);
            if constexpr (MODE == 1) {
                const double un = rhs * hd;
                write_level(a, n + 1, 0, i, un);
                e = un * un;
            } else {
                a.rhs[i] = rhs;
            }
        }
        if constexpr (MODE == 1) {
            const double s = block_sum(e, red);
            if (threadIdx.x == 0) epart_of(a, n + 1)[blk] = s;
        }
    }
}

// MODE 1 (the update kernel) runs one block more than there are row blocks: the last
// one closes the previous level and advances the counter.
template <int DT, int V, int U, int MODE>
__global__ __launch_bounds__(256) void k_cp_scatter1(Scat1Job jb, double* y_out) {
    if constexpr (MODE == 1) {
        if (blockIdx.x == gridDim.x - 1) {
            close_and_advance(jb.a, *jb.a.step, (int)gridDim.x - 1);
            return;
        }
        cp_scatter1_body<DT, V, U, MODE>(jb, y_out, blockIdx.x, *jb.a.step);
    } else {
        cp_scatter1_body<DT, V, U, MODE>(jb, y_out, blockIdx.x, MODE == 0 ? 0LL : *jb.a.step);
    }
}
template <int DT, int V, int U, int MODE>
__global__ __launch_bounds__(256) void k_cp_scatter1_group(const Scat1Job* __restrict__ jobs, int njobs) {
    const int p = find_job(jobs, njobs, (int)blockIdx.x);
    const Scat1Job& jb = jobs[p];
    const int blk = (int)blockIdx.x - jb.blk0;
    long long n = 0;
    if constexpr (MODE != 0) n = *jb.a.step;
    if constexpr (MODE == 1) {
        if (blk == 0) close_and_advance(jb.a, n, jb.nblk);
    }
    cp_scatter1_body<DT, V, U, MODE>(jb, nullptr, blk, n);
}

// ============================================================== Helmholtz apply and projections

// With a dense stiffness the step ends by applying Hinv_k to the right-hand side.  For
// a CP state the same kernel also forms the projections of the new level,
// s = Bf^T u^{n+1} and t = Cf^T u^{n+1}, and w = lam .* s .* t, from that right-hand side
// with the operator [Bf|Cf]^T Hinv_k built at context creation (the two products
// associate: Bf^T (Hinv_k rhs) = (Bf^T Hinv_k) rhs, with the same 2 N R flops as the
// projection of u^{n+1}).  The next step's scatter then starts at once, and a step is
// two kernels.  Blocks [0, nh) are Helmholtz row blocks, blocks [nh, nh + np)
// projection blocks (four row pairs each).
template <int DT, bool EVEN>
__device__ __forceinline__ void helm_proj_body(const HelmJob& jb, long long n, int blk) {
    if (blk < jb.nh) {
        helm_gemv_body<EVEN>(jb.a, n, blk);
        return;
    }
    typedef typename Store<DT>::T T;
    constexpr int V = 16 / (int)sizeof(T);
    const size_t rows = jb.layout ? (size_t)(jb.P + jb.R) : (size_t)2 * jb.Rp;
    const size_t mstride = (size_t)(bdf_order(n) - 1) * rows * jb.a.Np;
    Proj1Job pj{};
    pj.BCt = reinterpret_cast<const T*>(jb.Mst) + mstride;
    pj.BCt_lo = jb.Mst_lo ? jb.Mst_lo + mstride : nullptr;
    pj.lam = jb.lam;
    pj.N = jb.a.N;
    pj.Np = jb.a.Np;
    pj.Rp = jb.Rp;
    pj.layout = jb.layout;
    pj.P = jb.P;
    pj.R = jb.R;
    pj.u_base = jb.a.rhs;
    pj.w = jb.a.st;
    cp_proj_any_body<DT, V, 4>(pj, blk - jb.nh);
}

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

// Grouped states: the first block of each job also closes its state's previous level.
template <int DT>
__global__ __launch_bounds__(256) void k_helm_proj_group(const HelmJob* __restrict__ jobs, int njobs) {
    const int p = find_job(jobs, njobs, (int)blockIdx.x);
    const HelmJob& jb = jobs[p];
    const int blk = (int)blockIdx.x - jb.blk0;
    const long long n = *jb.a.step;
    if (blk == 0) close_and_advance(jb.a, n, jb.nh);
    if (jb.a.N % 2 == 0) helm_proj_body<DT, true>(jb, n, blk);
    else helm_proj_body<DT, false>(jb, n, blk);
}

// ============================================================== SVD-ROM, one trajectory

// First product of the SVD-ROM (Sec. 4.4): w_r = sigma_r sum_j U[j][r] u_j over the rows
// of Ut [Rsp][Np] (rows past the rank are zero, so w is zero there).  One wavefront per
// row, four per block; the second product is the streaming kernel with R weighted slabs.
struct SvdProj {
    const void* Ut;
    const unsigned short* Ut_lo;
    const void* sigma;
    int N, Np, Rsp;
    const double* u_base;
    const long long* stepp;
    long long slot_stride;
    void* w;
};

template <int DT, int V, int U>
__global__ __launch_bounds__(256) void k_svd_proj(SvdProj a) {
    typedef typename Store<DT>::T T;
    typedef typename Store<DT>::Acc Acc;
    constexpr int BYTES = V * (int)sizeof(T);
    constexpr bool X3 = (DT == DT_BF16X3);
    typedef typename RawT<BYTES>::T Raw;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int N = a.N, Np = a.Np;
    LdsU<DT> L;
    L.bind(smem, Np);
    const int lane = threadIdx.x % kWave;
    const int r = (int)blockIdx.x * 4 + (int)threadIdx.x / kWave;
    const bool live = r < a.Rsp;
    const T* row = reinterpret_cast<const T*>(a.Ut) + (size_t)(live ? r : 0) * Np;
    const unsigned short* rowlo = X3 ? a.Ut_lo + (size_t)(live ? r : 0) * Np : nullptr;
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
    L.fill(a.u_base + (a.stepp ? (size_t)slot_of(*a.stepp) * a.slot_stride : 0), N, Np);
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
    if (lane == 0) reinterpret_cast<Acc*>(a.w)[r] = reinterpret_cast<const Acc*>(a.sigma)[r] * z;
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
static void proj1_go(const Proj1Job& jb, const Proj1Job* jobs, int njobs, int blocks, int Npmax, hipStream_t s) {
    constexpr int V = 16 / (int)sizeof(typename Store<DT>::T);
    const size_t lds = proj_lds<DT>(Npmax);
    if (jobs) hipLaunchKernelGGL((k_cp_proj1_group<DT, V, 4>), dim3((unsigned)blocks), dim3(256), lds, s, jobs, njobs);
    else hipLaunchKernelGGL((k_cp_proj1<DT, V, 4>), dim3((unsigned)jb.nblk), dim3(256), lds, s, jb);
}

static void proj1_dispatch(int dt, const Proj1Job& jb, const Proj1Job* jobs, int njobs, int blocks, int Npmax,
                           hipStream_t s) {
    switch (dt) {
        case DT_F64: proj1_go<DT_F64>(jb, jobs, njobs, blocks, Npmax, s); break;
        case DT_F32: proj1_go<DT_F32>(jb, jobs, njobs, blocks, Npmax, s); break;
        case DT_BF16: proj1_go<DT_BF16>(jb, jobs, njobs, blocks, Npmax, s); break;
        default: proj1_go<DT_BF16X3>(jb, jobs, njobs, blocks, Npmax, s); break;
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
    proj1_dispatch(dt, jb, nullptr, 0, 0, Np, s);
    return 0;
}

void launch_cp_proj1_group(int dt, const Proj1Job* jobs_dev, int njobs, int blocks, int Npmax, hipStream_t s) {
    Proj1Job none{};
    proj1_dispatch(dt, none, jobs_dev, njobs, blocks, Npmax, s);
}

template <int DT, int MODE>
static void scat1_go(const Scat1Job& jb, double* y, const Scat1Job* jobs, int njobs, int blocks, int Rpmax,
                     hipStream_t s) {
    typedef typename Store<DT>::Acc Acc;
    constexpr int V = 16 / (int)sizeof(typename Store<DT>::T);
    const size_t lds = sizeof(Acc) * Rpmax;
    if (jobs) hipLaunchKernelGGL((k_cp_scatter1_group<DT, V, 8, MODE>), dim3((unsigned)blocks), dim3(256), lds, s, jobs, njobs);
    else hipLaunchKernelGGL((k_cp_scatter1<DT, V, 8, MODE>), dim3((unsigned)jb.nblk + (MODE == 1 ? 1u : 0u)), dim3(256),
                            lds, s, jb, y);
}

template <int DT>
static void scat1_mode(int mode, const Scat1Job& jb, double* y, const Scat1Job* jobs, int njobs, int blocks, int Rpmax,
                       hipStream_t s) {
    if (mode == 0) scat1_go<DT, 0>(jb, y, jobs, njobs, blocks, Rpmax, s);
    else if (mode == 1) scat1_go<DT, 1>(jb, y, jobs, njobs, blocks, Rpmax, s);
    else scat1_go<DT, 2>(jb, y, jobs, njobs, blocks, Rpmax, s);
}

static void scat1_dispatch(int dt, int mode, const Scat1Job& jb, double* y, const Scat1Job* jobs, int njobs,
                           int blocks, int Rpmax, hipStream_t s) {
    switch (dt) {
        case DT_F64: scat1_mode<DT_F64>(mode, jb, y, jobs, njobs, blocks, Rpmax, s); break;
        case DT_F32: scat1_mode<DT_F32>(mode, jb, y, jobs, njobs, blocks, Rpmax, s); break;
        case DT_BF16: scat1_mode<DT_BF16>(mode, jb, y, jobs, njobs, blocks, Rpmax, s); break;
        default: scat1_mode<DT_BF16X3>(mode, jb, y, jobs, njobs, blocks, Rpmax, s); break;
    }
}

int launch_cp_scatter1(int dt, const void* Af, const void* Af_lo, int N, int Rp, const void* w, double* y_out,
                       const StepArgs* sa, int mode, hipStream_t s) {
    Scat1Job jb{};
    jb.Af = Af;
    jb.Af_lo = (const unsigned short*)Af_lo;
    jb.N = N;
    jb.Rp = Rp;
    jb.w = w;
    if (sa) jb.a = *sa;
    jb.nblk = (N + 3) / 4;
    scat1_dispatch(dt, mode, jb, y_out, nullptr, 0, 0, Rp, s);
    return 0;
}

void launch_cp_scatter1_group(int dt, int mode, const Scat1Job* jobs_dev, int njobs, int blocks, int Rpmax,
                              hipStream_t s) {
    Scat1Job none{};
    scat1_dispatch(dt, mode, none, nullptr, jobs_dev, njobs, blocks, Rpmax, s);
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

template <int DT>
static void helm_proj_group_go(const HelmJob* jobs, int njobs, int blocks, int Nmax, int Npmax, bool proj,
                               hipStream_t s) {
    const size_t lds = helm_proj_lds<DT>(Nmax, Npmax, proj);
    hipLaunchKernelGGL((k_helm_proj_group<DT>), dim3((unsigned)blocks), dim3(256), lds, s, jobs, njobs);
}

void launch_helm_proj_group(int dt, const HelmJob* jobs_dev, int njobs, int blocks, int Nmax, int Npmax, int proj,
                            hipStream_t s) {
    if (njobs < 1 || blocks < 1) return;
    switch (dt) {
        case DT_F64: helm_proj_group_go<DT_F64>(jobs_dev, njobs, blocks, Nmax, Npmax, proj != 0, s); break;
        case DT_F32: helm_proj_group_go<DT_F32>(jobs_dev, njobs, blocks, Nmax, Npmax, proj != 0, s); break;
        case DT_BF16: helm_proj_group_go<DT_BF16>(jobs_dev, njobs, blocks, Nmax, Npmax, proj != 0, s); break;
        default: helm_proj_group_go<DT_BF16X3>(jobs_dev, njobs, blocks, Nmax, Npmax, proj != 0, s); break;
    }
}

}  // namespace rom
