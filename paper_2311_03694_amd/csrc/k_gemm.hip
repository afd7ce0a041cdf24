// k_gemm.hip -- skinny products of the batched path on the matrix cores:
//   Y[b][m] = sum_k A[m][k] X[b][k]     (M rows, K contracted, Bpad <= a few hundred columns)
// used for the CP projections [Bf|Cf]^T u and the CP scatter Af W (Sec. 3.1, eq. tc_ap)
// and for the batched Helmholtz apply Hinv_k rhs (eq. nse_d1, dense stiffness).
//
// Block = 4 wavefronts over one 16-row tile of A and 16*FN columns, over the whole of K:
// wavefront w takes the w-th quarter of the K steps (one step = one 16-byte lane vector
// per lane: 32 k in BF16, 16 in FP32, 8 in FP64) and streams its A and X fragments
// through a PF-deep register ring; the 4 partial tiles are added in LDS in a fixed
// order and written straight to Y (no partial buffers, no second pass).  With one block
// per output tile the grid is ceil(M/16) x (column tiles), which fills the device for
// the shapes of this path; A is read once per column tile (column tiles of one row tile
// run next to each other on one XCD and share its L2).
//
// Epilogues (EPI):
//  * PLAIN writes Y.
//  * PAIR (the CP projections): a block takes row tile r of Bf^T and the same tile of
//    Cf^T (rows pair_off apart), so it holds s[b][r] and t[b][r] together and writes the
//    Hadamard product W[b][r] = lam_r s t (eq. tc_ap) instead of the projections.
//  * UPDATE / RHS (the CP scatter of a step): each output y^n[b][i] goes straight into
//    the BDFk/EXTk right-hand side of eq. nse_d1; UPDATE (diagonal stiffness) also
//    solves for u^{n+1}, stores it and leaves the energy of its 16 rows per trajectory,
//    and one extra block closes the previous level and advances the step counter (this
//    kernel is then the step's update kernel); RHS stores the right-hand side for the
//    Helmholtz apply.
//  * FINISH (the batched Helmholtz apply of a step): the outputs are u^{n+1}; they are
//    stored with their energy partials, and one extra block closes the step.
//  * SKEW (the CP projections of factors with skew column pairs, Sec. 3.3): A is the pair
//    form [P + R][Np] (the P distinct columns of Bf, then the columns of Af); a block
//    takes 16 pairs, each lane three rows (beta, alpha, gamma of its pair), and writes
//    W[b][c0] = lam beta gamma and W[b][c1] = -lam beta alpha; pairs past P write the
//    zero padding of W.
#include "als.h"
#include "kmfma.h"
#include "kstep.h"

namespace rom {

struct GemmArgs {
    const void* A;                 // [M][lda] rows in the operator's storage format
    const unsigned short* Alo;     // BF16X3 low words of A
    const void* X;                 // [Bpad][ldx] in the MFMA operand format
    const unsigned short* Xlo;     // BF16X3 low words of X
    void* Y;                       // [Bpad][M] (accumulation type)
    int M, K, Bpad;
    long long lda, ldx;
    int gx, gy;                    // row tiles, column tiles
    int ksplit;                    // PLAIN: K ranges, one partial product each (Y + split * M * Bpad)
    int bstore;                    // PLAIN, PAIR: columns b of Y stored (0: all Bpad)
    const long long* kstep;        // non-null: A += (BDF order at *kstep - 1) * a_kstride
    long long a_kstride;
    long long pair_off;            // PAIR: elements from a row of A to its partner row
    const void* lam;               // PAIR, SKEW: lam (accumulation type)
    int skew_P, skew_layout;       // SKEW: pairs, layout (1 interleaved, 2 blocked)
    long long wstride;             // SKEW: row length of W (Rp)
    StepArgs st;                   // UPDATE, RHS: the state of the step (M = N rows)
};

enum { EPI_PLAIN = 0, EPI_PAIR = 1, EPI_UPDATE = 2, EPI_RHS = 3, EPI_FINISH = 4, EPI_SKEW = 5 };

template <int ADT, int MKD, int FN, int PF, int EPI>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs p) {
    constexpr bool PAIR = (EPI == EPI_PAIR);
    constexpr bool SKEW = (EPI == EPI_SKEW);
    constexpr bool CLOSE = (EPI == EPI_UPDATE || EPI == EPI_FINISH);   // writes level n+1
    typedef MfmaT<MKD> Tr;
    typedef typename Tr::X XT;
    typedef typename Tr::Acc Acc;
    typedef typename Tr::Acc4 Acc4;
    constexpr int KS = Tr::KS, VEC = Tr::VEC;
    constexpr bool X3 = (MKD == MK_BF16X3);
    // a FP32 product over BF16 words (the CP scatter of the BF16 formats) reads 4 words
    // per lane vector and converts them when the slot is consumed, not when it is
    // loaded (a conversion at load time would wait for the load right away)
    constexpr bool CVT = (MKD == MK_F32 && ADT != DT_F32);
    constexpr int AV = CVT ? 4 : (int)(16 / sizeof(typename Store<ADT>::T));
    static_assert(AV == VEC, "lane vectors of A and X must cover the same k");
    constexpr int NA = PAIR ? 2 : SKEW ? 3 : 1;          // A rows per lane (row and partner(s))
    extern __shared__ __attribute__((aligned(16))) char smem[];
    Acc* red = reinterpret_cast<Acc*>(smem);             // [NA][4][FN][4][64]

    const int nks = EPI == EPI_PLAIN ? p.ksplit : 1;
    const int nwork = p.gx * p.gy * nks + (CLOSE ? 1 : 0);
    const int per = (nwork + 7) / 8;
    const int wi = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (wi >= nwork) return;
    if constexpr (CLOSE) {
        if (wi == nwork - 1) {                           // the step-closing block
            close_and_advance(p.st, *p.st.step, p.gx);
            return;
        }
    }
    const long long n = EPI >= EPI_UPDATE ? *p.st.step : 0;
    // the K ranges of one tile are consecutive work items (one XCD, shared X rows)
    const int ks = wi % nks, tile = wi / nks;
    const int by = tile % p.gy, bx = tile / p.gy;

    const int lane = threadIdx.x & 63, g = lane >> 4, c16 = lane & 15;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int rowbase = bx * 16, b0 = by * 16 * FN;
    // this block's K steps [kb, kb + kn), split over the 4 wavefronts
    const int ksteps_all = (p.K + KS - 1) / KS;
    const int kper = (ksteps_all + nks - 1) / nks;
    const int kb = ks * kper;
    const int ksteps = kb < ksteps_all ? (ksteps_all - kb < kper ? ksteps_all - kb : kper) : 0;
    const int wsb = ksteps / 4, wse = ksteps - wsb * 4;
    const int ns = wsb + (w < wse ? 1 : 0);
    const int s0 = kb + w * wsb + (w < wse ? w : wse);

    // the lane's row (rows past M are clamped for loads and never stored) and columns
    int r = rowbase + c16;
    r = r < p.M ? r : p.M - 1;
    const size_t kbase = p.kstep ? (size_t)(bdf_order(*p.kstep) - 1) * p.a_kstride : 0;
    size_t arows[NA];
    if constexpr (SKEW) {
        const int c0 = p.skew_layout == 1 ? 2 * r : r, c1 = p.skew_layout == 1 ? 2 * r + 1 : p.skew_P + r;
        arows[0] = kbase + (size_t)r * p.lda;
        arows[1] = kbase + (size_t)(p.skew_P + c0) * p.lda;
        arows[2] = kbase + (size_t)(p.skew_P + c1) * p.lda;
    } else {
#pragma unroll
        for (int h = 0; h < NA; ++h) arows[h] = kbase + (size_t)r * p.lda + (h ? (size_t)p.pair_off : 0);
    }
    size_t xrow[FN];
#pragma unroll
    for (int t = 0; t < FN; ++t) {
        int b = b0 + t * 16 + c16;
        b = b < p.Bpad ? b : p.Bpad - 1;
        xrow[t] = (size_t)b * p.ldx;
    }

    Acc4 Z[NA][FN];
#pragma unroll
    for (int h = 0; h < NA; ++h)
#pragma unroll
        for (int t = 0; t < FN; ++t) Z[h][t] = Acc4{0, 0, 0, 0};

    if (ns > 0) {                                        // wavefront-uniform
        // Ring of PF steps.  Loads are unconditional: addresses past K are clamped to
        // the last lane vector of the row and their X fragments selected to zero when
        // consumed, so the loop has no branches and waits only for the slot it uses.
        u32x4 ah[NA][PF], al[NA][PF], xh[PF][FN], xl[PF][FN];
        int kq[PF];
        int sp = 0;                                      // producer step
        auto issue = [&](int d) {
            const int st = s0 + (sp < ns ? sp : ns - 1);
            int k = st * KS + g * VEC;
            kq[d] = k;
            k = k < p.K ? k : p.K - VEC;
#pragma unroll
            for (int h2 = 0; h2 < NA; ++h2) {
                const size_t ar = arows[h2];
                if constexpr (CVT) {
                    const u32x2 h = ld_plain<8>(reinterpret_cast<const unsigned short*>(p.A) + ar + k);
                    u32x2 l = u32x2{0u, 0u};
                    if constexpr (ADT == DT_BF16X3) l = ld_plain<8>(p.Alo + ar + k);
                    ah[h2][d] = u32x4{h[0], h[1], l[0], l[1]};
                } else {
                    load_a<ADT, MKD, false>(p.A, p.Alo, ar + k, ah[h2][d], al[h2][d]);
                }
            }
#pragma unroll
            for (int t = 0; t < FN; ++t) {
                xh[d][t] = ld_plain<16>(reinterpret_cast<const XT*>(p.X) + xrow[t] + k);
                if constexpr (X3) xl[d][t] = ld_plain<16>(p.Xlo + xrow[t] + k);
                else xl[d][t] = u32x4{0u, 0u, 0u, 0u};
            }
            ++sp;
        };
#pragma unroll
        for (int d = 0; d < PF; ++d) {
            issue(d);
            __builtin_amdgcn_sched_barrier(0);           // slot order: slot 0 lands first
        }
        const int ns_pad = (ns + PF - 1) / PF * PF;
        for (int q0 = 0; q0 < ns_pad; q0 += PF) {
#pragma unroll
            for (int d = 0; d < PF; ++d) {
                const bool live = (q0 + d < ns) && (kq[d] < p.K);
                const u32x4 z = u32x4{0u, 0u, 0u, 0u};
#pragma unroll
                for (int h2 = 0; h2 < NA; ++h2) {
                    u32x4 av = ah[h2][d];
                    if constexpr (CVT) {
                        // 4 BF16 words (plus their low words) -> 4 FP32 values, hi + lo exact
                        float f[4] = {bf16_lo_f(av[0]), bf16_hi_f(av[0]), bf16_lo_f(av[1]), bf16_hi_f(av[1])};
                        if constexpr (ADT == DT_BF16X3) {
                            f[0] += bf16_lo_f(av[2]);
                            f[1] += bf16_hi_f(av[2]);
                            f[2] += bf16_lo_f(av[3]);
                            f[3] += bf16_hi_f(av[3]);
                        }
                        av = u32x4{__float_as_uint(f[0]), __float_as_uint(f[1]), __float_as_uint(f[2]),
                                   __float_as_uint(f[3])};
                    }
#pragma unroll
                    for (int t = 0; t < FN; ++t) {
                        const u32x4 xv = live ? xh[d][t] : z;
                        const u32x4 xlv = live ? xl[d][t] : z;
                        mfma_step<MKD>(Z[h2][t], av, al[h2][d], xv, xlv);
                    }
                }
                issue(d);
                // nothing crosses: later slots' arithmetic hoisted above these loads
                // would push the loads to the end of the body and defeat the ring
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }

    // ---- add the 4 wavefront tiles (fixed order) and write Y (PAIR: W = lam s t)
    constexpr int RS = 4 * FN * 4 * 64;                  // one A row set of red
#pragma unroll
    for (int h = 0; h < NA; ++h)
#pragma unroll
        for (int t = 0; t < FN; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) red[h * RS + ((w * FN + t) * 4 + v) * 64 + lane] = Z[h][t][v];
    __syncthreads();
    Acc* out = reinterpret_cast<Acc*>(p.Y) + (size_t)ks * p.M * p.Bpad;
    for (int e = threadIdx.x; e < 256 * FN; e += 256) {
        const int cl = e >> 4, rr = e & 15;              // local column, local row
        const int t = cl >> 4, cc = cl & 15;
        const int gg = MKD == MK_F64 ? (rr & 3) : (rr >> 2);
        const int v = MKD == MK_F64 ? (rr >> 2) : (rr & 3);
        const int ln = gg * 16 + cc;
        Acc sum[NA];
#pragma unroll
        for (int h = 0; h < NA; ++h) {
            sum[h] = red[h * RS + (t * 4 + v) * 64 + ln];
#pragma unroll
            for (int w2 = 1; w2 < 4; ++w2) sum[h] += red[h * RS + ((w2 * FN + t) * 4 + v) * 64 + ln];
        }
        const int row = rowbase + rr, b = b0 + cl;
        if constexpr (SKEW) {
            if (b < p.Bpad) {
                Acc* wrow = out + (size_t)b * p.wstride;
                if (row < p.skew_P) {
                    const int c0 = p.skew_layout == 1 ? 2 * row : row;
                    const int c1 = p.skew_layout == 1 ? 2 * row + 1 : p.skew_P + row;
                    const Acc* lam = reinterpret_cast<const Acc*>(p.lam);
                    wrow[c0] = lam[c0] * sum[0] * sum[2];
                    wrow[c1] = lam[c1] * sum[0] * (-sum[1]);
                } else {
                    const long long e = 2LL * row;                // zero padding of W past R = 2P
                    if (e < p.wstride) wrow[e] = 0;
                    if (e + 1 < p.wstride) wrow[e + 1] = 0;
                }
            }
        } else if constexpr (EPI <= EPI_PAIR) {
            if (row < p.M && b < (p.bstore > 0 ? p.bstore : p.Bpad)) {
                if constexpr (PAIR) out[(size_t)b * p.M + row] = reinterpret_cast<const Acc*>(p.lam)[row] * sum[0] * sum[1];
                else out[(size_t)b * p.M + row] = sum[0];
            }
        } else {
            const StepArgs& a = p.st;
            double ev = 0.0;
            if (row < p.M && b < a.B) {
                if constexpr (EPI == EPI_FINISH) {
                    const double un = (double)sum[0];
                    write_level(a, n + 1, b, row, un);
                    ev = un * un;
                } else {
                    const int k = bdf_order(n);
                    const BdfCoef c = bdf_coef(k);
                    const double rhs = bdf_rhs_point(a, n, c, k, b, row, (double)sum[0]);
                    if constexpr (EPI == EPI_UPDATE) {
                        const double un = rhs * a.hdiag[(size_t)(k - 1) * a.N + row];
                        write_level(a, n + 1, b, row, un);
                        ev = un * un;
                    } else {
                        a.rhs[(size_t)b * a.Np + row] = rhs;
                    }
                }
            }
            if constexpr (CLOSE) {
                // the tile's 16 rows of trajectory b sit in 16 consecutive lanes
                ev += __shfl_xor(ev, 8, 16);
                ev += __shfl_xor(ev, 4, 16);
                ev += __shfl_xor(ev, 2, 16);
                ev += __shfl_xor(ev, 1, 16);
                if (rr == 0 && b < a.B) epart_of(a, n + 1)[(size_t)b * a.enmax + bx] = ev;
            }
        }
    }
}

// ---------------------------------------------------------------- planning, launch

// Variant 0 picks the column-tile width from the shape; 1, 2, 3 force FN = 1, 2, 4.
constexpr int kGemmVariants = 4;
int gemm_variants() { return kGemmVariants; }

static int gemm_fn(int M, int Bpad, int v) {
    const int nct = Bpad / 16;
    if (v == 1) return 1;
    if (v == 2) return nct % 2 == 0 ? 2 : 1;
    if (v == 3) return nct % 4 == 0 ? 4 : (nct % 2 == 0 ? 2 : 1);
    // widest tile that still gives about one block per CU
    const int gx = (M + 15) / 16;
    for (int fn : {4, 2})
        if (nct % fn == 0 && (long long)gx * (nct / fn) >= 224) return fn;
    return 1;
}

GemmPlan gemm_plan(int M, int Bpad, int variant) {
    GemmPlan pl{};
    pl.fn = gemm_fn(M, Bpad, variant < 0 ? 0 : variant);
    pl.gx = (M + 15) / 16;
    pl.gy = Bpad / (16 * pl.fn);
    pl.blocks = (pl.gx * pl.gy + 7) / 8 * 8;
    pl.ksplit = 1;
    return pl;
}

// The widest column tiles (each A fragment feeds up to four MFMA tiles; with one 16-column
// tile a block's loads run at the compute unit's vector-load rate), then K ranges where
// the output tiles leave compute units idle: about one block per compute unit (about two
// were slower: more prologues and reductions), each wavefront keeping at least 4 K steps
// (8 FP64 values a step), at most 8 ranges.  N = 1000, B = 64, K = 2000: 17.5 -> 14.0 us.
GemmPlan gemm_plan_splitk(int M, int K, int Bpad) {
    GemmPlan pl = gemm_plan(M, Bpad, 3);
    const int tiles = pl.gx * pl.gy, ksteps = (K + 7) / 8;
    int ks = 256 / tiles;
    ks = ks < 1 ? 1 : ks > 8 ? 8 : ks;
    while (ks > 1 && ksteps / ks < 16) --ks;
    pl.ksplit = ks;
    pl.blocks = (tiles * ks + 7) / 8 * 8;
    return pl;
}

template <int ADT, int MKD, int EPI = EPI_PLAIN>
static void gemm_go(const GemmArgs& a, const GemmPlan& pl, hipStream_t s) {
    const size_t lds = (size_t)1024 * pl.fn * sizeof(typename MfmaT<MKD>::Acc) *
                       (EPI == EPI_PAIR ? 2 : EPI == EPI_SKEW ? 3 : 1);
    if (pl.fn == 4) hipLaunchKernelGGL((k_gemm<ADT, MKD, 4, 4, EPI>), dim3(pl.blocks), dim3(256), lds, s, a);
    else if (pl.fn == 2) hipLaunchKernelGGL((k_gemm<ADT, MKD, 2, 6, EPI>), dim3(pl.blocks), dim3(256), lds, s, a);
    else hipLaunchKernelGGL((k_gemm<ADT, MKD, 1, 8, EPI>), dim3(pl.blocks), dim3(256), lds, s, a);
}

static GemmArgs gemm_args(const GemmPlan& pl, const void* A, const void* Alo, long long lda, const void* X,
                          const void* Xlo, long long ldx, void* Y, int M, int K, int Bpad) {
    GemmArgs a{};
    a.A = A;
    a.Alo = (const unsigned short*)Alo;
    a.X = X;
    a.Xlo = (const unsigned short*)Xlo;
    a.Y = Y;
    a.M = M;
    a.K = K;
    a.Bpad = Bpad;
    a.lda = lda;
    a.ldx = ldx;
    a.gx = pl.gx;
    a.gy = pl.gy;
    a.ksplit = pl.ksplit > 0 ? pl.ksplit : 1;
    return a;
}

// CP projections: P[b][r] over the rows of [Bf|Cf]^T [2Rp][Np] (partials layout with one
// split, in the accumulation type).
void launch_gemm_proj(int dt, const GemmPlan& pl, const void* BCt, const void* BCt_lo, int Np, int Rp, int Bpad,
                      const void* X, const void* Xlo, void* P, hipStream_t s) {
    const GemmArgs a = gemm_args(pl, BCt, BCt_lo, Np, X, Xlo, Np, P, 2 * Rp, Np, Bpad);
    switch (dt) {
        case DT_F64: gemm_go<DT_F64, MK_F64>(a, pl, s); break;
        case DT_F32: gemm_go<DT_F32, MK_F32>(a, pl, s); break;
        case DT_BF16: gemm_go<DT_BF16, MK_BF16>(a, pl, s); break;
        default: gemm_go<DT_BF16X3, MK_BF16X3>(a, pl, s); break;
    }
}

// CP projections and their Hadamard product in one pass: W[b][r] = lam_r (Bf^T u_b)_r
// (Cf^T u_b)_r over the row pairs (r, Rp + r) of [Bf|Cf]^T; W [Bpad][Rp] in the
// accumulation type.  The plan's column-tile width is kept, its row tiles are those of
// Rp rows.
void launch_gemm_proj_pair(int dt, const GemmPlan& pl0, const void* BCt, const void* BCt_lo, int Np, int Rp,
                           int Bpad, const void* X, const void* Xlo, const void* lam, void* W, hipStream_t s) {
    GemmPlan pl = pl0;
    pl.gx = (Rp + 15) / 16;
    pl.gy = Bpad / (16 * pl.fn);
    pl.blocks = (pl.gx * pl.gy + 7) / 8 * 8;
    GemmArgs a = gemm_args(pl, BCt, BCt_lo, Np, X, Xlo, Np, W, Rp, Np, Bpad);
    a.pair_off = (long long)Rp * Np;
    a.lam = lam;
    switch (dt) {
        case DT_F64: gemm_go<DT_F64, MK_F64, EPI_PAIR>(a, pl, s); break;
        case DT_F32: gemm_go<DT_F32, MK_F32, EPI_PAIR>(a, pl, s); break;
        case DT_BF16: gemm_go<DT_BF16, MK_BF16, EPI_PAIR>(a, pl, s); break;
        default: gemm_go<DT_BF16X3, MK_BF16X3, EPI_PAIR>(a, pl, s); break;
    }
}

// CP projections of factors with skew column pairs and their Hadamard product, from the
// pair form SK [P + R][Np] (SKEW epilogue): W [Bpad][Rp] in the accumulation type.
void launch_gemm_proj_skew(int dt, const GemmPlan& pl0, const void* SK, const void* SK_lo, int Np, int P, int layout,
                           int Rp, int Bpad, const void* X, const void* Xlo, const void* lam, void* W, hipStream_t s) {
    GemmPlan pl = pl0;
    pl.gx = (Rp / 2 + 15) / 16;
    pl.gy = Bpad / (16 * pl.fn);
    pl.blocks = (pl.gx * pl.gy + 7) / 8 * 8;
    GemmArgs a = gemm_args(pl, SK, SK_lo, Np, X, Xlo, Np, W, P, Np, Bpad);
    a.skew_P = P;
    a.skew_layout = layout;
    a.wstride = Rp;
    a.lam = lam;
    switch (dt) {
        case DT_F64: gemm_go<DT_F64, MK_F64, EPI_SKEW>(a, pl, s); break;
        case DT_F32: gemm_go<DT_F32, MK_F32, EPI_SKEW>(a, pl, s); break;
        case DT_BF16: gemm_go<DT_BF16, MK_BF16, EPI_SKEW>(a, pl, s); break;
        default: gemm_go<DT_BF16X3, MK_BF16X3, EPI_SKEW>(a, pl, s); break;
    }
}

// CP scatter: Y[b][i] = sum_r Af[i][r] W[b][r], W in FP32 (FP64 for DT_F64); the BF16
// formats contract their factor words with FP32 MFMA.
void launch_gemm_scatter(int dt, const GemmPlan& pl, const void* Af, const void* Af_lo, int N, int Rp, int Bpad,
                         const void* W, void* Y, hipStream_t s) {
    const GemmArgs a = gemm_args(pl, Af, Af_lo, Rp, W, nullptr, Rp, Y, N, Rp, Bpad);
    switch (dt) {
        case DT_F64: gemm_go<DT_F64, MK_F64>(a, pl, s); break;
        case DT_F32: gemm_go<DT_F32, MK_F32>(a, pl, s); break;
        case DT_BF16: gemm_go<DT_BF16, MK_F32>(a, pl, s); break;
        default: gemm_go<DT_BF16X3, MK_F32>(a, pl, s); break;
    }
}

// CP scatter of a step: y^n = Af W goes straight into the BDF right-hand side; with a
// diagonal stiffness (diag = 1) the kernel also solves for u^{n+1} and closes the step
// (one extra block), else it stores the right-hand side for the Helmholtz apply.
void launch_gemm_scatter_step(int dt, const GemmPlan& pl0, const void* Af, const void* Af_lo, int N, int Rp,
                              int Bpad, const void* W, const StepArgs& st, int diag, hipStream_t s) {
    GemmPlan pl = pl0;
    if (diag) pl.blocks = (pl.gx * pl.gy + 1 + 7) / 8 * 8;
    GemmArgs a = gemm_args(pl, Af, Af_lo, Rp, W, nullptr, Rp, nullptr, N, Rp, Bpad);
    a.st = st;
    if (diag) {
        switch (dt) {
            case DT_F64: gemm_go<DT_F64, MK_F64, EPI_UPDATE>(a, pl, s); break;
            case DT_F32: gemm_go<DT_F32, MK_F32, EPI_UPDATE>(a, pl, s); break;
            case DT_BF16: gemm_go<DT_BF16, MK_F32, EPI_UPDATE>(a, pl, s); break;
            default: gemm_go<DT_BF16X3, MK_F32, EPI_UPDATE>(a, pl, s); break;
        }
    } else {
        switch (dt) {
            case DT_F64: gemm_go<DT_F64, MK_F64, EPI_RHS>(a, pl, s); break;
            case DT_F32: gemm_go<DT_F32, MK_F32, EPI_RHS>(a, pl, s); break;
            case DT_BF16: gemm_go<DT_BF16, MK_F32, EPI_RHS>(a, pl, s); break;
            default: gemm_go<DT_BF16X3, MK_F32, EPI_RHS>(a, pl, s); break;
        }
    }
}

// Plain FP64 product Y[b][m] = sum_k A[m][k] X[b][k] (setup work).
void launch_gemm_f64(const GemmPlan& pl, const double* A, long long lda, const double* X, long long ldx, double* Y,
                     int M, int K, int Bpad, hipStream_t s) {
    const GemmArgs a = gemm_args(pl, A, nullptr, lda, X, nullptr, ldx, Y, M, K, Bpad);
    gemm_go<DT_F64, MK_F64>(a, pl, s);
}

void launch_gemm_f64_rows(const GemmPlan& pl, const double* A, long long lda, const double* X, long long ldx,
                          double* Y, int M, int K, int Bpad, int rows, hipStream_t s) {
    GemmArgs a = gemm_args(pl, A, nullptr, lda, X, nullptr, ldx, Y, M, K, Bpad);
    a.bstore = rows;
    gemm_go<DT_F64, MK_F64>(a, pl, s);
}

// Batched Helmholtz apply: U[b][i] = sum_m Hinv_k[i][m] rhs[b][m] (FP64), k from the
// device step counter; Hinv [3][N][Np], rhs [Bpad][Np].  With step arguments (st) U is
// u^{n+1}: stored into the state with its energy partials, and the step is closed (one
// extra block); else U goes to Y.
void launch_gemm_helm(const GemmPlan& pl0, const double* hinv, int N, int Np, int Bpad, const double* rhs,
                      const long long* stepp, double* Y, const StepArgs* st, hipStream_t s) {
    GemmPlan pl = pl0;
    if (st) pl.blocks = (pl.gx * pl.gy + 1 + 7) / 8 * 8;
    GemmArgs a = gemm_args(pl, hinv, nullptr, Np, rhs, nullptr, Np, Y, N, Np, Bpad);
    a.kstep = stepp;
    a.a_kstride = (long long)N * Np;
    if (st) {
        a.st = *st;
        gemm_go<DT_F64, MK_F64, EPI_FINISH>(a, pl, s);
    } else {
        gemm_go<DT_F64, MK_F64>(a, pl, s);
    }
}

}  // namespace rom
