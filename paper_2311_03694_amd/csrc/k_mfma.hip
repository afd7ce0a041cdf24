// k_mfma.hip -- batched contractions on the matrix cores (MFMA), for B trajectories.
//
// One kernel shape serves three products, Out[b][m] over a row operand A and a
// coefficient operand X ([Bpad][Kp], trajectory-major):
//   dense (Sec. 2.2, eq. Cu, the G-ROM term; "KR" = Khatri-Rao form):
//       Y[b][i] = sum_j S[j][b] * sum_k C[i][j][k] X[b][k],   S = X = u (per format),
//     i.e. C_(1) [N x N^2] times the Khatri-Rao columns u_b (x) u_b, without ever
//     forming u (x) u: the inner sum over k is an MFMA GEMM of the C slab at fixed j
//     against u, and each finished slab is weighted by u_j per column;
//   CP projections (Sec. 3.1, eq. tc_ap):  P[b][r] = sum_k [Bf|Cf]^T[r][k] X[b][k];
//   CP scatter:  Y[b][i] = sum_r Af[i][r] W[b][r],  W = lam .* s .* t (FP32 / FP64).
//
// Tiling (gfx950, wave64): a block is 4 wavefronts stacked along rows; a wavefront
// owns MW rows x BT columns as (MW/16) x (BT/16) tiles of 16x16 MFMA accumulators.
// The X tile [BT][kc] of the block's k-chunk is staged once in LDS (16-byte rows of
// odd stride: conflict-free fragment reads); A fragments stream from HBM straight
// into registers through a PF-deep prefetch ring.  The grid is (row tiles, column
// tiles, j-ranges x k-chunks); every block writes an FP32 (FP64) partial tile that the
// consumer sums in a fixed order.  Rows and the contracted index are padded to
// multiples of 8 with zeros, so every 16-byte lane vector is wholly inside or outside
// the k range and the tail is handled by predicated zero loads.
//
// MFMA kinds and accumulator layouts: kmfma.h.  A and X use the same (lane group,
// element) -> k map, so each issue pairs matching k.
#include "kmfma.h"

namespace rom {

// ---------------------------------------------------------------- the kernel

struct MfmaArgs {
    const void* A;                 // rows: [M][J][Kp] (KR) or [M][Kp]
    const unsigned short* Alo;     // BF16X3 low words of A
    const void* X;                 // [Bpad][Kp] in the MFMA operand format
    const unsigned short* Xlo;     // BF16X3 low words of X
    const void* S;                 // [J][s_stride] j-weights (KR): FP64 for MK_F64, else FP32
    void* part;                    // [nsplit][Bpad][M] partial sums (FP64 for MK_F64, else FP32)
    long long a_rowstride, a_jstride;
    int M, J, Kp, Bpad, s_stride;
    int kc, jc, nkc;               // k-chunk length (multiple of 2 KS), j-range length, k-chunks
    int kcp;                       // LDS row stride (elements) of the X tile
    int gx, gy, gz;                // work grid: row tiles, column tiles, splits
    const long long* kstep;        // non-null: A += (BDF order at *kstep - 1) * a_kstride
    long long a_kstride;
};

template <int ADT, int MKD, int MW, int BT, bool KR, bool NT>
__global__ __launch_bounds__(256) void k_mfma_rows(MfmaArgs p) {
    typedef MfmaT<MKD> Tr;
    typedef typename Tr::X XT;
    typedef typename Tr::Acc4 Acc4;
    typedef typename Tr::Acc Acc;
    // A lane loads two 16-byte halves (VEC elements each) of 32 contiguous bytes per row
    // and step, so the 16 rows of a fragment are read as whole 128-byte lines; half h
    // feeds the h-th group of MFMA issues.  One step covers KS2 = 2 KS of k.
    constexpr int KS = Tr::KS, VEC = Tr::VEC, VEC2 = 2 * VEC, KS2 = 2 * KS;
    constexpr int FM = MW / 16, FN = BT / 16, PF = (FM == 1 ? 6 : 3);
    constexpr bool X3 = (MKD == MK_BF16X3);
    extern __shared__ __attribute__((aligned(16))) char smem[];
    XT* xs = reinterpret_cast<XT*>(smem);
    unsigned short* xsl = reinterpret_cast<unsigned short*>(smem + (size_t)BT * p.kcp * sizeof(XT));
    Acc* ss = reinterpret_cast<Acc*>(smem + (size_t)BT * p.kcp * sizeof(XT) * (X3 ? 2 : 1));

    // XCD-aware decode of the linear block id: consecutive ids go round-robin to the 8
    // XCDs, so ids q, q+8, q+16, ... (one XCD) take consecutive work items, and the
    // column tiles of one (row tile, split) share that XCD's L2 for their C reads.
    const int T = p.gx * p.gy * p.gz;
    const int per = (T + 7) / 8;
    const int wi = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (wi >= T) return;
    const int by = wi % p.gy, rest = wi / p.gy;
    const int bx = rest % p.gx, bz = rest / p.gx;

    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, c16 = lane & 15;
    const int rowbase = (bx * 4 + w) * MW;
    const int b0 = by * BT;
    const int jr = bz / p.nkc, kci = bz - jr * p.nkc;
    const int kbeg = kci * p.kc;
    const int kend = min(p.Kp, kbeg + p.kc);
    const int jbeg = jr * p.jc;
    const int jend = min(p.J, jbeg + p.jc);
    const int klen = kend - kbeg;

    // ---- stage the X tile (and the j-weights of this block's j-range) in LDS
    {
        const int vecs_per_row = (p.kc + KS2) / VEC;     // the tile plus its zero region
        struct V2 { u32x4 h, l; };
        staged_copy<6, V2>(
            BT * vecs_per_row,
            [&](int idx) {
                const int col = idx / vecs_per_row, kv = (idx - col * vecs_per_row) * VEC;
                const int k = kbeg + kv;
                V2 v;
                v.h = u32x4{0u, 0u, 0u, 0u};
                v.l = u32x4{0u, 0u, 0u, 0u};
                if (k < kend) {
                    const size_t off = (size_t)(b0 + col) * p.Kp + k;
                    v.h = ld_plain<16>(reinterpret_cast<const XT*>(p.X) + off);
                    if constexpr (X3) v.l = ld_plain<16>(p.Xlo + off);
                }
                return v;
            },
            [&](int idx, const V2& v) {
                const int col = idx / vecs_per_row, kv = (idx - col * vecs_per_row) * VEC;
                *reinterpret_cast<u32x4*>(xs + (size_t)col * p.kcp + kv) = v.h;
                if constexpr (X3) *reinterpret_cast<u32x4*>(xsl + (size_t)col * p.kcp + kv) = v.l;
            });
        if constexpr (KR) {
            const int nj = jend - jbeg;
            staged_copy<8, Acc>(
                BT * nj,
                [&](int idx) {
                    const int jj = idx / BT, col = idx - jj * BT;
                    return reinterpret_cast<const Acc*>(p.S)[(size_t)(jbeg + jj) * p.s_stride + b0 + col];
                },
                [&](int idx, Acc v) {
                    const int jj = idx / BT, col = idx - jj * BT;
                    ss[col * p.jc + jj] = v;
                });
        }
    }

    // ---- per-lane row pointers (rows past M are clamped for loads, never stored);
    // an operator chosen by the BDF order of the current step starts at kbase
    const size_t kbase = p.kstep ? (size_t)(bdf_order(*p.kstep) - 1) * p.a_kstride : 0;
    size_t rowoff[FM];
#pragma unroll
    for (int f = 0; f < FM; ++f) {
        int r = rowbase + f * 16 + c16;
        r = r < p.M ? r : p.M - 1;
        rowoff[f] = kbase + (size_t)r * p.a_rowstride;
    }

    Acc4 Y[FM][FN], Z[FM][FN];
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int t = 0; t < FN; ++t) {
            Y[f][t] = Acc4{0, 0, 0, 0};
            Z[f][t] = Acc4{0, 0, 0, 0};
        }

    const int nks = (klen + KS2 - 1) / KS2;           // steps per j
    const int nj = jend - jbeg;
    const int nsteps = (nj > 0 && nks > 0) ? nj * nks : 0;
    const int nsteps_pad = (nsteps + PF - 1) / PF * PF;

    // Prefetch ring of A fragments, PF steps deep.  Steps past the end (the padding up
    // to a multiple of PF) reload the last valid step, which stays inside the
    // allocation, and read the zero region [kc, kc + KS2) of the LDS tile, so they add
    // nothing.  Lane vectors may run past kend inside a row (into the next row or the
    // zeroed slack after the tensor): they meet zeros of the LDS tile.
    u32x4 ah[PF][FM][2], al[PF][FM][2];
    int pj = 0, pks = 0;                                // producer position
    auto issue = [&](int d) {
        int jj = pj, ks = pks;
        if (jj >= nj) { jj = nj - 1; ks = nks - 1; }
        const size_t base = (size_t)(jbeg + jj) * p.a_jstride + kbeg + ks * KS2 + g * VEC2;
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int f = 0; f < FM; ++f)
                load_a<ADT, MKD, NT>(p.A, p.Alo, rowoff[f] + base + h * VEC, ah[d][f][h], al[d][f][h]);
        if (++pks == nks) { pks = 0; ++pj; }
    };
    if (nsteps > 0) {
#pragma unroll
        for (int d = 0; d < PF; ++d) issue(d);
    }
    __syncthreads();

    int cj = 0, cks = 0;                                // consumer position
    for (int s0 = 0; s0 < nsteps_pad; s0 += PF) {
#pragma unroll
        for (int d = 0; d < PF; ++d) {
            const int kl = (cj < nj ? cks * KS2 : p.kc) + g * VEC2;   // padding: zero region
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                u32x4 bh[FN], bl[FN];
#pragma unroll
                for (int t = 0; t < FN; ++t) {
                    const size_t o = (size_t)(t * 16 + c16) * p.kcp + kl + h * VEC;
                    bh[t] = *reinterpret_cast<const u32x4*>(xs + o);
                    if constexpr (X3) bl[t] = *reinterpret_cast<const u32x4*>(xsl + o);
                }
#pragma unroll
                for (int f = 0; f < FM; ++f)
#pragma unroll
                    for (int t = 0; t < FN; ++t) {
                        if constexpr (KR) mfma_step<MKD>(Z[f][t], ah[d][f][h], al[d][f][h], bh[t], bl[t]);
                        else mfma_step<MKD>(Y[f][t], ah[d][f][h], al[d][f][h], bh[t], bl[t]);
                    }
            }
            issue(d);
            if constexpr (KR) {
                if (cks == nks - 1 && cj < nj) {
#pragma unroll
                    for (int t = 0; t < FN; ++t) {
                        const Acc sj = ss[(t * 16 + c16) * p.jc + cj];
#pragma unroll
                        for (int f = 0; f < FM; ++f) {
                            Y[f][t] += sj * Z[f][t];
                            Z[f][t] = Acc4{0, 0, 0, 0};
                        }
                    }
                }
            }
            if (++cks == nks) { cks = 0; ++cj; }
        }
    }

    // ---- partial tile out: part[z][b][row]
    Acc* out = reinterpret_cast<Acc*>(p.part) + (size_t)bz * p.Bpad * p.M;
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int t = 0; t < FN; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = rowbase + f * 16 + (MKD == MK_F64 ? g + 4 * v : 4 * g + v);
                if (row < p.M) out[(size_t)(b0 + t * 16 + c16) * p.M + row] = Y[f][t][v];
            }
}

// ---------------------------------------------------------------- CP Hadamard

// W[b][r] = lam_r * s_r * t_r with s, t summed over the projection partials
// P[z][b][r] (r < Rp) and P[z][b][Rp + r]; padding trajectories get zeros.
template <class Acc>
__global__ void k_hadamard(const Acc* __restrict__ P, int nz, int Bpad, int B, int Rp,
                           const Acc* __restrict__ lam, Acc* __restrict__ W) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x, b = blockIdx.y;
    if (r >= Rp) return;
    Acc s = 0, t = 0;
    if (b < B) {
        // partials added in z order; 8 pairs of loads in flight
        const size_t zs = (size_t)Bpad * 2 * Rp;
        const Acc* pb = P + (size_t)b * 2 * Rp + r;
        int z = 0;
        for (; z + 8 <= nz; z += 8) {
            Acc vs[8], vt[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                vs[e] = pb[(size_t)(z + e) * zs];
                vt[e] = pb[(size_t)(z + e) * zs + Rp];
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                s += vs[e];
                t += vt[e];
            }
        }
        for (; z < nz; ++z) {
            s += pb[(size_t)z * zs];
            t += pb[(size_t)z * zs + Rp];
        }
    }
    W[(size_t)b * Rp + r] = lam[r] * s * t;
}

// ---------------------------------------------------------------- planning, launch

static const MfmaTile kMfmaTiles[] = {
    // rows per wavefront, columns per block (cap), blocks in the grid (target)
    {32, 64, 1024}, {16, 64, 1024}, {32, 64, 512}, {16, 64, 512},
    {32, 64, 2048}, {16, 64, 2048}, {32, 32, 1024}, {16, 32, 1024},
};

int mfma_variants() { return (int)(sizeof(kMfmaTiles) / sizeof(kMfmaTiles[0])); }
MfmaTile mfma_variant(int idx) {
    if (idx < 0 || idx >= mfma_variants()) idx = 0;
    return kMfmaTiles[idx];
}

// k covered by one kernel step (two MFMA issue groups)
static int mk_ks(int mk) { return 2 * (mk == MK_F64 ? 8 : mk == MK_F32 ? 16 : 32); }
static int mk_xbytes(int mk) { return mk == MK_F64 ? 8 : mk == MK_F32 ? 4 : 2; }

MfmaPlan mfma_plan(int mk, int M, int J, int Kp, int Bpad, MfmaTile t) {
    MfmaPlan pl{};
    pl.mw = t.mw;
    pl.bt = t.bt;
    while (pl.bt > 16 && Bpad % pl.bt != 0) pl.bt /= 2;
    const int KS = mk_ks(mk), eb = mk_xbytes(mk), xb = eb * (mk == MK_BF16X3 ? 2 : 1);
    const int kp_r = (Kp + KS - 1) / KS * KS;
    // k-chunk: the X tile gets at most 40 KB of LDS; chunks are balanced
    int kc_max = (40960 / (pl.bt * xb)) / KS * KS;
    if (kc_max < KS) kc_max = KS;
    const long long gxy = (long long)((M + 4 * pl.mw - 1) / (4 * pl.mw)) * (Bpad / pl.bt);
    const long long want = t.target > 0 ? t.target : 2048;     // blocks in the grid
    long long splits = (want + gxy - 1) / gxy;
    if (splits < 1) splits = 1;
    long long nk = (kp_r + kc_max - 1) / kc_max;
    if (J == 1 && splits > nk) {
        // no j index to split: cut the contracted index finer, keeping at least four
        // steps per block
        long long nk_max = kp_r / (4 * KS);
        if (nk_max < 1) nk_max = 1;
        nk = splits < nk_max ? splits : nk_max;
        if (nk < (kp_r + kc_max - 1) / kc_max) nk = (kp_r + kc_max - 1) / kc_max;
    }
    pl.kc = (int)(((kp_r / KS) + nk - 1) / nk) * KS;
    pl.nkc = (Kp + pl.kc - 1) / pl.kc;
    // j-ranges: enough splits for the block target; at most 16 KB of j-weights in LDS
    const int jc_max = 16384 / (pl.bt * (mk == MK_F64 ? 8 : 4));
    long long njr = (splits + pl.nkc - 1) / pl.nkc;
    if (njr < 1) njr = 1;
    if (njr > J) njr = J;
    pl.jc = (int)((J + njr - 1) / njr);
    if (J > 1 && pl.jc > jc_max) pl.jc = jc_max;
    pl.njr = (J + pl.jc - 1) / pl.jc;
    pl.nsplit = pl.njr * pl.nkc;
    // LDS row stride: the chunk plus a zero region of one step, rounded to an odd number
    // of 16-byte units (conflict-free fragment reads)
    int units = ((pl.kc + KS) * eb + 15) / 16;
    if (units % 2 == 0) units += 1;
    pl.kcp = units * 16 / eb;
    pl.lds = (size_t)pl.bt * pl.kcp * eb * (mk == MK_BF16X3 ? 2 : 1) +
             (J > 1 ? (size_t)pl.bt * pl.jc * (mk == MK_F64 ? 8 : 4) : 0);
    pl.grid_x = (M + 4 * pl.mw - 1) / (4 * pl.mw);
    pl.grid_y = Bpad / pl.bt;
    pl.blocks = (pl.grid_x * pl.grid_y * pl.nsplit + 7) / 8 * 8;
    return pl;
}

template <int ADT, int MKD, int MW, int BT, bool KR>
static void go(const MfmaArgs& a, const MfmaPlan& pl, hipStream_t s) {
    if (pl.grid_y > 1)
        hipLaunchKernelGGL((k_mfma_rows<ADT, MKD, MW, BT, KR, false>), dim3(pl.blocks), dim3(256), pl.lds, s, a);
    else
        hipLaunchKernelGGL((k_mfma_rows<ADT, MKD, MW, BT, KR, true>), dim3(pl.blocks), dim3(256), pl.lds, s, a);
}

template <int ADT, int MKD, bool KR>
static void go_tile(const MfmaArgs& a, const MfmaPlan& pl, hipStream_t s) {
    if (pl.mw == 16) {
        if (pl.bt == 64) go<ADT, MKD, 16, 64, KR>(a, pl, s);
        else if (pl.bt == 32) go<ADT, MKD, 16, 32, KR>(a, pl, s);
        else go<ADT, MKD, 16, 16, KR>(a, pl, s);
    } else {
        if (pl.bt == 64) go<ADT, MKD, 32, 64, KR>(a, pl, s);
        else if (pl.bt == 32) go<ADT, MKD, 32, 32, KR>(a, pl, s);
        else go<ADT, MKD, 32, 16, KR>(a, pl, s);
    }
}

static MfmaArgs fill_args(const MfmaPlan& pl, const void* A, const void* Alo, const void* X, const void* Xlo,
                          const void* S, void* part, long long rowstride, long long jstride, int M, int J,
                          int Kp, int Bpad, int s_stride) {
    MfmaArgs a{};
    a.A = A;
    a.Alo = (const unsigned short*)Alo;
    a.X = X;
    a.Xlo = (const unsigned short*)Xlo;
    a.S = S;
    a.part = part;
    a.a_rowstride = rowstride;
    a.a_jstride = jstride;
    a.M = M;
    a.J = J;
    a.Kp = Kp;
    a.Bpad = Bpad;
    a.s_stride = s_stride;
    a.kc = pl.kc;
    a.jc = pl.jc;
    a.nkc = pl.nkc;
    a.kcp = pl.kcp;
    a.gx = pl.grid_x;
    a.gy = pl.grid_y;
    a.gz = pl.nsplit;
    return a;
}

static int mk_of(int dt) { return dt == DT_F64 ? MK_F64 : dt == DT_F32 ? MK_F32 : dt == DT_BF16 ? MK_BF16 : MK_BF16X3; }

MfmaPlan mfma_dense_plan(int dt, int N, int Np, int Bpad, MfmaTile t) { return mfma_plan(mk_of(dt), N, N, Np, Bpad, t); }

void launch_mfma_dense(int dt, const MfmaPlan& pl, const void* C, const void* Clo, int N, int Np, int Bpad,
                       const void* X, const void* Xlo, const void* S, void* part, hipStream_t s) {
    const MfmaArgs a = fill_args(pl, C, Clo, X, Xlo, S, part, (long long)N * Np, Np, N, N, Np, Bpad, Bpad);
    switch (dt) {
        case DT_F64: go_tile<DT_F64, MK_F64, true>(a, pl, s); break;
        case DT_F32: go_tile<DT_F32, MK_F32, true>(a, pl, s); break;
        case DT_BF16: go_tile<DT_BF16, MK_BF16, true>(a, pl, s); break;
        default: go_tile<DT_BF16X3, MK_BF16X3, true>(a, pl, s); break;
    }
}

MfmaPlan mfma_proj_plan(int dt, int Np, int Rp, int Bpad, MfmaTile t) { return mfma_plan(mk_of(dt), 2 * Rp, 1, Np, Bpad, t); }

void launch_mfma_proj(int dt, const MfmaPlan& pl, const void* BCt, const void* BCt_lo, int Np, int Rp, int Bpad,
                      const void* X, const void* Xlo, void* part, hipStream_t s) {
    const MfmaArgs a = fill_args(pl, BCt, BCt_lo, X, Xlo, nullptr, part, Np, 0, 2 * Rp, 1, Np, Bpad, 0);
    switch (dt) {
        case DT_F64: go_tile<DT_F64, MK_F64, false>(a, pl, s); break;
        case DT_F32: go_tile<DT_F32, MK_F32, false>(a, pl, s); break;
        case DT_BF16: go_tile<DT_BF16, MK_BF16, false>(a, pl, s); break;
        default: go_tile<DT_BF16X3, MK_BF16X3, false>(a, pl, s); break;
    }
}

// The scatter's coefficient operand W is FP32 (FP64 for the FP64 format): the BF16
// formats contract their BF16 factor words against it with FP32 MFMA.
MfmaPlan mfma_scatter_plan(int dt, int N, int Rp, int Bpad, MfmaTile t) {
    return mfma_plan(dt == DT_F64 ? MK_F64 : MK_F32, N, 1, Rp, Bpad, t);
}

void launch_mfma_scatter(int dt, const MfmaPlan& pl, const void* Af, const void* Af_lo, int N, int Rp, int Bpad,
                         const void* W, void* part, hipStream_t s) {
    const MfmaArgs a = fill_args(pl, Af, Af_lo, W, nullptr, nullptr, part, Rp, 0, N, 1, Rp, Bpad, 0);
    switch (dt) {
        case DT_F64: go_tile<DT_F64, MK_F64, false>(a, pl, s); break;
        case DT_F32: go_tile<DT_F32, MK_F32, false>(a, pl, s); break;
        case DT_BF16: go_tile<DT_BF16, MK_F32, false>(a, pl, s); break;
        default: go_tile<DT_BF16X3, MK_F32, false>(a, pl, s); break;
    }
}

MfmaPlan mfma_helm_plan(int N, int Np, int Bpad, MfmaTile t) { return mfma_plan(MK_F64, N, 1, Np, Bpad, t); }

void launch_mfma_helm(const MfmaPlan& pl, const double* hinv, int N, int Np, int Bpad, const double* rhs,
                      const long long* stepp, double* part, hipStream_t s) {
    MfmaArgs a = fill_args(pl, hinv, nullptr, rhs, nullptr, nullptr, part, Np, 0, N, 1, Np, Bpad, 0);
    a.kstep = stepp;
    a.a_kstride = (long long)N * Np;
    go_tile<DT_F64, MK_F64, false>(a, pl, s);
}

void launch_hadamard(int dt, const void* P, int nz, int Bpad, int B, int Rp, const void* lam, void* W,
                     hipStream_t s) {
    dim3 grid((Rp + 255) / 256, Bpad);
    if (dt == DT_F64)
        hipLaunchKernelGGL(k_hadamard<double>, grid, dim3(256), 0, s, (const double*)P, nz, Bpad, B, Rp,
                           (const double*)lam, (double*)W);
    else
        hipLaunchKernelGGL(k_hadamard<float>, grid, dim3(256), 0, s, (const float*)P, nz, Bpad, B, Rp,
                           (const float*)lam, (float*)W);
}

}  // namespace rom
