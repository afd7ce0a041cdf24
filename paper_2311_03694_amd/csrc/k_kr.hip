// k_kr.hip -- the batched dense G-ROM term (Sec. 2.2, eq. Cu) on the matrix cores, with
// the coefficient operand held in registers.
//
//   Y[b][i] = sum_j S[j][b] Z_j[b][i],   Z_j[b][i] = sum_k C[i][j][k] X[b][k],
//
// X = u in the contraction format, S = u in the accumulation format (for BF16 the
// BF16-rounded value, so both positions see the same coefficient).  Over a fixed
// k-range the MFMA operand built from X does not depend on j: a wavefront loads its X
// fragments once, keeps them in registers and streams the slabs C[i][j][k-range] of
// its j's through a prefetch ring, so the inner loop reads only the tensor (each
// element once per column tile) and one LDS row of j-weights per j.  u (x) u is never
// formed; each finished Z_j is weighted per trajectory and added into Y (VALU).
//
// The tensor is read from a tiled copy made for this kernel,
//   Ct[i/16][j][k/VEC][i%16][k%VEC]   (VEC = elements per 16 bytes, rows padded to a
//   multiple of 16 and k to a multiple of one fragment step with zeros),
// in which one lane vector is 16 contiguous bytes of one row and the 64 lane vectors of
// a fragment load (16 rows x 4 k-groups) are 1 KB of contiguous memory; a block's loads
// walk one contiguous region.
//
// Block = 4 wavefronts over 16 rows i, 16*FN trajectories, a range of j and one
// k-chunk of at most 4 KW fragment steps (a step is one 16-byte lane vector: 32 k in
// BF16, 16 in FP32, 8 in FP64); wavefront w owns the w-th quarter of the chunk's steps
// and all wavefronts walk the same consecutive j's, so for each j the block reads one
// contiguous run of every row (and, when the chunk spans the row, consecutive j's are
// contiguous too: the tensor streams as in the single-trajectory kernel).  Column c16
// of accumulator tile t is trajectory b0 + c16*FN + t, so a lane's FN j-weights are
// contiguous in LDS.  The 4 wavefront tiles are added in LDS in a fixed order and the
// block writes one partial tile part[split][b][i] (split = j-range * chunks + chunk),
// which the consumer sums in a fixed order: results are deterministic.
//
// Prologue: the j-weights go straight from memory into LDS (global_load_lds) and the X
// fragments into registers; only after the barrier that publishes the j-weights is
// the tensor ring issued, so that barrier waits for small L2-resident loads rather
// than for the ring's HBM traffic.  A chunk's steps rarely split evenly over the 4
// wavefronts; a wavefront with one step fewer runs a copy of the loop with one
// MFMA step fewer per j instead of multiplying zero fragments.
#include <type_traits>

#include "kmfma.h"

namespace rom {

typedef __attribute__((address_space(1))) void* gptr_t;   // global (HBM) pointer
typedef __attribute__((address_space(3))) void* lptr_t;   // LDS pointer

struct KrArgs {
    const void* C;                 // tiled [ceil(M/16)][J][Kt/VEC][16][VEC], storage format
    const unsigned short* Clo;     // BF16X3 low words of C, same layout
    const void* X;                 // [Bpad][Kx] coefficients in the MFMA operand format
    const unsigned short* Xlo;     // BF16X3 low words of X
    const void* S;                 // [J][Bpad] j-weights (FP64 for MK_F64, else FP32)
    void* part;                    // [nsplit][Bpad][M] partial tiles (accumulation type)
    int M, J, Kt, Kx, Bpad;
    int ksteps, nkc, jc, njr, gx, gy;
};

// FN consecutive values from LDS (16-byte reads where the row allows them).
template <int FN, class Acc>
__device__ __forceinline__ void lds_row(const Acc* p, Acc (&v)[FN]) {
    constexpr int EV = 16 / (int)sizeof(Acc);
    if constexpr (FN % EV == 0) {
#pragma unroll
        for (int q = 0; q < FN / EV; ++q) {
            const u32x4 x = reinterpret_cast<const u32x4*>(p)[q];
            const Acc* e = reinterpret_cast<const Acc*>(&x);
#pragma unroll
            for (int i = 0; i < EV; ++i) v[q * EV + i] = e[i];
        }
    } else {
#pragma unroll
        for (int t = 0; t < FN; ++t) v[t] = p[t];
    }
}

template <int ADT, int MKD, int FN, int KW, int PF>
__global__ __launch_bounds__(256) void k_kr(KrArgs p) {
    typedef MfmaT<MKD> Tr;
    typedef typename Tr::X XT;
    typedef typename Tr::Acc Acc;
    typedef typename Tr::Acc4 Acc4;
    typedef typename Store<ADT>::T AT;
    constexpr int KS = Tr::KS, VEC = Tr::VEC, NC = 16 * FN;
    constexpr int EV = 16 / (int)sizeof(Acc);
    constexpr bool X3 = (MKD == MK_BF16X3);
    static_assert(1024 % (NC * (int)sizeof(Acc)) == 0, "a j-weight row must divide a 1 KB chunk");
    extern __shared__ __attribute__((aligned(16))) char smem[];
    Acc* sl = reinterpret_cast<Acc*>(smem);              // [jn + 1][NC] j-weights, row jn zero

    // XCD-aware decode: consecutive block ids go round-robin over the 8 XCDs, so ids
    // q, q+8, ... (one XCD) take consecutive work items; the column tiles of one (row
    // tile, chunk, j-range) are consecutive and share that XCD's L2 for their C reads.
    const int nwork = p.gx * p.gy * p.nkc * p.njr;
    const int per = (nwork + 7) / 8;
    const int wi = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (wi >= nwork) return;
    int rest = wi;
    const int by = rest % p.gy;
    rest /= p.gy;
    const int kci = rest % p.nkc;
    rest /= p.nkc;
    const int bx = rest % p.gx;
    const int jr = rest / p.gx;

    const int lane = threadIdx.x & 63, g = lane >> 4, c16 = lane & 15;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int rowbase = bx * 16, b0 = by * NC;
    // chunks hold ksteps / nkc or one more steps (at most 4 KW), split as evenly over
    // the wavefronts (at most KW each); a wavefront without steps points at the
    // chunk's first step and keeps zero X fragments
    const int nsb = p.ksteps / p.nkc, nse = p.ksteps - nsb * p.nkc;
    const int cs = nsb + (kci < nse ? 1 : 0);
    const int c0 = kci * nsb + (kci < nse ? kci : nse);
    const int wsb = cs / 4, wse = cs - wsb * 4;
    const int ns = wsb + (w < wse ? 1 : 0);
    const int s0 = ns > 0 ? c0 + w * wsb + (w < wse ? w : wse) : c0;
    const int nsa = ns > 0 ? ns : 1;                     // steps the loads address
    const int jbeg = jr * p.jc;
    const int jn = min(p.J, jbeg + p.jc) - jbeg;

    // ---- the lane's vectors of the tiled tensor: unit (s0 + s) * 4 + g of row c16 in
    // row tile bx (rows past M are zero rows of the tile and are never stored)
    const size_t nku = (size_t)(p.Kt / VEC);
    const size_t abase = ((((size_t)bx * p.J + jbeg) * nku + (size_t)s0 * 4 + g) * 16 + c16) * VEC;
    const size_t jstep = nku * 16 * VEC;
    constexpr size_t sstep = (size_t)64 * VEC;

    const int nq = jn;                                   // every wavefront walks all j's
    const int nq_pad = (nq + PF - 1) / PF * PF;

    // ---- j-weights of the block's j's and trajectories, copied straight into LDS
    // (global_load_lds: no registers, no wait until the barrier).  Wavefront w copies
    // the 1 KB chunks w, w+4, ... of the [jn][NC] rows; lane l's 16 bytes land at
    // byte 16 l of its chunk.  Lanes of rows past jn stay idle; columns past Bpad read
    // a valid weight instead (their X fragments are zero, so it multiplies zeros in
    // columns that are never stored).  Row jn (the weights of padding iterations) is
    // written as zeros with ordinary LDS stores.
    {
        constexpr int rowb = NC * (int)sizeof(Acc);     // divides 1024
        constexpr int rpc = 1024 / rowb;                 // rows per chunk
        const int nch = (jn + rpc - 1) / rpc;
        const int r_in = (lane * 16) / rowb, cb = (lane * 16) % rowb;
        const int col = cb / (int)sizeof(Acc);
        const int colc = b0 + col < p.Bpad ? col : 0;
        for (int c = w; c < nch; c += 4) {
            const int jj = c * rpc + r_in;
            if (jj < jn) {
                const Acc* src = reinterpret_cast<const Acc*>(p.S) + (size_t)(jbeg + jj) * p.Bpad + b0 + colc;
                __builtin_amdgcn_global_load_lds((gptr_t)src, (lptr_t)(smem + (size_t)c * 1024), 16, 0, 0);
            }
        }
        for (int e = threadIdx.x; e < NC / EV; e += 256)
            *reinterpret_cast<u32x4*>(sl + (size_t)jn * NC + e * EV) = u32x4{0u, 0u, 0u, 0u};
    }

    // ---- X fragments of the chunk for the lane's trajectories, zero past Kp, Bpad or
    // the chunk's last step (addresses clamped, zero selection after the barrier)
    u32x4 xh[KW][FN], xl[KW][FN];
    unsigned xok = 0;
#pragma unroll
    for (int s = 0; s < KW; ++s)
#pragma unroll
        for (int t = 0; t < FN; ++t) {
            const int k = (s0 + s) * KS + g * VEC;
            const int b = b0 + c16 * FN + t;
            if (s < ns && k < p.Kx && b < p.Bpad) xok |= 1u << (s * FN + t);
            const size_t o = (size_t)(b < p.Bpad ? b : p.Bpad - 1) * p.Kx + (k < p.Kx ? k : p.Kx - VEC);
            xh[s][t] = ld_plain<16>(reinterpret_cast<const XT*>(p.X) + o);
            if constexpr (X3) xl[s][t] = ld_plain<16>(p.Xlo + o);
            else xl[s][t] = u32x4{0u, 0u, 0u, 0u};
        }

    // The copies above must land before any wavefront reads the j-weights; the
    // tensor ring is issued after the barrier, so this wait covers only the small
    // L2-resident loads and the ring's HBM traffic starts right behind it.
    __syncthreads();
#pragma unroll
    for (int s = 0; s < KW; ++s)
#pragma unroll
        for (int t = 0; t < FN; ++t)
            if (!((xok >> (s * FN + t)) & 1u)) {
                xh[s][t] = u32x4{0u, 0u, 0u, 0u};
                xl[s][t] = u32x4{0u, 0u, 0u, 0u};
            }

    // Prefetch ring of PF iterations (one j each).  The loop body has no branches and
    // its loads are never predicated (issues past the last j repeat it, steps past the
    // wavefront's last step repeat that step), so the compiler counts them exactly and
    // waits only for the slot it consumes.  Padding iterations up to a multiple of PF
    // take the zero j-weight row.
    u32x4 ah[PF][KW], al[PF][KW];
    int qp = 0;
    auto issue = [&](int d) {
        const int q = qp < nq ? qp : nq - 1;
        const size_t o = abase + (size_t)q * jstep;
#pragma unroll
        for (int s = 0; s < KW; ++s) {
            const size_t os = o + (size_t)(s < nsa ? s : nsa - 1) * sstep;
            ah[d][s] = ld_plain<16>(reinterpret_cast<const AT*>(p.C) + os);
            if constexpr (X3) al[d][s] = ld_plain<16>(p.Clo + os);
        }
        ++qp;
    };
#pragma unroll
    for (int d = 0; d < PF; ++d) {
        issue(d);
        __builtin_amdgcn_sched_barrier(0);               // slot order: slot 0 lands first
    }

    Acc4 Y[FN];
#pragma unroll
    for (int t = 0; t < FN; ++t) Y[t] = Acc4{0, 0, 0, 0};

    // The loop issues NSC fragment steps per j.  A wavefront with one step fewer than
    // KW (the chunk's steps do not split evenly) runs the NSC = KW - 1 copy instead of
    // multiplying zero fragments; the rare other counts use the KW copy with zero
    // fragments past their last step.
    // The j-weights are read one iteration ahead, so the LDS latency overlaps the
    // matrix work instead of stalling the fold.
    auto run = [&](auto nsc) {
        constexpr int NSC = decltype(nsc)::value;
        Acc svn[FN];
        lds_row<FN>(sl + c16 * FN, svn);                 // row 0 (jn >= 1)
        for (int q0 = 0; q0 < nq_pad; q0 += PF) {
#pragma unroll
            for (int d = 0; d < PF; ++d) {
                const int q = q0 + d;
                Acc sv[FN];
#pragma unroll
                for (int t = 0; t < FN; ++t) sv[t] = svn[t];
                const int jnext = q + 1 < nq ? q + 1 : jn;
                lds_row<FN>(sl + (size_t)jnext * NC + c16 * FN, svn);
                Acc4 Z[FN];
#pragma unroll
                for (int t = 0; t < FN; ++t) Z[t] = Acc4{0, 0, 0, 0};
#pragma unroll
                for (int s = 0; s < NSC; ++s)
#pragma unroll
                    for (int t = 0; t < FN; ++t) mfma_step<MKD>(Z[t], ah[d][s], al[d][s], xh[s][t], xl[s][t]);
#pragma unroll
                for (int t = 0; t < FN; ++t) Y[t] += sv[t] * Z[t];
                issue(d);
                // keep this slot's loads ahead of the next iterations (arithmetic and
                // LDS may move across, global loads may not)
                __builtin_amdgcn_sched_barrier(0x78F);
            }
        }
    };
    if constexpr (KW > 1) {
        if (ns == KW - 1) run(std::integral_constant<int, KW - 1>{});
        else run(std::integral_constant<int, KW>{});
    } else {
        run(std::integral_constant<int, KW>{});
    }

    // ---- add the 4 wavefront tiles in LDS (fixed order) and write the partial tile
    __syncthreads();                                     // every wavefront is done with sl
    Acc* red = reinterpret_cast<Acc*>(smem);             // [4][FN][4][64]
#pragma unroll
    for (int t = 0; t < FN; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) red[((w * FN + t) * 4 + v) * 64 + lane] = Y[t][v];
    __syncthreads();
    Acc* out = reinterpret_cast<Acc*>(p.part) + (size_t)(jr * p.nkc + kci) * p.Bpad * p.M;
    for (int e = threadIdx.x; e < 256 * FN; e += 256) {
        const int cl = e >> 4, rr = e & 15;              // local trajectory, local row
        const int t = cl % FN, cc = cl / FN;
        const int gg = MKD == MK_F64 ? (rr & 3) : (rr >> 2);
        const int v = MKD == MK_F64 ? (rr >> 2) : (rr & 3);
        const int ln = gg * 16 + cc;
        Acc sum = red[(t * 4 + v) * 64 + ln];
#pragma unroll
        for (int w2 = 1; w2 < 4; ++w2) sum += red[((w2 * FN + t) * 4 + v) * 64 + ln];
        const int row = rowbase + rr, b = b0 + cl;
        if (row < p.M && b < p.Bpad) out[(size_t)b * p.M + row] = sum;
    }
}

// ---------------------------------------------------------------- variants and plans

// Per arithmetic kind: trajectories per block / 16 (FN), fragment steps per wavefront
// (KW), prefetch depth in j's (PF) and the number of blocks the device runs at once
// with this shape (256 CUs x blocks per CU), which the j-split is planned against.
struct KrTile { int fn, kw, pf, slots; };
constexpr int kKrVariants = 8;
template <int MKD> struct KrTab;
template <> struct KrTab<MK_F64> {
    static constexpr KrTile t[kKrVariants] = {{4, 4, 3, 256}, {4, 4, 3, 512}, {8, 2, 3, 256}, {4, 2, 4, 512},
                                              {2, 4, 3, 256}, {2, 8, 2, 256}, {1, 8, 3, 256}, {1, 4, 4, 512}};
};
template <> struct KrTab<MK_F32> {
    static constexpr KrTile t[kKrVariants] = {{8, 4, 3, 256}, {8, 4, 3, 512}, {16, 2, 3, 256}, {4, 8, 3, 256},
                                              {4, 8, 3, 512}, {8, 2, 4, 512}, {2, 8, 3, 256}, {1, 8, 4, 256}};
};
template <> struct KrTab<MK_BF16> {
    static constexpr KrTile t[kKrVariants] = {{16, 2, 6, 256}, {4, 4, 5, 512}, {8, 4, 4, 256}, {4, 4, 3, 512},
                                              {8, 2, 6, 512},  {2, 4, 4, 512},  {4, 4, 4, 512}, {1, 8, 4, 256}};
};
template <> struct KrTab<MK_BF16X3> {
    static constexpr KrTile t[kKrVariants] = {{8, 2, 4, 256}, {8, 2, 4, 512}, {16, 1, 6, 256}, {4, 4, 4, 256},
                                              {4, 4, 4, 512}, {4, 2, 6, 512}, {2, 4, 4, 256}, {1, 4, 4, 256}};
};

static int mk_of_dt(int dt) { return dt == DT_F64 ? MK_F64 : dt == DT_F32 ? MK_F32 : dt == DT_BF16 ? MK_BF16 : MK_BF16X3; }

static KrTile kr_tile(int mk, int v) {
    switch (mk) {
        case MK_F64: return KrTab<MK_F64>::t[v];
        case MK_F32: return KrTab<MK_F32>::t[v];
        case MK_BF16: return KrTab<MK_BF16>::t[v];
        default: return KrTab<MK_BF16X3>::t[v];
    }
}

int kr_variants() { return kKrVariants; }

// Default variant: the first one (in order of preference) whose column tile does not
// exceed the padded batch.
static int kr_default(int mk, int Bpad) {
    const int nct = Bpad / 16;
    for (int v = 0; v < kKrVariants; ++v)
        if (kr_tile(mk, v).fn <= nct) return v;
    return kKrVariants - 1;
}

int kr_tiled_k(int dt, int N) {
    const int KS = dt == DT_F64 ? 8 : dt == DT_F32 ? 16 : 32;
    return (N + KS - 1) / KS * KS;
}

KrPlan kr_plan(int dt, int M, int J, int Kt, int Bpad, int v, size_t lds_max) {
    const int mk = mk_of_dt(dt);
    if (v < 0 || v >= kKrVariants) v = kr_default(mk, Bpad);
    const KrTile t = kr_tile(mk, v);
    KrPlan pl{};
    pl.v = v;
    pl.fn = t.fn;
    pl.kw = t.kw;
    pl.pf = t.pf;
    const int KS = mk == MK_F64 ? 8 : mk == MK_F32 ? 16 : 32;
    const size_t accb = mk == MK_F64 ? 8 : 4;
    const int NC = 16 * t.fn;
    pl.ksteps = Kt / KS;
    pl.nkc = (pl.ksteps + 4 * t.kw - 1) / (4 * t.kw);
    pl.gx = (M + 15) / 16;
    pl.gy = (Bpad + NC - 1) / NC;
    // j-ranges: at least as many as the LDS copy of the j-weights needs (and at least
    // PF j per block); among those, the count that minimizes rounds of `slots`
    // concurrent blocks times the j's per block plus a prologue allowance of 8 j
    const long long base = (long long)pl.gx * pl.gy * pl.nkc;
    long long jc_max = (long long)(lds_max / ((size_t)NC * accb)) - 1;
    if (jc_max < 4) jc_max = 4;
    long long njr_lo = (J + jc_max - 1) / jc_max;
    long long njr_cap = (J + t.pf - 1) / t.pf;
    if (njr_cap < njr_lo) njr_cap = njr_lo;
    long long njr = njr_lo, best = -1;
    for (long long n = njr_lo; n <= njr_cap && n <= njr_lo + 256; ++n) {
        const long long rounds = (base * n + t.slots - 1) / t.slots;
        const long long cost = rounds * ((J + n - 1) / n + 8);
        if (best < 0 || cost < best) {
            best = cost;
            njr = n;
        }
    }
    // j per block: a multiple of PF (no padding iterations) unless that would exceed
    // the LDS copy
    const int jq = t.pf;
    pl.jc = (int)((J + njr - 1) / njr);
    if ((pl.jc + jq - 1) / jq * jq <= jc_max) pl.jc = (pl.jc + jq - 1) / jq * jq;
    pl.njr = (J + pl.jc - 1) / pl.jc;
    pl.nsplit = pl.nkc * pl.njr;
    const size_t s_bytes = (size_t)(pl.jc + 1) * NC * accb, r_bytes = (size_t)1024 * t.fn * accb;
    pl.lds = s_bytes > r_bytes ? s_bytes : r_bytes;
    pl.blocks = (int)((base * pl.njr + 7) / 8 * 8);
    return pl;
}

template <int ADT, int MKD, int V>
static void kr_go_v(const KrArgs& a, const KrPlan& pl, hipStream_t s) {
    constexpr KrTile t = KrTab<MKD>::t[V];
    hipLaunchKernelGGL((k_kr<ADT, MKD, t.fn, t.kw, t.pf>), dim3(pl.blocks), dim3(256), pl.lds, s, a);
}

template <int ADT, int MKD, int V>
static hipError_t kr_attr_v(size_t lds) {
    constexpr KrTile t = KrTab<MKD>::t[V];
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_kr<ADT, MKD, t.fn, t.kw, t.pf>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <int ADT, int MKD>
static void kr_go(const KrArgs& a, const KrPlan& pl, hipStream_t s) {
    switch (pl.v) {
        case 0: kr_go_v<ADT, MKD, 0>(a, pl, s); break;
        case 1: kr_go_v<ADT, MKD, 1>(a, pl, s); break;
        case 2: kr_go_v<ADT, MKD, 2>(a, pl, s); break;
        case 3: kr_go_v<ADT, MKD, 3>(a, pl, s); break;
        case 4: kr_go_v<ADT, MKD, 4>(a, pl, s); break;
        case 5: kr_go_v<ADT, MKD, 5>(a, pl, s); break;
        case 6: kr_go_v<ADT, MKD, 6>(a, pl, s); break;
        default: kr_go_v<ADT, MKD, 7>(a, pl, s); break;
    }
}

template <int ADT, int MKD>
static hipError_t kr_attr(size_t lds) {
    hipError_t e = hipSuccess, q;
    if ((q = kr_attr_v<ADT, MKD, 0>(lds)) != hipSuccess) e = q;
    if ((q = kr_attr_v<ADT, MKD, 1>(lds)) != hipSuccess) e = q;
    if ((q = kr_attr_v<ADT, MKD, 2>(lds)) != hipSuccess) e = q;
    if ((q = kr_attr_v<ADT, MKD, 3>(lds)) != hipSuccess) e = q;
    if ((q = kr_attr_v<ADT, MKD, 4>(lds)) != hipSuccess) e = q;
    if ((q = kr_attr_v<ADT, MKD, 5>(lds)) != hipSuccess) e = q;
    if ((q = kr_attr_v<ADT, MKD, 6>(lds)) != hipSuccess) e = q;
    if ((q = kr_attr_v<ADT, MKD, 7>(lds)) != hipSuccess) e = q;
    return e;
}

hipError_t krs_set_lds_limit(size_t lds);

hipError_t kr_set_lds_limit(size_t lds) {
    hipError_t e = hipSuccess, q;
    if ((q = kr_attr<DT_F64, MK_F64>(lds)) != hipSuccess) e = q;
    if ((q = kr_attr<DT_F32, MK_F32>(lds)) != hipSuccess) e = q;
    if ((q = kr_attr<DT_BF16, MK_BF16>(lds)) != hipSuccess) e = q;
    if ((q = kr_attr<DT_BF16X3, MK_BF16X3>(lds)) != hipSuccess) e = q;
    if ((q = krs_set_lds_limit(lds)) != hipSuccess) e = q;
    return e;
}

void launch_kr_dense(int dt, const KrPlan& pl, const void* Ct, const void* Ct_lo, int N, int Np, int Bpad,
                     const void* X, const void* Xlo, const void* S, void* part, hipStream_t s) {
    KrArgs a{};
    a.C = Ct;
    a.Clo = (const unsigned short*)Ct_lo;
    a.X = X;
    a.Xlo = (const unsigned short*)Xlo;
    a.S = S;
    a.part = part;
    a.M = N;
    a.J = N;
    a.Kt = kr_tiled_k(dt, N);
    a.Kx = Np;
    a.Bpad = Bpad;
    a.ksteps = pl.ksteps;
    a.nkc = pl.nkc;
    a.jc = pl.jc;
    a.njr = pl.njr;
    a.gx = pl.gx;
    a.gy = pl.gy;
    switch (dt) {
        case DT_F64: kr_go<DT_F64, MK_F64>(a, pl, s); break;
        case DT_F32: kr_go<DT_F32, MK_F32>(a, pl, s); break;
        case DT_BF16: kr_go<DT_BF16, MK_BF16>(a, pl, s); break;
        default: kr_go<DT_BF16X3, MK_BF16X3>(a, pl, s); break;
    }
}

// ---------------------------------------------------------------- shared-tile variant
//
// k_krs: the same contraction with the tensor tile shared through LDS.  A block is 8
// wavefronts over 16 rows, 4*16*FN trajectories, one k-chunk of at most KC fragment
// steps and a range of j.  Wavefront w takes column group w%4 (16*FN trajectories)
// and j parity w/4: in iteration it the block handles j = 2it and 2it+1, each half of
// the wavefronts one of them.  Every wavefront holds the X fragments of its columns
// over the whole chunk (KC steps), so the per-j weighting costs 4 FMAs per 16x16 tile
// against KC MFMA steps.  The two tensor slabs of an iteration are read from HBM once
// per block: each wavefront loads at most two 1 KB fragments of them into registers
// P iterations ahead, stores them into one of two LDS slots after the barrier that
// frees it, and all wavefronts read their A operands from LDS.  The two parities are
// added in LDS at the end, in a fixed order, and the block writes one partial tile
// part[split][b][i] like k_kr.
struct KrsTile { int fn, kc, p; };
constexpr int kKrsVariants = 4;
template <int MKD> struct KrsTab;
template <> struct KrsTab<MK_F64> {
    static constexpr KrsTile t[kKrsVariants] = {{2, 7, 3}, {2, 8, 2}, {2, 4, 3}, {1, 8, 3}};
};
template <> struct KrsTab<MK_F32> {
    static constexpr KrsTile t[kKrsVariants] = {{4, 7, 2}, {4, 8, 2}, {4, 4, 3}, {2, 8, 3}};
};
template <> struct KrsTab<MK_BF16> {
    static constexpr KrsTile t[kKrsVariants] = {{4, 7, 2}, {4, 8, 2}, {4, 4, 3}, {2, 8, 3}};
};
template <> struct KrsTab<MK_BF16X3> {
    static constexpr KrsTile t[kKrsVariants] = {{4, 3, 2}, {2, 7, 2}, {2, 4, 3}, {2, 8, 2}};
};

template <int ADT, int MKD, int FN, int KC, int P>
__global__ __launch_bounds__(512) void k_krs(KrArgs p) {
    typedef MfmaT<MKD> Tr;
    typedef typename Tr::X XT;
    typedef typename Tr::Acc Acc;
    typedef typename Tr::Acc4 Acc4;
    typedef typename Store<ADT>::T AT;
    constexpr int KS = Tr::KS, VEC = Tr::VEC;
    constexpr int NCW = 16 * FN, NCB = 4 * NCW;          // columns per wavefront, per block
    constexpr int EV = 16 / (int)sizeof(Acc);
    constexpr bool X3 = (MKD == MK_BF16X3);
    constexpr int NH = X3 ? 2 : 1;                       // A words per element
    constexpr int SLOT = 2 * KC * 1024 * NH;             // bytes of one ring slot
    static_assert(1024 % (NCB * (int)sizeof(Acc)) == 0 || (NCB * (int)sizeof(Acc)) % 1024 == 0,
                  "j-weight rows and 1 KB chunks must nest");
    extern __shared__ __attribute__((aligned(16))) char smem[];
    char* ring = smem;                                   // [2 slots][hi, lo][2 parities][KC][1 KB]
    Acc* sl = reinterpret_cast<Acc*>(smem + 2 * SLOT);   // [jn + 1][NCB] j-weights, row jn zero

    const int nwork = p.gx * p.gy * p.nkc * p.njr;
    const int per = (nwork + 7) / 8;
    const int wi = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (wi >= nwork) return;
    int rest = wi;
    const int by = rest % p.gy;
    rest /= p.gy;
    const int kci = rest % p.nkc;
    rest /= p.nkc;
    const int bx = rest % p.gx;
    const int jr = rest / p.gx;

    const int lane = threadIdx.x & 63, g = lane >> 4, c16 = lane & 15;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int cg = w & 3, jp = w >> 2;
    const int rowbase = bx * 16, b0 = by * NCB, cb0 = b0 + cg * NCW;
    const int nsb = p.ksteps / p.nkc, nse = p.ksteps - nsb * p.nkc;
    const int cs = nsb + (kci < nse ? 1 : 0);            // steps of this chunk (<= KC)
    const int c0 = kci * nsb + (kci < nse ? kci : nse);
    const int jbeg = jr * p.jc;
    const int jn = min(p.J, jbeg + p.jc) - jbeg;
    const int nit = (jn + 1) / 2;                        // iterations (pairs of j)

    // ---- j-weights straight into LDS (rows [0, jn), 1 KB chunks over the 8
    // wavefronts), row jn zero; columns past Bpad read a valid weight (their X
    // fragments are zero and they are never stored)
    {
        constexpr int rowb = NCB * (int)sizeof(Acc);
        const int nbytes = jn * rowb;
        const int nch = (nbytes + 1023) / 1024;
        for (int c = w; c < nch; c += 8) {
            const int byte = c * 1024 + lane * 16;
            const int jj = byte / rowb, col = (byte - jj * rowb) / (int)sizeof(Acc);
            if (jj < jn) {
                const int colc = b0 + col < p.Bpad ? col : 0;
                const Acc* src = reinterpret_cast<const Acc*>(p.S) + (size_t)(jbeg + jj) * p.Bpad + b0 + colc;
                __builtin_amdgcn_global_load_lds((gptr_t)src, (lptr_t)(reinterpret_cast<char*>(sl) + (size_t)c * 1024), 16,
                                                 0, 0);
            }
        }
        for (int e = threadIdx.x; e < NCB / EV; e += 512)
            *reinterpret_cast<u32x4*>(sl + (size_t)jn * NCB + e * EV) = u32x4{0u, 0u, 0u, 0u};
    }

    // ---- X fragments of the wavefront's columns over the chunk
    u32x4 xh[KC][FN], xl[KC][FN];
    unsigned long long xok = 0;
#pragma unroll
    for (int s = 0; s < KC; ++s)
#pragma unroll
        for (int t = 0; t < FN; ++t) {
            const int k = (c0 + s) * KS + g * VEC;
            const int b = cb0 + c16 * FN + t;
            if (s < cs && k < p.Kx && b < p.Bpad) xok |= 1ull << (s * FN + t);
            const size_t o = (size_t)(b < p.Bpad ? b : p.Bpad - 1) * p.Kx + (k < p.Kx ? k : p.Kx - VEC);
            xh[s][t] = ld_plain<16>(reinterpret_cast<const XT*>(p.X) + o);
            if constexpr (X3) xl[s][t] = ld_plain<16>(p.Xlo + o);
            else xl[s][t] = u32x4{0u, 0u, 0u, 0u};
        }
    __syncthreads();                                     // j-weights published
#pragma unroll
    for (int s = 0; s < KC; ++s)
#pragma unroll
        for (int t = 0; t < FN; ++t)
            if (!((xok >> (s * FN + t)) & 1ull)) {
                xh[s][t] = u32x4{0u, 0u, 0u, 0u};
                xl[s][t] = u32x4{0u, 0u, 0u, 0u};
            }

    // ---- the two tensor slabs of an iteration: fragment f = par * cs + s (step s of
    // j = 2 it + par); wavefront w carries fragments w and w + 8.  Loads are
    // unconditional (fragments past 2 cs repeat the last one and are not stored; j past
    // the range repeats its last j, whose weight row is zero).
    const size_t nku = (size_t)(p.Kt / VEC);
    int fpar[2], fs[2];
    bool fval[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int f = w + 8 * h;
        fval[h] = f < 2 * cs;
        const int ff = fval[h] ? f : 2 * cs - 1;
        fpar[h] = ff >= cs ? 1 : 0;
        fs[h] = ff - fpar[h] * cs;
    }
    auto goff = [&](int it, int h) -> size_t {
        int j = 2 * it + fpar[h];
        j = j < jn ? j : jn - 1;
        return ((((size_t)bx * p.J + jbeg + j) * nku + (size_t)(c0 + fs[h]) * 4) * 16) * VEC + (size_t)lane * VEC;
    };
    u32x4 rs[P][2], rl[P][2];
    auto gload = [&](int it, int st) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const size_t o = goff(it, h);
            rs[st][h] = ld_plain<16>(reinterpret_cast<const AT*>(p.C) + o);
            if constexpr (X3) rl[st][h] = ld_plain<16>(p.Clo + o);
        }
    };
    auto swrite = [&](int st, int slot) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
            if (fval[h]) {
                char* d = ring + (size_t)slot * SLOT + (size_t)(fpar[h] * KC + fs[h]) * 1024 + lane * 16;
                *reinterpret_cast<u32x4*>(d) = rs[st][h];
                if constexpr (X3) *reinterpret_cast<u32x4*>(d + 2 * KC * 1024) = rl[st][h];
            }
    };

#pragma unroll
    for (int q = 0; q < P; ++q) {
        gload(q, q);
        __builtin_amdgcn_sched_barrier(0);
    }
    swrite(0, 0);
    __syncthreads();
    gload(P, 0);
    __builtin_amdgcn_sched_barrier(0);

    Acc4 Y[FN];
#pragma unroll
    for (int t = 0; t < FN; ++t) Y[t] = Acc4{0, 0, 0, 0};

    auto run = [&](auto nsc) {
        constexpr int NSC = decltype(nsc)::value;
        Acc svn[FN];
        lds_row<FN>(sl + (size_t)(jp < jn ? jp : jn) * NCB + cg * NCW + c16 * FN, svn);
        // unrolled by P so that every register stage index is a constant (T(q) sits in
        // stage q % P); iterations past nit (up to a multiple of P) take the zero
        // j-weight row, so the body has no branches
        const int nit_pad = (nit + P - 1) / P * P;
        for (int it0 = 0; it0 < nit_pad; it0 += P) {
#pragma unroll
            for (int d = 0; d < P; ++d) {
                const int it = it0 + d;
                const int slot = it & 1;
                Acc sv[FN];
#pragma unroll
                for (int t = 0; t < FN; ++t) sv[t] = svn[t];
                const int jnext = 2 * (it + 1) + jp;
                lds_row<FN>(sl + (size_t)(jnext < jn ? jnext : jn) * NCB + cg * NCW + c16 * FN, svn);
                const char* base = ring + (size_t)slot * SLOT + (size_t)jp * KC * 1024 + lane * 16;
                Acc4 Z[FN];
#pragma unroll
                for (int t = 0; t < FN; ++t) Z[t] = Acc4{0, 0, 0, 0};
#pragma unroll
                for (int s = 0; s < NSC; ++s) {
                    // steps past the chunk (only in the rare copies with NSC > cs) read the
                    // chunk's last step, which holds finite data; their X fragments are zero
                    const int sr = s < cs ? s : cs - 1;
                    const u32x4 a = *reinterpret_cast<const u32x4*>(base + (size_t)sr * 1024);
                    u32x4 al = u32x4{0u, 0u, 0u, 0u};
                    if constexpr (X3) al = *reinterpret_cast<const u32x4*>(base + (size_t)sr * 1024 + 2 * KC * 1024);
#pragma unroll
                    for (int t = 0; t < FN; ++t) mfma_step<MKD>(Z[t], a, al, xh[s][t], xl[s][t]);
                }
#pragma unroll
                for (int t = 0; t < FN; ++t) Y[t] += sv[t] * Z[t];
                // iteration it + 1's slabs into the other slot (read last in iteration
                // it - 1), then the barrier that publishes them and frees this slot; the
                // stores stay after the matrix work (hoisted, they would wait for their
                // loads early and shorten the prefetch)
                __builtin_amdgcn_sched_barrier(0);
                swrite((d + 1) % P, slot ^ 1);
                __syncthreads();
                gload(it + 1 + P, (d + 1) % P);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    };
    // one copy of the loop: a chunk shorter than KC multiplies zero X fragments in its
    // last steps (a second copy for KC - 1 steps made the compiler drain the ring)
    run(std::integral_constant<int, KC>{});

    // ---- add the two parities in LDS (fixed order) and write the partial tile
    __syncthreads();
    Acc* red = reinterpret_cast<Acc*>(smem);             // [8][FN][4][64]
#pragma unroll
    for (int t = 0; t < FN; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) red[((w * FN + t) * 4 + v) * 64 + lane] = Y[t][v];
    __syncthreads();
    Acc* out = reinterpret_cast<Acc*>(p.part) + (size_t)(jr * p.nkc + kci) * p.Bpad * p.M;
    for (int e = threadIdx.x; e < 16 * NCB; e += 512) {
        const int cb = e >> 4, rr = e & 15;              // block column, local row
        const int gq = cb / NCW, cl = cb - gq * NCW;     // column group, column within it
        const int t = cl % FN, cc = cl / FN;
        const int gg = MKD == MK_F64 ? (rr & 3) : (rr >> 2);
        const int v = MKD == MK_F64 ? (rr >> 2) : (rr & 3);
        const int ln = gg * 16 + cc;
        const Acc sum = red[((gq * FN + t) * 4 + v) * 64 + ln] + red[(((gq + 4) * FN + t) * 4 + v) * 64 + ln];
        const int row = rowbase + rr, b = b0 + cb;
        if (row < p.M && b < p.Bpad) out[(size_t)b * p.M + row] = sum;
    }
}

template <int MKD>
static KrsTile krs_tile(int v) {
    return KrsTab<MKD>::t[v];
}

static KrsTile krs_tile_mk(int mk, int v) {
    switch (mk) {
        case MK_F64: return krs_tile<MK_F64>(v);
        case MK_F32: return krs_tile<MK_F32>(v);
        case MK_BF16: return krs_tile<MK_BF16>(v);
        default: return krs_tile<MK_BF16X3>(v);
    }
}

// Same split rules as kr_plan, for 256 concurrent blocks of 8 wavefronts; the LDS holds
// the two ring slots and the j-weights of a block's j's.
KrPlan krs_plan(int dt, int M, int J, int Kt, int Bpad, int v, size_t lds_max) {
    const int mk = mk_of_dt(dt);
    if (v < 0 || v >= kKrsVariants) v = 0;
    const KrsTile t = krs_tile_mk(mk, v);
    KrPlan pl{};
    pl.v = v;
    pl.fn = t.fn;
    pl.kw = t.kc;
    pl.pf = t.p;
    const int KS = mk == MK_F64 ? 8 : mk == MK_F32 ? 16 : 32;
    const size_t accb = mk == MK_F64 ? 8 : 4;
    const int NCB = 64 * t.fn;
    const size_t slot = (size_t)2 * t.kc * 1024 * (mk == MK_BF16X3 ? 2 : 1);
    pl.ksteps = Kt / KS;
    pl.nkc = (pl.ksteps + t.kc - 1) / t.kc;
    pl.gx = (M + 15) / 16;
    pl.gy = (Bpad + NCB - 1) / NCB;
    const long long base = (long long)pl.gx * pl.gy * pl.nkc;
    long long jc_max = (long long)((lds_max - 2 * slot) / ((size_t)NCB * accb)) - 1;
    if (jc_max < 2) jc_max = 2;
    long long njr_lo = (J + jc_max - 1) / jc_max, njr = njr_lo, best = -1;
    for (long long n = njr_lo; n <= njr_lo + 256 && n <= J; ++n) {
        const long long rounds = (base * n + 255) / 256;
        const long long cost = rounds * ((J + n - 1) / n + 8);
        if (best < 0 || cost < best) {
            best = cost;
            njr = n;
        }
    }
    // j per block: whole groups of P pairs (no padding iterations) when they fit
    const int jq = 2 * t.p;
    pl.jc = (int)((J + njr - 1) / njr);
    if ((pl.jc + jq - 1) / jq * jq <= jc_max) pl.jc = (pl.jc + jq - 1) / jq * jq;
    else if ((pl.jc + 1) / 2 * 2 <= jc_max) pl.jc = (pl.jc + 1) / 2 * 2;
    pl.njr = (J + pl.jc - 1) / pl.jc;
    pl.nsplit = pl.nkc * pl.njr;
    const size_t s_bytes = (size_t)(pl.jc + 1) * NCB * accb;
    const size_t r_bytes = (size_t)8 * 256 * t.fn * accb;
    const size_t need = 2 * slot + s_bytes;
    pl.lds = need > r_bytes ? need : r_bytes;
    pl.blocks = (int)((base * pl.njr + 7) / 8 * 8);
    return pl;
}

template <int ADT, int MKD, int V>
static void krs_go_v(const KrArgs& a, const KrPlan& pl, hipStream_t s) {
    constexpr KrsTile t = KrsTab<MKD>::t[V];
    hipLaunchKernelGGL((k_krs<ADT, MKD, t.fn, t.kc, t.p>), dim3(pl.blocks), dim3(512), pl.lds, s, a);
}

template <int ADT, int MKD, int V>
static hipError_t krs_attr_v(size_t lds) {
    constexpr KrsTile t = KrsTab<MKD>::t[V];
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_krs<ADT, MKD, t.fn, t.kc, t.p>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <int ADT, int MKD>
static void krs_go(const KrArgs& a, const KrPlan& pl, hipStream_t s) {
    switch (pl.v) {
        case 0: krs_go_v<ADT, MKD, 0>(a, pl, s); break;
        case 1: krs_go_v<ADT, MKD, 1>(a, pl, s); break;
        case 2: krs_go_v<ADT, MKD, 2>(a, pl, s); break;
        default: krs_go_v<ADT, MKD, 3>(a, pl, s); break;
    }
}

template <int ADT, int MKD>
static hipError_t krs_attr(size_t lds) {
    hipError_t e = hipSuccess, q;
    if ((q = krs_attr_v<ADT, MKD, 0>(lds)) != hipSuccess) e = q;
    if ((q = krs_attr_v<ADT, MKD, 1>(lds)) != hipSuccess) e = q;
    if ((q = krs_attr_v<ADT, MKD, 2>(lds)) != hipSuccess) e = q;
    if ((q = krs_attr_v<ADT, MKD, 3>(lds)) != hipSuccess) e = q;
    return e;
}

hipError_t krs_set_lds_limit(size_t lds) {
    hipError_t e = hipSuccess, q;
    if ((q = krs_attr<DT_F64, MK_F64>(lds)) != hipSuccess) e = q;
    if ((q = krs_attr<DT_F32, MK_F32>(lds)) != hipSuccess) e = q;
    if ((q = krs_attr<DT_BF16, MK_BF16>(lds)) != hipSuccess) e = q;
    if ((q = krs_attr<DT_BF16X3, MK_BF16X3>(lds)) != hipSuccess) e = q;
    return e;
}

void launch_krs_dense(int dt, const KrPlan& pl, const void* Ct, const void* Ct_lo, int N, int Np, int Bpad,
                      const void* X, const void* Xlo, const void* S, void* part, hipStream_t s) {
    KrArgs a{};
    a.C = Ct;
    a.Clo = (const unsigned short*)Ct_lo;
    a.X = X;
    a.Xlo = (const unsigned short*)Xlo;
    a.S = S;
    a.part = part;
    a.M = N;
    a.J = N;
    a.Kt = kr_tiled_k(dt, N);
    a.Kx = Np;
    a.Bpad = Bpad;
    a.ksteps = pl.ksteps;
    a.nkc = pl.nkc;
    a.jc = pl.jc;
    a.njr = pl.njr;
    a.gx = pl.gx;
    a.gy = pl.gy;
    switch (dt) {
        case DT_F64: krs_go<DT_F64, MK_F64>(a, pl, s); break;
        case DT_F32: krs_go<DT_F32, MK_F32>(a, pl, s); break;
        case DT_BF16: krs_go<DT_BF16, MK_BF16>(a, pl, s); break;
        default: krs_go<DT_BF16X3, MK_BF16X3>(a, pl, s); break;
    }
}

// ---------------------------------------------------------------- engine choice

// Variants: k_kr (kKrVariants), then k_krs (kKrsVariants), then the LDS-tile kernel.
int dense_batched_variants() { return kKrVariants + kKrsVariants + mfma_variants(); }

DensePlan dense_batched_plan(int dt, int N, int Np, int Bpad, int variant, size_t lds_max) {
    (void)Np;
    DensePlan d{};
    if (variant >= kKrVariants + kKrsVariants) {
        d.engine = 1;
        d.m = mfma_dense_plan(dt, N, Np, Bpad, mfma_variant(variant - kKrVariants - kKrsVariants));
        d.nsplit = d.m.nsplit;
    } else if (variant >= kKrVariants) {
        d.engine = 2;
        d.k = krs_plan(dt, N, N, kr_tiled_k(dt, N), Bpad, variant - kKrVariants, lds_max);
        d.nsplit = d.k.nsplit;
    } else {
        d.engine = 0;
        d.k = kr_plan(dt, N, N, kr_tiled_k(dt, N), Bpad, variant, lds_max);
        d.nsplit = d.k.nsplit;
    }
    return d;
}

void launch_dense_batched(int dt, const DensePlan& pl, const void* C, const void* Clo, const void* Ct,
                          const void* Ct_lo, int N, int Np, int Bpad, const void* X, const void* Xlo, const void* S,
                          void* part, hipStream_t s) {
    if (pl.engine == 1) launch_mfma_dense(dt, pl.m, C, Clo, N, Np, Bpad, X, Xlo, S, part, s);
    else if (pl.engine == 2) launch_krs_dense(dt, pl.k, Ct, Ct_lo, N, Np, Bpad, X, Xlo, S, part, s);
    else launch_kr_dense(dt, pl.k, Ct, Ct_lo, N, Np, Bpad, X, Xlo, S, part, s);
}

// ---------------------------------------------------------------- tiled copy

// dst unit q = ((tile * N + j) * (Kt / VEC) + ku) * 16 + r  <-  row i = 16 tile + r,
// elements [ku VEC, ku VEC + VEC) of row-major src [N][N][Np]; zero outside (i >= N or
// k >= Np).  Units are 16 bytes; VEC = 16 / element size divides Np.
__global__ void k_kr_tile(const u32x4* __restrict__ src, u32x4* __restrict__ dst, int N, int Np, int Kt,
                          int VEC, long long units) {
    const int nku = Kt / VEC;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < units;
         q += (long long)gridDim.x * blockDim.x) {
        const int r = (int)(q & 15);
        long long rest = q >> 4;
        const int ku = (int)(rest % nku);
        rest /= nku;
        const int j = (int)(rest % N);
        const long long i = (rest / N) * 16 + r;
        const long long k0 = (long long)ku * VEC;
        u32x4 v = u32x4{0u, 0u, 0u, 0u};
        if (i < N && k0 < Np) v = src[((i * N + j) * Np + k0) / VEC];
        dst[q] = v;
    }
}

size_t kr_tiled_bytes(int dt, int N, int eb) {
    return (size_t)((N + 15) / 16 * 16) * N * kr_tiled_k(dt, N) * eb;
}

void launch_kr_tile(int dt, int eb, const void* src, void* dst, int N, int Np, hipStream_t s) {
    const int VEC = 16 / eb, Kt = kr_tiled_k(dt, N);
    const long long units = (long long)kr_tiled_bytes(dt, N, eb) / 16;
    hipLaunchKernelGGL(k_kr_tile, dim3(4096), dim3(256), 0, s, (const u32x4*)src, (u32x4*)dst, N, Np, Kt, VEC, units);
}

}  // namespace rom
