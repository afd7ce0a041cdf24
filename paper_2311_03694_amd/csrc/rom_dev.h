// rom_dev.h -- internal declarations shared by the HIP sources of librom.so
// (kernels, launchers and the C ABI).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rom {

enum Dt { DT_F64 = 0, DT_F32 = 1, DT_BF16 = 2, DT_BF16X3 = 3 };

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

constexpr int kWave = 64;

// ---------------------------------------------------------------- step state

// Device pointers of one state (a batch of B trajectories of one context), plus the
// context's Helmholtz data, as passed to the kernels of the step from level n.  Levels
// are kept in rings of three slots: level n lives in slot n % 3.  The step counter has
// two slots; *step holds n, the level of the newest coefficients.
struct StepArgs {
    int N, B;
    double inv_dt;           // 1/dt
    double* uring;           // [3][B][N] FP64 coefficients
    double* yring;           // [3][B][N] FP64 advection terms C(u)u
    long long* step;         // counter slot holding the newest level n (slot n & 1)
    long long* step_next;    // the other slot, where the update kernel stores n + 1
    long long* bad;          // first non-finite level (LLONG_MAX: none)
    int* closep;             // 1: the energy of level n is still to be summed
    double* elog;            // [cap][B] energy per level
    long long elog_cap;
    double* rhs;             // [Bpad][Np] right-hand sides (dense stiffness; padding zero)
    double* epart;           // [2][B][enmax] per-block energy partials of a level,
                             // parity slot (level & 1)
    int* ecount;             // [2] partials per trajectory of a level, same parity slots
    int enmax;               // capacity per trajectory (at least any update kernel's blocks)
    const double* hdiag;     // [3][N] 1/(beta0_k/dt + nu A_ii) (diagonal stiffness)
    const double* hinv;      // [3][N][Np] (beta0_k/dt M + nu A)^-1, row pitch Np (dense stiffness)
    double* zfull;           // full form: [zsplit][Bpad][N] G x of the level's right-hand
                             // side (zeroth-mode linear terms and M - I), summed over the
                             // zsplit partial products in order; NULL otherwise
    int zsplit;              // partial products of zfull (1 for one trajectory)
    long long zstride;       // doubles from one partial product to the next
    const double* fz;        // full form: [N] constant of the bracket, (C1 + C2)[:, 0] - c0
    const double* az;        // full form: [N] nu a0
    // coefficient copies in the contraction's number format for the batched kernels,
    // laid out [Bpad][Np] (padding rows and columns stay zero); written by the update
    // of each step
    void* ucv;               // FP64 / FP32 / BF16 words (BF16X3: high words)
    void* ucv_lo;            // BF16X3 low words
    void* uj;                // [Np][Bpad] j-weights in the accumulation type: FP64 (DT_F64),
                             // else FP32 (the BF16-rounded value for DT_BF16)
    void* st;                // CP, one trajectory: w = lam .* (Bf^T u) .* (Cf^T u) of the
                             // newest level [Rp] (accumulation type)
    int Bpad, Np;
    int dtype;               // Dt of the contraction
    int batched;             // 1: write ucv/uj for the batched contraction
};

// ---------------------------------------------------------------- grouped launches

// A job is one kernel's work for one (context, state) pair; grouped launches run the
// jobs of many pairs (uneven N, R) in one grid, job p owning blocks [blk0, blk0+nblk).
struct GemvJob {           // dense contraction, one trajectory
    const void* C;                 // [N][J][Np]
    const unsigned short* Clo;
    int N, Np;
    int J;                         // slabs per row: N (dense tensor), or the SVD rank
    const void* wj;                // slab weights [J] (accumulation type); null: u itself
    const double* u_base;
    const long long* stepp;
    long long slot_stride;
    void* part;
    int nchunk;
    long long chunk_len;
    int blk0, nblk;
};
struct Proj1Job {          // CP projections and their Hadamard product, one trajectory
    const void* BCt;               // layout 0: [Bf|Cf]^T [2Rp][Np]; else the pair form [P + R][Np]
    const unsigned short* BCt_lo;
    const void* lam;
    int N, Np, Rp;
    int layout, P, R;              // skew column pairs (0 none, 1 interleaved, 2 blocked), R = 2P
    const double* u_base;
    const long long* stepp;
    long long slot_stride;
    void* w;
    int blk0, nblk;
};
struct Scat1Job {          // CP Hadamard-scatter with the fused BDF update
    const void* Af;
    const unsigned short* Af_lo;
    int N, Rp;
    const void* w;                 // lam .* s .* t [Rp]
    StepArgs a;
    const double* G;               // full form: G = [L | M - I] [N][2 Np], whose terms the
                                   // scatter forms itself (null: none, or read from a.zfull)
    int blk0, nblk;
};
struct BdfJob {            // BDF update from contraction partials, one trajectory
    StepArgs a;
    const void* part;
    int nchunk, pb;
    int blk0, nblk;
};
struct HelmJob {           // dense-stiffness Helmholtz apply, one trajectory; with CP
                           // factors also the projections of the new level (see
                           // launch_helm_proj)
    StepArgs a;
    const void* Mst;               // CP: [3][2Rp][Np] [Bf|Cf]^T Hinv_k, contraction format; else null
    const unsigned short* Mst_lo;  // BF16X3 low words of Mst
    const void* lam;               // CP: lam [Rp] (accumulation type)
    int Rp;
    int layout, P, R;              // skew column pairs of the factors (Mst in the pair form)
    int nh, np;                    // row blocks of the Helmholtz part, of the projections (0: none)
    int blk0, nblk;                // grouped launches: first block, blocks (nh + np)
};
struct SvdProj {           // SVD form, first product: w_r = sigma_r U[:,r]^T u, one trajectory
    const void* Ut;                // [Rsp][Np] columns of U as rows
    const unsigned short* Ut_lo;
    const void* sigma;             // [Rsp] (accumulation type)
    int N, Np, Rsp;
    const double* u_base;
    const long long* stepp;
    long long slot_stride;
    void* w;                       // [Rsp] (accumulation type)
};
struct FullJob {           // full form: zeroth-mode and mass terms of a level, one trajectory
    StepArgs a;
    const double* G;               // [N][2 Np]
};
struct FinJob {            // closing energy sum of the newest level, one state
    StepArgs a;
};

// A job of a mixed launch over a heterogeneous work table (rom_step_multi): one phase of
// one one-trajectory state, of any kind and number format.  A step is at most four such
// launches, whatever the mix of N, R, formats, stiffness kinds and operator forms:
//   phase 0: full-form terms (MIX_FULL), SVD first products (MIX_SVDP)
//   phase 1: dense / SVD slab streams (MIX_GEMV), CP projections, diagonal stiffness (MIX_PROJ)
//   phase 2: BDF update or right-hand side from partials (MIX_BDF), CP scatter (MIX_SCAT)
//   phase 3: Helmholtz apply, with the next projections for CP states (MIX_HELM)
enum MixKind { MIX_GEMV = 0, MIX_PROJ = 1, MIX_BDF = 2, MIX_SCAT = 3, MIX_HELM = 4, MIX_SVDP = 5, MIX_FULL = 6 };
struct MixJob {
    int kind, dtype;
    int mode;                      // MIX_BDF: 1 = diagonal-stiffness update; MIX_SCAT: scatter mode 1 or 2
    int blk0, nblk;
    union {
        GemvJob g;
        Proj1Job p;
        BdfJob b;
        Scat1Job s;
        HelmJob h;
        SvdProj v;
        FullJob f;
    };
};
// Blocks and dynamic LDS bytes a mixed job needs; the launch over a table (jobs sorted by
// blk0, `blocks` in total, `lds` the largest need).
int mix_job_blocks(const MixJob& jb);
size_t mix_job_lds(const MixJob& jb);
void launch_mix(const MixJob* jobs_dev, int njobs, int blocks, size_t lds, hipStream_t s);

// ---------------------------------------------------------------- launchers (k_*.hip)

// Operator staging (a one-time conversion, round to nearest even): `rows` rows of
// `cols` FP64 values into rows of pitch `dpitch` elements (padding left untouched).
void launch_cvt_f64_to(int dt, const double* src, void* dst, void* dst_lo, long long rows, int cols,
                       int dpitch, hipStream_t s);
// Scaled-weight copy: out[r] = lambda[r] rounded as the dtype prescribes.
void launch_cvt_lambda(int dt, const double* src, void* dst, long long n, hipStream_t s);

// Dense contraction, one trajectory: partial sums part[c][i] of
// y_i = sum_j u_j sum_k C[i][j][k] u_k over chunk c of the (j,k) plane.
struct GemvTile { int threads, unroll, chunk_target; };
int dense_gemv_variants();
GemvTile dense_gemv_variant(int idx);
int dense_gemv_nchunk(int N, GemvTile t);
int launch_dense_gemv(int dt, const void* C, const void* Clo, int N, int Np, int J, const void* wj,
                      const double* u_base, const long long* stepp, long long slot_stride, void* part, int nchunk,
                      GemvTile t, hipStream_t s);
// SVD-ROM first product: w_r = sigma_r U[:,r]^T u over the rows of Ut [Rsp][Np]
void launch_svd_proj(int dt, const void* Ut, const void* Ut_lo, const void* sigma, int N, int Np, int Rs,
                     const double* u_base, const long long* stepp, long long slot_stride, void* w, hipStream_t s);

GemvJob make_gemv_job(int dt, const void* C, const void* Clo, int N, int Np, int J, const void* wj,
                      const double* u_base, const long long* stepp, long long slot_stride, void* part, int nchunk,
                      GemvTile t);
// Dense-stiffness apply of a step with, for CP states (np > 0), the projections of the
// new level (k_contract.hip), one state.
void launch_helm_proj(int dt, const HelmJob& jb, hipStream_t s);
// Closing energy sum of the newest level when it is still pending (after the last step
// of a sequence; one block per state).
void launch_close(const StepArgs& a, hipStream_t s);
void launch_close_group(const FinJob* jobs_dev, int njobs, hipStream_t s);

// Batched MFMA contraction (dense Khatri-Rao form, CP projections and CP scatter).
struct MfmaTile { int mw, bt, target; };
int mfma_variants();
MfmaTile mfma_variant(int idx);
// Launch geometry of one batched contraction: wave rows, block columns, k-chunk, j-range,
// splits (= partial tiles), LDS bytes and grid.
struct MfmaPlan {
    int mw, bt, kc, nkc, jc, njr, nsplit, kcp;
    size_t lds;
    int grid_x, grid_y, blocks;
};

// CP, one trajectory.
// st [2Rp]: s then t; factors padded to Np / Rp with zeros.
struct SkewPairs { int layout, P, R; };   // layout 0: general factors
int launch_cp_proj1(int dt, const void* BCt, const void* BCt_lo, const void* lam, int N, int Np, int Rp,
                    SkewPairs sk, const double* u_base, const long long* stepp, long long slot_stride,
                    void* w, hipStream_t s);
int proj1_blocks(int Rp, SkewPairs sk);
int launch_cp_scatter1(int dt, const void* Af, const void* Af_lo, int N, int Rp, const void* w, double* y_out,
                       const StepArgs* sa, int mode, hipStream_t s, const double* G = nullptr);

// CP, one trajectory, resident operator (k_res.hip): from level 2 on, a run of steps in
// one launch (one block per compute unit at most) whose blocks keep their rows of the
// order-3 operators in LDS.
struct ResJob {
    StepArgs a;                    // counter slots of level n0
    long long n0;                  // first level of the run (n0 >= 2)
    int nsteps;                    // levels n0 + 1 .. n0 + nsteps are produced
    int dense_h;                   // 1: dense stiffness (Hinv_3 rows, M_3 projections)
    const void* Af;                // [N][Rp]
    const unsigned short* Af_lo;
    const void* Pop;               // projection rows of order 3: pair form [P + R][Np] or
    const unsigned short* Pop_lo;  // [Bf|Cf]^T [2Rp][Np] (times Hinv_3 with a dense stiffness)
    const void* lam;               // [Rp] accumulation type
    int Rp, layout, P, R;
    int nrg, npg;                  // row groups (4 rows), projection groups (4 waves)
    int rg_per, pg_per;            // groups of each kind per block, at most
    unsigned long long* xmsg;      // [2N] tagged halves of x (rhs, or u^{n+1} with a diagonal stiffness)
    unsigned long long* wmsg;      // [Rp * words per entry] tagged words of w
    double* epall;                 // [nsteps][nrg] energy partials of the levels produced
    const unsigned* seq;           // tag base of the run
    int* err;                      // raised when a wait gives up
    unsigned spin_max;             // polling rounds before a wait gives up
};

// Bytes of the LDS image of N coefficients in format dt (LdsU<DT>::bytes).
__host__ __device__ inline size_t lds_u_bytes(int dt, int N) {
    const size_t eb = dt == DT_F64 ? 8 : dt == DT_F32 ? 4 : 2;
    const size_t r = ((size_t)N * eb + 15) & ~(size_t)15;
    if (dt == DT_F64 || dt == DT_F32) return r;
    const size_t l = dt == DT_BF16X3 ? (((size_t)N * 2 + 15) & ~(size_t)15) : 0;
    return r + l + (size_t)N * 4;
}

// LDS layout of a resident block: w [Rp], x [N] (FP64), the images of x (and -x for the
// BF16 formats' pair form), then the block's rows: Af (and its low words), Hinv_3, the
// projection rows (and their low words).
struct ResLayout { size_t W, xr, L, Ln, af, aflo, hv, pr, prlo, total; };
__host__ __device__ inline ResLayout res_layout(int dt, int N, int Np, int Rp, int layout, int dense_h, int rg_per,
                                                int pg_per) {
    const size_t eb = dt == DT_F64 ? 8 : dt == DT_F32 ? 4 : 2, ab = dt == DT_F64 ? 8 : 4;
    const bool x3 = dt == DT_BF16X3, neg = (dt == DT_BF16 || x3) && layout;
    const size_t ph = layout ? 3 : 2;
    ResLayout r{};
    size_t o = 0;
    auto put = [&](size_t& at, size_t bytes) {
        at = o;
        o = (o + bytes + 15) & ~(size_t)15;
    };
    put(r.W, (size_t)Rp * ab);
    put(r.xr, (size_t)N * 8);
    put(r.L, lds_u_bytes(dt, Np));
    put(r.Ln, neg ? lds_u_bytes(dt, Np) : 0);
    put(r.af, (size_t)rg_per * 4 * Rp * eb);
    put(r.aflo, x3 ? (size_t)rg_per * 4 * Rp * 2 : 0);
    put(r.hv, dense_h ? (size_t)rg_per * 4 * Np * 8 : 0);
    put(r.pr, (size_t)pg_per * 4 * ph * Np * eb);
    put(r.prlo, x3 ? (size_t)pg_per * 4 * ph * Np * 2 : 0);
    r.total = o;
    return r;
}
constexpr int kResWaitWords = 4096;    // message words a block waits for at most (x or w)
// Launch of the run (dynamic LDS `lds`, G blocks of 256 threads, all resident at once),
// then the closing kernel: it logs the energies of levels n0 .. n0 + nsteps - 1, leaves
// n0 + nsteps pending as the step kernels do (or, with close_last, the run ending a
// sequence of steps, closes it too), and advances the counter and the tag base.
hipError_t res_launch(int dt, const ResJob& jb, int G, size_t lds, hipStream_t s);
void res_close_launch(const StepArgs& a0, const StepArgs& aL, long long n0, int nsteps, const double* epall,
                      int nrg, unsigned* seq, bool close_last, hipStream_t s);
// Raise the kernel's dynamic LDS limit to `cap` (the same for every context: the
// attribute belongs to the kernel) and report how many of its blocks with `lds` bytes
// fit on one compute unit.
hipError_t res_attr(int dt, int N, size_t cap, size_t lds, int* blocks_per_cu);

// BDF update from contraction partials part[c][b][i] (row stride pb trajectories) in
// the accumulation type (FP64 for DT_F64, FP32 otherwise).  diag = 1: diagonal
// stiffness (update, energy partials, step close); diag = 0: right-hand side only.
void launch_bdf_from_partials(const StepArgs& a, int acc_f64, const void* part, int nchunk,
                              int pb, int diag, hipStream_t s);
// Dense stiffness, one trajectory: u^{n+1} = Hinv_k rhs, energy partials, step close.
void launch_helm_apply(const StepArgs& a, hipStream_t s);
// Write the batched coefficient copies from the current level (state create / set).
void launch_prep_ucv(const StepArgs& a, const double* u_src, hipStream_t s);
// Sum partials into FP64 y [B][N] (rom_nonlinear).
void launch_sum_partials(int acc_f64, const void* part, int nchunk, int pb, int B, int N,
                         double* y, hipStream_t s);

// Helmholtz setup on the device: H = (beta0/dt) I + nu A, Cholesky, inverse.
int helm_setup_dense(int N, int Np, double nu, double dt, const double* A_dev, const double* M_dev,
                     double* hinv_dev, double* work_dev, int* info_dev, hipStream_t s);
void helm_setup_diag(int N, double nu, double dt, const double* A_dev, const double* M_dev, double* hdiag_dev,
                     hipStream_t s);
// Full form of eq. nse_d1 (k_bdf.hip).  Setup: G = [L | M - I] [N][2 Np] with
// L = (C1 + C2)[:, 1:], fz = (C1 + C2)[:, 0] - c0, az = nu a0 (each input nullable: zero,
// M: the identity).  Per step: zfull of the level from the step counter.
void full_setup(int N, int Np, double nu, const double* M, const double* C1, const double* C2,
                const double* c0, const double* a0, double* G, double* fz, double* az, hipStream_t s);
void launch_full_terms(const StepArgs& a, const double* G, hipStream_t s);
// Batches: X [Bpad][2 Np] = [uhat | h] per trajectory (padding stays zero), the operand
// of zfull = X G^T (launch_gemm_f64).
void launch_full_x(const StepArgs& a, double* X, hipStream_t s);

// Batched contraction launchers (k_mfma.hip).  Partials are [nsplit][Bpad][M] in the
// accumulation type (FP64 for DT_F64, FP32 otherwise).
//   dense:   M = N rows of C [N][N][Np], X = u [Bpad][Np] and j-weights S [Np][Bpad]
//   proj:    M = 2Rp rows of [Bf|Cf]^T [2Rp][Np], X = u [Bpad][Np]
//   scatter: M = N rows of Af [N][Rp], X = W [Bpad][Rp] (FP32, FP64 for DT_F64)
MfmaPlan mfma_dense_plan(int dt, int N, int Np, int Bpad, MfmaTile t);
void launch_mfma_dense(int dt, const MfmaPlan& pl, const void* C, const void* Clo, int N, int Np, int Bpad,
                       const void* X, const void* Xlo, const void* S, void* part, hipStream_t s);
MfmaPlan mfma_proj_plan(int dt, int Np, int Rp, int Bpad, MfmaTile t);
void launch_mfma_proj(int dt, const MfmaPlan& pl, const void* BCt, const void* BCt_lo, int Np, int Rp, int Bpad,
                      const void* X, const void* Xlo, void* part, hipStream_t s);
MfmaPlan mfma_scatter_plan(int dt, int N, int Rp, int Bpad, MfmaTile t);
void launch_mfma_scatter(int dt, const MfmaPlan& pl, const void* Af, const void* Af_lo, int N, int Rp, int Bpad,
                         const void* W, void* part, hipStream_t s);
// Batched Helmholtz apply: partials [nsplit][Bpad][N] (FP64) of Hinv_k rhs, with k read
// from the device step counter; Hinv [3][N][Np], rhs [Bpad][Np].
MfmaPlan mfma_helm_plan(int N, int Np, int Bpad, MfmaTile t);
void launch_mfma_helm(const MfmaPlan& pl, const double* hinv, int N, int Np, int Bpad, const double* rhs,
                      const long long* stepp, double* part, hipStream_t s);
// Batched dense contraction with the coefficient fragments held in registers
// (k_kr.hip).  Partials [nsplit][Bpad][N]; X = u [Bpad][Np], j-weights S [Np][Bpad];
// the tensor comes from the tiled copy Ct [ceil(N/16)][N][Kt/VEC][16][VEC] made by
// launch_kr_tile (Kt = kr_tiled_k, VEC = 16 bytes / element size).
struct KrPlan {
    int v, fn, kw, pf;             // variant and its shape
    int ksteps, nkc, jc, njr;      // fragment steps, k-chunks, j per block, j-ranges
    int gx, gy, nsplit, blocks;
    size_t lds;
};
int kr_variants();
int kr_tiled_k(int dt, int N);
size_t kr_tiled_bytes(int dt, int N, int eb);
void launch_kr_tile(int dt, int eb, const void* src, void* dst, int N, int Np, hipStream_t s);
KrPlan kr_plan(int dt, int M, int J, int Kt, int Bpad, int variant, size_t lds_max);
void launch_kr_dense(int dt, const KrPlan& pl, const void* Ct, const void* Ct_lo, int N, int Np, int Bpad,
                     const void* X, const void* Xlo, const void* S, void* part, hipStream_t s);
// Allow every variant up to `lds` bytes of dynamic LDS.
hipError_t kr_set_lds_limit(size_t lds);

// The batched dense contraction of a context: variants [0, kr_variants()) select the
// register kernel, the following mfma_variants() the LDS-tile kernel; -1 = default.
struct DensePlan {
    int engine;                    // 0 = k_kr, 1 = k_mfma_rows, 2 = k_krs
    KrPlan k;
    MfmaPlan m;
    int nsplit;
};
int dense_batched_variants();
DensePlan dense_batched_plan(int dt, int N, int Np, int Bpad, int variant, size_t lds_max);
void launch_dense_batched(int dt, const DensePlan& pl, const void* C, const void* Clo, const void* Ct,
                          const void* Ct_lo, int N, int Np, int Bpad, const void* X, const void* Xlo, const void* S,
                          void* part, hipStream_t s);

// Skinny products of the batched path (k_gemm.hip): one block per output tile over the
// whole contracted index; outputs in the partials layout with a single split.
struct GemmPlan { int fn, gx, gy, blocks, ksplit; };
int gemm_variants();
GemmPlan gemm_plan(int M, int Bpad, int variant);
// The plan of an FP64 product over K whose short column side leaves the device
// underfilled: K split into ksplit ranges, one partial product each.
GemmPlan gemm_plan_splitk(int M, int K, int Bpad);
void launch_gemm_proj(int dt, const GemmPlan& pl, const void* BCt, const void* BCt_lo, int Np, int Rp, int Bpad,
                      const void* X, const void* Xlo, void* P, hipStream_t s);
void launch_gemm_proj_skew(int dt, const GemmPlan& pl0, const void* SK, const void* SK_lo, int Np, int P, int layout,
                           int Rp, int Bpad, const void* X, const void* Xlo, const void* lam, void* W, hipStream_t s);
void launch_gemm_proj_pair(int dt, const GemmPlan& pl, const void* BCt, const void* BCt_lo, int Np, int Rp,
                           int Bpad, const void* X, const void* Xlo, const void* lam, void* W, hipStream_t s);
void launch_gemm_scatter_step(int dt, const GemmPlan& pl, const void* Af, const void* Af_lo, int N, int Rp,
                              int Bpad, const void* W, const StepArgs& st, int diag, hipStream_t s);
void launch_gemm_scatter(int dt, const GemmPlan& pl, const void* Af, const void* Af_lo, int N, int Rp, int Bpad,
                         const void* W, void* Y, hipStream_t s);
void launch_gemm_f64(const GemmPlan& pl, const double* A, long long lda, const double* X, long long ldx, double* Y,
                     int M, int K, int Bpad, hipStream_t s);
void launch_gemm_helm(const GemmPlan& pl, const double* hinv, int N, int Np, int Bpad, const double* rhs,
                      const long long* stepp, double* Y, const StepArgs* st, hipStream_t s);

// A batched CP product of a context: variants [0, gemm_variants()) select k_gemm, the
// following mfma_variants() the LDS-tile kernel; -1 = default.
struct SkinnyPlan {
    int engine;                    // 0 = k_gemm, 1 = k_mfma_rows
    GemmPlan g;
    MfmaPlan m;
    int nsplit;
};

// W[b][r] = lam_r s_r t_r from projection partials P [nz][Bpad][2Rp].
void launch_hadamard(int dt, const void* P, int nz, int Bpad, int B, int Rp, const void* lam, void* W,
                     hipStream_t s);

}  // namespace rom
