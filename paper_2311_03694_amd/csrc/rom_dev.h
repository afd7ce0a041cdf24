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
// context's Helmholtz data.  Levels are kept in rings of three slots: level n lives
// in slot n % 3.  *step holds n, the level of the newest coefficients.
struct StepArgs {
    int N, B;
    double inv_dt;           // 1/dt
    double* uring;           // [3][B][N] FP64 coefficients
    double* yring;           // [3][B][N] FP64 advection terms C(u)u
    long long* step;         // newest level n
    long long* bad;          // first non-finite level (LLONG_MAX: none)
    double* elog;            // [cap][B] energy per level
    long long elog_cap;
    double* rhs;             // [B][N] right-hand sides (dense stiffness)
    double* epart;           // [B][nblk] energy partial sums
    unsigned* ticket;        // arrival counter of the last-block reduction (0 at rest)
    const double* hdiag;     // [3][N] 1/(beta0_k/dt + nu A_ii) (diagonal stiffness)
    const double* hinv;      // [3][N][N] (beta0_k/dt I + nu A)^-1 (dense stiffness)
    // coefficient copies in the contraction's number format for the batched kernels,
    // laid out [Bpad][N] (padding rows stay zero); written by the update of each step
    void* ucv;               // FP64 / FP32 / BF16 words (BF16X3: high words)
    void* ucv_lo;            // BF16X3 low words
    float* uscale;           // FP32 (BF16: BF16-rounded) values used as the j-weight
    int Bpad;
    int dtype;               // Dt of the contraction
    int batched;             // 1: write ucv/uscale for the batched contraction
};

// ---------------------------------------------------------------- launchers (k_*.hip)

// Operator staging (a one-time conversion, round to nearest even).
void launch_cvt_f64_to(int dt, const double* src, void* dst, void* dst_lo, long long n,
                       hipStream_t s);
// Scaled-weight copy: out[r] = lambda[r] rounded as the dtype prescribes.
void launch_cvt_lambda(int dt, const double* src, void* dst, long long n, hipStream_t s);

// Dense contraction, one trajectory: partial sums part[c][i] of
// y_i = sum_j u_j sum_k C[i][j][k] u_k over chunk c of the (j,k) plane.
struct GemvTile { int threads, unroll, chunk_target; };
int dense_gemv_variants();
GemvTile dense_gemv_variant(int idx);
int dense_gemv_nchunk(int N, GemvTile t);
int launch_dense_gemv(int dt, const void* C, const void* Clo, int N, const double* u_base,
                      const long long* stepp, long long slot_stride, void* part, int nchunk,
                      GemvTile t, hipStream_t s);

// Batched MFMA contraction (dense Khatri-Rao form, CP projections and CP scatter).
struct MfmaTile { int mw, bt, kc, jc; };
int mfma_variants();
MfmaTile mfma_variant(int idx);

// CP, one trajectory.
int launch_cp_proj1(int dt, const void* BCt, const void* BCt_lo, int N, int R,
                    const double* u_base, const long long* stepp, long long slot_stride,
                    void* st, hipStream_t s);
int launch_cp_scatter1(int dt, const void* Af, const void* Af_lo, const void* lam, int N,
                       int R, const void* st, double* y_out, const StepArgs* sa, int mode,
                       hipStream_t s);

// BDF update from contraction partials part[c][b][i] (row stride pb trajectories) in
// the accumulation type (FP64 for DT_F64, FP32 otherwise).  diag = 1: diagonal
// stiffness (update, energy, finalize); diag = 0: right-hand side only.
void launch_bdf_from_partials(const StepArgs& a, int acc_f64, const void* part, int nchunk,
                              int pb, int diag, hipStream_t s);
// Dense stiffness: u^{n+1} = Hinv_k rhs, energy, finalize.
void launch_helm_apply(const StepArgs& a, hipStream_t s);
// Write the batched coefficient copies from the current level (state create / set).
void launch_prep_ucv(const StepArgs& a, const double* u_src, hipStream_t s);
// Sum partials into FP64 y [B][N] (rom_nonlinear).
void launch_sum_partials(int acc_f64, const void* part, int nchunk, int pb, int B, int N,
                         double* y, hipStream_t s);

// Helmholtz setup on the device: H = (beta0/dt) I + nu A, Cholesky, inverse.
int helm_setup_dense(int N, double nu, double dt, const double* A_dev, double* hinv_dev,
                     double* work_dev, int* info_dev, hipStream_t s);
void helm_setup_diag(int N, double nu, double dt, const double* A_dev, double* hdiag_dev,
                     hipStream_t s);

// Batched contraction launchers (k_mfma.hip).
// dense: Y partials [nchunk][Bpad][N] FP32/FP64 from C [N][N][N] and ucv [Bpad][N].
int mfma_dense_nchunk(int N, int Bpad, MfmaTile t);
int launch_mfma_dense(int dt, const void* C, const void* Clo, int N, int Bpad,
                      const StepArgs& a, const void* ucv_override, const void* ucvlo_override,
                      const float* uscale_override, void* part, MfmaTile t, hipStream_t s);
// CP projections ST partials [nchunk][Bpad][2R] from BCt [2R][N] and ucv [Bpad][N].
int mfma_proj_nchunk(int N, int R, MfmaTile t);
int launch_mfma_proj(int dt, const void* BCt, const void* BCt_lo, int N, int R, int Bpad,
                     const void* ucv, const void* ucv_lo, void* part, MfmaTile t,
                     hipStream_t s);
// CP scatter partials [nchunk][Bpad][N] from Af [N][R] and W = lam .* S .* T, where
// S, T are the reduced projections summed from the proj partials.
int mfma_scatter_nchunk(int N, int R, MfmaTile t);
int launch_mfma_scatter(int dt, const void* Af, const void* Af_lo, const void* lam, int N,
                        int R, int Bpad, int B, const void* proj_part, int proj_nchunk,
                        void* part, MfmaTile t, hipStream_t s);

}  // namespace rom
