/*
 * rom.h -- C ABI of librom.so: the online stage of a Galerkin reduced-order model
 * (ROM) on one AMD Instinct MI355X (gfx950), with the advection tensor either dense
 * (the standard G-ROM) or in CP form (the CPD-ROM), following arXiv 2311.03694.
 *
 * The model (Sec. 2.2, eq. nse_ode, identity mass matrix, core tensor without the
 * zeroth mode) is
 *     du/dt = -C(u)u - nu A u,   [C(u)u]_i = sum_{j,k} C[i][j][k] u_j u_k,
 * integrated by the semi-implicit BDFk/EXTk scheme of eq. nse_d1: the viscous term is
 * implicit, the advection term is extrapolated, k = 1, 2 for the first two steps and
 * k = 3 afterwards.  In CP form (Sec. 3.1, eqs. approx_tensor and tc_ap)
 *     C[i][j][k] ~ sum_r lam_r Af[i][r] Bf[j][r] Cf[k][r],
 *     C(u)u      = Af (lam .* (Bf^T u) .* (Cf^T u)).
 *
 * Conventions for every call:
 *  - Host arrays are FP64, row-major, 0-based; the library deep-copies what it keeps,
 *    so the caller may free its buffers after the call returns.
 *  - Device arrays named *_dev are caller-owned device memory (e.g. torch tensors);
 *    the library reads/writes them on the context's stream and never frees them.
 *  - Work is asynchronous on the context's stream unless a call says it synchronizes.
 *  - No call aborts or throws; each returns a rom_status and, on failure, leaves a
 *    message for rom_last_error() (thread-local, valid until the next call on the
 *    same thread).
 *  - Contexts and states are independent; one context must not be used from two
 *    threads at once.
 */
#ifndef ROM_H
#define ROM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rom_ctx_s *rom_ctx;     /* device operators, Helmholtz inverses, kernels  */
typedef struct rom_state_s *rom_state; /* batch of trajectories: FP64 histories, energy  */

typedef enum {
    ROM_OK = 0,
    ROM_E_INVALID = 1,     /* bad argument, or a Helmholtz matrix that is not SPD        */
    ROM_E_NOMEM = 2,       /* device or host allocation failed                           */
    ROM_E_DEVICE = 3,      /* a HIP runtime call failed                                  */
    ROM_E_NONFINITE = 4,   /* a trajectory produced Inf/NaN (Sec. 4.3's unstable ROMs)   */
    ROM_E_UNSUPPORTED = 5  /* valid request this library does not implement              */
} rom_status;

/* Arithmetic of the advection contraction.  The state update, the Helmholtz solve and
 * the energy are always FP64.
 *   ROM_FP64   : FP64 operator, FP64 arithmetic.
 *   ROM_FP32   : FP32 operator and coefficients, FP32 accumulation.
 *   ROM_BF16   : BF16 operator and BF16 coefficients (round to nearest even from FP32),
 *                exact products, FP32 accumulation.
 *   ROM_BF16X3 : operator and coefficients split x = hi + lo into two BF16 words;
 *                products hi*hi + hi*lo + lo*hi, FP32 accumulation. */
typedef enum { ROM_FP64 = 0, ROM_FP32 = 1, ROM_BF16 = 2, ROM_BF16X3 = 3 } rom_dtype;

/* Problem description handed to rom_create (Sec. 2.2, eqs. nse_ode / nse_d1).
 *   N         number of modes, 1 <= N.
 *   nu        viscosity, the paper's 1/Re (>= 0).
 *   dt        time step (> 0).
 *   A         host [N][N] symmetric stiffness; nu*A + (beta0/dt)*I must be SPD for
 *             beta0 in {1, 3/2, 11/6}.  A diagonal A is detected and solved by division.
 *   C         host [N][N][N] dense advection tensor, C[i][j][k] multiplies u_j*u_k in
 *             row i; or NULL to use the CP factors below.
 *   R         CP rank (columns), >= 1 when C is NULL.
 *   lambda    host [R] weights; Af, Bf, Cf host [N][R] factors of tensor positions 1,2,3.
 *   dtype     rom_dtype of the contraction.
 *   max_batch largest batch a state of this context may hold (>= 1).
 *   stream    hipStream_t for all work of this context; NULL = a non-blocking stream the
 *             context creates and destroys (it does not wait for the null stream). */
typedef struct rom_desc {
    int32_t N;
    int32_t R;
    double nu;
    double dt;
    const double *A;
    const double *C;
    const double *lambda;
    const double *Af;
    const double *Bf;
    const double *Cf;
    int32_t dtype;
    int32_t max_batch;
    void *stream;
} rom_desc;

/* Stage the operators on the device (a conversion to the contraction dtype), form the
 * three FP64 Helmholtz inverses (one Cholesky factorisation and triangular solves per
 * BDF order, on the device) and size the workspaces.  Synchronizes.
 * Errors: ROM_E_INVALID (sizes, nu < 0, dt <= 0, missing operator, non-SPD Helmholtz
 * matrix), ROM_E_NOMEM, ROM_E_DEVICE. */
rom_status rom_create(const rom_desc *d, rom_ctx *out);

/* The same with the advection tensor in the SVD form of the SVD-ROM (Sec. 4.4): the
 * mode-3 matricization is replaced by its rank-R SVD, C_(3) ~ U_R Sigma_R V_R^T.  The
 * mode-3 index is the second index j of C[i][j][k] (the advected coefficient), so
 *     C[i][j][k] ~ sum_r U[j][r] sigma_r V[i][k][r],
 *     y_i = sum_r sigma_r (U[:,r]^T u) (sum_k V[i][k][r] u_k)      (2 N^2 R flops).
 * U host [N][R], sigma host [R], V host [N][N][R] (row (i, k), then r); R >= 1.  d->C,
 * d->lambda and the CP factors must be NULL (d->R is ignored).  The formats apply as for
 * the dense tensor (U and V in the contraction format, sigma like the CP weights).  States
 * hold one trajectory (max_batch must be 1; ROM_E_UNSUPPORTED otherwise, or for N > 4096);
 * rom_step_multi steps such states one by one.  Errors as rom_create. */
rom_status rom_create_svd(const rom_desc *d, int32_t R, const double *U, const double *sigma,
                          const double *V, rom_ctx *out);

/* Full form of the reduced system (Sec. 2.2, eqs. nse_ode, nse_d1 and
 * zeroth_contribution): a mass matrix and the terms of the zeroth mode phi_0, whose
 * coefficient is 1 in the augmented vector ubar = [1, u_1 .. u_N].  Every pointer is host
 * FP64, row-major, read during rom_create_full only, and nullable:
 *   M       [N][N] symmetric positive definite mass matrix; NULL = the identity.
 *   C1, C2  [N][N+1] zeroth-mode advection matrices, column 0 for phi_0; NULL = zero.
 *   c0, a0  [N] zeroth-mode advection and stiffness vectors; NULL = zero.
 * Each step then solves (beta0/dt M + nu A) u^{n+1} = - sum_q alpha_q [C(u)u + (C1 + C2) ubar
 * - c0]^{n+1-q} - M (1/dt) sum_q beta_q u^{n+1-q} - nu a0, the -c0 removing the phi_0-phi_0
 * entry that C1 ubar and C2 ubar both contain. */
typedef struct rom_full_terms {
    const double *M;
    const double *C1;
    const double *C2;
    const double *c0;
    const double *a0;
} rom_full_terms;

/* rom_create with the full form (dense tensor or CP factors; not the SVD form).  States
 * of the context take one more FP64 kernel per step (the zeroth-mode and mass terms, an
 * N x 2N GEMV); rom_nonlinear still returns C(u)u alone, and so does the y history of
 * rom_state_get / rom_state_set (each step recomputes the zeroth-mode and mass terms
 * from the u history).  The energy logged for such states stays |u|^2/2 (the coefficient
 * norm that the plain form logs), not u^T M u/2: it is the quantity the blow-up check
 * and the oracle compare, and it bounds u^T M u/2 within the extreme eigenvalues of M.
 * Errors as rom_create, plus ROM_E_INVALID for f == NULL or a
 * non-symmetric M (a non-SPD M shows as a non-SPD Helmholtz matrix) and
 * ROM_E_UNSUPPORTED for N > 4096. */
rom_status rom_create_full(const rom_desc *d, const rom_full_terms *f, rom_ctx *out);
void rom_destroy(rom_ctx ctx);

/* CP-ALS (Sec. 2.3, eqs. cp_nls and cp_als): `sweeps` sweeps of alternating least squares
 * fitting [[A1, A2, A3]] (CP weights one) to a dense tensor.  Each sweep solves the three
 * subproblems in turn, each through its normal equations, e.g. for the first factor
 *   A1 <- M1 V1^{-1},  M1[i][r] = sum_jk C[i][j][k] A2[j][r] A3[k][r],
 *   V1 = (A2^T A2) .* (A3^T A3),
 * V inverted in FP64 on the device by blocked Gauss-Jordan elimination without pivoting
 * (every pivot block of an SPD matrix is SPD).
 *   C        device FP64 [N][N][N], C[i][j][k] (position 1 = i, as rom_desc.C); read only.
 *   A1..A3   device FP64 [N][R] factors for positions 1, 2, 3: the initial guess on entry
 *            (the caller chooses it), the fitted factors on return.
 *   stream   hipStream_t or NULL (the null stream); the sweeps themselves run on a stream
 *            of the call's own, ordered after it.  Synchronizes; allocates and frees its own
 *            workspace: two padded unfoldings of C and their product with a factor, about
 *            2 N^3 + N^2 R + 4 R^2 doubles (ROM_E_NOMEM when that does not fit).
 * Errors: ROM_E_INVALID (N or R outside [1, 4096], sweeps < 0, NULL pointers, or a
 * normal matrix that is not positive definite: rank-deficient factors; the factors then
 * hold non-finite values), ROM_E_NOMEM, ROM_E_DEVICE.  sweeps = 0 does nothing. */
rom_status rom_cp_als(int32_t N, int32_t R, const double *C, double *A1, double *A2, double *A3,
                      int32_t sweeps, void *stream);

/* ALS-skew (Sec. 3.3, eqs. skew_abc_struct and cp_als_quad): `sweeps` sweeps fitting the
 * skew-symmetry preserving CP structure with P column pairs (rank R = 2P, weights one)
 *   A1 = [A11 A12],  A2 = [B1 B1],  A3 = [A12 -A11]
 * to a dense tensor (for a tensor skew in positions 1 and 3, C[i][j][k] = -C[k][j][i]).
 * Each sweep updates B1 by least squares with the two halves of A2 tied (the ALS update
 * of the second factor), then runs `subiters` subiterations on the first factor: the
 * least-squares solution A1_next with A3 held fixed, the momentum update
 * A1 <- momentum A1 + (1 - momentum) A1_next, and A3 tied again.  The paper fixes neither
 * the momentum nor the subiteration count (1/2 averages as the Babylonian square-root
 * iteration the paper cites does).  Normal equations as in rom_cp_als, FP64 on the device.
 *   C             device FP64 [N][N][N] (as rom_cp_als); read only.
 *   A11, A12, B1  device FP64 [N][P]: the initial blocks on entry, the fitted ones on return.
 *   stream        as rom_cp_als.  Synchronizes; allocates and frees its own workspace
 *                 (about N^3 + 2 N^2 P doubles).
 * Errors: ROM_E_INVALID (N outside [1, 4096], P outside [1, 2048], sweeps or subiters < 0,
 * momentum outside [0, 1), NULL pointers, or a normal matrix that is not positive
 * definite), ROM_E_NOMEM, ROM_E_DEVICE.  sweeps = 0 does nothing. */
rom_status rom_cp_als_skew(int32_t N, int32_t P, const double *C, double *A11, double *A12, double *B1,
                           int32_t sweeps, int32_t subiters, double momentum, void *stream);

/* y = C(u)u for `batch` coefficient vectors (Sec. 2.2, eq. Cu; CP form: eq. tc_ap).
 * u_dev, y_dev: device FP64 [batch][N], caller-owned; 1 <= batch <= max_batch.
 * The contraction runs in the context's dtype; y is returned in FP64.  Asynchronous. */
rom_status rom_nonlinear(rom_ctx ctx, int32_t batch, const double *u_dev, double *y_dev);

/* rom_nonlinear for callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same kernels and
 * results as rom_nonlinear, but the workspace (partial sums, CP projections, operand
 * copies) is a fixed 32 MiB array that the library's code object holds on each GPU until
 * the process ends, instead of the context's workspace; the call allocates and frees
 * nothing and launches only kernels (the workspace it uses is cleared by a kernel, no
 * memset).  Every call on one GPU shares that array: calls that overlap in time on one
 * GPU (several streams, several threads) race and must be ordered by the caller.
 * Errors as rom_nonlinear, plus ROM_E_UNSUPPORTED when the evaluation's workspace
 * exceeds the 32 MiB (large batches of large N; rom_nonlinear has no such limit). */
rom_status rom_nonlinear_noalloc(rom_ctx ctx, int32_t batch, const double *u_dev, double *y_dev);

/* Measurement entry point: y = C(u)u exactly as rom_nonlinear computes it, but with the
 * contraction kernels (dense: the stream or MFMA contraction; CP: projections, Hadamard
 * product and scatter) captured `reps` >= 1 times into a HIP graph, launched once to warm
 * up and once between two HIP events on the context's stream; *kernel_us receives their
 * average duration per repetition (operand copies and the final sum of partial results
 * are outside the events).  For profiling and roofline reports; the context's stream
 * must not be capturing.  Synchronizes.  Errors as rom_nonlinear, plus ROM_E_INVALID for
 * reps < 1 or a NULL kernel_us. */
rom_status rom_nonlinear_timed(rom_ctx ctx, int32_t batch, const double *u_dev, double *y_dev,
                               int32_t reps, double *kernel_us);

/* A batch of trajectories at step 0 with initial coefficients u0_host [batch][N].
 * Synchronizes (one upload). */
rom_status rom_state_create(rom_ctx ctx, int32_t batch, const double *u0_host,
                            rom_state *out);
void rom_state_destroy(rom_state st);

/* Advance every trajectory of the state by nsteps BDFk/EXTk steps (eq. nse_d1 with
 * the 1-2-3 start-up ramp) and log the energy E = |u|^2/2 after each step.  Runs on the
 * context's stream as replays of captured graphs (see rom_step_prepare); synchronizes
 * once at the end to read the health flag.  Returns ROM_E_NONFINITE if any trajectory became non-finite, with the
 * first such step number in *first_bad_step (nullable; -1 if none). */
rom_status rom_step(rom_ctx ctx, rom_state st, int64_t nsteps, int64_t *first_bad_step);

/* Capture, without running any step, the HIP graphs that a later rom_step or
 * rom_step_async of nsteps replays, and move them to the device.  A call of nsteps
 * replays (nsteps - 1) / 64 graphs of 64 steps and one graph of the remaining 1..64 steps
 * ending with the step close; graphs depend on the parity of the first level only, and
 * both parities are prepared, so other steps may run in between.  A length is otherwise
 * captured the first time it is stepped.  Graphs are dropped when the energy log or a
 * workspace moves (it grows by doubling): the energy log is sized here for nsteps more
 * steps from the current level.  Synchronizes.  Errors as rom_step_async. */
rom_status rom_step_prepare(rom_ctx ctx, rom_state st, int64_t nsteps);

/* Enqueue nsteps without the final synchronization; rom_step_sync later waits and
 * reports the health flag exactly as rom_step does. */
rom_status rom_step_async(rom_ctx ctx, rom_state st, int64_t nsteps);
rom_status rom_step_sync(rom_ctx ctx, rom_state st, int64_t *first_bad_step);

/* Energies (eq. ene_fluc, first quantity, with identity mass matrix): 1/2 |u|^2 per level,
 * also for a full-form state, whose mass matrix M the log does not weight (it is the
 * quantity the non-finite check and the oracle's log use).  Synchronizes.
 * E_host [batch] (nullable): energy of the current level of each trajectory.
 * Elog_host (nullable): [steps+1][batch], level 0..steps of the state's step counter. */
rom_status rom_energy(rom_ctx ctx, rom_state st, double *E_host, double *Elog_host);

/* Checkpoint/resume.  u_hist [3][batch][N] = levels n, n-1, n-2; y_hist [2][batch][N] =
 * C(u)u at levels n-1, n-2; *step = n.  Levels below 0 are zero.  rom_state_set
 * restarts at step n from the given history (the energy log restarts at level n).  A
 * one-trajectory CP state with a dense stiffness carries lam .* (Bf^T u) .* (Cf^T u) from
 * step to step; a restart recomputes it for level n from u^n, so it continues an
 * uninterrupted run to rounding rather than bit for bit.  Both synchronize. */
rom_status rom_state_get(rom_ctx ctx, rom_state st, double *u_hist, double *y_hist,
                         int64_t *step);
rom_status rom_state_set(rom_ctx ctx, rom_state st, const double *u_hist,
                         const double *y_hist, int64_t step);

/* Continuous batching: replace trajectory b (0 <= b < batch) of a state by another one at
 * the state's current level n, leaving the other trajectories as they are.  u_hist [3][N]
 * holds the new trajectory's u at levels n, n-1, n-2 and y_hist [2][N] its C(u)u at
 * levels n-1, n-2 (host FP64), as rom_state_set takes for a whole state; E^n of trajectory
 * b is logged from u_hist[0].  A trajectory that has taken its own start-up steps (BDF1
 * and BDF2 from its level 0) joins a state at n >= 2 and continues with BDF3, as from its
 * own level 2; zeros make an idle slot (it stays zero).  clear_health != 0 also clears
 * the state's non-finite flag (for a caller that replaced every failed trajectory; see
 * rom_query what = 10 and rom_energy).  Every form and format (a full-form state
 * recomputes its zeroth-mode and mass terms from the u history; a one-trajectory CP state
 * with a dense stiffness recomputes the projections of level n).  Synchronizes. */
rom_status rom_state_set_slot(rom_ctx ctx, rom_state st, int32_t b, const double *u_hist, const double *y_hist,
                              int32_t clear_health);

/* Copy the current coefficients u^n [batch][N] into caller device memory.  Async. */
rom_status rom_state_u(rom_ctx ctx, rom_state st, double *u_dev);

/* Several (context, state) pairs advanced together by nsteps steps each, on the stream
 * of ctxs[0].  The one-trajectory states, whatever their N, CP rank, format, stiffness
 * kind (diagonal or dense) and operator form (dense, CP general or pair form, SVD, full
 * form), share at most four launches per step, one per phase of the step, each over a
 * device work table of all their jobs; batches (B > 1) run their own kernels inside the
 * same captured steps.  A state's results equal those of rom_step on it alone, to the bit.
 * The work tables and captured graphs of a set of pairs are built on its first call and
 * reused by later calls with the same pairs in the same order and level parities (they
 * are dropped when a member is destroyed).  Synchronizes at the end.  Returns
 * ROM_E_NONFINITE with the earliest non-finite level over all pairs; rom_query(what = 10)
 * tells which states failed. */
rom_status rom_step_multi(int32_t n, const rom_ctx *ctxs, const rom_state *states,
                          int64_t nsteps, int64_t *first_bad_step);

/* Introspection.  what: 0 = device bytes held by the context, 1 = device bytes held by
 * the state, 2 = N, 3 = R (0 if dense), 4 = dtype, 5 = state batch, 6 = state step,
 * 7 = skew column-pair layout the one-trajectory CP kernels use (rom_cp_skew_layout's
 * codes; 0 = general form), 8 = operator form (0 dense, 1 CP, 2 SVD), 9 = SVD rank
 * (0 unless SVD), 10 = the state's first non-finite level, -1 if none (synchronizes with
 * the context's stream; lets a caller of rom_step_multi find which states failed),
 * 11 = blocks of the resident runs the state's steps take from level 2 on (0: none; see
 * rom_set_tile kind 5). */
rom_status rom_query(rom_ctx ctx, rom_state st, int32_t what, int64_t *value);

/* Kernel tile selection (the autotuner's knob).  kind: 0 = dense single-trajectory
 * streaming contraction, 1 = dense batched MFMA contraction, 2 = CP projections,
 * 3 = CP scatter, 4 = pair form of the CP projections (0 = general form, 1 = pair form
 * for one trajectory and for batches, ROM_E_UNSUPPORTED if the factors have no skew column
 * pairs), 5 = resident runs of one-trajectory CP steps (0 = off: every step through the
 * per-step kernels; 1 or -1 = on where the operator fits on chip).  value: an index into
 * that kernel's variant table (see rom_tile_count); -1 restores the built-in choice (for
 * kind 4: the pair form for one trajectory whenever the factors allow it, the general
 * form for batches).  Applies to later launches.
 *
 * Resident runs: from level 2 on, a one-trajectory CP state (not the full form) takes runs
 * of 16 to 512 steps in one launch whose blocks, one per compute unit at most, keep their
 * rows of Af, the projection operator and (dense stiffness) Hinv_3 in LDS, and pass the
 * right-hand side and w = lam .* s .* t between them as tagged messages.  Every block of a
 * run must be on the device at once: the library orders the runs of a process across
 * streams (a run waits for the previous run on another stream), and a device shared with
 * another kernel that waits for all of its own blocks may delay a run until that kernel
 * ends.  They
 * apply when 2N <= 4096, Rp (FP64: 2 Rp) <= 4096 and the rows fit the device's LDS; the
 * results equal the per-step kernels' to the bit.  A wait for another block's data that
 * does not end within a bounded number of polling rounds (seconds) makes rom_step_sync
 * return ROM_E_DEVICE.  A run is not captured into graphs (a capturing stream takes the
 * per-step kernels).  When the runtime refuses a run's launch, the context takes the
 * per-step kernels from then on, with the same results. */
rom_status rom_set_tile(rom_ctx ctx, int32_t kind, int32_t value);
int32_t rom_tile_count(int32_t kind);

/* Skew column pairs of CP factors (Sec. 3.3, eq. skew_abc_struct), checked exactly on
 * the host (no device work; callable without a GPU).  Pair p = (c0, c1) must satisfy
 * lambda[c0] == lambda[c1], Bf[:,c0] == Bf[:,c1], Cf[:,c0] == Af[:,c1] and
 * Cf[:,c1] == -Af[:,c0].  Returns 1 for c0 = 2p, c1 = 2p + 1 (interleaved pairs), 2 for
 * c0 = p, c1 = R/2 + p (the paper's blocks [A1 A2], [B1 B1], [A2 -A1]), 0 otherwise
 * (also for odd R or NULL arrays).  Arrays: host [N][R] factors, lambda [R].
 * rom_create runs the same check: with pairs, the one-trajectory CP projections read the
 * P distinct columns of Bf and the R columns of Af (1.5 N R values instead of 2 N R) and
 * give the same result to the bit. */
int32_t rom_cp_skew_layout(int32_t N, int32_t R, const double *lambda, const double *Af,
                           const double *Bf, const double *Cf);

const char *rom_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ROM_H */
