/*
 * rom_oracle.c -- plain FP64 CPU oracle for the online stage of a Galerkin
 * reduced-order model whose advection tensor may be given in CP form
 * (arXiv 2311.03694, "Accelerating Galerkin Reduced-Order Models for Turbulent
 * Flows with Tensor Decomposition").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark load this file's library.  The product path never links,
 * calls or includes it, and it shares no code with the HIP sources.
 *
 * Every routine is a loop nest written in the order of the definition it cites, in IEEE
 * FP64 (built with -ffp-contract=off, no fast-math).  Loops over independent output rows
 * may be shared among host threads (OpenMP, orc_set_threads; one thread unless asked):
 * each row is still summed by one thread in the written order, so the results are the
 * same to the bit for any thread count.
 *
 * Storage (row-major, 0-based):
 *   C[i][j][k]  = the paper's C_{i k j} with output row i; the pair (j, k) is the pair
 *                 of advecting/advected coefficients.  The contraction is symmetric in
 *                 j and k, so y_i = sum_j sum_k C[i][j][k] u_j u_k  (Sec. 2.2, eq. Cu).
 *   Af,Bf,Cf    = [N][R] CP factors for tensor positions 1, 2, 3; lam = [R] weights.
 *   A           = [N][N] reduced stiffness; M = [N][N] reduced mass matrix (NULL: the
 *                 identity).
 *   C1, C2      = [N][N+1] zeroth-mode matrices of eq. zeroth_contribution, column 0
 *                 belonging to the zeroth mode (coefficient 1 in the augmented vector
 *                 ubar = [1, u_1 .. u_N]); c0, a0 = [N] zeroth-mode vectors.
 *
 * Parity status: every function below is pinned by a CPU test (closed forms,
 * invariants, brute force, library routines); none is "parity unpinned".
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ threads */

static int g_threads = 1;

/* Host threads for the row loops (>= 1); returns the previous count. */
int orc_set_threads(int n)
{
    int old = g_threads;
    g_threads = n < 1 ? 1 : n;
    return old;
}

int orc_get_threads(void) { return g_threads; }

/* ------------------------------------------------------------------ contractions */

/* Dense advection term of the G-ROM (Sec. 2.2, eq. Cu and the C(u)u term of eq. nse_d1):
 *   y_i = sum_{j} u_j * ( sum_{k} C[i][j][k] * u_k ),  2 N^3 flops. */
void orc_nonlinear_dense(int64_t N, const double *C, const double *u, double *y)
{
#pragma omp parallel for schedule(static) num_threads(g_threads)
    for (int64_t i = 0; i < N; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < N; ++j) {
            const double *row = C + (i * N + j) * N;
            double t = 0.0;
            for (int64_t k = 0; k < N; ++k)
                t += row[k] * u[k];
            s += u[j] * t;
        }
        y[i] = s;
    }
}

/* The same definition for a chosen subset of output rows (used at sizes where the
 * full N^3 contraction is too slow for a test): y_out[q] = y_{rows[q]}. */
void orc_nonlinear_dense_rows(int64_t N, const double *C, const double *u,
                              int64_t nrows, const int64_t *rows, double *y_out)
{
#pragma omp parallel for schedule(static) num_threads(g_threads)
    for (int64_t q = 0; q < nrows; ++q) {
        int64_t i = rows[q];
        double s = 0.0;
        for (int64_t j = 0; j < N; ++j) {
            const double *row = C + (i * N + j) * N;
            double t = 0.0;
            for (int64_t k = 0; k < N; ++k)
                t += row[k] * u[k];
            s += u[j] * t;
        }
        y_out[q] = s;
    }
}

/* CP contraction (Sec. 3.1, eq. tc_ap), with the weight vector lam:
 *   s_r = sum_k Bf[k][r] u_k,   t_r = sum_j Cf[j][r] u_j,
 *   y_i = sum_r Af[i][r] * (lam_r * s_r * t_r).               6 N R flops. */
void orc_nonlinear_cp(int64_t N, int64_t R, const double *lam, const double *Af,
                      const double *Bf, const double *Cf, const double *u, double *y)
{
    double *s = (double *)malloc(sizeof(double) * (size_t)(R > 0 ? R : 1));
    double *t = (double *)malloc(sizeof(double) * (size_t)(R > 0 ? R : 1));
#pragma omp parallel for schedule(static) num_threads(g_threads)
    for (int64_t r = 0; r < R; ++r) {
        double sr = 0.0, tr = 0.0;
        for (int64_t k = 0; k < N; ++k)
            sr += Bf[k * R + r] * u[k];
        for (int64_t j = 0; j < N; ++j)
            tr += Cf[j * R + r] * u[j];
        s[r] = sr;
        t[r] = tr;
    }
#pragma omp parallel for schedule(static) num_threads(g_threads)
    for (int64_t i = 0; i < N; ++i) {
        double acc = 0.0;
        for (int64_t r = 0; r < R; ++r)
            acc += Af[i * R + r] * (lam[r] * s[r] * t[r]);
        y[i] = acc;
    }
    free(s);
    free(t);
}

/* CP contraction of a decomposition that keeps the partial skew-symmetry
 * (Sec. 3.3, eq. skew_abc_struct): rank R = 2P with factor matrices
 *   A^(1) = [A11 A12],  A^(2) = [A21 A21],  A^(3) = [A12 -A11]   (each block N x P)
 * and one weight per pair of columns.  For pair p write a = A11[:,p], c = A12[:,p],
 * b = A21[:,p]; its two rank-1 terms of eq. tc_ap give
 *   y += lam_p (b^T u) (c^T u) a  +  lam_p (b^T u) (-(a^T u)) c,
 * so with beta_p = b^T u, alpha_p = a^T u, gamma_p = c^T u:
 *   y_i = sum_p lam_p beta_p (A11[i][p] gamma_p - A12[i][p] alpha_p).   5 N P flops. */
void orc_nonlinear_cp_skew(int64_t N, int64_t P, const double *lam, const double *A11,
                           const double *A12, const double *A21, const double *u, double *y)
{
    double *al = (double *)malloc(sizeof(double) * (size_t)(P > 0 ? P : 1));
    double *be = (double *)malloc(sizeof(double) * (size_t)(P > 0 ? P : 1));
    double *ga = (double *)malloc(sizeof(double) * (size_t)(P > 0 ? P : 1));
    for (int64_t p = 0; p < P; ++p) {
        double a = 0.0, b = 0.0, c = 0.0;
        for (int64_t k = 0; k < N; ++k) {
            a += A11[k * P + p] * u[k];
            b += A21[k * P + p] * u[k];
            c += A12[k * P + p] * u[k];
        }
        al[p] = a;
        be[p] = b;
        ga[p] = c;
    }
    for (int64_t i = 0; i < N; ++i) {
        double acc = 0.0;
        for (int64_t p = 0; p < P; ++p)
            acc += lam[p] * be[p] * (A11[i * P + p] * ga[p] - A12[i * P + p] * al[p]);
        y[i] = acc;
    }
    free(al);
    free(be);
    free(ga);
}

/* SVD-ROM contraction (Sec. 4.4): the mode-3 matricization of the tensor is replaced by
 * its rank-R SVD, C_(3) ~ U_R Sigma_R V_R^T.  In the storage order used here the mode-3
 * index is the second index j of C[i][j][k] (the advected coefficient), so
 *   C[i][j][k] ~ sum_r U[j][r] sigma_r V[i][k][r],
 * with U [N][R] and V [N][N][R] (row (i, k) of V_R), and
 *   s_r = sum_j U[j][r] u_j,   y_i = sum_r sigma_r s_r (sum_k V[i][k][r] u_k).   2 N^2 R flops. */
void orc_nonlinear_svd(int64_t N, int64_t R, const double *U, const double *sigma, const double *V,
                       const double *u, double *y)
{
    double *s = (double *)malloc(sizeof(double) * (size_t)(R > 0 ? R : 1));
    for (int64_t r = 0; r < R; ++r) {
        double acc = 0.0;
        for (int64_t j = 0; j < N; ++j)
            acc += U[j * R + r] * u[j];
        s[r] = acc;
    }
#pragma omp parallel for schedule(static) num_threads(g_threads)
    for (int64_t i = 0; i < N; ++i) {
        double yi = 0.0;
        for (int64_t r = 0; r < R; ++r) {
            double vr = 0.0;
            for (int64_t k = 0; k < N; ++k)
                vr += V[(i * N + k) * R + r] * u[k];
            yi += sigma[r] * s[r] * vr;
        }
        y[i] = yi;
    }
    free(s);
}

/* Kruskal tensor (Sec. 2.3, eq. cpd, with weights):
 *   T[i][j][k] = sum_r lam_r Af[i][r] Bf[j][r] Cf[k][r]. */
void orc_reconstruct(int64_t N, int64_t R, const double *lam, const double *Af,
                     const double *Bf, const double *Cf, double *T)
{
    for (int64_t i = 0; i < N; ++i)
        for (int64_t j = 0; j < N; ++j)
            for (int64_t k = 0; k < N; ++k) {
                double acc = 0.0;
                for (int64_t r = 0; r < R; ++r)
                    acc += lam[r] * Af[i * R + r] * Bf[j * R + r] * Cf[k * R + r];
                T[(i * N + j) * N + k] = acc;
            }
}

/* ------------------------------------------------------------------ linear algebra */

/* Cholesky factor H = L L^T of a symmetric positive definite matrix (textbook
 * column-by-column form).  L is written lower-triangular, zeros above.
 * Returns 0, or -1 if a pivot is not positive. */
int orc_cholesky(int64_t N, const double *H, double *L)
{
    memset(L, 0, sizeof(double) * (size_t)(N * N));
    for (int64_t j = 0; j < N; ++j) {
        double d = H[j * N + j];
        for (int64_t m = 0; m < j; ++m)
            d -= L[j * N + m] * L[j * N + m];
        if (!(d > 0.0))
            return -1;
        double ljj = sqrt(d);
        L[j * N + j] = ljj;
        for (int64_t i = j + 1; i < N; ++i) {
            double v = H[i * N + j];
            for (int64_t m = 0; m < j; ++m)
                v -= L[i * N + m] * L[j * N + m];
            L[i * N + j] = v / ljj;
        }
    }
    return 0;
}

/* Solve L L^T x = b: forward substitution, then back substitution. */
void orc_chol_solve(int64_t N, const double *L, const double *b, double *x)
{
    double *z = (double *)malloc(sizeof(double) * (size_t)N);
    for (int64_t i = 0; i < N; ++i) {
        double v = b[i];
        for (int64_t m = 0; m < i; ++m)
            v -= L[i * N + m] * z[m];
        z[i] = v / L[i * N + i];
    }
    for (int64_t i = N - 1; i >= 0; --i) {
        double v = z[i];
        for (int64_t m = i + 1; m < N; ++m)
            v -= L[m * N + i] * x[m];
        x[i] = v / L[i * N + i];
    }
    free(z);
}

/* ------------------------------------------------------------------ energy */

/* Kinetic energy of the reduced state with identity mass matrix (eq. ene_fluc,
 * first quantity): E = 1/2 sum_i u_i^2. */
double orc_energy(int64_t N, const double *u)
{
    double s = 0.0;
    for (int64_t i = 0; i < N; ++i)
        s += u[i] * u[i];
    return 0.5 * s;
}

/* ------------------------------------------------------------------ BDFk / EXTk */

/* Coefficients of the k-th order backward difference (beta) and extrapolation
 * (alpha) used by the semi-implicit scheme of eq. nse_d1.  beta[0] multiplies the
 * new level on the left; beta[q], alpha[q-1] (q = 1..k) multiply level n+1-q on the
 * right.  They follow from differentiating (BDF) and evaluating (EXT) at t^{n+1} the
 * Lagrange polynomial through the last k (EXT) or k+1 (BDF) equispaced levels. */
static void bdf_ext(int k, double beta[4], double alpha[3])
{
    memset(beta, 0, 4 * sizeof(double));
    memset(alpha, 0, 3 * sizeof(double));
    if (k == 1) {
        beta[0] = 1.0;  beta[1] = -1.0;
        alpha[0] = 1.0;
    } else if (k == 2) {
        beta[0] = 1.5;  beta[1] = -2.0; beta[2] = 0.5;
        alpha[0] = 2.0; alpha[1] = -1.0;
    } else {
        beta[0] = 11.0 / 6.0; beta[1] = -3.0; beta[2] = 1.5; beta[3] = -1.0 / 3.0;
        alpha[0] = 3.0; alpha[1] = -3.0; alpha[2] = 1.0;
    }
}

/* The advection operator of a run: the dense tensor (C), the CP factors (R, lam, Af, Bf,
 * Cf) or the SVD form of the SVD-ROM (Rs, U, sigma, V), in that order of precedence. */
typedef struct {
    const double *C;
    int64_t R;
    const double *lam, *Af, *Bf, *Cf;
    int64_t Rs;
    const double *U, *sigma, *V;
} orc_adv;

static void advection(int64_t N, const orc_adv *op, const double *u, double *y)
{
    if (op->C)
        orc_nonlinear_dense(N, op->C, u, y);
    else if (op->U)
        orc_nonlinear_svd(N, op->Rs, op->U, op->sigma, op->V, u, y);
    else
        orc_nonlinear_cp(N, op->R, op->lam, op->Af, op->Bf, op->Cf, u, y);
}

/* Explicit term of eq. nse_d1 at one level (Sec. 2.2):
 *   g = C(u)u + (C1 + C2) ubar - c0,   ubar = [1, u_1 .. u_N],
 * C1, C2, c0 each optional (NULL: zero). */
static void explicit_full(int64_t N, const orc_adv *op, const double *C1, const double *C2,
                          const double *c0, const double *u, double *g)
{
    advection(N, op, u, g);
    for (int64_t i = 0; i < N; ++i) {
        double v = 0.0;
        for (int64_t j = 0; j <= N; ++j) {
            const double ub = j == 0 ? 1.0 : u[j - 1];
            const double m = (C1 ? C1[i * (N + 1) + j] : 0.0) + (C2 ? C2[i * (N + 1) + j] : 0.0);
            v += m * ub;
        }
        g[i] += v - (c0 ? c0[i] : 0.0);
    }
}

/* The same with C(u)u the dense contraction if C != NULL, else the CP contraction. */
void orc_explicit_full(int64_t N, const double *C, int64_t R, const double *lam, const double *Af,
                       const double *Bf, const double *Cf, const double *C1, const double *C2,
                       const double *c0, const double *u, double *g)
{
    const orc_adv op = {C, R, lam, Af, Bf, Cf, 0, NULL, NULL, NULL};
    explicit_full(N, &op, C1, C2, c0, u, g);
}

/* Time integration of  M du/dt = -C(ubar)ubar - nu A ubar  (eq. nse_ode; M = I and no
 * zeroth-mode terms in orc_run) by the semi-implicit BDFk/EXTk scheme of eq. nse_d1:
 *
 *   (beta0/dt M + nu A) u^{n+1} = - sum_{q=1..k} alpha_q g^{n+1-q}
 *                                 - M (1/dt) sum_{q=1..k} beta_q u^{n+1-q} - nu a0,
 *   g^m = C(u^m) u^m + (C1 + C2) ubar^m - c0   (orc_explicit_full),
 *
 * with k = min(n+1, 3): the first step is BDF1/EXT1, the second BDF2/EXT2, then
 * BDF3/EXT3.
 *
 * State (in/out): step n, uh = [u^n, u^{n-1}, u^{n-2}] ([3][N]), yh = [g^{n-1},
 * g^{n-2}] ([2][N]); levels that do not exist yet are ignored.  The advection term is
 * the dense contraction if C != NULL, else the CP contraction.
 * Outputs (optional): E[0..nsteps] = energies of u^{n}..u^{n+nsteps};
 * traj[(s)][N] = u^{n+s}.
 * Returns 0 ok, 1 if a Helmholtz matrix is not SPD, 2 on allocation failure,
 * 4 if a state became non-finite (first_bad = that step index, integration stops). */
static int run_core(int64_t N, double nu, double dt, const double *A, const double *M,
                    const orc_adv *op, const double *C1, const double *C2,
                    const double *c0, const double *a0, int64_t step0, double *uh, double *yh,
                    int64_t nsteps, double *E, double *traj, int64_t *first_bad)
{
    size_t nn = (size_t)(N * N);
    double *L[3] = {NULL, NULL, NULL};
    double *H = (double *)malloc(sizeof(double) * nn);
    double *y = (double *)malloc(sizeof(double) * (size_t)N);
    double *rhs = (double *)malloc(sizeof(double) * (size_t)N);
    double *un = (double *)malloc(sizeof(double) * (size_t)N);
    int status = 0;
    if (first_bad)
        *first_bad = -1;
    if (!H || !y || !rhs || !un) {
        status = 2;
        goto done;
    }
    if (E)
        E[0] = orc_energy(N, uh);
    if (traj)
        memcpy(traj, uh, sizeof(double) * (size_t)N);

    for (int64_t s = 0; s < nsteps; ++s) {
        int64_t n = step0 + s;
        int k = (int)(n + 1 < 3 ? n + 1 : 3);
        double beta[4], alpha[3];
        bdf_ext(k, beta, alpha);

        if (!L[k - 1]) {
            L[k - 1] = (double *)malloc(sizeof(double) * nn);
            if (!L[k - 1]) {
                status = 2;
                goto done;
            }
            for (int64_t i = 0; i < N; ++i)
                for (int64_t j = 0; j < N; ++j)
                    H[i * N + j] = nu * A[i * N + j] +
                                   (beta[0] / dt) * (M ? M[i * N + j] : (i == j ? 1.0 : 0.0));
            if (orc_cholesky(N, H, L[k - 1]) != 0) {
                status = 1;
                goto done;
            }
        }

        /* g^n (the advection term, plus the zeroth-mode terms when given) */
        explicit_full(N, op, C1, C2, c0, uh, y);

        /* right-hand side: levels n, n-1, n-2 are uh[0..2] and y, yh[0], yh[1] */
        for (int64_t i = 0; i < N; ++i) {
            const double *ylev[3] = {y, yh, yh + N};
            double v = 0.0;
            for (int q = 1; q <= k; ++q)
                v -= alpha[q - 1] * ylev[q - 1][i];
            if (M) {
                for (int64_t j = 0; j < N; ++j) {
                    double h = 0.0;
                    for (int q = 1; q <= k; ++q)
                        h += (beta[q] / dt) * uh[(size_t)(q - 1) * N + j];
                    v -= M[i * N + j] * h;
                }
            } else {
                for (int q = 1; q <= k; ++q)
                    v -= (beta[q] / dt) * uh[(size_t)(q - 1) * N + i];
            }
            if (a0)
                v -= nu * a0[i];
            rhs[i] = v;
        }
        orc_chol_solve(N, L[k - 1], rhs, un);

        /* shift histories */
        memcpy(uh + 2 * N, uh + N, sizeof(double) * (size_t)N);
        memcpy(uh + N, uh, sizeof(double) * (size_t)N);
        memcpy(uh, un, sizeof(double) * (size_t)N);
        memcpy(yh + N, yh, sizeof(double) * (size_t)N);
        memcpy(yh, y, sizeof(double) * (size_t)N);

        double e = orc_energy(N, uh);
        if (E)
            E[s + 1] = e;
        if (traj)
            memcpy(traj + (size_t)(s + 1) * N, uh, sizeof(double) * (size_t)N);
        if (!isfinite(e)) {
            if (first_bad)
                *first_bad = n + 1;
            status = 4;
            goto done;
        }
    }
done:
    for (int q = 0; q < 3; ++q)
        free(L[q]);
    free(H);
    free(y);
    free(rhs);
    free(un);
    return status;
}

/* The run with the dense tensor (C != NULL) or the CP factors as the advection term. */
int orc_run_full(int64_t N, double nu, double dt, const double *A, const double *M,
                 const double *C, int64_t R, const double *lam, const double *Af,
                 const double *Bf, const double *Cf, const double *C1, const double *C2,
                 const double *c0, const double *a0, int64_t step0, double *uh, double *yh,
                 int64_t nsteps, double *E, double *traj, int64_t *first_bad)
{
    const orc_adv op = {C, R, lam, Af, Bf, Cf, 0, NULL, NULL, NULL};
    return run_core(N, nu, dt, A, M, &op, C1, C2, c0, a0, step0, uh, yh, nsteps, E, traj, first_bad);
}

/* orc_run_full with the identity mass matrix and no zeroth-mode terms. */
int orc_run(int64_t N, double nu, double dt, const double *A, const double *C, int64_t R,
            const double *lam, const double *Af, const double *Bf, const double *Cf,
            int64_t step0, double *uh, double *yh, int64_t nsteps, double *E, double *traj,
            int64_t *first_bad)
{
    return orc_run_full(N, nu, dt, A, NULL, C, R, lam, Af, Bf, Cf, NULL, NULL, NULL, NULL, step0, uh,
                        yh, nsteps, E, traj, first_bad);
}

/* orc_run with the SVD form of the SVD-ROM (Sec. 4.4, orc_nonlinear_svd) as the advection
 * term: U [N][Rs], sigma [Rs], V [N][N][Rs]. */
int orc_run_svd(int64_t N, double nu, double dt, const double *A, int64_t Rs, const double *U,
                const double *sigma, const double *V, int64_t step0, double *uh, double *yh,
                int64_t nsteps, double *E, double *traj, int64_t *first_bad)
{
    const orc_adv op = {NULL, 0, NULL, NULL, NULL, NULL, Rs, U, sigma, V};
    return run_core(N, nu, dt, A, NULL, &op, NULL, NULL, NULL, NULL, step0, uh, yh, nsteps, E, traj,
                    first_bad);
}

/* ------------------------------------------------------------------ storage rounding */

/* FP64 -> FP32, round to nearest even (the C conversion in the default rounding mode). */
void orc_round_f32(int64_t n, const double *x, double *out)
{
    for (int64_t i = 0; i < n; ++i)
        out[i] = (double)(float)x[i];
}

/* FP32 -> BF16 (1 sign, 8 exponent, 7 stored fraction bits), round to nearest, ties to
 * even, by comparing the 16 dropped bits with one half unit in the last place. */
static float bf16_of_f32(float f)
{
    uint32_t b;
    memcpy(&b, &f, 4);
    if ((b & 0x7f800000u) == 0x7f800000u) {            /* inf or NaN: keep, quiet NaN */
        if (b & 0x007fffffu)
            b |= 0x00400000u;
        b &= 0xffff0000u;
    } else {
        uint32_t low = b & 0xffffu;
        uint32_t high = b & 0xffff0000u;
        int up = (low > 0x8000u) || (low == 0x8000u && (high & 0x10000u));
        b = up ? high + 0x10000u : high;                  /* carry may reach inf: correct */
    }
    float r;
    memcpy(&r, &b, 4);
    return r;
}

/* FP64 -> FP32 -> BF16, each step round-to-nearest-even. */
void orc_round_bf16(int64_t n, const double *x, double *out)
{
    for (int64_t i = 0; i < n; ++i)
        out[i] = (double)bf16_of_f32((float)x[i]);
}

/* Split into two BF16 words: hi = bf16(fp32(x)), lo = bf16(fp32(x) - hi). */
void orc_split_bf16x3(int64_t n, const double *x, double *hi, double *lo)
{
    for (int64_t i = 0; i < n; ++i) {
        float f = (float)x[i];
        float h = bf16_of_f32(f);
        float l = bf16_of_f32(f - h);
        hi[i] = (double)h;
        lo[i] = (double)l;
    }
}
