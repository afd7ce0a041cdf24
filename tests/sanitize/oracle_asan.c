/* oracle_asan.c -- drives every function of the FP64 oracle (oracle/rom_oracle.c) in a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer (test infrastructure).
 *
 * Each call is checked against a relation the functions must satisfy, so the run is a
 * test and not only a memory check:
 *   - the CP contraction equals the dense contraction of the reconstructed tensor
 *     (Sec. 3.1, eq. tc_ap against eq. Cu);
 *   - the skew-pair contraction equals the CP contraction of its expanded factors
 *     (Sec. 3.3, eq. skew_abc_struct);
 *   - the SVD-ROM contraction equals the dense contraction of the tensor its factors
 *     define (Sec. 4.4);
 *   - the row subset equals the full dense contraction bitwise;
 *   - the Cholesky solve leaves a small residual;
 *   - the explicit full-form term without mass matrix or zeroth-mode terms equals the
 *     advection term, and the full-form run with M = I and no terms equals the plain run
 *     to rounding (it sums the history before applying M);
 *   - every run is bitwise the same on one and on four OpenMP threads;
 *   - storage rounding is idempotent and the BF16 split reconstructs the FP32 value.
 * Exit status 0 when every check holds. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int orc_set_threads(int n);
void orc_nonlinear_dense(int64_t N, const double *C, const double *u, double *y);
void orc_nonlinear_dense_rows(int64_t N, const double *C, const double *u, int64_t nrows, const int64_t *rows,
                              double *y_out);
void orc_nonlinear_cp(int64_t N, int64_t R, const double *lam, const double *Af, const double *Bf, const double *Cf,
                      const double *u, double *y);
void orc_nonlinear_cp_skew(int64_t N, int64_t P, const double *lam, const double *A11, const double *A12,
                           const double *A21, const double *u, double *y);
void orc_nonlinear_svd(int64_t N, int64_t R, const double *U, const double *sigma, const double *V, const double *u,
                       double *y);
void orc_reconstruct(int64_t N, int64_t R, const double *lam, const double *Af, const double *Bf, const double *Cf,
                     double *T);
int orc_cholesky(int64_t N, const double *H, double *L);
void orc_chol_solve(int64_t N, const double *L, const double *b, double *x);
double orc_energy(int64_t N, const double *u);
void orc_explicit_full(int64_t N, const double *C, int64_t R, const double *lam, const double *Af, const double *Bf,
                       const double *Cf, const double *C1, const double *C2, const double *c0, const double *u,
                       double *g);
int orc_run_full(int64_t N, double nu, double dt, const double *A, const double *M, const double *C, int64_t R,
                 const double *lam, const double *Af, const double *Bf, const double *Cf, const double *C1,
                 const double *C2, const double *c0, const double *a0, int64_t step0, double *uh, double *yh,
                 int64_t nsteps, double *E, double *traj, int64_t *first_bad);
int orc_run(int64_t N, double nu, double dt, const double *A, const double *C, int64_t R, const double *lam,
            const double *Af, const double *Bf, const double *Cf, int64_t step0, double *uh, double *yh,
            int64_t nsteps, double *E, double *traj, int64_t *first_bad);
int orc_run_svd(int64_t N, double nu, double dt, const double *A, int64_t Rs, const double *U, const double *sigma,
                const double *V, int64_t step0, double *uh, double *yh, int64_t nsteps, double *E, double *traj,
                int64_t *first_bad);
void orc_round_f32(int64_t n, const double *x, double *out);
void orc_round_bf16(int64_t n, const double *x, double *out);
void orc_split_bf16x3(int64_t n, const double *x, double *hi, double *lo);

static int failures = 0;

static void check(int ok, const char *what)
{
    if (!ok) {
        fprintf(stderr, "FAIL: %s\n", what);
        ++failures;
    }
}

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;

static double uniform(void) /* splitmix64 -> [-1, 1) */
{
    uint64_t z = (rng_state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

static double *vec(int64_t n)
{
    double *v = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i)
        v[i] = uniform();
    return v;
}

static double *zeros(int64_t n) { return (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double)); }

static double rel_diff(int64_t n, const double *a, const double *b)
{
    double d = 0.0, m = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        d = fmax(d, fabs(a[i] - b[i]));
        m = fmax(m, fabs(b[i]));
    }
    return d / (m > 0.0 ? m : 1.0);
}

/* Both runs of a problem (1 and 4 threads) must agree bitwise; returns the status. */
typedef int (*run_fn)(void *ctx, double *uh, double *yh, double *E, double *traj, int64_t *first_bad);

static void run_both(run_fn f, void *ctx, int64_t N, int64_t nsteps, const char *what)
{
    double *out[2][4];
    int64_t fb[2];
    int st[2];
    for (int t = 0; t < 2; ++t) {
        orc_set_threads(t ? 4 : 1);
        rng_state = 42;
        out[t][0] = zeros(3 * N);
        for (int64_t i = 0; i < N; ++i)
            out[t][0][i] = 0.1 * uniform();
        out[t][1] = zeros(2 * N);
        out[t][2] = zeros(nsteps + 1);
        out[t][3] = zeros((nsteps + 1) * N);
        st[t] = f(ctx, out[t][0], out[t][1], out[t][2], out[t][3], &fb[t]);
    }
    orc_set_threads(1);
    char msg[160];
    snprintf(msg, sizeof msg, "%s: status 0", what);
    check(st[0] == 0 && st[1] == 0, msg);
    snprintf(msg, sizeof msg, "%s: 1 and 4 threads bitwise equal", what);
    check(memcmp(out[0][3], out[1][3], sizeof(double) * (size_t)((nsteps + 1) * N)) == 0 &&
              memcmp(out[0][2], out[1][2], sizeof(double) * (size_t)(nsteps + 1)) == 0,
          msg);
    snprintf(msg, sizeof msg, "%s: finite energies", what);
    int fin = 1;
    for (int64_t s = 0; s <= nsteps; ++s)
        fin = fin && isfinite(out[0][2][s]);
    check(fin, msg);
    for (int t = 0; t < 2; ++t)
        for (int q = 0; q < 4; ++q)
            free(out[t][q]);
}

typedef struct {
    int64_t N, R, Rs;
    const double *A, *M, *C, *lam, *Af, *Bf, *Cf, *C1, *C2, *c0, *a0, *U, *sigma, *V;
} prob;

static const int64_t kSteps = 25;

static int run_dense(void *c, double *uh, double *yh, double *E, double *traj, int64_t *fb)
{
    const prob *p = (const prob *)c;
    return orc_run(p->N, 1e-2, 1e-2, p->A, p->C, 0, NULL, NULL, NULL, NULL, 0, uh, yh, kSteps, E, traj, fb);
}

static int run_cp(void *c, double *uh, double *yh, double *E, double *traj, int64_t *fb)
{
    const prob *p = (const prob *)c;
    return orc_run(p->N, 1e-2, 1e-2, p->A, NULL, p->R, p->lam, p->Af, p->Bf, p->Cf, 0, uh, yh, kSteps, E, traj, fb);
}

static int run_svd(void *c, double *uh, double *yh, double *E, double *traj, int64_t *fb)
{
    const prob *p = (const prob *)c;
    return orc_run_svd(p->N, 1e-2, 1e-2, p->A, p->Rs, p->U, p->sigma, p->V, 0, uh, yh, kSteps, E, traj, fb);
}

static int run_full(void *c, double *uh, double *yh, double *E, double *traj, int64_t *fb)
{
    const prob *p = (const prob *)c;
    return orc_run_full(p->N, 1e-2, 1e-2, p->A, p->M, NULL, p->R, p->lam, p->Af, p->Bf, p->Cf, p->C1, p->C2, p->c0,
                        p->a0, 0, uh, yh, kSteps, E, traj, fb);
}

int main(void)
{
    const int64_t N = 7, R = 5, P = 3, Rs = 4;
    const int64_t N3 = N * N * N;

    /* CP against the dense contraction of its Kruskal tensor */
    double *lam = vec(R), *Af = vec(N * R), *Bf = vec(N * R), *Cf = vec(N * R), *u = vec(N);
    double *T = zeros(N3), *y1 = zeros(N), *y2 = zeros(N), *y3 = zeros(N);
    orc_reconstruct(N, R, lam, Af, Bf, Cf, T);
    orc_nonlinear_dense(N, T, u, y1);
    orc_nonlinear_cp(N, R, lam, Af, Bf, Cf, u, y2);
    check(rel_diff(N, y2, y1) < 1e-13, "cp equals dense of the reconstruction");

    /* row subset, bitwise */
    int64_t rows[3] = {N - 1, 0, 3};
    orc_nonlinear_dense_rows(N, T, u, 3, rows, y3);
    check(y3[0] == y1[N - 1] && y3[1] == y1[0] && y3[2] == y1[3], "row subset equals the dense rows");

    /* skew pairs against the expanded factors [A11 A12], [A21 A21], [A12 -A11] */
    double *lp = vec(P), *A11 = vec(N * P), *A12 = vec(N * P), *A21 = vec(N * P);
    double *lx = zeros(2 * P), *Ax = zeros(N * 2 * P), *Bx = zeros(N * 2 * P), *Cx = zeros(N * 2 * P);
    for (int64_t p = 0; p < P; ++p) {
        lx[p] = lx[P + p] = lp[p];
        for (int64_t i = 0; i < N; ++i) {
            Ax[i * 2 * P + p] = A11[i * P + p];
            Ax[i * 2 * P + P + p] = A12[i * P + p];
            Bx[i * 2 * P + p] = Bx[i * 2 * P + P + p] = A21[i * P + p];
            Cx[i * 2 * P + p] = A12[i * P + p];
            Cx[i * 2 * P + P + p] = -A11[i * P + p];
        }
    }
    orc_nonlinear_cp_skew(N, P, lp, A11, A12, A21, u, y1);
    orc_nonlinear_cp(N, 2 * P, lx, Ax, Bx, Cx, u, y2);
    check(rel_diff(N, y1, y2) < 1e-13, "skew pairs equal the expanded CP factors");

    /* SVD-ROM against the tensor C[i][j][k] = sum_r U[j][r] sigma_r V[i][k][r] */
    double *U = vec(N * Rs), *sg = vec(Rs), *V = vec(N * N * Rs), *Cs = zeros(N3);
    for (int64_t i = 0; i < N; ++i)
        for (int64_t j = 0; j < N; ++j)
            for (int64_t k = 0; k < N; ++k) {
                double a = 0.0;
                for (int64_t r = 0; r < Rs; ++r)
                    a += U[j * Rs + r] * sg[r] * V[(i * N + k) * Rs + r];
                Cs[(i * N + j) * N + k] = a;
            }
    orc_nonlinear_svd(N, Rs, U, sg, V, u, y1);
    orc_nonlinear_dense(N, Cs, u, y2);
    check(rel_diff(N, y1, y2) < 1e-13, "svd equals dense of its tensor");

    /* SPD solve: H = B B^T + N I */
    double *B = vec(N * N), *H = zeros(N * N), *L = zeros(N * N), *b = vec(N), *x = zeros(N), *Hx = zeros(N);
    for (int64_t i = 0; i < N; ++i)
        for (int64_t j = 0; j < N; ++j) {
            double a = i == j ? (double)N : 0.0;
            for (int64_t m = 0; m < N; ++m)
                a += B[i * N + m] * B[j * N + m];
            H[i * N + j] = a;
        }
    check(orc_cholesky(N, H, L) == 0, "cholesky of an SPD matrix succeeds");
    orc_chol_solve(N, L, b, x);
    for (int64_t i = 0; i < N; ++i) {
        Hx[i] = 0.0;
        for (int64_t j = 0; j < N; ++j)
            Hx[i] += H[i * N + j] * x[j];
    }
    check(rel_diff(N, Hx, b) < 1e-13, "cholesky solve residual");
    double *Hn = zeros(N * N);
    memcpy(Hn, H, sizeof(double) * (size_t)(N * N));
    Hn[0] = -1.0;
    check(orc_cholesky(N, Hn, L) == -1, "cholesky rejects a non-positive pivot");

    /* energy */
    double e = 0.0;
    for (int64_t i = 0; i < N; ++i)
        e += u[i] * u[i];
    check(orc_energy(N, u) == 0.5 * e, "energy is half the squared norm");

    /* explicit full-form term without terms equals the advection term */
    orc_explicit_full(N, T, 0, NULL, NULL, NULL, NULL, NULL, NULL, NULL, u, y1);
    orc_nonlinear_dense(N, T, u, y2);
    check(memcmp(y1, y2, sizeof(double) * (size_t)N) == 0, "explicit term without terms equals dense");

    /* runs: stiffness A SPD (H / N), full form with M = I and zero terms */
    double *A = zeros(N * N), *M = zeros(N * N);
    for (int64_t i = 0; i < N * N; ++i)
        A[i] = H[i] / (double)N;
    for (int64_t i = 0; i < N; ++i)
        M[i * N + i] = 1.0;
    double *C1 = zeros(N * (N + 1)), *C2 = zeros(N * (N + 1)), *c0 = zeros(N), *a0 = zeros(N);
    prob pr = {N, R, Rs, A, M, T, lam, Af, Bf, Cf, C1, C2, c0, a0, U, sg, V};
    run_both(run_dense, &pr, N, kSteps, "dense run");
    run_both(run_cp, &pr, N, kSteps, "cp run");
    run_both(run_svd, &pr, N, kSteps, "svd run");
    run_both(run_full, &pr, N, kSteps, "full-form run");
    {
        double *uh[2], *yh[2], *E[2], *tr[2];
        int64_t fb[2];
        for (int t = 0; t < 2; ++t) {
            rng_state = 7;
            uh[t] = zeros(3 * N);
            for (int64_t i = 0; i < N; ++i)
                uh[t][i] = 0.1 * uniform();
            yh[t] = zeros(2 * N);
            E[t] = zeros(kSteps + 1);
            tr[t] = zeros((kSteps + 1) * N);
        }
        orc_run(N, 1e-2, 1e-2, A, NULL, R, lam, Af, Bf, Cf, 0, uh[0], yh[0], kSteps, E[0], tr[0], &fb[0]);
        orc_run_full(N, 1e-2, 1e-2, A, M, NULL, R, lam, Af, Bf, Cf, C1, C2, c0, a0, 0, uh[1], yh[1], kSteps, E[1],
                     tr[1], &fb[1]);
        check(rel_diff((kSteps + 1) * N, tr[1], tr[0]) < 1e-12,
              "full-form run with M = I and no terms equals the plain run");
        for (int t = 0; t < 2; ++t) {
            free(uh[t]);
            free(yh[t]);
            free(E[t]);
            free(tr[t]);
        }
    }

    /* storage rounding */
    double *r1 = zeros(N), *r2 = zeros(N), *hi = zeros(N), *lo = zeros(N);
    orc_round_f32(N, u, r1);
    orc_round_f32(N, r1, r2);
    check(memcmp(r1, r2, sizeof(double) * (size_t)N) == 0, "fp32 rounding is idempotent");
    orc_round_bf16(N, u, r1);
    orc_round_bf16(N, r1, r2);
    check(memcmp(r1, r2, sizeof(double) * (size_t)N) == 0, "bf16 rounding is idempotent");
    orc_split_bf16x3(N, u, hi, lo);
    orc_round_f32(N, u, r2);
    int close = 1;
    for (int64_t i = 0; i < N; ++i)
        close = close && fabs(hi[i] + lo[i] - r2[i]) <= 0x1p-16 * fabs(r2[i]);
    check(close, "bf16 split reconstructs the fp32 value to 2^-16");

    double *all[] = {lam, Af, Bf, Cf, u, T, y1, y2, y3, lp, A11, A12, A21, lx, Ax, Bx, Cx, U, sg, V, Cs,
                     B, H, L, b, x, Hx, Hn, A, M, C1, C2, c0, a0, r1, r2, hi, lo};
    for (size_t q = 0; q < sizeof all / sizeof all[0]; ++q)
        free(all[q]);
    if (failures) {
        fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    printf("oracle sanitizer run: all checks hold\n");
    return 0;
}
