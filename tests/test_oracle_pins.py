"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: hand-worked exact
rationals (tests/golden), closed forms, invariants, library routines, or a
convergence order.  Together they catch a dropped term, a wrong sign or index, a
transposed operand or a wrong scheme coefficient anywhere in rom_oracle.c.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

import romsynth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    vals = {}
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = (s.strip() for s in line.split("="))
            vals[k] = Fraction(v)
    return vals


# ---------------------------------------------------------------- contraction

def test_worked_example_contraction(orc):
    g = _golden("n2_worked_example.txt")
    C = np.zeros((2, 2, 2))
    C[0, 0, 1] = float(g["a"])
    C[0, 1, 1] = float(g["b"])
    C[1, 0, 0] = -float(g["a"])
    C[1, 1, 0] = -float(g["b"])
    u = np.array([float(g["u0_0"]), float(g["u0_1"])])
    y = orc.nonlinear_dense(C, u)
    assert y[0] == float(g["y0_0"]) and y[1] == float(g["y0_1"])


def test_unit_tensor_index_positions(orc):
    """A tensor with one non-zero entry selects exactly one product u_j u_k into row i.
    This fixes which position is the output and which two are contracted."""
    N = 4
    u = np.array([1.0, 2.0, 3.0, 5.0])
    for (i, j, k) in [(0, 1, 2), (3, 0, 0), (2, 3, 1), (1, 2, 3)]:
        C = np.zeros((N, N, N))
        C[i, j, k] = 1.0
        y = orc.nonlinear_dense(C, u)
        expect = np.zeros(N)
        expect[i] = u[j] * u[k]
        assert np.array_equal(y, expect)


def test_unit_factors_cp_positions(orc):
    """Rank-1 CP with unit vectors: only row i of y is non-zero, equal to lam*u_j*u_k,
    where i, j, k index the non-zeros of the first, second and third factor."""
    N = 5
    u = np.array([1.0, -2.0, 3.0, 0.5, 7.0])
    for (i, j, k) in [(0, 1, 2), (4, 3, 3), (2, 0, 4)]:
        Af = np.zeros((N, 1)); Af[i, 0] = 1.0
        Bf = np.zeros((N, 1)); Bf[j, 0] = 1.0
        Cf = np.zeros((N, 1)); Cf[k, 0] = 1.0
        lam = np.array([0.25])
        y = orc.nonlinear_cp(lam, Af, Bf, Cf, u)
        expect = np.zeros(N)
        expect[i] = 0.25 * u[j] * u[k]
        assert np.array_equal(y, expect)
        T = orc.reconstruct(lam, Af, Bf, Cf)
        Texp = np.zeros((N, N, N))
        Texp[i, j, k] = 0.25
        assert np.array_equal(T, Texp)


def test_energy_identity_skew(orc):
    """Skew symmetry in positions 1 and 3 (Sec. 3.2) makes u . C(u)u vanish."""
    for N, seed in [(16, 0), (33, 1)]:
        C = romsynth.dense_rough(N, seed, cfg=7)
        u = romsynth.initial_u(N, [seed], cfg=7)[0]
        y = orc.nonlinear_dense(C, u)
        scale = np.einsum("ijk,i,j,k->", np.abs(C), np.abs(u), np.abs(u), np.abs(u))
        assert abs(u @ y) <= 1e-14 * scale
        # a non-skew tensor does not satisfy it (the check has teeth)
        y2 = orc.nonlinear_dense(C + np.abs(C), u)
        assert abs(u @ y2) > 1e-6 * scale


def test_homogeneity_and_symmetry_in_pair(orc):
    N = 12
    rng = np.random.default_rng(3)
    C = rng.standard_normal((N, N, N))
    u = rng.standard_normal(N)
    y = orc.nonlinear_dense(C, u)
    assert np.array_equal(orc.nonlinear_dense(C, 2.0 * u), 4.0 * y)
    # positions 2 and 3 enter symmetrically
    y_sw = orc.nonlinear_dense(np.ascontiguousarray(C.transpose(0, 2, 1)), u)
    assert np.allclose(y, y_sw, rtol=1e-13, atol=1e-13)


def test_cp_equals_dense_of_reconstruction(orc):
    rng = np.random.default_rng(11)
    N, R = 9, 7
    lam = rng.standard_normal(R)
    Af, Bf, Cf = (rng.standard_normal((N, R)) for _ in range(3))
    u = rng.standard_normal(N)
    T = orc.reconstruct(lam, Af, Bf, Cf)
    y_cp = orc.nonlinear_cp(lam, Af, Bf, Cf, u)
    y_d = orc.nonlinear_dense(T, u)
    assert np.allclose(y_cp, y_d, rtol=1e-12, atol=1e-12 * np.abs(y_d).max())


def test_skew_paired_factors_give_skew_tensor(orc):
    """Sec. 3.3: with A(1) = [A1 A2], A(2) = [B1 B1], A(3) = [A2 -A1] the Kruskal
    tensor is skew in positions 1 and 3; the generator's interleaved pairs are that
    structure up to a column permutation."""
    lam, Af, Bf, Cf = romsynth.skew_cp_factors(7, 4, seed=2, cfg=9)
    T = orc.reconstruct(lam, Af, Bf, Cf)
    assert np.allclose(T, -T.transpose(2, 1, 0), rtol=0, atol=1e-15)
    # and the generator's vectorised dense build agrees with the oracle's loops
    D = romsynth.dense_from_skew_cp(7, 4, eps=0.0, seed=2, cfg=9)
    assert np.allclose(D, T, rtol=0, atol=1e-14)


def _skew_scale(lam, A11, A12, A21, u):
    """sum over pairs of |lam beta| (|u.a| |gamma| + |u.c| |alpha|): the size of the
    terms that cancel in u . y."""
    al, be, ga = A11.T @ u, A21.T @ u, A12.T @ u
    return float(np.sum(np.abs(lam * be) * (np.abs(u @ A11) * np.abs(ga) + np.abs(u @ A12) * np.abs(al))))


def test_cp_skew_contraction(orc):
    """Sec. 3.3, eq. skew_abc_struct: the pair form of the contraction equals the general
    CP contraction of the expanded factors [A11 A12], [A21 A21], [A12 -A11] (and the
    dense contraction of their Kruskal tensor), and u . y vanishes to rounding."""
    rng = np.random.default_rng(21)
    for N, P in [(11, 5), (6, 1), (17, 8)]:
        lam = rng.standard_normal(P)
        A11, A12, A21 = (rng.standard_normal((N, P)) for _ in range(3))
        u = rng.standard_normal(N)
        y = orc.nonlinear_cp_skew(lam, A11, A12, A21, u)
        Af = np.hstack([A11, A12])
        Bf = np.hstack([A21, A21])
        Cf = np.hstack([A12, -A11])
        lr = np.concatenate([lam, lam])
        y_cp = orc.nonlinear_cp(lr, Af, Bf, Cf, u)
        tol = 1e-13 * float(np.abs(lr) @ (np.abs(Bf.T @ u) * np.abs(Cf.T @ u))) * float(np.abs(Af).max())
        assert np.max(np.abs(y - y_cp)) <= tol
        y_d = orc.nonlinear_dense(orc.reconstruct(lr, Af, Bf, Cf), u)
        assert np.max(np.abs(y - y_d)) <= 1e2 * tol
        assert abs(u @ y) <= 1e-14 * _skew_scale(lam, A11, A12, A21, u)
        # a sign error in the third factor breaks both the match and the cancellation
        y_bad = orc.nonlinear_cp(lr, Af, Bf, np.hstack([A12, A11]), u)
        assert np.max(np.abs(y_bad - y)) > 1e3 * tol


def test_cp_skew_interleaved_generator(orc):
    """The generator's interleaved pairs (columns 2p, 2p+1 = (a, b, c), (c, b, -a)) are
    the structure of Sec. 3.3 up to a column permutation."""
    lam, Af, Bf, Cf = romsynth.skew_cp_factors(13, 6, seed=4, cfg=9)
    assert np.array_equal(Bf[:, 0::2], Bf[:, 1::2])
    assert np.array_equal(Af[:, 1::2], Cf[:, 0::2]) and np.array_equal(Cf[:, 1::2], -Af[:, 0::2])
    u = romsynth.initial_u(13, [4], cfg=9)[0]
    y = orc.nonlinear_cp_skew(lam[0::2], Af[:, 0::2], Af[:, 1::2], Bf[:, 0::2], u)
    y_cp = orc.nonlinear_cp(lam, Af, Bf, Cf, u)
    assert np.allclose(y, y_cp, rtol=1e-12, atol=1e-13 * np.abs(y_cp).max())


def test_svd_contraction(orc):
    """Sec. 4.4: the SVD-ROM contraction equals the dense contraction of its own
    reconstruction C[i][j][k] = sum_r U[j][r] sigma_r V[i][k][r]; with the full SVD of
    a tensor's mode-3 matricization (numpy's SVD; the mode-3 index is j here) it equals
    the dense contraction of the tensor itself; with the index roles swapped it does not."""
    rng = np.random.default_rng(31)
    N, R = 9, 4
    U = rng.standard_normal((N, R))
    sig = rng.standard_normal(R)
    V = rng.standard_normal((N, N, R))
    u = rng.standard_normal(N)
    T = np.einsum("jr,r,ikr->ijk", U, sig, V)
    y = orc.nonlinear_svd(U, sig, V, u)
    y_d = orc.nonlinear_dense(T, u)
    scale = np.einsum("ijk,j,k->i", np.abs(T), np.abs(u), np.abs(u))
    assert np.all(np.abs(y - y_d) <= 1e-13 * scale + 1e-300)
    # full SVD of C_(3): rows j, columns (i, k)
    C = romsynth.dense_rough(N, 2, cfg=5)
    M = np.ascontiguousarray(C.transpose(1, 0, 2).reshape(N, N * N))
    Uf, sf, Vh = np.linalg.svd(M, full_matrices=False)
    Vf = np.ascontiguousarray(Vh.T.reshape(N, N, N))          # [i][k][r]
    y_svd = orc.nonlinear_svd(Uf, sf, Vf, u)
    y_c = orc.nonlinear_dense(C, u)
    sc = np.einsum("ijk,j,k->i", np.abs(C), np.abs(u), np.abs(u))
    assert np.all(np.abs(y_svd - y_c) <= 1e-12 * sc.max())
    # the other unfolding (k as the mode-3 index) is a different operator on a
    # non-symmetric tensor: the check has teeth
    M2 = np.ascontiguousarray(C.transpose(2, 0, 1).reshape(N, N * N))
    U2, s2, Vh2 = np.linalg.svd(M2, full_matrices=False)
    T2 = np.einsum("jr,r,ikr->ijk", U2, s2, Vh2.T.reshape(N, N, N))
    assert not np.allclose(T2, C, atol=1e-6)


def test_rows_variant_matches_full(orc):
    C = romsynth.dense_rough(10, 4, cfg=5)
    u = romsynth.initial_u(10, [4], cfg=5)[0]
    y = orc.nonlinear_dense(C, u)
    rows = np.array([0, 3, 9, 3])
    assert np.array_equal(orc.nonlinear_dense_rows(C, u, rows), y[rows])


# ---------------------------------------------------------------- linear algebra, energy

def test_cholesky_against_numpy(orc):
    rng = np.random.default_rng(5)
    G = rng.standard_normal((20, 20))
    H = G @ G.T + 20 * np.eye(20)
    L = orc.cholesky(H)
    assert np.allclose(L, np.linalg.cholesky(H), rtol=1e-13, atol=1e-13)
    b = rng.standard_normal(20)
    assert np.allclose(orc.chol_solve(L, b), np.linalg.solve(H, b), rtol=1e-12, atol=1e-13)
    with pytest.raises(np.linalg.LinAlgError):
        orc.cholesky(-H)


def test_energy_closed_form(orc):
    assert orc.energy(np.array([3.0, 4.0])) == 12.5


# ---------------------------------------------------------------- time stepping

def test_worked_example_two_steps(orc):
    g = _golden("n2_worked_example.txt")
    C = np.zeros((2, 2, 2))
    C[0, 0, 1] = float(g["a"]); C[0, 1, 1] = float(g["b"])
    C[1, 0, 0] = -float(g["a"]); C[1, 1, 0] = -float(g["b"])
    A = np.diag([float(g["A_0"]), float(g["A_1"])])
    u0 = np.array([float(g["u0_0"]), float(g["u0_1"])])
    r = orc.run(2, float(g["nu"]), float(g["dt"]), A, 2, u0=u0, C=C, traj=True)
    assert r["status"] == 0
    T = r["traj"]
    for n, name in [(1, "u1"), (2, "u2")]:
        for i in range(2):
            assert T[n, i] == pytest.approx(float(g[f"{name}_{i}"]), rel=1e-15, abs=0)
    for n in range(3):
        assert r["E"][n] == pytest.approx(float(g[f"E{n}"]), rel=1e-15)
    # history bookkeeping: y_hist = (y^1, y^0)
    assert r["y_hist"][0][0] == pytest.approx(float(g["y1_0"]), rel=1e-15)
    assert r["y_hist"][0][1] == pytest.approx(float(g["y1_1"]), rel=1e-15)
    assert r["y_hist"][1][0] == float(g["y0_0"])


def _closed_form_modes(mu, nu, dt, z0, nsteps):
    """Linear test equation z' = -nu*mu*z under BDFk with the 1,2,3 ramp.

    For n >= 2 each level obeys (11/6 + h) z^{n+1} = 3 z^n - 3/2 z^{n-1} + 1/3 z^{n-2}
    (h = dt*nu*mu), whose solution is sum_q c_q xi_q^n with xi_q the roots of the
    characteristic cubic; z^1 = z^0/(1+h) and z^2 = (2 z^1 - z^0/2)/(3/2+h) start it."""
    h = dt * nu * mu
    z1 = z0 / (1 + h)
    z2 = (2 * z1 - 0.5 * z0) / (1.5 + h)
    xi = np.roots([11.0 / 6.0 + h, -3.0, 1.5, -1.0 / 3.0])
    V = np.array([[x ** n for x in xi] for n in range(3)], dtype=complex)
    c = np.linalg.solve(V, np.array([z0, z1, z2], dtype=complex))
    n = np.arange(nsteps + 1)
    return np.real(sum(c[q] * xi[q] ** n for q in range(3)))


def test_linear_closed_form_diag(orc):
    N, nu, dt, steps = 6, 0.7, 0.01, 60
    A = romsynth.stiffness_diag(N)
    u0 = romsynth.initial_u(N, [1], cfg=8)[0]
    r = orc.run(N, nu, dt, A, steps, u0=u0, C=np.zeros((N, N, N)), traj=True)
    mu = np.diag(A)
    for i in range(N):
        z = _closed_form_modes(mu[i], nu, dt, u0[i], steps)
        assert np.allclose(r["traj"][:, i], z, rtol=1e-11, atol=1e-14)


def test_linear_closed_form_spd(orc):
    N, nu, dt, steps = 8, 0.3, 0.02, 40
    A = romsynth.stiffness_spd(N, seed=1, cfg=8, norm=2.0)
    u0 = romsynth.initial_u(N, [2], cfg=8)[0]
    r = orc.run(N, nu, dt, A, steps, u0=u0, C=np.zeros((N, N, N)), traj=True)
    w, Q = np.linalg.eigh(A)
    z0 = Q.T @ u0
    Z = np.stack([_closed_form_modes(w[q], nu, dt, z0[q], steps) for q in range(N)], axis=1)
    assert np.allclose(r["traj"], Z @ Q.T, rtol=1e-10, atol=1e-13)


def test_inviscid_linear_is_constant(orc):
    """nu = 0, C = 0: the BDF weights sum to zero, so every level equals u^0."""
    N = 5
    u0 = romsynth.initial_u(N, [3], cfg=8)[0]
    r = orc.run(N, 0.0, 0.1, romsynth.stiffness_diag(N), 25, u0=u0, C=np.zeros((N, N, N)),
                traj=True)
    assert np.allclose(r["traj"], u0[None, :], rtol=1e-14, atol=0)


def _logistic_exact(t, u0, a, c):
    # u' = -c u^2 - a u  (Bernoulli):  1/u = (1/u0 + c/a) e^{a t} - c/a
    return 1.0 / ((1.0 / u0 + c / a) * np.exp(a * t) - c / a)


def test_third_order_convergence(orc):
    """N = 1: y = c u^2, A = [a].  Started from exact levels, BDF3/EXT3 must converge
    with order 3; a wrong BDF or EXT weight lowers the order or breaks consistency."""
    a, c, u0, T = 1.0, 1.0, 0.5, 1.0
    errs = []
    for n in (50, 100, 200):
        dt = T / n
        ex = [_logistic_exact(m * dt, u0, a, c) for m in range(3)]
        uh = np.array([[ex[2]], [ex[1]], [ex[0]]])
        yh = np.array([[c * ex[1] ** 2], [c * ex[0] ** 2]])
        r = orc.run(1, 1.0, dt, np.array([[a]]), n - 2, C=np.array([[[c]]]), step0=2,
                    uh=uh, yh=yh)
        errs.append(abs(r["u_hist"][0][0] - _logistic_exact(T, u0, a, c)))
    ratios = [errs[0] / errs[1], errs[1] / errs[2]]
    assert all(7.0 < q < 9.0 for q in ratios), (errs, ratios)


def test_nonfinite_and_not_spd_status(orc):
    N = 3
    C = np.zeros((N, N, N))
    u0 = np.array([1.0, np.nan, 0.0])
    r = orc.run(N, 1.0, 0.1, np.eye(N), 5, u0=u0, C=C)
    assert r["status"] == 4 and r["first_bad"] == 1
    r = orc.run(N, 1.0, 0.1, -100.0 * np.eye(N), 5, u0=np.ones(N), C=C)
    assert r["status"] == 1


def test_config0_energy_decays(orc):
    """Config 0 (N=32): with skew C and SPD A the continuous energy decays as
    dE/dt = -nu u.A u; the discrete run follows it monotonically."""
    p = romsynth.make_config(0)
    r = orc.run(p.N, p.nu, p.dt, p.A, 200, u0=p.u0[0], C=p.C)
    assert r["status"] == 0
    assert np.all(np.diff(r["E"]) < 0)


# ---------------------------------------------------------------- storage rounding

def test_bf16_rounding_special_values(orc):
    x = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -8 + 2.0 ** -20,
                  -(1.0 + 3 * 2.0 ** -8), 3.4e38, np.inf, 0.0])
    expect = np.array([1.0, 1.0, 1.0 + 2.0 ** -6, 1.0 + 2.0 ** -7, -(1.0 + 2.0 ** -6), np.inf,
                       np.inf, 0.0])
    assert np.array_equal(orc.round_bf16(x), expect)
    assert np.isnan(orc.round_bf16(np.array([np.nan]))[0])


def test_bf16_rounding_matches_torch(orc):
    import torch
    x = np.random.default_rng(0).standard_normal(100000) * 10.0 ** np.random.default_rng(1).uniform(-20, 20, 100000)
    ref = torch.from_numpy(x).to(torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(orc.round_bf16(x), ref)
    ref32 = torch.from_numpy(x).to(torch.float32).to(torch.float64).numpy()
    assert np.array_equal(orc.round_f32(x), ref32)


def test_bf16x3_split(orc):
    x = np.random.default_rng(2).standard_normal(10000)
    hi, lo = orc.split_bf16x3(x)
    assert np.array_equal(hi, orc.round_bf16(x))
    x32 = orc.round_f32(x)
    assert np.all(np.abs(x32 - hi - lo) <= 2.0 ** -16 * np.abs(x32))
    assert np.array_equal(orc.round_bf16(lo), lo)


# ---------------------------------------------------------------- full form (zeroth mode, mass)

def test_full_explicit_term_is_augmented_contraction(orc):
    """Eq. nse_d1's bracket C(u)u + (C1 + C2) ubar - c0 equals the contraction of the full
    tensor (Sec. 4.2: indices 0..N in both contracted positions) with ubar = [1, u]: C1 is
    the slice with the zeroth mode advecting, C2 the slice with it advected, and c0 their
    shared corner, counted twice by (C1 + C2) ubar.  Brute force over the full tensor."""
    rng = np.random.default_rng(41)
    N = 7
    T = rng.standard_normal((N, N + 1, N + 1))
    u = rng.standard_normal(N)
    ub = np.concatenate([[1.0], u])
    want = np.array([sum(T[i, j, k] * ub[j] * ub[k] for j in range(N + 1) for k in range(N + 1))
                     for i in range(N)])
    C1, C2, c0 = T[:, 0, :].copy(), T[:, :, 0].copy(), T[:, 0, 0].copy()
    core = np.ascontiguousarray(T[:, 1:, 1:])
    g = orc.explicit_full(u, C=core, C1=C1, C2=C2, c0=c0)
    assert np.max(np.abs(g - want)) <= 1e-13 * np.max(np.abs(want))
    # the CP core gives the same bracket
    R = 5
    lam, Af, Bf, Cf = rng.standard_normal(R), *(rng.standard_normal((N, R)) for _ in range(3))
    core_cp = np.einsum("r,ir,jr,kr->ijk", lam, Af, Bf, Cf)
    T2 = T.copy()
    T2[:, 1:, 1:] = core_cp
    want2 = np.einsum("ijk,j,k->i", T2, ub, ub)
    g2 = orc.explicit_full(u, lam=lam, Af=Af, Bf=Bf, Cf=Cf, C1=C1, C2=C2, c0=c0)
    assert np.max(np.abs(g2 - want2)) <= 1e-12 * np.max(np.abs(want2))


def test_full_mass_matrix_change_of_variables(orc):
    """With M = L L^T and v = L^T u, M du/dt = -g(u) - nu (A u + a0) becomes
    dv/dt = -L^{-1} g(L^{-T} v) - nu (L^{-1} A L^{-T} v + L^{-1} a0): identity mass, every
    operator transformed.  BDFk/EXTk are linear in the levels, so the two discrete
    trajectories agree up to rounding.  Pins M in the Helmholtz matrix and in the history
    term together, and the zeroth-mode terms under the transformation."""
    N, nu, dt, steps = 12, 2e-2, 1e-2, 60
    A = romsynth.stiffness_spd(N, seed=2, cfg=9, norm=1.0)
    M = romsynth.mass_spd(N, seed=3, cfg=9, norm=0.5)
    lam, Af, Bf, Cf = romsynth.skew_cp_factors(N, 4, seed=4, cfg=9)
    C1, C2, c0, a0 = romsynth.zeroth_terms(N, seed=5, cfg=9, scale=0.3)
    u0 = romsynth.initial_u(N, [6], cfg=9)[0]
    r1 = orc.run(N, nu, dt, A, steps, u0=u0, lam=lam, Af=Af, Bf=Bf, Cf=Cf, M=M, C1=C1, C2=C2,
                 c0=c0, a0=a0, traj=True)
    L = np.linalg.cholesky(M)
    Li = np.linalg.inv(L)

    def tr(Z):   # zeroth-mode matrix: column 0 maps like a vector, columns 1..N like L^-1 Z L^-T
        out = np.empty_like(Z)
        out[:, 0] = Li @ Z[:, 0]
        out[:, 1:] = Li @ Z[:, 1:] @ Li.T
        return out
    r2 = orc.run(N, nu, dt, Li @ A @ Li.T, steps, u0=L.T @ u0, lam=lam, Af=Li @ Af, Bf=Li @ Bf,
                 Cf=Li @ Cf, C1=tr(C1), C2=tr(C2), c0=Li @ c0, a0=Li @ a0, traj=True)
    assert r1["status"] == 0 and r2["status"] == 0
    V = r1["traj"] @ L
    assert np.max(np.abs(V - r2["traj"])) <= 1e-10 * np.max(np.abs(r2["traj"]))
    # the identity mass really differs: the untransformed operators give another trajectory
    r3 = orc.run(N, nu, dt, A, steps, u0=u0, lam=lam, Af=Af, Bf=Bf, Cf=Cf, C1=C1, C2=C2, c0=c0,
                 a0=a0, traj=True)
    assert np.max(np.abs(r3["traj"] - r1["traj"])) > 1e-4 * np.max(np.abs(r1["traj"]))


def test_full_fixed_point(orc):
    """Linear full form (zero core tensor): the steady state u* solves
    (L + nu A) u* = -(f + nu a0), L = (C1 + C2)[:, 1:], f = (C1 + C2)[:, 0] - c0.  BDFk and
    EXTk reproduce constants exactly (their weights sum to beta0 and to 1), so started at
    u* every level stays there whatever M is.  u* comes from numpy's solver."""
    N, nu, dt, steps = 10, 1e-2, 1e-2, 200
    A = romsynth.stiffness_spd(N, seed=7, cfg=9, norm=1.0)
    M = romsynth.mass_spd(N, seed=8, cfg=9, norm=0.5)
    C1, C2, c0, a0 = romsynth.zeroth_terms(N, seed=9, cfg=9, scale=0.3)
    L = (C1 + C2)[:, 1:]
    f = (C1 + C2)[:, 0] - c0
    us = np.linalg.solve(L + nu * A, -(f + nu * a0))
    r = orc.run(N, nu, dt, A, steps, u0=us, C=np.zeros((N, N, N)), M=M, C1=C1, C2=C2, c0=c0, a0=a0,
                traj=True)
    assert r["status"] == 0
    assert np.max(np.abs(r["traj"] - us)) <= 1e-11 * np.max(np.abs(us))
    # a sign error in a0 moves the state off u*
    r2 = orc.run(N, nu, dt, A, steps, u0=us, C=np.zeros((N, N, N)), M=M, C1=C1, C2=C2, c0=c0,
                 a0=-a0, traj=True)
    assert np.max(np.abs(r2["traj"][-1] - us)) > 1e-6 * np.max(np.abs(us))


# ---------------------------------------------------------------- CP-ALS (Sec. 2.3)

def _als_problem(N, R, seed):
    rng = np.random.default_rng(seed)
    T = [rng.standard_normal((N, R)) for _ in range(3)]
    X = np.einsum("ir,jr,kr->ijk", *T) + 1e-3 * rng.standard_normal((N, N, N))
    F0 = [rng.standard_normal((N, R)) for _ in range(3)]
    return X, T, F0


def test_als_update_is_least_squares(orc):
    """Each update of eq. cp_als is the least-squares solution of its subproblem: numpy's
    lstsq on the unfolded problem (X_(n) against the Khatri-Rao product of the two fixed
    factors) gives the same factor.  A transposed operand or a wrong unfolding fails."""
    N, R = 7, 3
    X, _, F = _als_problem(N, R, 3)
    A1, A2, A3 = F
    KR = np.einsum("jr,kr->jkr", A2, A3).reshape(N * N, R)          # rows (j, k)
    want1 = np.linalg.lstsq(KR, X.reshape(N, N * N).T, rcond=None)[0].T
    (B1, B2, B3), _ = orc.als.cp_als(X, A1, A2, A3, 1)
    assert np.max(np.abs(B1 - want1)) <= 1e-9 * np.max(np.abs(want1))
    KR2 = np.einsum("ir,kr->ikr", B1, A3).reshape(N * N, R)          # rows (i, k)
    X2 = X.transpose(1, 0, 2).reshape(N, N * N)
    want2 = np.linalg.lstsq(KR2, X2.T, rcond=None)[0].T
    assert np.max(np.abs(B2 - want2)) <= 1e-9 * np.max(np.abs(want2))
    KR3 = np.einsum("ir,jr->ijr", B1, B2).reshape(N * N, R)          # rows (i, j)
    X3 = X.transpose(2, 0, 1).reshape(N, N * N)
    want3 = np.linalg.lstsq(KR3, X3.T, rcond=None)[0].T
    assert np.max(np.abs(B3 - want3)) <= 1e-9 * np.max(np.abs(want3))


def test_als_exact_factors_fixed_point(orc):
    """A tensor of exact CP rank R: its own factors minimise every subproblem, so a sweep
    returns them (up to rounding) with residual ~0."""
    N, R = 8, 3
    rng = np.random.default_rng(4)
    T = [rng.standard_normal((N, R)) for _ in range(3)]
    X = np.einsum("ir,jr,kr->ijk", *T)
    F, res = orc.als.cp_als(X, *T, 2)
    for a, b in zip(F, T):
        assert np.max(np.abs(a - b)) <= 1e-10 * np.max(np.abs(b))
    assert res[-1] < 1e-12


def test_als_residual_never_grows(orc):
    """Every subproblem is minimised exactly, so the fit residual of eq. cp_nls does not
    increase from sweep to sweep; from a random start it falls well below its start."""
    N, R = 9, 4
    X, _, F0 = _als_problem(N, R, 5)
    r0 = orc.als.residual(X, F0)
    _, res = orc.als.cp_als(X, *F0, 40)
    assert all(b <= a * (1 + 1e-12) for a, b in zip(res, res[1:]))
    assert res[-1] < 0.5 * min(r0, 1.0)


def test_run_svd_form_equals_reconstructed_dense(orc):
    """The stepper with the SVD form (Sec. 4.4) as its advection term follows the stepper
    with the dense tensor that form reconstructs, C[i][j][k] = sum_r U[j][r] s_r V[i][k][r]."""
    N, R = 12, 5
    rng = np.random.default_rng(7)
    U = rng.standard_normal((N, R)) / np.sqrt(N)
    sig = 1.0 / (1.0 + np.arange(R))
    V = rng.standard_normal((N, N, R)) / N
    T = np.einsum("jr,r,ikr->ijk", U, sig, V)
    A = romsynth.stiffness_spd(N, 1, cfg=9)
    u0 = romsynth.initial_u(N, [2], cfg=9)[0]
    a = orc.run(N, 1e-2, 1e-2, A, 30, u0=u0, U=U, sigma=sig, V=V, traj=True)
    b = orc.run(N, 1e-2, 1e-2, A, 30, u0=u0, C=T, traj=True)
    assert a["status"] == b["status"] == 0
    assert np.max(np.abs(a["traj"] - b["traj"])) <= 1e-13 * np.max(np.abs(b["traj"]))
    assert np.max(np.abs(a["E"] - b["E"]) / b["E"]) <= 1e-13


def test_threads_give_identical_results(orc):
    """The oracle's row loops on several host threads give the one-thread results to the
    bit (dense, CP, SVD forms; evaluations and runs)."""
    N, pairs = 40, 12
    C = romsynth.dense_from_skew_cp(N, pairs, 1e-6, seed=1, cfg=8)
    lam, Af, Bf, Cf = romsynth.skew_cp_factors(N, pairs, seed=1, cfg=8)
    rng = np.random.default_rng(8)
    U = rng.standard_normal((N, 6))
    sig = np.ones(6)
    V = rng.standard_normal((N, N, 6)) / N
    A = romsynth.stiffness_spd(N, 2, cfg=8)
    u0 = romsynth.initial_u(N, [1], cfg=8)[0]
    kinds = [dict(C=C), dict(lam=lam, Af=Af, Bf=Bf, Cf=Cf), dict(U=U, sigma=sig, V=V)]
    one = [orc.run(N, 1e-3, 1e-3, A, 25, u0=u0, traj=True, **k) for k in kinds]
    ev1 = [orc.nonlinear_dense(C, u0), orc.nonlinear_cp(lam, Af, Bf, Cf, u0), orc.nonlinear_svd(U, sig, V, u0)]
    with orc.threads(4):
        assert orc.get_threads() == 4
        many = [orc.run(N, 1e-3, 1e-3, A, 25, u0=u0, traj=True, **k) for k in kinds]
        ev4 = [orc.nonlinear_dense(C, u0), orc.nonlinear_cp(lam, Af, Bf, Cf, u0), orc.nonlinear_svd(U, sig, V, u0)]
    assert orc.get_threads() == 1
    for a, b in zip(one, many):
        assert np.array_equal(a["traj"], b["traj"]) and np.array_equal(a["E"], b["E"])
    for a, b in zip(ev1, ev4):
        assert np.array_equal(a, b)


# ------------------------------------------------------------------ ALS-skew (Sec. 3.3)

def _skew_problem(N, P, seed, noise):
    rng = np.random.default_rng(seed)
    a, c, b = (rng.standard_normal((N, P)) for _ in range(3))
    from oracle import als
    X = np.einsum("ir,jr,kr->ijk", *als.skew_factors(a, c, b))
    if noise:
        G = rng.standard_normal((N, N, N))
        X = X + noise * 0.5 * (G - G.transpose(2, 1, 0))
    return X, (a, c, b), rng


def test_als_skew_structure_and_fixed_point(orc):
    """Sec. 3.3, eq. skew_abc_struct: the structured factors give a tensor skew in positions
    1 and 3, and exact structured factors are a fixed point of ALS-skew (with a planted
    sign error in the third factor the fixed point is lost)."""
    X, (a, c, b), _ = _skew_problem(11, 3, 1, 0.0)
    assert np.max(np.abs(X + X.transpose(2, 1, 0))) <= 1e-13 * np.max(np.abs(X))
    (A11, A12, B1), res = orc.als.als_skew(X, a, c, b, sweeps=3, subiters=2)
    assert max(res) < 1e-12
    for u, v in ((A11, a), (A12, c), (B1, b)):
        assert np.max(np.abs(u - v)) <= 1e-10 * np.max(np.abs(v))
    Xbad = np.einsum("ir,jr,kr->ijk", np.hstack([a, c]), np.hstack([b, b]), np.hstack([c, a]))
    assert np.max(np.abs(Xbad + Xbad.transpose(2, 1, 0))) > 1e-3 * np.max(np.abs(Xbad))


def test_als_skew_updates_are_least_squares(orc):
    """Each ALS-skew update solves its linear least-squares problem (numpy's lstsq on the
    unfolded system): the tied second factor B1 over the P columns of vec(a_p c_p^T -
    c_p a_p^T), and the subiteration's first factor over the Khatri-Rao columns with the
    third factor held fixed (eq. cp_als_quad).  For a skew tensor the untied ALS update of
    the second factor has equal halves, i.e. equals the tied one."""
    N, P = 9, 3
    X, _, rng = _skew_problem(N, P, 2, 0.3)
    a, c, b = (rng.standard_normal((N, P)) for _ in range(3))
    als = orc.als
    # tied second factor
    (_, _, B1), _ = als.als_skew(X, a, c, b, sweeps=1, subiters=0)
    Z = (np.einsum("ip,kp->ikp", a, c) - np.einsum("ip,kp->ikp", c, a)).reshape(N * N, P)
    X2 = X.transpose(1, 0, 2).reshape(N, N * N)                       # rows j, columns (i, k)
    B1_ls = np.linalg.lstsq(Z, X2.T, rcond=None)[0].T
    assert np.max(np.abs(B1 - B1_ls)) <= 1e-10 * np.max(np.abs(B1_ls))
    F = als.skew_factors(a, c, b)
    A2u = np.linalg.solve(als.normal_matrix(F, 1), als.mttkrp(X, F, 1).T).T
    assert np.max(np.abs(A2u[:, :P] - A2u[:, P:])) <= 1e-10 * np.max(np.abs(A2u))
    assert np.max(np.abs(A2u[:, :P] - B1_ls)) <= 1e-10 * np.max(np.abs(B1_ls))
    # one subiteration without momentum: the least-squares first factor with A3 fixed
    (A11, A12, B1b), _ = als.als_skew(X, a, c, b, sweeps=1, subiters=1, momentum=0.0)
    F = als.skew_factors(a, c, B1b)
    KR = np.einsum("jr,kr->jkr", F[1], F[2]).reshape(N * N, 2 * P)    # rows (j, k)
    A1_ls = np.linalg.lstsq(KR, X.reshape(N, N * N).T, rcond=None)[0].T
    assert np.max(np.abs(np.hstack([A11, A12]) - A1_ls)) <= 1e-9 * np.max(np.abs(A1_ls))
    # with momentum m the new first factor lies between the old one and that solution
    (A11m, A12m, _), _ = als.als_skew(X, a, c, b, sweeps=1, subiters=1, momentum=0.25)
    assert np.allclose(np.hstack([A11m, A12m]), 0.25 * np.hstack([a, c]) + 0.75 * A1_ls, rtol=0, atol=1e-9)


def test_als_skew_fit_residual(orc):
    """From a random start on a noisy rank-6 skew tensor (3 pairs): the residual of eq.
    cp_nls does not grow from sweep to sweep (seeded case) and reaches the noise level; the
    fitted Kruskal tensor stays skew in positions 1 and 3."""
    N, P = 14, 3
    X, _, rng = _skew_problem(N, P, 3, 1e-3)
    init = [rng.standard_normal((N, P)) for _ in range(3)]
    (A11, A12, B1), res = orc.als.als_skew(X, *init, sweeps=60, subiters=3)
    assert all(r1 <= r0 * (1 + 1e-12) for r0, r1 in zip(res, res[1:])), res
    assert res[-1] < 1e-2
    T = np.einsum("ir,jr,kr->ijk", *orc.als.skew_factors(A11, A12, B1))
    assert np.max(np.abs(T + T.transpose(2, 1, 0))) <= 1e-12 * np.max(np.abs(T))
