"""The seeded synthetic inputs (romsynth) against the recipe they state: shapes of the named
workloads, determinism of the seeded streams, independence of the streams, SPD stiffness
and mass matrices with the stated perturbation norm, the skew column pairs and their skew
Kruskal tensor, and the zeroth-mode terms' shared column.  The generators hold none of the
method's arithmetic; these checks keep the inputs what the tests and the bench say they
are."""
import numpy as np
import pytest

import romsynth as rs


def test_named_workload_shapes():
    p0 = rs.make_config(0)
    assert p0.N == 32 and p0.C.shape == (32, 32, 32) and p0.u0.shape == (1, 32)
    assert np.allclose(p0.C, -p0.C.transpose(2, 1, 0))          # skew in positions 1 and 3
    p3 = rs.make_config(3, dense=False, batch=4)
    assert p3.N == 1000 and p3.Af.shape == (1000, 2000) and p3.lam.shape == (2000,)
    assert p3.u0.shape == (4, 1000) and (p3.nu, p3.dt) == (5e-4, 5e-4)
    p2 = rs.make_config(2, dense=False, batch=3)
    assert p2.Af.shape == (400, 400)                             # truncated to R = 400
    # config 2 reuses config 1's tensor streams and draws its own initial states
    p1 = rs.make_config(1, dense=False, batch=3)
    assert np.array_equal(p2.Af, p1.Af[:, :400])
    assert not np.array_equal(p2.u0, p1.u0)


def test_streams_are_deterministic_and_independent():
    a1 = rs.skew_cp_factors(30, 6, seed=2, cfg=5)
    a2 = rs.skew_cp_factors(30, 6, seed=2, cfg=5)
    for x, y in zip(a1, a2):
        assert np.array_equal(x, y)
    b = rs.skew_cp_factors(30, 6, seed=3, cfg=5)
    assert not np.array_equal(a1[1], b[1])
    u = rs.initial_u(30, [0, 1, 2], cfg=5)
    assert u.shape == (3, 30) and not np.array_equal(u[0], u[1])
    # each trajectory's row depends on its own seed only
    assert np.array_equal(rs.initial_u(30, [1], cfg=5)[0], u[1])
    # spectrum law u_k ~ k^(-5/6)
    k = np.arange(1, 31, dtype=np.float64)
    z = u / k ** (-5.0 / 6.0)
    assert np.all(np.isfinite(z)) and 0.3 < np.std(z) < 3.0


def test_skew_pairs_and_kruskal_tensor():
    N, P = 9, 4
    lam, Af, Bf, Cf = rs.skew_cp_factors(N, P, seed=1, cfg=7)
    assert np.array_equal(lam[0::2], lam[1::2]) and np.allclose(lam[0::2], 1.0 / np.arange(1, P + 1))
    assert np.array_equal(Bf[:, 0::2], Bf[:, 1::2])
    assert np.array_equal(Af[:, 1::2], Cf[:, 0::2]) and np.array_equal(Cf[:, 1::2], -Af[:, 0::2])
    assert np.allclose(np.linalg.norm(Af[:, 0::2], axis=0), 1.0)
    T = np.einsum("r,ir,jr,kr->ijk", lam, Af, Bf, Cf)
    assert np.allclose(T, -T.transpose(2, 1, 0), atol=1e-14)
    # without noise the dense tensor is S - S^(13), S the first columns' Kruskal tensor,
    # which is the Kruskal tensor of all 2P columns
    D = rs.dense_from_skew_cp(N, P, 0.0, seed=1, cfg=7)
    assert np.allclose(D, T, atol=1e-14)
    # truncation keeps whole leading pairs
    t = rs.truncate_cp(lam, Af, Bf, Cf, 4)
    assert t[1].shape == (N, 4) and np.array_equal(t[1], Af[:, :4])


@pytest.mark.parametrize("N", [17, 64])
def test_stiffness_and_mass_are_spd_with_the_stated_norm(N):
    A = rs.stiffness_spd(N, seed=0, cfg=3)
    P = A - rs.stiffness_diag(N)
    assert np.allclose(A, A.T)
    assert np.min(np.linalg.eigvalsh(P)) > -1e-12                 # P = 0.1 M / |M|, M = G G^T
    assert abs(np.linalg.norm(P, 2) - 0.1) < 1e-12
    M = rs.mass_spd(N, seed=2, cfg=3)
    assert np.allclose(M, M.T) and abs(np.linalg.norm(M - np.eye(N), 2) - 0.1) < 1e-12
    assert np.min(np.linalg.eigvalsh(M)) >= 1.0 - 1e-12
    Md = rs.mass_spd(N, seed=2, cfg=3, diag=True)
    assert np.count_nonzero(Md - np.diag(np.diag(Md))) == 0 and np.all(np.diag(Md) >= 1.0)
    G = rs.stiffness_graded(N, 1.0, 1e4, seed=0, cfg=3)
    w = np.linalg.eigvalsh(G)
    assert np.allclose([w[0], w[-1]], [1.0, 1e4], rtol=1e-9)


def test_zeroth_terms_share_the_self_advection_column():
    C1, C2, c0, a0 = rs.zeroth_terms(12, seed=1, cfg=3, scale=0.1)
    assert C1.shape == (12, 13) and C2.shape == (12, 13) and c0.shape == (12,) and a0.shape == (12,)
    assert np.array_equal(C1[:, 0], c0) and np.array_equal(C2[:, 0], c0)
    assert not np.array_equal(C1[:, 1:], C2[:, 1:])


def test_integer_inputs_are_exact_small_integers():
    C = rs.integer_dense(6, vmax=1)
    assert np.array_equal(C, np.round(C)) and np.max(np.abs(C)) <= 2
    assert np.array_equal(C, -C.transpose(2, 1, 0))
    lam, Af, Bf, Cf = rs.integer_cp_factors(6, 4, vmax=1)
    for x in (lam, Af, Bf, Cf):
        assert np.array_equal(x, np.round(x))
    assert np.array_equal(Cf[:, 1::2], -Af[:, 0::2])
    u = rs.integer_u(6, [0, 1], vmax=2)
    assert np.array_equal(u, np.round(u)) and np.max(np.abs(u)) <= 2
