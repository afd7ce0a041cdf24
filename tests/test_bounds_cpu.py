"""The per-row parity bounds (helpers.bound_dense / bound_cp) have teeth.

The GPU parity tests accept a contraction result when every row lies within a bound
derived from the rounding each term passes through.  These CPU tests plant, in the
oracle's output, the mistakes such a test must catch, and check that the bound of the
format under test rejects them, while the result of correctly rounded operands stays
inside it:
  - a BF16X3 path that lost its low words computes the BF16-rounded contraction: the
    BF16X3 bound must reject it;
  - an FP32 result must pass the FP32 bound and fail the FP64 bound;
  - a BF16 result must pass the BF16 bound, and a y that is zero, 20% off, taken from the
    wrong tensor positions or missing the CP weights must fail it;
  - a 1e-3 relative error must fail the FP32 and BF16X3 bounds.
Workloads: the rough dense tensor and the skew-paired CP factors of the GPU tests, at
sizes those tests use."""
import numpy as np
import pytest

import oracle as orc
import romsynth
from helpers import bound_cp, bound_dense, cond_traj_bar, elem_violations


def _rb(x):
    return orc.round_bf16(x).reshape(np.shape(x))


def _rf(x):
    return orc.round_f32(x).reshape(np.shape(x))


def _frac_bad(y, y_ref, bound):
    return elem_violations(y, y_ref, bound).size / len(y_ref)


@pytest.mark.parametrize("N,kind", [(32, "rough"), (37, "rough"), (40, "skew")])
def test_dense_bounds_have_teeth(N, kind):
    if kind == "rough":
        C = romsynth.dense_rough(N, seed=1, cfg=60)
    else:
        C = romsynth.dense_from_skew_cp(N, N // 2, 1e-6, seed=1, cfg=60)
    u = romsynth.initial_u(N, [3], cfg=60)[0]
    y = orc.nonlinear_dense(C, u)
    y_b = orc.nonlinear_dense(_rb(C), _rb(u))
    y_f = orc.nonlinear_dense(_rf(C), _rf(u))
    # correctly rounded operands stay inside their format's bound
    assert _frac_bad(y_f, y, bound_dense("fp32", C, u)) == 0
    assert _frac_bad(y_b, y, bound_dense("bf16", C, u)) == 0
    # lost BF16X3 low words, FP32 in place of FP64
    assert _frac_bad(y_b, y, bound_dense("bf16x3", C, u)) > 0.25
    assert _frac_bad(y_f, y, bound_dense("fp64", C, u)) > 0.9
    # planted mistakes
    assert _frac_bad(np.zeros(N), y, bound_dense("bf16", C, u)) > 0.5
    assert _frac_bad(1.2 * y, y, bound_dense("bf16", C, u)) > 0.1
    y_pos = orc.nonlinear_dense(np.ascontiguousarray(C.transpose(1, 0, 2)), u)    # output from position 2
    assert _frac_bad(y_pos, y, bound_dense("bf16", C, u)) > 0.5
    assert _frac_bad(y * (1 + 1e-3), y, bound_dense("fp32", C, u)) > 0.5
    assert _frac_bad(y * (1 + 1e-3), y, bound_dense("bf16x3", C, u)) > 0.1
    # BF16 against BF16-rounded operands: only the FP32 accumulation remains
    assert _frac_bad(y_b, y_b, bound_dense("bf16", _rb(C), _rb(u), rounded=True)) == 0
    assert _frac_bad(y, y_b, bound_dense("bf16", _rb(C), _rb(u), rounded=True)) > 0.5


@pytest.mark.parametrize("N,pairs", [(37, 25), (40, 20), (64, 32)])
def test_cp_bounds_have_teeth(N, pairs):
    lam, Af, Bf, Cf = romsynth.skew_cp_factors(N, pairs, seed=2, cfg=61)
    u = romsynth.initial_u(N, [3], cfg=61)[0]
    ops = (lam, Af, Bf, Cf)
    y = orc.nonlinear_cp(*ops, u)
    y_b = orc.nonlinear_cp(*map(_rb, ops), _rb(u))
    y_f = orc.nonlinear_cp(*map(_rf, ops), _rf(u))
    b = {dt: bound_cp(dt, *ops, u) for dt in ("fp64", "fp32", "bf16", "bf16x3")}
    assert _frac_bad(y_f, y, b["fp32"]) == 0
    assert _frac_bad(y_b, y, b["bf16"]) == 0
    assert _frac_bad(y_b, y, b["bf16x3"]) > 0.5
    assert _frac_bad(y_f, y, b["fp64"]) > 0.9
    assert _frac_bad(np.zeros(N), y, b["bf16"]) > 0.5
    assert _frac_bad(1.2 * y, y, b["bf16"]) > 0.05
    assert _frac_bad(orc.nonlinear_cp(np.ones_like(lam), Af, Bf, Cf, u), y, b["bf16"]) > 0.5    # weights dropped
    assert _frac_bad(orc.nonlinear_cp(lam, Af, Bf, Bf, u), y, b["bf16"]) > 0.5                  # t from the wrong factor
    assert _frac_bad(y * (1 + 1e-3), y, b["fp32"]) > 0.5
    assert _frac_bad(y * (1 + 1e-3), y, b["bf16x3"]) > 0.1


def test_cp_bound_from_right_hand_side():
    """Projections formed as ([B|C]^T Hinv) rhs: the bound takes S = |B^T Hinv| |rhs|.  A
    result with the projections rounded to BF16 in the FP32 path must fail it, the FP32
    result of the rounded operator must pass."""
    N, pairs = 40, 20
    lam, Af, Bf, Cf = romsynth.skew_cp_factors(N, pairs, seed=4, cfg=62)
    A = romsynth.stiffness_spd(N, 0, cfg=62)
    u = romsynth.initial_u(N, [1], cfg=62)[0]
    H = (11.0 / 6.0) / 1e-3 * np.eye(N) + 1e-3 * A
    Hinv = np.linalg.inv(H)
    rhs = H @ u
    MB, MC = Bf.T @ Hinv, Cf.T @ Hinv
    S = np.abs(MB) @ np.abs(rhs)
    T = np.abs(MC) @ np.abs(rhs)
    y = orc.nonlinear_cp(lam, Af, Bf, Cf, u)
    bd = bound_cp("fp32", lam, Af, Bf, Cf, u, S=S, T=T)
    # the FP32 path: operator M and rhs rounded to FP32, projections accumulated exactly
    s32 = _rf(MB) @ _rf(rhs)
    t32 = _rf(MC) @ _rf(rhs)
    y32 = _rf(Af) @ (_rf(lam) * s32 * t32)
    assert _frac_bad(y32, y, bd) == 0
    sb = _rb(MB) @ _rb(rhs)
    tb = _rb(MC) @ _rb(rhs)
    yb = Af @ (lam * sb * tb)
    assert _frac_bad(yb, y, bd) > 0.5


def test_ill_conditioned_bar_is_the_problems_own_sensitivity():
    """The FP64 bar for an ill-conditioned Helmholtz matrix (cond ~ 1e4) is neither loose
    nor tight by more than a factor ten: flipping the last bit of the stiffness entries
    (symmetric random signs) moves the oracle's own trajectory by 0.1 to 1 times
    cond_traj_bar at every level."""
    N = 48
    A = romsynth.stiffness_graded(N, 1.0, 2e10, seed=1, cfg=25)
    p = romsynth.make_problem(N, pairs=20, eps=1e-6, nu=1e-3, dt=1e-3, cfg=25, dense=False)
    w = np.linalg.eigvalsh((11.0 / 6.0) / 1e-3 * np.eye(N) + 1e-3 * A)
    cond = w[-1] / w[0]
    assert 1e4 < cond < 2e4
    kw = dict(u0=p.u0[0], lam=p.lam, Af=p.Af, Bf=p.Bf, Cf=p.Cf, traj=True)
    ref = orc.run(N, 1e-3, 1e-3, A, 200, **kw)["traj"]
    R = np.triu(np.random.default_rng(7).choice([-1.0, 1.0], size=(N, N)))
    R = R + np.triu(R, 1).T
    T = orc.run(N, 1e-3, 1e-3, A * (1.0 + 2.0 ** -53 * R), 200, **kw)["traj"]
    for m in (10, 60, 200):
        d = np.linalg.norm(T[m] - ref[m]) / np.linalg.norm(ref[m])
        assert 0.1 * cond_traj_bar(cond, m) < d < cond_traj_bar(cond, m), (m, d)
