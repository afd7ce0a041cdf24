"""Parity of the HIP path (through the C ABI) with the FP64 oracle, single trajectory.

Every case prints what names it before it touches the GPU, so a failing run can be
attributed from its last lines."""
import sys

import numpy as np
import pytest

import oracle as orc
import paper_2311_03694_amd as rg
import romsynth
from helpers import TRAJ_TOL, bf16_bound, cond_traj_bar, check_eval, eval_bound_cp, eval_bound_dense, rel, traj_rel

pytestmark = pytest.mark.gpu

DTS = ["fp64", "fp32", "bf16", "bf16x3"]


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _gpu_nonlinear(torch, rom, u):
    ud = torch.tensor(np.atleast_2d(u), dtype=torch.float64, device="cuda")
    yd = torch.empty_like(ud)
    torch.cuda.synchronize()
    rg.rom_nonlinear(rom.handle, ud.shape[0], ud, yd)
    torch.cuda.synchronize()
    return yd.cpu().numpy().reshape(np.shape(u))


def _rounded_operands(dt, arrays):
    if dt == "bf16":
        return [orc.round_bf16(a).reshape(np.shape(a)) for a in arrays]
    return arrays


# ---------------------------------------------------------------- single evaluations

@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("N", [32, 37, 100, 130])
def test_dense_nonlinear(torch_gpu, dt, N):
    _say(f"dense nonlinear N={N} {dt}")
    C = romsynth.dense_rough(N, seed=N, cfg=11)
    u = romsynth.initial_u(N, [N], cfg=11)[0]
    rom = rg.Rom(N, 1e-3, 1e-3, romsynth.stiffness_diag(N), C=C, dtype=dt)
    y = _gpu_nonlinear(torch_gpu, rom, u)
    Cr, ur = _rounded_operands(dt, [C, u])
    y_ref = orc.nonlinear_dense(Cr, ur)
    check_eval(dt, y, y_ref, eval_bound_dense(dt, C, u))
    if dt == "bf16":
        y_ex = orc.nonlinear_dense(C, u)
        assert np.all(np.abs(y - y_ex) <= bf16_bound(C, u))


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("N,pairs", [(37, 25), (100, 50), (96, 160)])
def test_cp_nonlinear(torch_gpu, dt, N, pairs):
    _say(f"cp nonlinear N={N} R={2 * pairs} {dt}")
    lam, Af, Bf, Cf = romsynth.skew_cp_factors(N, pairs, seed=3, cfg=12)
    u = romsynth.initial_u(N, [5], cfg=12)[0]
    rom = rg.Rom(N, 1e-3, 1e-3, romsynth.stiffness_diag(N), lam=lam, Af=Af, Bf=Bf, Cf=Cf, dtype=dt)
    y = _gpu_nonlinear(torch_gpu, rom, u)
    ops = _rounded_operands(dt, [lam, Af, Bf, Cf, u])
    y_ref = orc.nonlinear_cp(*ops)
    check_eval(dt, y, y_ref, eval_bound_cp(dt, lam, Af, Bf, Cf, u))


def test_unit_tensor_positions(torch_gpu):
    """One non-zero entry C[i][j][k] must land in row i with weight u_j u_k."""
    N = 8
    u = np.arange(1.0, N + 1.0)
    for (i, j, k) in [(0, 1, 2), (7, 3, 5), (2, 6, 0)]:
        _say(f"unit tensor {(i, j, k)}")
        C = np.zeros((N, N, N))
        C[i, j, k] = 1.0
        rom = rg.Rom(N, 1e-3, 1e-3, np.eye(N), C=C, dtype="fp64")
        y = _gpu_nonlinear(torch_gpu, rom, u)
        e = np.zeros(N)
        e[i] = u[j] * u[k]
        assert np.array_equal(y, e)


# ---------------------------------------------------------------- trajectories

def _run_gpu(p, dense, dt, nsteps, chunks=None):
    rom = rg.Rom.from_problem(p, dense=dense, dtype=dt)
    st = rom.state(p.u0[0])
    levels = [p.u0[0].copy()]
    marks = chunks or [nsteps]
    done = 0
    for m in marks:
        st.step(m - done)
        done = m
        levels.append(st.u()[0].copy())
    E, Elog = st.energy()
    return levels, Elog[:, 0], st


def _oracle_levels(p, dense, nsteps, marks, rounded=None):
    kw = dict(C=p.C) if dense else dict(lam=p.lam, Af=p.Af, Bf=p.Bf, Cf=p.Cf)
    if rounded:
        kw = {k: rounded(v) for k, v in kw.items()}
    r = orc.run(p.N, p.nu, p.dt, p.A, nsteps, u0=p.u0[0], traj=True, **kw)
    assert r["status"] == 0
    return [r["traj"][0]] + [r["traj"][m] for m in marks], r["E"]


@pytest.mark.parametrize("dt", ["fp64", "fp32"])
def test_config0_trajectory(torch_gpu, dt):
    """N=32 rough dense tensor, diagonal stiffness, 1000 BDF3/EXT3 steps."""
    _say(f"config0 trajectory {dt}")
    p = romsynth.make_config(0)
    marks = [1, 2, 3, 100, 640, 1000]
    lv, E, _ = _run_gpu(p, True, dt, 1000, marks)
    lref, Eref = _oracle_levels(p, True, 1000, marks)
    assert traj_rel(lv, lref) < TRAJ_TOL[dt]
    assert np.max(np.abs(E - Eref) / Eref) < TRAJ_TOL[dt]


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("dense", [True, False])
def test_skew_cp_trajectory(torch_gpu, dt, dense):
    """N=100 skew-paired tensor (50 pairs, eps 1e-6), 600 steps; dense and CP forms."""
    _say(f"N=100 trajectory dense={dense} {dt}")
    p = romsynth.make_problem(100, pairs=50, eps=1e-6, nu=1e-3, dt=1e-3, nsteps=600, cfg=13,
                              dense=dense, cp=not dense)
    marks = [1, 2, 5, 128, 300, 600]
    lv, E, _ = _run_gpu(p, dense, dt, 600, marks)
    lref, Eref = _oracle_levels(p, dense, 600, marks)
    assert traj_rel(lv, lref) < TRAJ_TOL[dt], traj_rel(lv, lref)
    assert np.max(np.abs(E - Eref) / Eref) < TRAJ_TOL[dt]


@pytest.mark.parametrize("dt", ["fp64", "fp32", "bf16", "bf16x3"])
@pytest.mark.parametrize("dense", [True, False])
def test_spd_stiffness_trajectory(torch_gpu, dt, dense):
    """Dense SPD stiffness A = diag(k^2) + P: FP64 Helmholtz inverses built on the GPU
    (CP: the projections of each new level through [Bf|Cf]^T Hinv_k in every format)."""
    _say(f"spd stiffness dense={dense} {dt}")
    p = romsynth.make_problem(70, pairs=40, eps=1e-7, nu=5e-4, dt=5e-4, A="spd", nsteps=300,
                              cfg=14, dense=dense, cp=not dense)
    marks = [1, 2, 3, 150, 300]
    lv, E, _ = _run_gpu(p, dense, dt, 300, marks)
    lref, Eref = _oracle_levels(p, dense, 300, marks)
    assert traj_rel(lv, lref) < TRAJ_TOL[dt], traj_rel(lv, lref)
    assert np.max(np.abs(E - Eref) / Eref) < TRAJ_TOL[dt]


def test_checkpoint_resume_bitwise(torch_gpu):
    _say("checkpoint/resume")
    p = romsynth.make_problem(48, pairs=30, eps=1e-6, nsteps=0, cfg=15, dense=False)
    rom = rg.Rom.from_problem(p, dense=False, dtype="fp32")
    a = rom.state(p.u0[0])
    a.step(200)
    b = rom.state(p.u0[0])
    b.step(73)
    uh, yh, n = b.get()
    assert n == 73
    c = rom.state(np.zeros(48))
    c.set(uh, yh, n)
    c.step(127)
    ua, ya, na = a.get()
    uc, yc, nc = c.get()
    assert na == nc == 200
    assert np.array_equal(ua, uc) and np.array_equal(ya, yc)
    Ea, _ = a.energy()
    Ec, _ = c.energy()
    assert np.array_equal(Ea, Ec)


@pytest.mark.parametrize("dense,A", [(True, "diag"), (False, "spd")])
def test_restart_from_oracle_history(torch_gpu, dense, A):
    """rom_state_set with an oracle history continues exactly like the oracle (for a CP
    trajectory with a dense stiffness the restart recomputes the projections of the
    restart level, which later steps carry from one Helmholtz kernel to the next)."""
    _say(f"restart from oracle history dense={dense} A={A}")
    p = romsynth.make_problem(40, pairs=20, eps=1e-6, A=A, cfg=16, dense=dense, cp=not dense)
    kw = dict(C=p.C) if dense else dict(lam=p.lam, Af=p.Af, Bf=p.Bf, Cf=p.Cf)
    r1 = orc.run(p.N, p.nu, p.dt, p.A, 30, u0=p.u0[0], **kw)
    rom = rg.Rom.from_problem(p, dense=dense, dtype="fp64")
    s = rom.state(p.u0[0])
    s.set(r1["u_hist"][:, None, :], r1["y_hist"][:, None, :], 30)
    s.step(40)
    r2 = orc.run(p.N, p.nu, p.dt, p.A, 40, step0=30, uh=r1["u_hist"], yh=r1["y_hist"], **kw)
    assert rel(s.u()[0], r2["u_hist"][0]) < 1e-12


def test_nonfinite_reported(torch_gpu):
    _say("non-finite initial state")
    N = 16
    C = romsynth.dense_rough(N, 0, cfg=17)
    rom = rg.Rom(N, 1e-3, 1e-3, romsynth.stiffness_diag(N), C=C, dtype="fp32")
    u0 = np.ones(N)
    u0[3] = np.nan
    s = rom.state(u0)
    with pytest.raises(rg.NonFinite) as ei:
        s.step(5)
    assert ei.value.first_bad == 0
    _say("blow-up")
    # u_i' = -c u_i^2 from u_i(0) < 0 (one tensor entry per mode): the explicit term
    # grows past the FP64 range at a step the oracle and the GPU agree on exactly
    N = 4
    C = np.zeros((N, N, N))
    for i in range(N):
        C[i, i, i] = 1.0 + i
    u0 = -np.array([2.0, 1.5, 1.0, 0.5])
    r = orc.run(N, 0.0, 0.05, np.eye(N), 400, u0=u0, C=C)
    assert r["status"] == 4 and r["first_bad"] > 5
    big = rg.Rom(N, 0.0, 0.05, np.eye(N), C=C, dtype="fp64")
    s2 = big.state(u0)
    with pytest.raises(rg.NonFinite) as ei:
        s2.step(400)
    assert ei.value.first_bad == r["first_bad"], (ei.value.first_bad, r["first_bad"])


def test_explicit_inverse_ill_conditioned(torch_gpu):
    """The dense-stiffness solve applies an explicit inverse built from the Cholesky
    factor.  With cond(beta0/dt I + nu A) near 1e4 (eigenvalues of A log-spaced over ten
    decades) every FP64 level m stays within m * cond * u64 of the oracle's triangular
    solves: the spread any two FP64 solvers show on this problem (a last-bit change of
    the stiffness alone moves the oracle by a fifth of it)."""
    N = 48
    A = romsynth.stiffness_graded(N, 1.0, 2e10, seed=1, cfg=25)
    w = np.linalg.eigvalsh((11.0 / 6.0) / 1e-3 * np.eye(N) + 1e-3 * A)
    cond = w[-1] / w[0]
    assert cond > 1e4
    p = romsynth.make_problem(N, pairs=20, eps=1e-6, nu=1e-3, dt=1e-3, cfg=25, dense=False)
    rom = rg.Rom(N, 1e-3, 1e-3, A, lam=p.lam, Af=p.Af, Bf=p.Bf, Cf=p.Cf, dtype="fp64")
    _say(f"ill-conditioned stiffness, cond(H) = {cond:.2e}")
    st = rom.state(p.u0[0])
    ref = orc.run(N, 1e-3, 1e-3, A, 200, u0=p.u0[0], lam=p.lam, Af=p.Af, Bf=p.Bf, Cf=p.Cf, traj=True)
    assert ref["status"] == 0
    done = 0
    for m in (1, 2, 3, 10, 60, 200):
        st.step(m - done)
        done = m
        err = rel(st.u()[0], ref["traj"][m])
        _say(f"  level {m}: {err:.2e} = {err / cond_traj_bar(cond, m):.3f} of the bar")
        assert err < cond_traj_bar(cond, m), (m, err)


def test_not_spd_rejected(torch_gpu):
    _say("non-SPD Helmholtz")
    N = 12
    A = romsynth.stiffness_spd(N, 0, cfg=18) - 1e6 * np.eye(N)
    with pytest.raises(rg.RomError) as ei:
        rg.Rom(N, 1.0, 1e-3, A, C=np.zeros((N, N, N)), dtype="fp64")
    assert ei.value.status == 1


@pytest.mark.parametrize("dense,A,B", [(False, "diag", 1), (True, "spd", 1), (True, "diag", 1), (False, "spd", 1),
                                       (False, "spd", 3)])
def test_step_splits_agree(torch_gpu, dense, A, B):
    """The step counter has two slots and captured chunks are cached per parity of
    their first level: 301 steps at once equal 1 + 130 + 3 + 167 steps (chunks that
    start at odd and at even levels, eager steps between), energies included."""
    _say(f"step splits dense={dense} A={A} B={B}")
    p = romsynth.make_problem(40, pairs=20, eps=1e-6, nu=1e-3, dt=1e-3, A=A, batch=B, cfg=23,
                              dense=dense, cp=not dense)
    rom = rg.Rom.from_problem(p, dense=dense, dtype="fp64", max_batch=B)
    a = rom.state(p.u0)
    a.step(301)
    b = rom.state(p.u0)
    for k in (1, 130, 3, 167):
        b.step(k)
    ua, _, na = a.get()
    ub, _, nb = b.get()
    assert na == nb == 301
    assert np.array_equal(ua, ub)
    Ea, La = a.energy()
    Eb, Lb = b.energy()
    assert np.array_equal(La, Lb)
    assert np.all(np.isfinite(La))


def test_graph_and_eager_agree(torch_gpu):
    """A run that crosses graph-replay chunks equals a run of single eager steps."""
    _say("graph vs eager")
    p = romsynth.make_problem(64, pairs=32, eps=1e-6, cfg=19, dense=True, cp=False)
    rom = rg.Rom.from_problem(p, dense=True, dtype="fp32")
    a = rom.state(p.u0[0])
    a.step(300)
    b = rom.state(p.u0[0])
    for _ in range(300):
        b.step(1)
    assert np.array_equal(a.get()[0], b.get()[0])


def test_prepare_runs_no_step(torch_gpu):
    """rom_step_prepare captures graphs without stepping; a prepared call of 20 steps and
    calls of other lengths (one graph, a 64-step graph plus the rest) give the same
    trajectory as an unprepared one, to the bit."""
    _say("prepare")
    p = romsynth.make_problem(40, pairs=20, eps=1e-6, A="spd", cfg=24, dense=False)
    rom = rg.Rom.from_problem(p, dense=False, dtype="fp32")
    a = rom.state(p.u0[0])
    a.step(3)
    u3 = a.get()
    a.prepare(20)
    a.prepare(150)
    assert a.step_count == 3
    ub = a.get()
    assert all(np.array_equal(x, y) for x, y in zip(u3[:2], ub[:2]))
    a.step(20)
    a.step(150)
    b = rom.state(p.u0[0])
    for k in (3, 20, 64, 86):
        b.step(k)
    assert np.array_equal(a.get()[0], b.get()[0])
    assert np.array_equal(a.energy()[1], b.energy()[1])
