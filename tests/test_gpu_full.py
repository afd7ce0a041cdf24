"""The full form of the reduced system (Sec. 2.2, eqs. nse_ode, nse_d1 and
zeroth_contribution) on the GPU: a mass matrix M (identity, diagonal or dense SPD) and the
zeroth-mode terms C1, C2, c0, a0, with the dense tensor and the CP factors, one
trajectory and batches, against the oracle's full-form integration; with no terms and
M = I, the full-form context steps to the bit like the plain one; grouped launches."""
import sys

import numpy as np
import pytest

import oracle as orc
import paper_2311_03694_amd as rg
import romsynth
from helpers import TRAJ_TOL, rel, traj_rel

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _terms(N, mass, cfg):
    C1, C2, c0, a0 = romsynth.zeroth_terms(N, seed=1, cfg=cfg, scale=0.1)
    M = None
    if mass == "diag":
        M = romsynth.mass_spd(N, seed=2, cfg=cfg, norm=0.3, diag=True)
    elif mass == "dense":
        M = romsynth.mass_spd(N, seed=2, cfg=cfg, norm=0.3)
    return dict(M=M, C1=C1, C2=C2, c0=c0, a0=a0)


def _ref(p, form, full, steps, u0):
    core = dict(C=p.C) if form == "dense" else dict(lam=p.lam, Af=p.Af, Bf=p.Bf, Cf=p.Cf)
    return orc.run(p.N, p.nu, p.dt, p.A, steps, u0=u0, **core, **full)


def _rom(p, form, full, dt, B):
    core = dict(C=p.C) if form == "dense" else dict(lam=p.lam, Af=p.Af, Bf=p.Bf, Cf=p.Cf)
    return rg.Rom(p.N, p.nu, p.dt, p.A, **core, full=full, dtype=dt, max_batch=B)


@pytest.mark.parametrize("mass", ["identity", "diag", "dense"])
@pytest.mark.parametrize("A", ["diag", "spd"])
@pytest.mark.parametrize("dt", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("form", ["dense", "cp"])
def test_full_trajectory(torch_gpu, form, dt, A, mass):
    """One trajectory, 150 steps (N = 44: a ragged tail), coefficients and every energy
    against the oracle (the terms themselves are FP64 in every format)."""
    N, steps = 44, 150
    _say(f"full form {form} {dt} A={A} M={mass}")
    p = romsynth.make_problem(N, pairs=22, eps=1e-6, A=A, cfg=81, dense=form == "dense", cp=form == "cp")
    full = _terms(N, mass, 81)
    rom = _rom(p, form, full, dt, 1)
    s = rom.state(p.u0[0])
    s.step(steps)
    uh, _, n = s.get()
    _, Elog = s.energy()
    ref = _ref(p, form, full, steps, p.u0[0])
    assert ref["status"] == 0 and n == steps
    assert rel(uh[0][0], ref["u_hist"][0]) < TRAJ_TOL[dt]
    assert float(np.max(np.abs(Elog.reshape(-1) - ref["E"]) / ref["E"])) < TRAJ_TOL[dt]
    # the terms matter: the plain system drifts away from the full one
    plain = orc.run(p.N, p.nu, p.dt, p.A, steps, u0=p.u0[0],
                    **(dict(C=p.C) if form == "dense" else dict(lam=p.lam, Af=p.Af, Bf=p.Bf, Cf=p.Cf)))
    assert rel(plain["u_hist"][0], ref["u_hist"][0]) > 100 * TRAJ_TOL[dt]
    s.close()
    rom.close()


@pytest.mark.parametrize("A,mass", [("spd", "dense"), ("diag", "diag")])
@pytest.mark.parametrize("dt", ["fp64", "fp32"])
@pytest.mark.parametrize("form", ["dense", "cp"])
def test_full_batched(torch_gpu, form, dt, A, mass):
    """Five trajectories through the batched kernels, with a dense mass matrix and an SPD
    stiffness (Helmholtz product) or both diagonal (the update in the contraction's
    epilogue); each against its own oracle run."""
    N, B, steps = 40, 5, 120
    _say(f"full form batched {form} {dt} B={B} A={A} M={mass}")
    p = romsynth.make_problem(N, pairs=20, eps=1e-6, A=A, batch=B, cfg=82, dense=form == "dense",
                              cp=form == "cp")
    full = _terms(N, mass, 82)
    rom = _rom(p, form, full, dt, B)
    s = rom.state(p.u0)
    s.step(steps)
    uh, _, n = s.get()
    _, Elog = s.energy()
    assert n == steps
    for b in range(B):
        ref = _ref(p, form, full, steps, p.u0[b])
        assert ref["status"] == 0
        assert rel(uh[0][b], ref["u_hist"][0]) < TRAJ_TOL[dt], b
        assert float(np.max(np.abs(Elog[:, b] - ref["E"]) / ref["E"])) < TRAJ_TOL[dt], b
    s.close()
    rom.close()


@pytest.mark.parametrize("A", ["diag", "spd"])
@pytest.mark.parametrize("form", ["dense", "cp"])
def test_full_without_terms_is_plain(torch_gpu, form, A):
    """No zeroth-mode terms and M = I given explicitly: the full-form context takes one more
    kernel per step whose terms are zero, and its trajectory equals the plain context's
    to the bit."""
    N, steps = 36, 100
    _say(f"full form without terms {form} A={A}")
    p = romsynth.make_problem(N, pairs=18, eps=1e-6, A=A, cfg=83, dense=form == "dense", cp=form == "cp")
    r_full = _rom(p, form, dict(M=np.eye(N)), "fp32", 1)
    r_plain = _rom(p, form, None, "fp32", 1)
    sf, sp = r_full.state(p.u0[0]), r_plain.state(p.u0[0])
    sf.step(steps)
    sp.step(steps)
    assert np.array_equal(sf.get()[0], sp.get()[0])
    assert np.array_equal(sf.energy()[1], sp.energy()[1])
    for x in (sf, sp, r_full, r_plain):
        x.close()


def test_full_in_grouped_launches(torch_gpu):
    """rom_step_multi with a full-form state beside a plain CP state equals each run alone."""
    _say("full + cp grouped")
    N = 40
    p = romsynth.make_problem(N, pairs=20, eps=1e-6, A="spd", cfg=84, dense=False, cp=True)
    rf = _rom(p, "cp", _terms(N, "dense", 84), "fp32", 1)
    rc = _rom(p, "cp", None, "fp32", 1)
    u0 = p.u0[0]
    mf, mc = rf.state(u0), rc.state(u0)
    rg.rom_step_multi([rf.handle, rc.handle], [mf.handle, mc.handle], 90)
    a_f, a_c = rf.state(u0), rc.state(u0)
    a_f.step(90)
    a_c.step(90)
    assert np.array_equal(mf.get()[0], a_f.get()[0])
    assert np.array_equal(mc.get()[0], a_c.get()[0])
    for x in (mf, mc, a_f, a_c):
        x.close()
    rf.close()
    rc.close()


@pytest.mark.slow
def test_full_headline_size(torch_gpu):
    """The benchmark's full-form workload (N = 1000, CP rank 2000 FP32, SPD stiffness, dense
    SPD mass matrix, zeroth-mode terms; tile table applied as the benchmark does): 30 steps
    and every energy against the oracle."""
    from paper_2311_03694_amd import tune
    _say("full form N=1000 CP rank 2000 fp32, 30 steps")
    p = romsynth.make_config(3, R=2000, batch=1, dense=False)
    N, steps = p.N, 30
    C1, C2, c0, a0 = romsynth.zeroth_terms(N, seed=1, cfg=3, scale=0.1)
    full = dict(M=romsynth.mass_spd(N, seed=2, cfg=3, norm=0.1), C1=C1, C2=C2, c0=c0, a0=a0)
    rom = _rom(p, "cp", full, "fp32", 1)
    tune.apply(rom, 1, dense=False, R=2000)
    s = rom.state(p.u0[0])
    s.step(steps)
    uh, _, n = s.get()
    _, Elog = s.energy()
    ref = _ref(p, "cp", full, steps, p.u0[0])
    assert ref["status"] == 0 and n == steps
    assert rel(uh[0][0], ref["u_hist"][0]) < TRAJ_TOL["fp32"]
    assert float(np.max(np.abs(Elog.reshape(-1) - ref["E"]) / ref["E"])) < TRAJ_TOL["fp32"]
    s.close()
    rom.close()


@pytest.mark.parametrize("A", ["diag", "spd"])
@pytest.mark.parametrize("form", ["dense", "cp"])
def test_full_restart(torch_gpu, form, A):
    """A checkpoint of a full-form state (rom_state_get: the u levels and the y levels,
    which hold C(u)u alone) restored into a new state continues like the uninterrupted
    run: each step recomputes the zeroth-mode and mass terms from the u levels.  Both
    against the oracle's uninterrupted full-form run."""
    N, n1, n2 = 40, 30, 40
    _say(f"full form restart {form} A={A}")
    p = romsynth.make_problem(N, pairs=20, eps=1e-6, A=A, cfg=85, dense=form == "dense", cp=form == "cp")
    full = _terms(N, "dense", 85)
    rom = _rom(p, form, full, "fp64", 1)
    s1 = rom.state(p.u0[0])
    s1.step(n1)
    uh, yh, n = s1.get()
    assert n == n1
    s2 = rom.state(p.u0[0])
    s2.set(uh, yh, n1)
    s2.step(n2)
    s1.step(n2)
    ref = _ref(p, form, full, n1 + n2, p.u0[0])
    assert ref["status"] == 0
    assert rel(s2.get()[0][0][0], ref["u_hist"][0]) < TRAJ_TOL["fp64"]
    assert rel(s2.get()[0][0][0], s1.get()[0][0][0]) < 1e-13
    for x in (s1, s2, rom):
        x.close()


@pytest.mark.parametrize("dt", ["fp64", "fp32"])
def test_full_form_ragged_large_n(torch_gpu, dt):
    """N = 1100 (padded to 1104 > 1024): the full-form terms kernel stages the history in
    more than one pass and walks each row of G in more than one chunk.  CP rank 120, SPD
    stiffness, dense SPD mass matrix, zeroth-mode terms; every level of 25 steps against
    the oracle."""
    import romsynth as syn
    N = 1100
    _say(f"full form N={N} {dt}")
    p = syn.make_problem(N, pairs=60, eps=1e-7, nu=5e-4, dt=5e-4, A="spd", cfg=31, dense=False)
    C1, C2, c0, a0 = syn.zeroth_terms(N, seed=2, cfg=31, scale=0.1)
    full = dict(M=syn.mass_spd(N, seed=3, cfg=31, norm=0.1), C1=C1, C2=C2, c0=c0, a0=a0)
    rom = rg.Rom(N, p.nu, p.dt, p.A, lam=p.lam, Af=p.Af, Bf=p.Bf, Cf=p.Cf, full=full, dtype=dt)
    st = rom.state(p.u0[0])
    lv = [p.u0[0].copy()]
    for _ in range(25):
        st.step(1)
        lv.append(st.u()[0].copy())
    ref = orc.run(N, p.nu, p.dt, p.A, 25, u0=p.u0[0], lam=p.lam, Af=p.Af, Bf=p.Bf, Cf=p.Cf, traj=True, **full)
    assert ref["status"] == 0
    err = traj_rel(lv, ref["traj"])
    _say(f"  max level error {err:.2e}")
    assert err < TRAJ_TOL[dt], err
    E = st.energy()[1][:, 0]
    assert np.max(np.abs(E - ref["E"]) / ref["E"]) < 2 * TRAJ_TOL[dt]
