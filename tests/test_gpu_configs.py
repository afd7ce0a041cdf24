"""Parity over long horizons on the stated workloads, every level against the oracle.

* N = 400 with 400 skew pairs and 1e-6 noise (the shape of Sec. 4.1.3's 3D lid-driven
  cavity ROM): the dense G-ROM and the CP-ROM truncated to R = 100, 200, 400, 800, FP64
  and FP32, 2000 steps, u and E at every level.
* N = 400 with 256 trajectories: dense BF16, BF16X3 and FP32 and CP R = 400 in FP32 over
  5000 graph-replayed steps; sampled trajectories, E at every level and u at marks.
* N = 1000 with SPD stiffness: CP R = 500 and 1000 one trajectory in FP64 and BF16
  (1000 steps, every level), R = 2000 FP32 over 10,000 steps (E every level, u every
  100th), and batches of 16 (CP R = 2000, dense) on sampled trajectories.

Each GPU result is compared with the oracle of the same operator (dense with dense, CP
rank R with the same factors): relative error of u per level below the format's bar (FP64
1e-12, FP32 and BF16X3 1e-5, BF16 1e-3), of the energy below twice that (the relative
error of |u|^2 / 2 is at most twice that of u).  The oracle's row loops run on the host's
cores (results identical to one thread)."""
import os
import sys

import numpy as np
import pytest

import oracle as orc
import paper_2311_03694_amd as rg
import romsynth
from helpers import ENERGY_TOL, TRAJ_TOL, traj_rel
from paper_2311_03694_amd import tune

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

THREADS = max(1, min(16, os.cpu_count() or 1))


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _ops(p, dense, R=None):
    if dense:
        return dict(C=p.C)
    lam, Af, Bf, Cf = (p.lam, p.Af, p.Bf, p.Cf) if R is None else romsynth.truncate_cp(p.lam, p.Af, p.Bf, p.Cf, R)
    return dict(lam=lam, Af=Af, Bf=Bf, Cf=Cf)


def _oracle(p, ops, nsteps, u0, traj=True):
    with orc.threads(THREADS):
        r = orc.run(p.N, p.nu, p.dt, p.A, nsteps, u0=u0, traj=traj, **ops)
    assert r["status"] == 0
    return r


def _gpu_every_level(torch, rom, u0, nsteps):
    """u at every level 0..nsteps of a one-trajectory state (one step per call, the
    level copied on the context's stream) and the energy log."""
    N = rom.N
    st = rom.state(u0)
    st.prepare(1)
    U = torch.empty((nsteps + 1, N), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    rg.rom_state_u(rom.handle, st.handle, U[0])
    for n in range(nsteps):
        st.step_async(1)
        rg.rom_state_u(rom.handle, st.handle, U[n + 1])
    st.sync()
    torch.cuda.synchronize()
    E = st.energy()[1][:, 0]
    st.close()
    return U.cpu().numpy(), E


def _check_traj(dt, U, E, ref, what):
    err_u = traj_rel(U, ref["traj"])
    err_e = float(np.max(np.abs(E - ref["E"]) / ref["E"]))
    _say(f"  {what}: max level error u {err_u:.2e}, E {err_e:.2e} ({len(E)} levels)")
    assert err_u < TRAJ_TOL[dt], (what, err_u)
    assert err_e < ENERGY_TOL[dt], (what, err_e)


# ------------------------------------------------------------------ N = 400, one trajectory

@pytest.fixture(scope="module")
def cfg1(torch_gpu):
    _say("generating the N=400 workload (dense tensor, 400 skew pairs)")
    return romsynth.make_config(1)


@pytest.fixture(scope="module")
def cfg1_dense_ref(cfg1):
    _say("oracle: N=400 dense, 2000 steps")
    return _oracle(cfg1, _ops(cfg1, True), 2000, cfg1.u0[0])


@pytest.mark.timeout(400)
@pytest.mark.parametrize("dt", ["fp64", "fp32"])
def test_config1_dense_every_level(torch_gpu, cfg1, cfg1_dense_ref, dt):
    p = cfg1
    _say(f"N=400 dense {dt}, 2000 steps")
    rom = rg.Rom.from_problem(p, dense=True, dtype=dt)
    U, E = _gpu_every_level(torch_gpu, rom, p.u0[0], 2000)
    _check_traj(dt, U, E, cfg1_dense_ref, f"dense {dt}")
    rom.close()


@pytest.mark.timeout(200)
@pytest.mark.parametrize("dt", ["fp64", "fp32"])
@pytest.mark.parametrize("R", [100, 200, 400, 800])
def test_config1_cp_every_level(torch_gpu, cfg1, R, dt):
    p = cfg1
    _say(f"N=400 CP R={R} {dt}, 2000 steps")
    ops = _ops(p, False, R)
    ref = _oracle(p, ops, 2000, p.u0[0])
    rom = rg.Rom(p.N, p.nu, p.dt, p.A, **ops, dtype=dt)
    U, E = _gpu_every_level(torch_gpu, rom, p.u0[0], 2000)
    _check_traj(dt, U, E, ref, f"CP R={R} {dt}")
    rom.close()


def test_config1_model_error_decreases(cfg1, cfg1_dense_ref):
    """The CP-ROM's distance from the G-ROM (Sec. 4.1, errors relative to the G-ROM),
    oracle against oracle: truncating fewer skew pairs brings the trajectory closer."""
    p = cfg1
    errs = []
    for R in (100, 200, 400, 800):
        ref = _oracle(p, _ops(p, False, R), 2000, p.u0[0])
        errs.append(traj_rel(ref["traj"], cfg1_dense_ref["traj"]))
    _say(f"CP-vs-dense model error over 2000 steps, R = 100..800: {errs}")
    assert all(a > b for a, b in zip(errs, errs[1:])), errs


# ------------------------------------------------------------------ N = 400, 256 trajectories

MARKS = [1, 2, 3, 64, 1000, 2500, 5000]


@pytest.fixture(scope="module")
def cfg2(torch_gpu):
    _say("generating the N=400 workload with 256 trajectories")
    return romsynth.make_config(2, R=400)


@pytest.fixture(scope="module")
def cfg2_dense_ref(cfg2):
    b = 137
    _say(f"oracle: N=400 dense, trajectory {b}, 5000 steps")
    return b, _oracle(cfg2, _ops(cfg2, True), 5000, cfg2.u0[b])


def _gpu_marks(rom, u0, marks):
    st = rom.state(u0)
    U = {}
    done = 0
    for m in marks:
        st.step(m - done)
        done = m
        U[m] = st.get()[0][0].copy()
    E = st.energy()[1]
    st.close()
    return U, E


@pytest.mark.timeout(400)
@pytest.mark.parametrize("dt", ["bf16", "bf16x3", "fp32"])
def test_config2_dense_5000_steps(torch_gpu, cfg2, cfg2_dense_ref, dt):
    p = cfg2
    b, ref = cfg2_dense_ref
    B = p.u0.shape[0]
    _say(f"N=400 B={B} dense {dt}, 5000 steps")
    rom = rg.Rom.from_problem(p, dense=True, dtype=dt, max_batch=B)
    tune.apply(rom, B, dense=True)
    U, E = _gpu_marks(rom, p.u0, MARKS)
    _check_traj(dt, np.stack([p.u0[b]] + [U[m][b] for m in MARKS]), E[:, b],
                dict(traj=np.stack([ref["traj"][0]] + [ref["traj"][m] for m in MARKS]), E=ref["E"]),
                f"trajectory {b}")
    assert np.all(np.isfinite(E))
    rom.close()


@pytest.mark.timeout(300)
def test_config2_cp_5000_steps(torch_gpu, cfg2):
    p = cfg2
    B = p.u0.shape[0]
    _say(f"N=400 B={B} CP R=400 fp32, 5000 steps")
    rom = rg.Rom.from_problem(p, dense=False, dtype="fp32", max_batch=B)
    tune.apply(rom, B, dense=False, R=400)
    U, E = _gpu_marks(rom, p.u0, MARKS)
    for b in (0, 15, 16, 200, 255):
        ref = _oracle(p, _ops(p, False), 5000, p.u0[b])
        _check_traj("fp32", np.stack([p.u0[b]] + [U[m][b] for m in MARKS]), E[:, b],
                    dict(traj=np.stack([ref["traj"][0]] + [ref["traj"][m] for m in MARKS]), E=ref["E"]),
                    f"trajectory {b}")
    rom.close()


# ------------------------------------------------------------------ N = 1000

@pytest.fixture(scope="module")
def cfg3(torch_gpu):
    _say("generating the N=1000 CP workload (rank 2000)")
    return romsynth.make_config(3, dense=False)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("R", [500, 1000])
def test_config3_cp_fp64_bf16_every_level(torch_gpu, cfg3, R):
    p = cfg3
    ops = _ops(p, False, R)
    _say(f"oracle: N=1000 CP R={R}, 1000 steps")
    ref = _oracle(p, ops, 1000, p.u0[0])
    for dt in ("fp64", "bf16"):
        _say(f"N=1000 CP R={R} {dt}, 1000 steps")
        rom = rg.Rom(p.N, p.nu, p.dt, p.A, **ops, dtype=dt)
        U, E = _gpu_every_level(torch_gpu, rom, p.u0[0], 1000)
        _check_traj(dt, U, E, ref, f"CP R={R} {dt}")
        rom.close()


@pytest.mark.timeout(400)
def test_config3_cp_10000_steps(torch_gpu, cfg3):
    p = cfg3
    _say("oracle: N=1000 CP R=2000, 10000 steps")
    ref = _oracle(p, _ops(p, False), 10000, p.u0[0])
    _say("N=1000 CP R=2000 fp32, 10000 steps")
    rom = rg.Rom.from_problem(p, dense=False, dtype="fp32")
    tune.apply(rom, 1, dense=False, R=2000)
    marks = list(range(100, 10001, 100))
    U, E = _gpu_marks(rom, p.u0[0], marks)
    _check_traj("fp32", np.stack([p.u0[0]] + [U[m][0] for m in marks]), E[:, 0],
                dict(traj=np.stack([ref["traj"][0]] + [ref["traj"][m] for m in marks]), E=ref["E"]), "10000 steps")
    rom.close()


@pytest.mark.timeout(300)
@pytest.mark.parametrize("dt", ["fp32", "bf16"])
def test_config3_cp_batch16(torch_gpu, cfg3, dt):
    p = cfg3
    B = 16
    U0 = romsynth.initial_u(p.N, range(B), cfg=3)
    _say(f"N=1000 CP R=2000 B={B} {dt}, 300 steps")
    rom = rg.Rom.from_problem(p, dense=False, dtype=dt, max_batch=B)
    tune.apply(rom, B, dense=False, R=2000)
    marks = [1, 2, 3, 50, 150, 300]
    U, E = _gpu_marks(rom, U0, marks)
    for b in (0, 9, 15):
        ref = _oracle(p, _ops(p, False), 300, U0[b])
        _check_traj(dt, np.stack([U0[b]] + [U[m][b] for m in marks]), E[:, b],
                    dict(traj=np.stack([ref["traj"][0]] + [ref["traj"][m] for m in marks]), E=ref["E"]),
                    f"trajectory {b}")
    rom.close()


@pytest.mark.timeout(600)
def test_config3_dense_batch16(torch_gpu):
    _say("generating the N=1000 dense workload")
    p = romsynth.make_config(3, dense=True, cp=False)
    B = 16
    U0 = romsynth.initial_u(p.N, range(B), cfg=3)
    b = 11
    _say(f"oracle: N=1000 dense trajectory {b}, 20 steps")
    ref = _oracle(p, _ops(p, True), 20, U0[b])
    for dt in ("fp32", "bf16"):
        _say(f"N=1000 dense B={B} {dt}, 20 steps")
        rom = rg.Rom.from_problem(p, dense=True, dtype=dt, max_batch=B)
        tune.apply(rom, B, dense=True)
        marks = [1, 2, 3, 10, 20]
        U, E = _gpu_marks(rom, U0, marks)
        _check_traj(dt, np.stack([U0[b]] + [U[m][b] for m in marks]), E[:, b],
                    dict(traj=np.stack([ref["traj"][0]] + [ref["traj"][m] for m in marks]), E=ref["E"]),
                    f"dense trajectory {b}")
        rom.close()
