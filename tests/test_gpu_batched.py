"""Parity of the batched (MFMA) path with the FP64 oracle, through the C ABI."""
import sys

import numpy as np
import pytest

import oracle as orc
import paper_2311_03694_amd as rg
import romsynth
from helpers import TRAJ_TOL, check_eval, eval_bound_cp, eval_bound_dense, rel, traj_rel

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


def _gpu_nonlinear(torch, rom, U):
    ud = torch.tensor(U, dtype=torch.float64, device="cuda")
    yd = torch.empty_like(ud)
    torch.cuda.synchronize()
    rg.rom_nonlinear(rom.handle, ud.shape[0], ud, yd)
    torch.cuda.synchronize()
    return yd.cpu().numpy()


def _round(dt, arrays):
    if dt == "bf16":
        return [orc.round_bf16(a).reshape(np.shape(a)) for a in arrays]
    return arrays


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("N,B", [(37, 3), (100, 20), (130, 64), (64, 17)])
def test_dense_batched_nonlinear(torch_gpu, dt, N, B):
    _say(f"dense batched nonlinear N={N} B={B} {dt}")
    C = romsynth.dense_rough(N, seed=N + 1, cfg=21)
    U = romsynth.initial_u(N, range(B), cfg=21)
    rom = rg.Rom(N, 1e-3, 1e-3, romsynth.stiffness_diag(N), C=C, dtype=dt, max_batch=B)
    Y = _gpu_nonlinear(torch_gpu, rom, U)
    Cr, Ur = _round(dt, [C, U])
    for b in range(B):
        yr = orc.nonlinear_dense(Cr, Ur[b])
        check_eval(dt, Y[b], yr, eval_bound_dense(dt, C, U[b]))


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("N,B", [(130, 40), (203, 17)])
def test_dense_batched_every_variant(torch_gpu, dt, N, B):
    """Every tile variant of the batched dense contraction (register kernel and LDS-tile
    kernel) against the oracle: ragged rows, k-chunks, j-ranges and column tiles."""
    C = romsynth.dense_rough(N, seed=N + 3, cfg=23)
    U = romsynth.initial_u(N, range(B), cfg=23)
    rom = rg.Rom(N, 1e-3, 1e-3, romsynth.stiffness_diag(N), C=C, dtype=dt, max_batch=B)
    Cr, Ur = _round(dt, [C, U])
    refs = [orc.nonlinear_dense(Cr, Ur[b]) for b in range(B)]
    bounds = [eval_bound_dense(dt, C, U[b]) for b in range(B)]
    for v in range(rg.rom_tile_count(1)):
        _say(f"dense batched variant {v} N={N} B={B} {dt}")
        rg.rom_set_tile(rom.handle, 1, v)
        Y = _gpu_nonlinear(torch_gpu, rom, U)
        for b in range(B):
            check_eval(dt, Y[b], refs[b], bounds[b])


@pytest.mark.parametrize("dense", [True, False])
def test_nonlinear_after_workspace_layout_changes(torch_gpu, dense):
    """rom_nonlinear with batch sizes that move the workspace regions between calls:
    the operand copies are rebuilt with their zero padding every time, so stale
    workspace bytes (which read as BF16 can be NaN) never reach the products."""
    N, dt = 70, "bf16"
    U = romsynth.initial_u(N, range(48), cfg=24)
    if dense:
        C = romsynth.dense_rough(N, seed=5, cfg=24)
        rom = rg.Rom(N, 1e-3, 1e-3, romsynth.stiffness_diag(N), C=C, dtype=dt, max_batch=48)
        Cr, Ur = _round(dt, [C, U])
        refs = [orc.nonlinear_dense(Cr, Ur[b]) for b in range(48)]
        bounds = [eval_bound_dense(dt, C, U[b]) for b in range(48)]
    else:
        lam, Af, Bf, Cf = romsynth.skew_cp_factors(N, 30, seed=5, cfg=24)
        rom = rg.Rom(N, 1e-3, 1e-3, romsynth.stiffness_diag(N), lam=lam, Af=Af, Bf=Bf, Cf=Cf, dtype=dt,
                     max_batch=48)
        lr, Ar, Br, Crr, Ur = _round(dt, [lam, Af, Bf, Cf, U])
        refs = [orc.nonlinear_cp(lr, Ar, Br, Crr, Ur[b]) for b in range(48)]
        bounds = [eval_bound_cp(dt, lam, Af, Bf, Cf, U[b]) for b in range(48)]
    for B in (40, 17, 48, 2, 33, 40):
        _say(f"nonlinear after layout change dense={dense} B={B}")
        Y = _gpu_nonlinear(torch_gpu, rom, U[:B])
        assert np.all(np.isfinite(Y))
        for b in range(B):
            check_eval(dt, Y[b], refs[b], bounds[b])


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("N,pairs,B", [(37, 25, 3), (100, 50, 20), (96, 160, 40)])
def test_cp_batched_nonlinear(torch_gpu, dt, N, pairs, B):
    _say(f"cp batched nonlinear N={N} R={2 * pairs} B={B} {dt}")
    lam, Af, Bf, Cf = romsynth.skew_cp_factors(N, pairs, seed=4, cfg=22)
    U = romsynth.initial_u(N, range(B), cfg=22)
    rom = rg.Rom(N, 1e-3, 1e-3, romsynth.stiffness_diag(N), lam=lam, Af=Af, Bf=Bf, Cf=Cf, dtype=dt, max_batch=B)
    Y = _gpu_nonlinear(torch_gpu, rom, U)
    ops = _round(dt, [lam, Af, Bf, Cf])
    Ur = _round(dt, [U])[0]
    for b in range(B):
        yr = orc.nonlinear_cp(*ops, Ur[b])
        check_eval(dt, Y[b], yr, eval_bound_cp(dt, lam, Af, Bf, Cf, U[b]))


@pytest.mark.parametrize("dt", DTS)
def test_cp_batched_every_variant(torch_gpu, dt):
    """Every tile variant of the batched CP projections and scatter (skinny-GEMM kernel
    and LDS-tile kernel) against the oracle, with ragged rows, rank and batch."""
    N, pairs, B = 130, 75, 40
    lam, Af, Bf, Cf = romsynth.skew_cp_factors(N, pairs, seed=6, cfg=25)
    U = romsynth.initial_u(N, range(B), cfg=25)
    rom = rg.Rom(N, 1e-3, 1e-3, romsynth.stiffness_diag(N), lam=lam, Af=Af, Bf=Bf, Cf=Cf, dtype=dt, max_batch=B)
    ops = _round(dt, [lam, Af, Bf, Cf])
    Ur = _round(dt, [U])[0]
    refs = [orc.nonlinear_cp(*ops, Ur[b]) for b in range(B)]
    bounds = [eval_bound_cp(dt, lam, Af, Bf, Cf, U[b]) for b in range(B)]
    for kind in (2, 3):
        for v in range(rg.rom_tile_count(kind)):
            _say(f"cp batched kind {kind} variant {v} {dt}")
            rg.rom_set_tile(rom.handle, kind, v)
            Y = _gpu_nonlinear(torch_gpu, rom, U)
            for b in range(B):
                check_eval(dt, Y[b], refs[b], bounds[b])
        rg.rom_set_tile(rom.handle, kind, -1)


def test_batched_unit_positions(torch_gpu):
    """One non-zero tensor entry / rank-1 unit factors, through the MFMA path: the
    output must land in row i of every trajectory with weight u_j u_k."""
    N, B = 24, 5
    U = np.arange(1.0, B * N + 1.0).reshape(B, N) / 10.0
    for (i, j, k) in [(0, 1, 2), (23, 7, 19), (5, 22, 0)]:
        _say(f"batched unit tensor {(i, j, k)}")
        C = np.zeros((N, N, N))
        C[i, j, k] = 1.0
        rom = rg.Rom(N, 1e-3, 1e-3, np.eye(N), C=C, dtype="fp64", max_batch=B)
        Y = _gpu_nonlinear(torch_gpu, rom, U)
        E = np.zeros((B, N))
        E[:, i] = U[:, j] * U[:, k]
        assert np.allclose(Y, E, rtol=1e-15, atol=0)
        Af = np.zeros((N, 1)); Af[i, 0] = 1.0
        Bf = np.zeros((N, 1)); Bf[j, 0] = 1.0
        Cf = np.zeros((N, 1)); Cf[k, 0] = 1.0
        rom2 = rg.Rom(N, 1e-3, 1e-3, np.eye(N), lam=np.array([0.5]), Af=Af, Bf=Bf, Cf=Cf, dtype="fp64",
                      max_batch=B)
        Y2 = _gpu_nonlinear(torch_gpu, rom2, U)
        assert np.allclose(Y2, 0.5 * E, rtol=1e-15, atol=0)


def _oracle_traj(p, dense, b, nsteps):
    kw = dict(C=p.C) if dense else dict(lam=p.lam, Af=p.Af, Bf=p.Bf, Cf=p.Cf)
    r = orc.run(p.N, p.nu, p.dt, p.A, nsteps, u0=p.u0[b], **kw)
    assert r["status"] == 0
    return r


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("dense,A", [(True, "diag"), (False, "diag"), (True, "spd"), (False, "spd")])
def test_batched_trajectories(torch_gpu, dt, dense, A):
    """B=6 trajectories, 300 steps (crosses graph chunks): each column against its own
    oracle run, and against the same trajectory run alone (single-trajectory kernels)."""
    B, steps = 6, 300
    _say(f"batched trajectories dense={dense} A={A} {dt}")
    p = romsynth.make_problem(56, pairs=28, eps=1e-6, nu=1e-3, dt=1e-3, A=A, batch=B, cfg=23,
                              dense=dense, cp=not dense)
    rom = rg.Rom.from_problem(p, dense=dense, dtype=dt, max_batch=B)
    st = rom.state(p.u0)
    st.step(steps)
    uh, _, n = st.get()
    assert n == steps
    _, Elog = st.energy()
    tol = TRAJ_TOL[dt]
    for b in range(B):
        r = _oracle_traj(p, dense, b, steps)
        assert rel(uh[0][b], r["u_hist"][0]) < tol, (b, rel(uh[0][b], r["u_hist"][0]))
        assert np.max(np.abs(Elog[:, b] - r["E"]) / r["E"]) < tol
    # alone vs in the batch
    # (a CP trajectory alone with a dense stiffness projects the right-hand side through
    # [Bf|Cf]^T Hinv_k, so its BF16 roundings fall on other operands than in the batch:
    # the two agree to the BF16 trajectory tolerance only)
    single = rom.state(p.u0[2])
    single.step(steps)
    alone_tol = 1e-12 if dt == "fp64" else 1e-5
    if dt == "bf16" and not dense and A == "spd":
        alone_tol = TRAJ_TOL["bf16"]
    assert rel(uh[0][2], single.u()[0]) < alone_tol


def test_batched_checkpoint_resume(torch_gpu):
    _say("batched checkpoint/resume")
    B = 9
    p = romsynth.make_problem(40, pairs=20, eps=1e-6, batch=B, cfg=24, dense=True, cp=False)
    rom = rg.Rom.from_problem(p, dense=True, dtype="bf16x3", max_batch=B)
    a = rom.state(p.u0)
    a.step(150)
    b = rom.state(p.u0)
    b.step(61)
    uh, yh, n = b.get()
    c = rom.state(np.zeros_like(p.u0))
    c.set(uh, yh, n)
    c.step(89)
    assert np.array_equal(a.get()[0], c.get()[0])


@pytest.mark.parametrize("dense,B", [(True, 1), (True, 20), (False, 1), (False, 20)])
def test_nonlinear_timed_matches(torch_gpu, dense, B):
    """The measurement entry point returns the same y as rom_nonlinear (bit for bit),
    a positive kernel time, and rejects reps < 1."""
    _say(f"nonlinear_timed dense={dense} B={B}")
    torch = torch_gpu
    N = 64
    U = romsynth.initial_u(N, range(B), cfg=26)
    if dense:
        rom = rg.Rom(N, 1e-3, 1e-3, romsynth.stiffness_diag(N), C=romsynth.dense_rough(N, seed=7, cfg=26),
                     dtype="fp32", max_batch=max(B, 2))
    else:
        lam, Af, Bf, Cf = romsynth.skew_cp_factors(N, 20, seed=7, cfg=26)
        rom = rg.Rom(N, 1e-3, 1e-3, romsynth.stiffness_diag(N), lam=lam, Af=Af, Bf=Bf, Cf=Cf, dtype="fp32",
                     max_batch=max(B, 2))
    ud = torch.tensor(U, dtype=torch.float64, device="cuda")
    y1 = torch.empty_like(ud)
    y2 = torch.empty_like(ud)
    rg.rom_nonlinear(rom.handle, B, ud, y1)
    us = rg.rom_nonlinear_timed(rom.handle, B, ud, y2, 3)
    torch.cuda.synchronize()
    assert us > 0
    assert torch.equal(y1, y2)
    with pytest.raises(rg.RomError):
        rg.rom_nonlinear_timed(rom.handle, B, ud, y2, 0)
