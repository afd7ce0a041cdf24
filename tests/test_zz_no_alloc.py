"""rom_nonlinear_noalloc (workspace in the library's fixed device scratch, no allocation)
against rom_nonlinear (the context's allocated workspace): the same kernels, so the
results must be equal to the bit, for dense and CP contexts, one trajectory and batches,
in all four formats, on two calls in a row of which the second is smaller (the scratch
keeps the first call's contents), and with a second context of smaller N in between."""
import sys

import numpy as np
import pytest

import paper_2311_03694_amd as rg
import romsynth

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


def _ctx(form, N, dt, B, seed):
    A = romsynth.stiffness_diag(N)
    if form == "dense":
        C = romsynth.dense_from_skew_cp(N, N // 2, 1e-6, seed=seed, cfg=80)
        return rg.Rom(N, 1e-3, 1e-3, A, C=C, dtype=dt, max_batch=B)
    lam, Af, Bf, Cf = romsynth.skew_cp_factors(N, N // 2, seed=seed, cfg=80)
    return rg.Rom(N, 1e-3, 1e-3, A, lam=lam, Af=Af, Bf=Bf, Cf=Cf, dtype=dt, max_batch=B)


def _both(torch, rom, u):
    ud = torch.tensor(u, dtype=torch.float64, device="cuda")
    y1 = torch.full_like(ud, float("nan"))
    y2 = torch.full_like(ud, float("nan"))
    torch.cuda.synchronize()
    rg.rom_nonlinear(rom.handle, u.shape[0], ud, y1)
    rg.rom_nonlinear_noalloc(rom.handle, u.shape[0], ud, y2)
    torch.cuda.synchronize()
    return y1.cpu().numpy(), y2.cpu().numpy()


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("form", ["dense", "cp"])
@pytest.mark.parametrize("N,B", [(70, 1), (53, 19)])
def test_noalloc_equals_nonlinear(torch_gpu, dt, form, N, B):
    _say(f"noalloc {form} N={N} B={B} {dt}")
    rom = _ctx(form, N, dt, B, seed=N)
    u = romsynth.initial_u(N, range(B), cfg=81)
    y1, y2 = _both(torch_gpu, rom, u)
    assert np.all(np.isfinite(y1)) and np.array_equal(y1, y2)
    # a second, smaller call on the same context: the scratch still holds the first
    Bs = max(1, B // 3)
    u2 = 0.5 * romsynth.initial_u(N, range(7, 7 + Bs), cfg=81)
    y1, y2 = _both(torch_gpu, rom, u2)
    assert np.all(np.isfinite(y1)) and np.array_equal(y1, y2)
    # then a smaller context
    small = _ctx(form, N // 2 + 1, dt, Bs, seed=N + 1)
    u3 = romsynth.initial_u(N // 2 + 1, range(Bs), cfg=82)
    y1, y2 = _both(torch_gpu, small, u3)
    assert np.all(np.isfinite(y1)) and np.array_equal(y1, y2)
    small.close()
    rom.close()


def test_noalloc_after_nonfinite_input(torch_gpu):
    """A call with NaN coefficients leaves NaN in the scratch; the next call must not see it."""
    _say("noalloc after NaN input")
    N, B = 45, 9
    rom = _ctx("dense", N, "bf16", B, seed=3)
    u = romsynth.initial_u(N, range(B), cfg=83)
    bad = u.copy()
    bad[:, :] = np.nan
    _both(torch_gpu, rom, bad)
    y1, y2 = _both(torch_gpu, rom, u)
    assert np.all(np.isfinite(y2)) and np.array_equal(y1, y2)
    rom.close()


def test_noalloc_rejects_large_workspace(torch_gpu):
    """A batch whose workspace exceeds the fixed scratch is refused with ROM_E_UNSUPPORTED
    (CP N=500, R=1000, 4096 trajectories: the projection partials alone take 32 MB), and
    rom_nonlinear still serves it."""
    _say("noalloc size limit")
    N, B = 500, 4096
    rom = _ctx("cp", N, "fp32", B, seed=5)
    u = romsynth.initial_u(N, range(B), cfg=84)
    ud = torch_gpu.tensor(u, dtype=torch_gpu.float64, device="cuda")
    yd = torch_gpu.empty_like(ud)
    with pytest.raises(rg.RomError) as ei:
        rg.rom_nonlinear_noalloc(rom.handle, B, ud, yd)
    assert ei.value.status == rg.binding.ROM_E_UNSUPPORTED and "workspace" in str(ei.value)
    rg.rom_nonlinear(rom.handle, B, ud, yd)
    torch_gpu.cuda.synchronize()
    assert bool(torch_gpu.isfinite(yd).all())
    y1, y2 = _both(torch_gpu, rom, u[:16])          # a batch that fits still matches
    assert np.array_equal(y1, y2)
    rom.close()
