"""The tile autotuner on the GPU: tune() times every variant of the kernels a batch uses
on a real context (dense batched contraction; CP projections and scatter), keeps the
fastest, records it in the table, and a context stepped with the tuned tiles gives the
same trajectory as with the built-in choice, to the format's rounding."""
import sys

import numpy as np
import pytest

import paper_2311_03694_amd as rg
import romsynth
from paper_2311_03694_amd import tune

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


@pytest.mark.parametrize("dense", [True, False])
def test_tune_and_apply(torch_gpu, dense):
    _say(f"autotuner, {'dense' if dense else 'CP'} batch of 16, N=40, fp32")
    B, N = 16, 40
    p = romsynth.make_problem(N, pairs=8, eps=1e-6, nu=1e-3, dt=1e-3, A="diag", batch=B, cfg=31,
                              dense=dense, cp=not dense)
    R = 0 if dense else p.R
    rom = rg.Rom.from_problem(p, dense=dense, dtype="fp32", max_batch=B)
    table = {}
    out = tune.tune(rom, p.u0, dense=dense, R=R, steps=2, reps=1, table=table)
    kinds = tune.kinds_for(dense, B)
    assert sorted(out) == sorted(tune.key(k, N, R, B, "fp32") for k in kinds)
    for k in kinds:
        rec = out[tune.key(k, N, R, B, "fp32")]
        times = rec["seconds_per_step"]
        assert len(times) == rg.rom_tile_count(k)
        assert all(np.isfinite(t) and t > 0 for t in times)
        assert rec["best"] == int(np.argmin(times))
        assert table[tune.key(k, N, R, B, "fp32")] == rec["best"]
    # a second context of the same shape takes the table's tiles; both step alike
    rom2 = rg.Rom.from_problem(p, dense=dense, dtype="fp32", max_batch=B)
    assert tune.apply(rom2, B, dense=dense, R=R, table=table) == len(kinds)
    rom3 = rg.Rom.from_problem(p, dense=dense, dtype="fp32", max_batch=B)
    s2, s3 = rom2.state(p.u0), rom3.state(p.u0)
    s2.step(30)
    s3.step(30)
    u2, u3 = s2.u(), s3.u()
    assert np.max(np.abs(u2 - u3)) <= 1e-5 * np.max(np.abs(u3))
    for x in (s2, s3, rom2, rom3, rom):
        x.close()
