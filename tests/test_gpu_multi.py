"""Uneven-N batching: rom_step_multi advances pairs of different N, R, dtype and
stiffness together (grouped launches over device job tables) and must give the same
trajectories as stepping each pair alone."""
import sys

import numpy as np
import pytest

import oracle as orc
import paper_2311_03694_amd as rg
import romsynth
from helpers import TRAJ_TOL, rel

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


SPECS = [
    # (N, pairs, dense, dtype, stiffness, batch)
    (37, 20, True, "fp32", "diag", 1),
    (64, 30, True, "fp64", "spd", 1),
    (100, 30, False, "bf16", "diag", 1),
    (48, 20, False, "fp32", "spd", 1),
    (24, 12, True, "bf16x3", "diag", 5),
    (130, 70, False, "fp64", "diag", 1),
]


def _build(spec, cfg):
    N, pairs, dense, dt, A, B = spec
    p = romsynth.make_problem(N, pairs=pairs, eps=1e-6, nu=1e-3, dt=1e-3, A=A, batch=B, cfg=cfg,
                              dense=dense, cp=not dense)
    return p, rg.Rom.from_problem(p, dense=dense, dtype=dt, max_batch=B)


def test_multi_equals_alone(torch_gpu):
    steps = 300
    probs, roms = [], []
    for q, spec in enumerate(SPECS):
        p, r = _build(spec, 40 + q)
        probs.append(p)
        roms.append(r)
    # a second state on the context of pair 2 (shares the operator)
    extra_u0 = romsynth.initial_u(probs[2].N, [77], cfg=42)
    ctxs = [r.handle for r in roms] + [roms[2].handle]
    multi = [r.state(p.u0) for r, p in zip(roms, probs)] + [roms[2].state(extra_u0)]
    _say(f"rom_step_multi over {len(ctxs)} pairs, {steps} steps")
    rg.rom_step_multi(ctxs, [s.handle for s in multi], steps)
    alone = [r.state(p.u0) for r, p in zip(roms, probs)] + [roms[2].state(extra_u0)]
    for q, s in enumerate(alone):
        _say(f"alone pair {q}")
        s.step(steps)
    for q in range(len(ctxs)):
        um, ym, nm = multi[q].get()
        ua, ya, na = alone[q].get()
        assert nm == na == steps
        assert np.array_equal(um, ua), q
        assert np.array_equal(multi[q].energy()[1], alone[q].energy()[1]), q


def test_multi_against_oracle(torch_gpu):
    steps = 150
    probs, roms, states = [], [], []
    for q, spec in enumerate(SPECS[:4]):
        p, r = _build(spec, 50 + q)
        probs.append(p)
        roms.append(r)
        states.append(r.state(p.u0))
    _say("rom_step_multi vs oracle")
    rg.rom_step_multi([r.handle for r in roms], [s.handle for s in states], steps)
    for q, (p, s) in enumerate(zip(probs, states)):
        kw = dict(C=p.C) if p.C is not None else dict(lam=p.lam, Af=p.Af, Bf=p.Bf, Cf=p.Cf)
        ref = orc.run(p.N, p.nu, p.dt, p.A, steps, u0=p.u0[0], **kw)
        dt = SPECS[q][3]
        assert rel(s.u()[0], ref["u_hist"][0]) < TRAJ_TOL[dt], (q, rel(s.u()[0], ref["u_hist"][0]))


def test_multi_rejects_bad_input(torch_gpu):
    p, r = _build(SPECS[0], 60)
    s = r.state(p.u0)
    with pytest.raises(rg.RomError):
        rg.rom_step_multi([r.handle, r.handle], [s.handle, s.handle], 3)
    p2, r2 = _build(SPECS[1], 61)
    with pytest.raises(rg.RomError):
        rg.rom_step_multi([r2.handle], [s.handle], 3)


def test_multi_mixed_level_parities(torch_gpu):
    """States whose levels have different parities share grouped launches: the kernels
    of each step take the step-counter slots of each state's own level.  One step alone
    for half of the states, then 131 steps together (a captured chunk launched twice,
    then three eager steps), then one more step for the other half, must equal 132
    steps alone, energies included."""
    probs, roms = [], []
    for q, spec in enumerate(SPECS):
        p, r = _build(spec, 60 + q)
        probs.append(p)
        roms.append(r)
    multi = [r.state(p.u0) for r, p in zip(roms, probs)]
    for q in (0, 2, 4):
        _say(f"pair {q}: one step alone (odd level)")
        multi[q].step(1)
    _say("rom_step_multi, 131 steps, levels of both parities")
    rg.rom_step_multi([r.handle for r in roms], [s.handle for s in multi], 131)
    for q in (1, 3, 5):
        multi[q].step(1)
    for q, (r, p) in enumerate(zip(roms, probs)):
        _say(f"pair {q} alone, 132 steps")
        a = r.state(p.u0)
        a.step(132)
        um, ym, nm = multi[q].get()
        ua, ya, na = a.get()
        assert nm == na == 132, (q, nm, na)
        assert np.array_equal(um, ua), q
        assert np.array_equal(multi[q].energy()[1], a.energy()[1]), q
