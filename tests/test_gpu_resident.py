"""Resident one-trajectory CP steps (k_res.hip): a run of steps in one cooperative launch
whose blocks keep their operator rows in LDS and exchange the right-hand side and w as
tagged messages.  Every level, y history and energy equals the per-step kernels' to the
bit (the same dot products in the same order), across runs, restarts and formats, and the
trajectories follow the FP64 oracle."""
import sys

import numpy as np
import pytest

import oracle as orc
import paper_2311_03694_amd as rg
import romsynth
from helpers import TRAJ_TOL, traj_rel

pytestmark = pytest.mark.gpu

RESIDENT = 5           # rom_set_tile kind: resident one-trajectory CP steps


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _pair(p, dt, pair):
    """Resident context and per-step context of one problem."""
    kw = dict(lam=p.lam, Af=p.Af, Bf=p.Bf, Cf=p.Cf, dtype=dt)
    res = rg.Rom(p.N, p.nu, p.dt, p.A, **kw)
    ref = rg.Rom(p.N, p.nu, p.dt, p.A, **kw)
    ref.set_tile(RESIDENT, 0)
    if not pair:
        res.set_tile(4, 0)
        ref.set_tile(4, 0)
    return res, ref


def _same(a, b, what):
    ua, ya, na = a.get()
    ub, yb, nb = b.get()
    assert na == nb
    assert np.array_equal(ua, ub), (what, float(np.max(np.abs(ua - ub))))
    assert np.array_equal(ya, yb), (what, float(np.max(np.abs(ya - yb))))
    Ea, Eb = a.energy()[1], b.energy()[1]
    assert np.array_equal(Ea, Eb, equal_nan=True), what          # NaN below a restart level


@pytest.mark.parametrize("N,pairs", [(37, 18), (130, 70)])
@pytest.mark.parametrize("A", ["diag", "spd"])
@pytest.mark.parametrize("pair", [True, False])
@pytest.mark.parametrize("dt", ["fp64", "fp32", "bf16", "bf16x3"])
def test_resident_equals_per_step(torch_gpu, dt, pair, A, N, pairs):
    _say(f"resident {dt} pair={pair} A={A} N={N} R={2 * pairs}")
    p = romsynth.make_problem(N, pairs=pairs, eps=1e-6, nu=1e-3, dt=1e-3, A=A, cfg=91, dense=False)
    res, ref = _pair(p, dt, pair)
    a, b = res.state(p.u0[0]), ref.state(p.u0[0])
    assert a.resident_blocks > 0 and b.resident_blocks == 0
    # two start-up levels, then runs of 40 and 600 steps (two runs and a tail) and a
    # short call below the run length
    for k in (42, 600, 7):
        a.step(k)
        b.step(k)
        _same(a, b, f"after {a.step_count} steps")
    ref_o = orc.run(N, p.nu, p.dt, p.A, a.step_count, u0=p.u0[0], lam=p.lam, Af=p.Af, Bf=p.Bf, Cf=p.Cf)
    err = float(np.linalg.norm(a.u() - ref_o["u_hist"][0]) / np.linalg.norm(ref_o["u_hist"][0]))
    _say(f"  oracle error {err:.2e}")
    assert err < TRAJ_TOL[dt]


def test_resident_restart_and_reuse(torch_gpu):
    """A restart to an earlier level and a second state of the same context: the message
    tags of earlier runs never match a later run's.  (A restart recomputes the dense-
    stiffness projections from u^n, so the per-step reference takes the same restart.)"""
    N, pairs = 64, 40
    p = romsynth.make_problem(N, pairs=pairs, eps=1e-6, nu=1e-3, dt=1e-3, A="spd", cfg=92, dense=False)
    res, ref = _pair(p, "fp32", True)
    a, b = res.state(p.u0[0]), ref.state(p.u0[0])
    a.step(100)
    b.step(100)
    uh, yh, n = a.get()
    a.step(50)
    a.set(uh, yh, n)                   # back to level 100, then over the same levels again
    b.set(uh, yh, n)
    a.step(50)
    b.step(50)
    _same(a, b, "restart")
    c, d = res.state(p.u0[0]), ref.state(p.u0[0])
    c.step(150)
    d.step(150)
    _same(c, d, "second state")


def test_resident_headline_size(torch_gpu):
    """N = 1000, CP rank 2000 in the pair form, SPD stiffness, FP32 and BF16X3: the
    benchmark's configuration; 300 steps against the per-step kernels, bitwise."""
    p = romsynth.make_config(3, dense=False, nsteps=300)
    for dt in ("fp32", "bf16x3"):
        _say(f"headline size {dt}")
        res, ref = _pair(p, dt, True)
        a, b = res.state(p.u0[0]), ref.state(p.u0[0])
        assert a.resident_blocks == 250
        a.step(300)
        b.step(300)
        _same(a, b, dt)
        a.close(); b.close(); res.close(); ref.close()


def test_resident_many_row_groups(torch_gpu):
    """N = 1100 > 4 x 256 rows: blocks own two row groups (diagonal stiffness)."""
    N, pairs = 1100, 32
    p = romsynth.make_problem(N, pairs=pairs, eps=1e-6, nu=5e-4, dt=5e-4, A="diag", cfg=93, dense=False)
    res, ref = _pair(p, "fp32", True)
    a, b = res.state(p.u0[0]), ref.state(p.u0[0])
    assert a.resident_blocks > 0
    a.step(120)
    b.step(120)
    _same(a, b, "N=1100")


def test_resident_first_bad_level(torch_gpu):
    """u_i' = -c_i u_i^2 from u_i(0) < 0 as CP factors (Af = Bf = Cf = I, lam = c): the
    first non-finite level of a resident run is the oracle's."""
    N = 4
    I = np.eye(N)
    lam = 1.0 + np.arange(N)
    u0 = -np.array([2.0, 1.5, 1.0, 0.5])
    r = orc.run(N, 0.0, 0.01, np.eye(N), 400, u0=u0, lam=lam, Af=I, Bf=I, Cf=I)
    assert r["status"] == 4 and r["first_bad"] > 20
    rom = rg.Rom(N, 0.0, 0.01, np.eye(N), lam=lam, Af=I, Bf=I, Cf=I, dtype="fp64")
    s = rom.state(u0)
    assert s.resident_blocks > 0
    with pytest.raises(rg.NonFinite) as ei:
        s.step(400)
    assert ei.value.first_bad == r["first_bad"]


def test_resident_in_a_second_process(torch_gpu, tmp_path):
    """This process takes a resident run first; then a child process steps the same
    problem.  The runtime may refuse the child's cooperative launch while this process
    holds the device's resource for such launches: the child's steps must then go through
    the per-step kernels, and either way its levels equal the per-step kernels' to the bit."""
    import os
    import subprocess
    _say("resident run here, then the same steps in a child process")
    p = romsynth.make_problem(64, pairs=40, eps=1e-6, nu=1e-3, dt=1e-3, A="spd", cfg=93, dense=False)
    res, ref = _pair(p, "fp32", True)
    a, b = res.state(p.u0[0]), ref.state(p.u0[0])
    assert a.resident_blocks > 0
    a.step(100)
    b.step(100)
    _same(a, b, "this process")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = tmp_path / "child.npz"
    code = f"""
import sys
sys.path.insert(0, {root!r})
import numpy as np, romsynth, paper_2311_03694_amd as rg
p = romsynth.make_problem(64, pairs=40, eps=1e-6, nu=1e-3, dt=1e-3, A="spd", cfg=93, dense=False)
rom = rg.Rom(p.N, p.nu, p.dt, p.A, lam=p.lam, Af=p.Af, Bf=p.Bf, Cf=p.Cf, dtype="fp32")
st = rom.state(p.u0[0])
st.step(100)
u, y, n = st.get()
np.savez({str(out)!r}, u=u, y=y, E=st.energy()[1], n=n)
print("child done", flush=True)
"""
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=180)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    got = np.load(out)
    ub, yb, nb = b.get()
    assert int(got["n"]) == nb
    assert np.array_equal(got["u"], ub) and np.array_equal(got["y"], yb)
    assert np.array_equal(got["E"], b.energy()[1])


def test_resident_runs_on_two_streams(torch_gpu):
    """Two contexts on two streams whose resident runs are enqueued interleaved and
    asynchronously: the library orders the runs across the streams (each run needs the
    whole device), so both sequences finish and equal the per-step kernels to the bit."""
    torch = torch_gpu
    _say("resident runs of two contexts on two streams, interleaved")
    p = romsynth.make_problem(130, pairs=70, eps=1e-6, nu=1e-3, dt=1e-3, A="spd", cfg=95, dense=False)
    q = romsynth.make_problem(97, pairs=40, eps=1e-6, nu=1e-3, dt=1e-3, A="diag", cfg=96, dense=False)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    roms = [rg.Rom(x.N, x.nu, x.dt, x.A, lam=x.lam, Af=x.Af, Bf=x.Bf, Cf=x.Cf, dtype="fp32", stream=st)
            for x, st in zip((p, q), streams)]
    states = [r.state(x.u0[0]) for r, x in zip(roms, (p, q))]
    for st in states:
        assert st.resident_blocks > 0
        st.step(2)
    for _ in range(3):
        for st in states:
            st.step_async(300)
    for st in states:
        st.sync()
    for x in (p, q):
        ref = rg.Rom(x.N, x.nu, x.dt, x.A, lam=x.lam, Af=x.Af, Bf=x.Bf, Cf=x.Cf, dtype="fp32")
        ref.set_tile(RESIDENT, 0)
        b = ref.state(x.u0[0])
        b.step(902)
        a = states[0 if x is p else 1]
        _same(a, b, f"N={x.N} on its own stream")
