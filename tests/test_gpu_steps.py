"""Parity of the kernels inside a time step, row by row, on every step path.

Two kinds of checks, both through the C ABI:

1. Integer pin (bitwise).  Operators and coefficients are small integers (tensor entries
   |C| <= 2, CP factors |a| <= 1 with weights 1 or 2, |u| <= 2).  Every product and
   partial sum is then an integer below 2^24, exact in FP64, FP32, BF16 (exact BF16
   products, FP32 accumulation) and BF16X3 (zero low words), whatever the summation
   order, so the GPU must reproduce the oracle's y = C(u)u to the bit (eq. Cu; CP form
   eq. tc_ap).  This holds for rom_nonlinear and for the contraction a step performs:
   a state restarted (rom_state_set) from an integer history at level n computes y^n
   inside its first step, and the y history of rom_state_get returns it.  The new level
   u^{n+1} then differs from the oracle's step only by FP64 rounding, in every format.

2. Elementwise y history.  After a run on random (non-integer) operators the y levels of
   rom_state_get are compared with the oracle evaluated at the GPU's own u of the same
   level; each row must lie within the rounding bound of helpers.bound_dense /
   helpers.bound_cp (test_bounds_cpu.py shows these bounds reject a lost BF16X3 low word,
   a 20% error in a BF16 y and a 1e-3 error in FP32).  A one-trajectory CP state with a
   dense stiffness forms the projections of a level from the right-hand side of the step
   before, as ([B|C]^T Hinv_k) rhs: its bound takes S = |B^T Hinv_k| |rhs|.

Paths: dense and CP (general and pair form of skew column pairs), one trajectory and
batches, diagonal and dense SPD stiffness, plain and full form (mass matrix and zeroth
mode terms), and grouped launches of several pairs (rom_step_multi); four formats."""
import sys

import numpy as np
import pytest

import oracle as orc
import paper_2311_03694_amd as rg
import romsynth
from helpers import bound_cp, bound_dense, check_elem

pytestmark = pytest.mark.gpu

DTS = ["fp64", "fp32", "bf16", "bf16x3"]
NU, DT = 1e-2, 1e-2


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


class Case:
    """One operator set and the context built from it."""

    def __init__(self, form, N, R, dt, A_kind, B, full, integer, seed=0, nu=NU, dtstep=DT):
        self.form, self.N, self.B, self.dt = form, N, B, dt
        self.nu, self.dtstep = nu, dtstep
        self.A = romsynth.stiffness_diag(N) if A_kind == "diag" else romsynth.stiffness_spd(N, seed, cfg=70)
        if form == "dense":
            self.C = (romsynth.integer_dense(N, seed) if integer
                      else romsynth.dense_from_skew_cp(N, R // 2, 1e-6, seed=seed, cfg=71))
            self.ops = dict(C=self.C)
        else:
            if integer:
                lam, Af, Bf, Cf = romsynth.integer_cp_factors(N, R, seed, skew=True)
            else:
                lam, Af, Bf, Cf = romsynth.skew_cp_factors(N, R // 2, seed=seed, cfg=71)
            self.ops = dict(lam=lam, Af=Af, Bf=Bf, Cf=Cf)
        self.full = None
        if full:
            C1, C2, c0, a0 = romsynth.zeroth_terms(N, seed=seed, cfg=72, scale=0.5 if integer else 0.1)
            self.full = dict(M=romsynth.mass_spd(N, seed=seed, cfg=72, norm=0.2), C1=C1, C2=C2, c0=c0, a0=a0)
        self.rom = rg.Rom(N, nu, dtstep, self.A, **self.ops, full=self.full, dtype=dt, max_batch=B)
        if form in ("cp_pair", "cp_general"):
            rg.rom_set_tile(self.rom.handle, 4, 1 if form == "cp_pair" else 0)
            assert rg.rom_query(self.rom.handle, None, 7) == (1 if form == "cp_pair" else 0)

    def y_oracle(self, u):
        if self.form == "dense":
            return orc.nonlinear_dense(self.C, u)
        o = self.ops
        return orc.nonlinear_cp(o["lam"], o["Af"], o["Bf"], o["Cf"], u)

    def bound(self, u, level_order=3):
        if self.form == "dense":
            return bound_dense(self.dt, self.C, u)
        o = self.ops
        S = T = None
        diagA = np.count_nonzero(self.A - np.diag(np.diag(self.A))) == 0
        if self.B == 1 and not diagA:
            # projections from the right-hand side of the step that produced u:
            # s = (B^T Hinv_k) rhs with rhs = H_k u
            b0 = {1: 1.0, 2: 1.5, 3: 11.0 / 6.0}[level_order]
            M = self.full["M"] if self.full else np.eye(self.N)
            H = b0 / self.dtstep * M + self.nu * self.A
            Hinv = np.linalg.inv(H)
            rhs = np.abs(H @ u)
            au = np.abs(u)
            S = np.maximum(np.abs(o["Bf"].T @ Hinv) @ rhs, np.abs(o["Bf"]).T @ au)
            T = np.maximum(np.abs(o["Cf"].T @ Hinv) @ rhs, np.abs(o["Cf"]).T @ au)
        return bound_cp(self.dt, o["lam"], o["Af"], o["Bf"], o["Cf"], u, S=S, T=T)

    def oracle_step(self, uh, yh_core, n):
        """One oracle step per trajectory from history (uh [3][B][N] levels n, n-1, n-2;
        yh_core [2][B][N] = C(u)u at n-1, n-2).  The oracle's y history holds the whole
        explicit term (C(u)u plus the zeroth-mode terms), formed here from the oracle."""
        out = np.empty((self.B, self.N))
        f = self.full or {}
        for b in range(self.B):
            yh = yh_core[:, b, :].copy()
            if self.full:
                Z = np.zeros((self.N, self.N, self.N))
                for q in range(2):
                    yh[q] += orc.explicit_full(uh[q + 1, b], C=Z, C1=f["C1"], C2=f["C2"], c0=f["c0"])
            r = orc.run(self.N, self.nu, self.dtstep, self.A, 1, step0=n, uh=uh[:, b, :], yh=yh,
                        M=f.get("M"), C1=f.get("C1"), C2=f.get("C2"), c0=f.get("c0"), a0=f.get("a0"),
                        **self.ops)
            assert r["status"] == 0
            out[b] = r["u_hist"][0]
        return out

    def close(self):
        self.rom.close()


def _integer_history(N, B, seed, n=7):
    uh = np.stack([romsynth.integer_u(N, [seed * 100 + 10 * q + b for b in range(B)]) for q in range(3)])
    yh = np.stack([romsynth.integer_u(N, [seed * 100 + 50 + 10 * q + b for b in range(B)], vmax=9)
                   for q in range(2)])
    return uh, yh, n


# ------------------------------------------------------------------ integer pin, rom_nonlinear

@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("form", ["dense", "cp_general", "cp_pair"])
@pytest.mark.parametrize("N,R,B", [(4, 6, 1), (4, 6, 3), (37, 40, 1), (37, 40, 5), (130, 64, 19)])
def test_integer_nonlinear_bitwise(torch_gpu, dt, form, N, R, B):
    _say(f"integer nonlinear {form} N={N} R={R} B={B} {dt}")
    cs = Case(form, N, R, dt, "diag", B, False, True, seed=N + B)
    u = romsynth.integer_u(N, range(B))
    ud = torch_gpu.tensor(u, dtype=torch_gpu.float64, device="cuda")
    yd = torch_gpu.empty_like(ud)
    torch_gpu.cuda.synchronize()
    rg.rom_nonlinear(cs.rom.handle, B, ud, yd)
    torch_gpu.cuda.synchronize()
    y = yd.cpu().numpy()
    y_ref = np.stack([cs.y_oracle(u[b]) for b in range(B)])
    assert np.array_equal(y, y_ref), np.max(np.abs(y - y_ref))
    cs.close()


# ------------------------------------------------------------------ integer pin, one step

STEP_PATHS = [
    # form, stiffness, batch, full
    ("dense", "diag", 1, False), ("dense", "spd", 1, False),
    ("cp_pair", "diag", 1, False), ("cp_pair", "spd", 1, False),
    ("cp_general", "diag", 1, False), ("cp_general", "spd", 1, False),
    ("dense", "diag", 5, False), ("dense", "spd", 5, False),
    ("cp_general", "diag", 5, False), ("cp_general", "spd", 5, False),
    ("cp_pair", "spd", 5, False),
    ("dense", "spd", 1, True), ("cp_pair", "spd", 1, True), ("cp_general", "diag", 1, True),
    ("dense", "diag", 5, True), ("cp_general", "spd", 5, True),
]


def _pid(p):
    return f"{p[0]}-{p[1]}-B{p[2]}{'-full' if p[3] else ''}"


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("path", STEP_PATHS, ids=_pid)
def test_integer_step_bitwise(torch_gpu, dt, path):
    form, A_kind, B, full = path
    N, R = 37, 40
    _say(f"integer step {_pid(path)} N={N} {dt}")
    cs = Case(form, N, R, dt, A_kind, B, full, True, seed=3)
    uh, yh, n = _integer_history(N, B, seed=5)
    st = cs.rom.state(uh[0])
    st.set(uh, yh, n)
    st.step(1)
    uh1, yh1, n1 = st.get()
    assert n1 == n + 1
    y_ref = np.stack([cs.y_oracle(uh[0, b]) for b in range(B)])
    assert np.array_equal(yh1[0], y_ref), np.max(np.abs(yh1[0] - y_ref))
    assert np.array_equal(yh1[1], yh[0])
    u_ref = cs.oracle_step(uh, yh, n)
    scale = np.max(np.abs(u_ref))
    assert np.max(np.abs(uh1[0] - u_ref)) <= 1e-13 * scale, np.max(np.abs(uh1[0] - u_ref)) / scale
    st.close()
    cs.close()


def test_integer_step_grouped(torch_gpu):
    """rom_step_multi over pairs of different N, form, format and stiffness (one
    trajectory each, plus a batch and a full-form state, which step on their own inside
    the call): y^n of every pair to the bit, u^{n+1} to FP64 rounding."""
    specs = [("dense", 37, 40, "fp32", "diag", 1, False), ("cp_pair", 53, 40, "bf16", "spd", 1, False),
             ("cp_general", 29, 24, "bf16x3", "diag", 1, False), ("cp_pair", 61, 80, "fp64", "spd", 1, False),
             ("dense", 45, 40, "bf16", "spd", 1, False), ("cp_general", 37, 40, "fp32", "spd", 4, False),
             ("cp_pair", 37, 40, "fp32", "spd", 1, True)]
    cases, states, hist = [], [], []
    for q, (form, N, R, dt, A_kind, B, full) in enumerate(specs):
        _say(f"grouped integer step pair {q}: {form} N={N} {dt} {A_kind} B={B} full={full}")
        cs = Case(form, N, R, dt, A_kind, B, full, True, seed=10 + q)
        uh, yh, n = _integer_history(N, B, seed=20 + q, n=6 + (q % 2))
        st = cs.rom.state(uh[0])
        st.set(uh, yh, n)
        cases.append(cs)
        states.append(st)
        hist.append((uh, yh, n))
    rg.rom_step_multi([c.rom.handle for c in cases], [s.handle for s in states], 1)
    for cs, st, (uh, yh, n) in zip(cases, states, hist):
        uh1, yh1, n1 = st.get()
        assert n1 == n + 1
        y_ref = np.stack([cs.y_oracle(uh[0, b]) for b in range(cs.B)])
        assert np.array_equal(yh1[0], y_ref)
        u_ref = cs.oracle_step(uh, yh, n)
        assert np.max(np.abs(uh1[0] - u_ref)) <= 1e-13 * np.max(np.abs(u_ref))
    for st in states:
        st.close()
    for cs in cases:
        cs.close()


# ------------------------------------------------------------------ elementwise y history

def _check_history(cs, st, what):
    uh, yh, n = st.get()
    for q in range(2):                   # y levels n-1, n-2 at the GPU's own u levels
        lev = n - 1 - q
        order = min(lev, 3)
        for b in range(cs.B):
            u = uh[q + 1, b]
            y_ref = cs.y_oracle(u)
            check_elem(yh[q, b], y_ref, cs.bound(u, order), f"{what} level {lev} trajectory {b}")


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("path", STEP_PATHS, ids=_pid)
def test_history_elementwise(torch_gpu, dt, path):
    form, A_kind, B, full = path
    N, R = 70, 64
    _say(f"history elementwise {_pid(path)} N={N} {dt}")
    cs = Case(form, N, R, dt, A_kind, B, full, False, seed=4, nu=1e-3, dtstep=1e-3)
    u0 = romsynth.initial_u(N, range(B), cfg=73)
    st = cs.rom.state(u0)
    st.step(41)                          # crosses the 1-2-3 ramp and three ladder chunks
    _check_history(cs, st, _pid(path))
    st.step(2)
    _check_history(cs, st, _pid(path))
    st.close()
    cs.close()


@pytest.mark.parametrize("dt", DTS)
def test_history_elementwise_grouped(torch_gpu, dt):
    specs = [("dense", 37, 40, "diag", 1, False), ("cp_pair", 70, 64, "spd", 1, False),
             ("cp_general", 53, 40, "diag", 1, False), ("dense", 45, 40, "spd", 1, False),
             ("cp_general", 37, 40, "spd", 3, False), ("cp_pair", 41, 40, "spd", 1, True)]
    cases, states = [], []
    for q, (form, N, R, A_kind, B, full) in enumerate(specs):
        _say(f"grouped history pair {q}: {form} N={N} {dt} {A_kind} B={B} full={full}")
        cs = Case(form, N, R, dt, A_kind, B, full, False, seed=q, nu=1e-3, dtstep=1e-3)
        st = cs.rom.state(romsynth.initial_u(N, range(B), cfg=74 + q))
        cases.append(cs)
        states.append(st)
    rg.rom_step_multi([c.rom.handle for c in cases], [s.handle for s in states], 150)
    for q, (cs, st) in enumerate(zip(cases, states)):
        _check_history(cs, st, f"grouped pair {q}")
    for st in states:
        st.close()
    for cs in cases:
        cs.close()
