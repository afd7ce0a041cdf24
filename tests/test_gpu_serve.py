"""The serving loop on the device: requests of different N, operator kind and format
arrive while others run, share pools of slots (batched states) on their operators, and
each result equals the same request solved alone and the FP64 oracle within the
format's tolerance.  The slot writes the loop is built on (rom_state_set_slot) are
checked on their own."""
import sys

import numpy as np
import pytest

import oracle as orc
import paper_2311_03694_amd as rg
import romsynth
from helpers import ENERGY_TOL, TRAJ_TOL, rel
from paper_2311_03694_amd.serve import RomBackend, Server, poisson_requests, summarize

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


@pytest.mark.parametrize("dense,A,dt,B", [(True, "diag", "fp32", 4), (True, "spd", "bf16x3", 4),
                                          (False, "spd", "fp32", 4), (False, "diag", "bf16", 3),
                                          (False, "spd", "fp64", 1), (True, "spd", "fp64", 1)])
def test_set_slot_joins_a_running_state(torch_gpu, dense, A, dt, B):
    """A trajectory that took its two start-up steps alone joins slot 1 of a state at level
    7: the other slots continue exactly as without the write, and the new one follows the
    oracle's trajectory from its own level 2."""
    N = 37
    _say(f"set_slot dense={dense} A={A} {dt} B={B}")
    p = romsynth.make_problem(N, pairs=18, eps=1e-6, nu=1e-3, dt=1e-3, A=A, batch=B, cfg=85, dense=dense, cp=not dense)
    rom = rg.Rom.from_problem(p, dense=dense, dtype=dt, max_batch=B)
    ops = dict(C=p.C) if dense else dict(lam=p.lam, Af=p.Af, Bf=p.Bf, Cf=p.Cf)
    u_new = romsynth.initial_u(N, [99], cfg=85)[0]
    ramp = rom.state(u_new)
    ramp.step(2)
    uh, yh, _ = ramp.get()
    a, b = rom.state(p.u0), rom.state(p.u0)
    a.step(7)
    b.step(7)
    slot = 1 % B
    b.set_slot(slot, uh[:, 0, :], yh[:, 0, :])
    a.step(30)
    b.step(30)
    ua, ub = a.get()[0][0], b.get()[0][0]
    for q in range(B):
        if q != slot:
            assert np.array_equal(ua[q], ub[q]), q
    ref = orc.run(N, p.nu, p.dt, p.A, 32, u0=u_new, **ops)
    assert rel(ub[slot], ref["u_hist"][0]) < TRAJ_TOL[dt], rel(ub[slot], ref["u_hist"][0])
    E = b.energy()[1][:, slot]
    assert abs(E[-1] - ref["E"][-1]) <= ENERGY_TOL[dt] * ref["E"][-1]
    e_join = 0.5 * float(np.sum(uh[0, 0] ** 2))
    assert abs(E[7] - e_join) <= 1e-14 * e_join                          # the join level's energy
    # an idle slot: zeros stay zeros
    b.set_slot(slot, np.zeros((3, N)), np.zeros((2, N)))
    b.step(5)
    assert np.array_equal(b.get()[0][0][slot], np.zeros(N))


def _oracle_of(be, r):
    A = romsynth.stiffness_spd(r.N, r.seed, be.cfg)
    if r.kind == "dense":
        kw = dict(C=romsynth.dense_from_skew_cp(r.N, r.N, be.eps, r.seed, be.cfg))
    else:
        lam, Af, Bf, Cf = romsynth.skew_cp_factors(r.N, r.N, r.seed, be.cfg)
        kw = dict(lam=lam, Af=Af, Bf=Bf, Cf=Cf)
    return orc.run(r.N, be.nu, be.dt, A, r.nsteps, u0=be.u0(r), **kw)


def test_serving_matches_oracle_and_alone(torch_gpu):
    reqs = poisson_requests(24, rate=400.0, Ns=(24, 40, 64), dense_frac=0.4, dtypes=("fp32", "bf16x3"),
                            steps_range=(1, 400), seeds=(0, 1), rng_seed=11)
    be = RomBackend(pool_slots=4)
    srv = Server(be, hbm_budget=8 << 30, max_slots=16, chunk=64)
    _say(f"serving {len(reqs)} requests")
    recs = srv.run(reqs)
    s = summarize(recs, max(r.done for r in recs))
    assert s["requests"] == s["completed"] == len(reqs)
    assert max(srv.batches) > 1                        # requests really shared launches
    # a request admitted while another was still running (continuous batching)
    assert any(b.admitted < a.done and b.arrival > a.admitted for a in recs for b in recs)
    for r, rec in zip(reqs, recs):
        _say(f"request {r.rid} N={r.N} {r.kind} {r.dtype} steps={r.nsteps}: oracle and alone")
        ref = _oracle_of(be, r)
        assert rel(rec.u, ref["u_hist"][0]) < TRAJ_TOL[r.dtype], (r.rid, rel(rec.u, ref["u_hist"][0]))
        assert abs(rec.energy - ref["E"][-1]) <= ENERGY_TOL[r.dtype] * ref["E"][-1]
        op, _ = be.create_op((r.N, r.seed, r.kind, r.dtype))
        st = op.state(be.u0(r))
        st.step(r.nsteps)
        assert rel(rec.u, st.u()[0]) <= TRAJ_TOL[r.dtype], (r.rid, rel(rec.u, st.u()[0]))
        st.close()
        be.destroy_op(op)
    srv.close()


class _PoisoningBackend(RomBackend):
    """Hands the pool a non-finite history for one request (as if its trajectory had blown
    up), to check that only that request fails."""

    def __init__(self, bad_rid, **kw):
        super().__init__(**kw)
        self.bad_rid = bad_rid

    def start(self, op, r):
        hist, res = super().start(op, r)
        if r.rid == self.bad_rid and hist is not None:
            hist[0][0, 3] = np.nan
        return hist, res


def test_serving_isolates_a_failed_trajectory(torch_gpu):
    reqs = poisson_requests(8, rate=1000.0, Ns=(32,), dense_frac=0.5, dtypes=("fp32",), steps_range=(100, 300),
                            seeds=(3,), rng_seed=5)
    be = _PoisoningBackend(bad_rid=2, pool_slots=8)
    srv = Server(be, hbm_budget=4 << 30, max_slots=8, chunk=32)
    _say("serving with one poisoned trajectory")
    recs = srv.run(reqs)
    assert recs[2].error and "non-finite" in recs[2].error
    for r, rec in zip(reqs, recs):
        if r.rid == 2:
            continue
        assert rec.error is None, (r.rid, rec.error)
        ref = _oracle_of(be, r)
        assert rel(rec.u, ref["u_hist"][0]) < TRAJ_TOL[r.dtype]
    srv.close()
