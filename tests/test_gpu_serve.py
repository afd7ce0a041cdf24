"""The serving loop on the device: requests of different N, operator kind and format
arrive while others run, share grouped launches, and each result equals the same
request solved alone (and the FP64 oracle) within the format's tolerance."""
import sys

import numpy as np
import pytest

import oracle as orc
import romsynth
from helpers import TRAJ_TOL, rel
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


def test_serving_alone_equals_mix(torch_gpu):
    reqs = poisson_requests(24, rate=400.0, Ns=(24, 40, 64), dense_frac=0.4, dtypes=("fp32", "bf16x3"),
                            steps_range=(50, 400), seeds=(0, 1), rng_seed=11)
    be = RomBackend()
    srv = Server(be, hbm_budget=8 << 30, max_slots=16, chunk=64)
    _say(f"serving {len(reqs)} requests")
    recs = srv.run(reqs)
    s = summarize(recs, max(r.done for r in recs))
    assert s["requests"] == len(reqs)
    assert max(srv.batches) > 1                        # requests really shared launches
    # a request admitted while another was still running (continuous batching)
    assert any(b.admitted < a.done and b.arrival > a.admitted for a in recs for b in recs)
    for r, rec in zip(reqs, recs):
        _say(f"alone request {r.rid} N={r.N} {r.kind} {r.dtype} steps={r.nsteps}")
        op, _ = be.create_op((r.N, r.seed, r.kind, r.dtype))
        st = op.state(be.u0(r))
        st.step(r.nsteps)
        u_alone = st.u()[0]
        assert rel(rec.u, u_alone) <= TRAJ_TOL[r.dtype], (r.rid, rel(rec.u, u_alone))
        st.close()
        op.close()
    srv.close()


def test_serving_matches_oracle(torch_gpu):
    reqs = poisson_requests(6, rate=1000.0, Ns=(32, 48), dense_frac=0.5, dtypes=("fp32",),
                            steps_range=(60, 200), seeds=(3,), rng_seed=5)
    be = RomBackend()
    srv = Server(be, hbm_budget=4 << 30, max_slots=8, chunk=32)
    _say("serving vs oracle")
    recs = srv.run(reqs)
    for r, rec in zip(reqs, recs):
        A = romsynth.stiffness_spd(r.N, r.seed, be.cfg)
        u0 = be.u0(r)
        if r.kind == "dense":
            kw = dict(C=romsynth.dense_from_skew_cp(r.N, r.N, be.eps, r.seed, be.cfg))
        else:
            lam, Af, Bf, Cf = romsynth.skew_cp_factors(r.N, r.N, r.seed, be.cfg)
            kw = dict(lam=lam, Af=Af, Bf=Bf, Cf=Cf)
        ref = orc.run(r.N, be.nu, be.dt, A, r.nsteps, u0=u0, **kw)
        assert rel(rec.u, ref["u_hist"][0]) < TRAJ_TOL[r.dtype]
        assert abs(rec.energy - ref["E"][-1]) <= TRAJ_TOL[r.dtype] * ref["E"][-1]
    srv.close()
