"""Scheduling logic of the serving loop on the host, with a fake device backend
(deterministic step-time model, byte accounting)."""
import numpy as np
import pytest

from paper_2311_03694_amd.serve import Request, Server, op_key, poisson_requests, summarize


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 0.0)


class FakeBackend:
    """Operators cost N^2 bytes, states N bytes; a chunk of n steps over the active pairs
    costs n * (1e-6 + 1e-9 * sum N) seconds of virtual time."""

    def __init__(self, clock):
        self.clock = clock
        self.created = []
        self.destroyed = []
        self.live = 0
        self.peak = 0
        self.steps = {}

    def estimate_op_bytes(self, key):
        return key[0] ** 2

    def estimate_state_bytes(self, key):
        return key[0]

    def create_op(self, key):
        self.created.append(key)
        self.live += key[0] ** 2
        self.peak = max(self.peak, self.live)
        return ("op", key), key[0] ** 2

    def destroy_op(self, op):
        self.destroyed.append(op[1])
        self.live -= op[1][0] ** 2

    def create_state(self, op, r):
        self.steps[r.rid] = 0
        self.live += r.N
        self.peak = max(self.peak, self.live)
        return ("st", r), r.N

    def destroy_state(self, st):
        self.live -= st[1].N

    def step(self, pairs, n):
        self.clock.t += n * (1e-6 + 1e-9 * sum(st[1].N for _, st in pairs))
        for _, st in pairs:
            self.steps[st[1].rid] += n

    def result(self, st):
        return np.full(3, float(self.steps[st[1].rid])), float(st[1].rid)


def _run(reqs, budget, slots=64, chunk=50):
    clk = Clock()
    be = FakeBackend(clk)
    srv = Server(be, budget, max_slots=slots, chunk=chunk, clock=clk, sleep=clk.sleep)
    recs = srv.run(reqs)
    return srv, be, recs, clk


def test_every_request_runs_its_steps():
    reqs = poisson_requests(200, rate=2000.0, Ns=(10, 20, 40), steps_range=(10, 1000), rng_seed=3)
    srv, be, recs, clk = _run(reqs, budget=10 ** 6)
    assert len(recs) == len(reqs)
    for r, rec in zip(reqs, recs):
        assert rec.rid == r.rid
        assert be.steps[r.rid] == r.nsteps           # exactly nsteps, never more
        assert rec.u[0] == r.nsteps
        assert r.arrival <= rec.admitted <= rec.done
    s = summarize(recs, clk.t)
    lat = np.array([x.latency for x in recs])
    assert s["latency_p50_s"] == pytest.approx(np.percentile(lat, 50))
    assert s["latency_p99_s"] == pytest.approx(np.percentile(lat, 99))
    assert s["trajectory_steps"] == sum(r.nsteps for r in reqs)


def test_budget_is_respected_and_operators_shared():
    reqs = [Request(i, 0.0, N=30 if i % 2 else 20, seed=0, kind="cp", dtype="fp32", nsteps=100, u0_seed=i)
            for i in range(40)]
    budget = 30 ** 2 + 20 ** 2 + 40 * 30
    srv, be, recs, _ = _run(reqs, budget)
    assert be.peak <= budget
    assert sorted(set(be.created)) == sorted({op_key(r) for r in reqs})
    assert len(be.created) == 2                        # each operator built once, then shared


def test_eviction_makes_room():
    # two operators that do not fit together: the second waits until the first is
    # unreferenced, then replaces it
    reqs = [Request(0, 0.0, 100, 0, "dense", "fp32", 300, 0), Request(1, 0.0, 90, 0, "dense", "fp32", 100, 1)]
    srv, be, recs, _ = _run(reqs, budget=100 ** 2 + 200)
    assert be.peak <= 100 ** 2 + 200
    assert be.destroyed == [(100, 0, "dense", "fp32")]
    assert recs[1].admitted >= recs[0].done


def test_continuous_batching_admits_mid_flight():
    # a long request is running when a short one arrives: the short one joins the
    # running batch and finishes first
    reqs = [Request(0, 0.0, 20, 0, "cp", "fp32", 5000, 0), Request(1, 1e-3, 20, 0, "cp", "fp32", 100, 1)]
    srv, be, recs, _ = _run(reqs, budget=10 ** 6, chunk=100)
    assert recs[1].admitted < recs[0].done
    assert recs[1].done < recs[0].done
    assert max(srv.batches) == 2


def test_oversized_request_rejected():
    with pytest.raises(ValueError):
        _run([Request(0, 0.0, 100, 0, "dense", "fp32", 10, 0)], budget=100)
