"""Continuous-batching request loop for ROM solves (host scheduler over librom.so).

A request asks for `nsteps` BDF3/EXT3 steps of one trajectory of a reduced model with
N modes, given either as a dense advection tensor or as rank-R CP factors, in one
contraction format.  The loop

  * admits waiting requests whose arrival time has passed while a slot is free and the
    HBM budget holds the request's operator (shared by all requests on the same
    operator, reference counted, evicted least-recently-used once unreferenced) plus its
    trajectory state;
  * advances every admitted request by one chunk of steps with a single
    rom_step_multi call, so requests of different N and R share the device in the same
    grouped launches (continuous batching: new requests join at chunk boundaries
    while older ones are still running);
  * retires requests whose step count is reached and records their latency
    (completion minus arrival), final coefficients and energy.

The device work is behind a small backend interface: RomBackend drives the C ABI;
tests use a deterministic fake backend to check the scheduling logic on the host.
"""
from __future__ import annotations

import dataclasses
import math
import time
from collections import OrderedDict
from typing import Callable, Dict, List, Optional, Tuple

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float            # seconds after the start of the run
    N: int
    seed: int                 # operator seed (requests with equal (N, seed, kind, dtype) share it)
    kind: str                 # "cp" or "dense"
    dtype: str                # "fp32", "bf16x3", "bf16", "fp64"
    nsteps: int
    u0_seed: int


@dataclasses.dataclass
class Record:
    rid: int
    arrival: float
    admitted: float
    done: float
    nsteps: int
    N: int
    kind: str
    dtype: str
    u: Optional[np.ndarray] = None
    energy: Optional[float] = None
    error: Optional[str] = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def op_key(r: Request) -> Tuple:
    return (r.N, r.seed, r.kind, r.dtype)


# ----------------------------------------------------------------------------- backends

class RomBackend:
    """The real device: operators from the seeded generator (N modes, N skew pairs, i.e.
    CP rank 2N, 1e-7 noise, SPD stiffness, nu = dt = 5e-4), states through the C ABI."""

    def __init__(self, cfg: int = 4, eps: float = 1e-7, nu: float = 5e-4, dt: float = 5e-4, stream=None):
        import paper_2311_03694_amd as rg
        import romsynth
        self.rg = rg
        self.syn = romsynth
        self.cfg, self.eps, self.nu, self.dt = cfg, eps, nu, dt
        self.stream = stream
        self._host_ops: Dict[Tuple, object] = {}

    def estimate_op_bytes(self, key) -> int:
        N, _seed, kind, dtype = key
        eb = {"fp64": 8, "fp32": 4, "bf16": 2, "bf16x3": 4}[dtype]
        Np = (N + 7) // 8 * 8
        helm = 3 * N * N * 8
        if kind == "dense":
            return N * N * Np * eb + helm
        R = 2 * N
        return 3 * R * Np * eb + helm

    def estimate_state_bytes(self, key) -> int:
        N = key[0]
        return 8 * N * 10 + 8 * 4096 + 65536

    def create_op(self, key):
        N, seed, kind, dtype = key
        syn = self.syn
        A = syn.stiffness_spd(N, seed, self.cfg)
        if kind == "dense":
            C = syn.dense_from_skew_cp(N, N, self.eps, seed, self.cfg)
            rom = self.rg.Rom(N, self.nu, self.dt, A, C=C, dtype=dtype, stream=self.stream)
        else:
            lam, Af, Bf, Cf = syn.skew_cp_factors(N, N, seed, self.cfg)
            rom = self.rg.Rom(N, self.nu, self.dt, A, lam=lam, Af=Af, Bf=Bf, Cf=Cf, dtype=dtype,
                              stream=self.stream)
        return rom, rom.bytes()

    def destroy_op(self, op):
        op.close()

    def u0(self, r: Request) -> np.ndarray:
        return self.syn.initial_u(r.N, [r.u0_seed], cfg=self.cfg)[0]

    def create_state(self, op, r: Request):
        st = op.state(self.u0(r))
        return st, st.bytes()

    def destroy_state(self, st):
        st.close()

    def step(self, pairs: List[Tuple[object, object]], nsteps: int):
        self.rg.rom_step_multi([op.handle for op, _ in pairs], [st.handle for _, st in pairs], nsteps)

    def result(self, st) -> Tuple[np.ndarray, float]:
        E, _ = st.energy(log=False)
        return st.u()[0].copy(), float(E[0])


# ----------------------------------------------------------------------------- the loop

class Server:
    """Admission by slots and HBM budget, continuous batching in chunks of steps."""

    def __init__(self, backend, hbm_budget: int, max_slots: int = 256, chunk: int = 256,
                 clock: Optional[Callable[[], float]] = None, sleep: Optional[Callable[[float], None]] = None):
        self.be = backend
        self.budget = int(hbm_budget)
        self.max_slots = int(max_slots)
        self.chunk = int(chunk)
        self.clock = clock or time.perf_counter
        self.sleep = sleep or time.sleep
        self.ops: "OrderedDict[Tuple, list]" = OrderedDict()   # key -> [op, bytes, refcount]
        self.used = 0
        self.peak_used = 0
        self.batches: List[int] = []                           # active requests per chunk

    # -- memory
    def _evict_for(self, need: int) -> bool:
        for key in list(self.ops.keys()):
            if self.used + need <= self.budget:
                break
            op, nbytes, refs = self.ops[key]
            if refs == 0:
                self.be.destroy_op(op)
                self.used -= nbytes
                del self.ops[key]
        return self.used + need <= self.budget

    def _try_admit(self, r: Request):
        key = op_key(r)
        need = self.be.estimate_state_bytes(key)
        if key not in self.ops:
            need += self.be.estimate_op_bytes(key)
        if need > self.budget:
            raise ValueError(f"request {r.rid} needs {need} bytes, more than the HBM budget")
        if not self._evict_for(need):
            return None
        if key not in self.ops:
            op, nbytes = self.be.create_op(key)
            self.ops[key] = [op, nbytes, 0]
            self.used += nbytes
        self.ops.move_to_end(key)
        entry = self.ops[key]
        st, sbytes = self.be.create_state(entry[0], r)
        entry[2] += 1
        self.used += sbytes
        self.peak_used = max(self.peak_used, self.used)
        return [r, entry[0], st, sbytes, 0]        # request, op, state, bytes, steps done

    def run(self, requests: List[Request]) -> List[Record]:
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        qi = 0
        waiting: List[Request] = []
        active: List[list] = []
        records: Dict[int, Record] = {}
        t0 = self.clock()
        now = lambda: self.clock() - t0
        while qi < len(pending) or waiting or active:
            t = now()
            while qi < len(pending) and pending[qi].arrival <= t:
                waiting.append(pending[qi])
                qi += 1
            # admit in arrival order while slots and memory allow (no overtaking)
            while waiting and len(active) < self.max_slots:
                slot = self._try_admit(waiting[0])
                if slot is None:
                    break
                r = waiting.pop(0)
                records[r.rid] = Record(r.rid, r.arrival, now(), math.nan, r.nsteps, r.N, r.kind, r.dtype)
                active.append(slot)
            if not active:
                if qi < len(pending):
                    self.sleep(max(0.0, pending[qi].arrival - now()))
                    continue
                if waiting:
                    raise RuntimeError("a waiting request can never be admitted")
                break
            n = min(self.chunk, min(a[0].nsteps - a[4] for a in active))
            self.batches.append(len(active))
            self.be.step([(a[1], a[2]) for a in active], n)
            for a in active:
                a[4] += n
            t_done = now()
            still = []
            for a in active:
                r, op, st, sbytes, done = a
                if done >= r.nsteps:
                    rec = records[r.rid]
                    rec.done = t_done
                    rec.u, rec.energy = self.be.result(st)
                    self.be.destroy_state(st)
                    self.used -= sbytes
                    self.ops[op_key(r)][2] -= 1
                else:
                    still.append(a)
            active = still
        return [records[r.rid] for r in requests]

    def close(self):
        for key in list(self.ops.keys()):
            self.be.destroy_op(self.ops[key][0])
        self.ops.clear()
        self.used = 0


def summarize(records: List[Record], wall: float) -> dict:
    lat = np.array([r.latency for r in records])
    steps = sum(r.nsteps for r in records)
    return {
        "requests": len(records),
        "trajectory_steps": int(steps),
        "wall_s": wall,
        "throughput_traj_steps_per_s": steps / wall if wall > 0 else float("nan"),
        "requests_per_s": len(records) / wall if wall > 0 else float("nan"),
        "latency_p50_s": float(np.percentile(lat, 50)),
        "latency_p99_s": float(np.percentile(lat, 99)),
        "latency_max_s": float(lat.max()),
    }


def poisson_requests(n: int, rate: float, *, Ns=(100, 200, 400, 700, 1000), dense_frac: float = 0.5,
                     dtypes=("fp32", "bf16x3"), steps_range=(1000, 100000), seeds=(0, 1),
                     rng_seed: int = 0) -> List[Request]:
    """Seeded request stream: exponential inter-arrival times at `rate` per second, N
    uniform over Ns, dense with probability dense_frac (else CP of rank 2N), dtype
    uniform over dtypes, step count log-uniform over steps_range, operator seed uniform
    over seeds, one initial-state seed per request."""
    g = np.random.default_rng(rng_seed)
    t = 0.0
    out = []
    lo, hi = math.log(steps_range[0]), math.log(steps_range[1])
    for i in range(n):
        t += g.exponential(1.0 / rate)
        out.append(Request(rid=i, arrival=t, N=int(g.choice(Ns)), seed=int(g.choice(seeds)),
                           kind="dense" if g.random() < dense_frac else "cp",
                           dtype=str(g.choice(list(dtypes))),
                           nsteps=int(round(math.exp(g.uniform(lo, hi)))), u0_seed=1000 + i))
    return out
