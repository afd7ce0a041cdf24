"""Continuous-batching request loop for ROM solves (host scheduler over librom.so).

A request asks for `nsteps` BDF3/EXT3 steps of one trajectory of a reduced model with
N modes, given either as a dense advection tensor or as rank-R CP factors, in one
contraction format.  The loop

  * keeps operators resident (created on first use, or all up front with `warm`, so that
    their creation stays out of request latency), shared by every request on the same
    operator and evicted least-recently-used once unreferenced, within an HBM budget;
  * runs the requests of one operator as the slots of pools: batched states whose steps
    read the operator once for all slots (a dense tensor is streamed once per step for up
    to `pool_slots` trajectories).  A request first takes its two start-up steps (BDF1,
    BDF2) alone on a one-trajectory state of its operator, then its history is written
    into a free slot of a pool that is past its own start-up (rom_state_set_slot) and it
    continues with BDF3 there, at the pool's level;
  * advances the pools with an occupied slot in rounds (continuous batching: requests
    join and leave at round boundaries while others keep running).  With a backend that
    steps pools concurrently (RomBackend: each operator's context on a stream of its own,
    every pool's steps enqueued asynchronously, then all of them awaited), each pool takes
    its own number of steps in a round, more for a pool whose step is cheaper (up to
    `max_ratio` chunks, by the backend's step-time estimate), so that the pools of small
    operators are not held to the pace of the largest one; otherwise every pool takes one
    chunk in a single rom_step_multi call;
  * retires finished requests (their slot's coefficients and energy), and failed ones: a
    non-finite trajectory ends its own request with an error and its slot is cleared;
    the other requests continue.  A request whose operator and pool cannot fit the budget
    even with nothing else resident is rejected with an error instead of stopping the run.

The device work is behind a small backend interface: RomBackend drives the C ABI; tests
use a deterministic fake backend to check the scheduling logic on the host.
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


RAMP = 2          # start-up steps a request takes alone (BDF1, BDF2) before joining a pool


# ----------------------------------------------------------------------------- backends

class RomBackend:
    """The real device: operators from the seeded generator (N modes, N skew pairs, i.e.
    CP rank 2N, 1e-7 noise, SPD stiffness, nu = dt = 5e-4), pools and start-up states
    through the C ABI."""

    def __init__(self, cfg: int = 4, eps: float = 1e-7, nu: float = 5e-4, dt: float = 5e-4, stream=None,
                 pool_slots: int = 16):
        import paper_2311_03694_amd as rg
        import romsynth
        self.rg = rg
        self.syn = romsynth
        self.cfg, self.eps, self.nu, self.dt = cfg, eps, nu, dt
        self.stream = stream
        self.pool_slots = pool_slots
        self._tensors: Dict[Tuple, np.ndarray] = {}       # host dense tensors per (N, seed)

    # -- operators
    def estimate_op_bytes(self, key) -> int:
        N, _seed, kind, dtype = key
        eb = {"fp64": 8, "fp32": 4, "bf16": 2, "bf16x3": 4}[dtype]
        Np = (N + 7) // 8 * 8
        helm = 3 * N * Np * 8
        if kind == "dense":
            return 2 * N * N * Np * eb + helm              # stream layout and the batched kernel's tiles
        R = 2 * N
        return 2 * 3 * R * Np * eb + helm                  # factors and the projection operators

    def host_tensor(self, N, seed):
        k = (N, seed)
        if k not in self._tensors:
            self._tensors[k] = self.syn.dense_from_skew_cp(N, N, self.eps, seed, self.cfg)
        return self._tensors[k]

    def create_op(self, key):
        N, seed, kind, dtype = key
        syn = self.syn
        A = syn.stiffness_spd(N, seed, self.cfg)
        if kind == "dense":
            rom = self.rg.Rom(N, self.nu, self.dt, A, C=self.host_tensor(N, seed), dtype=dtype,
                              max_batch=self.pool_slots, stream=self.stream)
        else:
            lam, Af, Bf, Cf = syn.skew_cp_factors(N, N, seed, self.cfg)
            rom = self.rg.Rom(N, self.nu, self.dt, A, lam=lam, Af=Af, Bf=Bf, Cf=Cf, dtype=dtype,
                              max_batch=self.pool_slots, stream=self.stream)
        rom.ramp = rom.state(np.zeros(N))                  # the start-up state of this operator
        return rom, rom.bytes() + rom.ramp.bytes()

    def destroy_op(self, op):
        op.ramp.close()
        op.close()

    def u0(self, r: Request) -> np.ndarray:
        return self.syn.initial_u(r.N, [r.u0_seed], cfg=self.cfg)[0]

    # -- pools
    def estimate_pool_bytes(self, key) -> int:
        N = key[0]
        Np = (N + 7) // 8 * 8
        B, Bp = self.pool_slots, (self.pool_slots + 15) // 16 * 16
        return 8 * B * N * 6 + Bp * Np * 8 * 3 + 8 * 4096 * B + (1 << 20)

    def create_pool(self, op):
        """A batched state of zero trajectories, stepped past its own start-up."""
        st = op.state(np.zeros((self.pool_slots, op.N)))
        st.step(RAMP)
        return st, st.bytes()

    def destroy_pool(self, pool):
        pool.close()

    def pool_bytes(self, pool) -> int:
        return pool.bytes()

    # -- trajectories
    def start(self, op, r: Request):
        """The request's start-up steps alone: (history for a slot, None), or (None, result)
        when the request needs no more steps, or (None, None) if they became non-finite."""
        N = op.N
        uh = np.zeros((3, 1, N))
        uh[0, 0] = self.u0(r)
        op.ramp.set(uh, np.zeros((2, 1, N)), 0)
        n = min(RAMP, r.nsteps)
        try:
            op.ramp.step(n)
        except self.rg.NonFinite:
            return None, None
        u_hist, y_hist, _ = op.ramp.get()
        if r.nsteps <= RAMP:
            E, _ = op.ramp.energy(log=False)
            return None, (u_hist[0, 0].copy(), float(E[0]))
        return (u_hist[:, 0, :].copy(), y_hist[:, 0, :].copy()), None

    def set_slot(self, pool, slot, hist, clear_health=False):
        N = pool.rom.N
        if hist is None:
            hist = (np.zeros((3, N)), np.zeros((2, N)))
        pool.set_slot(slot, hist[0], hist[1], clear_health)

    def step(self, pools: List[object], nsteps: int) -> bool:
        """Advance the pools; False if a trajectory became non-finite (the others advanced)."""
        try:
            self.rg.rom_step_multi([p.rom.handle for p in pools], [p.handle for p in pools], nsteps)
        except self.rg.NonFinite:
            return False
        return True

    def step_pools(self, items) -> List[object]:
        """Advance each pool by its own number of steps, all enqueued before any is awaited
        (pools of different operators run on their contexts' streams side by side); the
        pools in which a trajectory became non-finite."""
        for pool, n in items:
            pool.step_async(n)
        bad = []
        for pool, _ in items:
            try:
                pool.sync()
            except self.rg.NonFinite:
                bad.append(pool)
        return bad

    def estimate_step_seconds(self, key) -> float:
        """Time of one step of a pool of `key`: the operator bytes a step streams (the dense
        tensor once for all slots, or the CP factors and projection operators, and the FP64
        Helmholtz inverse) at 5 TB/s, plus 20 us of latency."""
        N, _seed, kind, dtype = key
        eb = {"fp64": 8, "fp32": 4, "bf16": 2, "bf16x3": 4}[dtype]
        nbytes = N ** 3 * eb if kind == "dense" else 3 * N * (2 * N) * eb
        return 2e-5 + (nbytes + 8 * N * N) / 5e12

    def slot_finite(self, pool) -> np.ndarray:
        E, _ = pool.energy(log=False)
        return np.isfinite(E)

    def slot_results(self, pool, slots) -> Dict[int, Tuple[np.ndarray, float]]:
        u_hist, _, _ = pool.get()
        E, _ = pool.energy(log=False)
        return {b: (u_hist[0, b].copy(), float(E[b])) for b in slots}


# ----------------------------------------------------------------------------- the loop

class _Pool:
    def __init__(self, handle, nbytes, slots):
        self.handle = handle
        self.bytes = nbytes
        self.free = list(range(slots))
        self.occupant: Dict[int, list] = {}               # slot -> active entry


class Server:
    """Admission by slots and HBM budget, continuous batching in chunks of steps."""

    def __init__(self, backend, hbm_budget: int, max_slots: int = 256, chunk: int = 256,
                 pool_slots: Optional[int] = None, clock: Optional[Callable[[], float]] = None,
                 sleep: Optional[Callable[[float], None]] = None, max_ratio: int = 32):
        self.be = backend
        self.max_ratio = int(max_ratio)
        self.budget = int(hbm_budget)
        self.max_slots = int(max_slots)
        self.chunk = int(chunk)
        self.pool_slots = int(pool_slots if pool_slots is not None else getattr(backend, "pool_slots", 16))
        self.clock = clock or time.perf_counter
        self.sleep = sleep or time.sleep
        self.ops: "OrderedDict[Tuple, list]" = OrderedDict()   # key -> [op, bytes, active requests]
        self.pools: Dict[Tuple, List[_Pool]] = {}
        self.used = 0
        self.peak_used = 0
        self.batches: List[int] = []                           # active requests per chunk
        self.create_seconds = 0.0                              # time spent creating operators

    # -- memory
    def _free_pool(self, key, pool):
        self.be.destroy_pool(pool.handle)
        self.used -= pool.bytes
        self.pools[key].remove(pool)

    def _evict_for(self, need: int) -> bool:
        # unreferenced operators (least recently used first) with their idle pools
        for key in list(self.ops.keys()):
            if self.used + need <= self.budget:
                break
            op, nbytes, refs = self.ops[key]
            if refs == 0:
                for pool in list(self.pools.get(key, [])):
                    self._free_pool(key, pool)
                self.be.destroy_op(op)
                self.used -= nbytes
                del self.ops[key]
        # idle pools of operators still in use
        for key, plist in self.pools.items():
            for pool in list(plist):
                if self.used + need <= self.budget:
                    break
                if not pool.occupant:
                    self._free_pool(key, pool)
        return self.used + need <= self.budget

    def _ensure_op(self, key) -> bool:
        if key in self.ops:
            return True
        need = self.be.estimate_op_bytes(key)
        if not self._evict_for(need):
            return False
        t = self.clock()
        op, nbytes = self.be.create_op(key)
        self.create_seconds += self.clock() - t
        self.ops[key] = [op, nbytes, 0]
        self.used += nbytes
        self.peak_used = max(self.peak_used, self.used)
        return True

    def _round(self, stepped) -> Dict[int, int]:
        """Steps of each pool in this round: the pool with the costliest step takes at most
        one chunk, a pool whose step is k times cheaper up to k chunks (at most max_ratio),
        and no pool more than its occupants' fewest remaining steps."""
        est = getattr(self.be, "estimate_step_seconds", None)
        cost = {id(p): (est(key) if est else 1.0) for key, p in stepped}
        worst = max(cost.values())
        out = {}
        for key, p in stepped:
            ratio = max(1, min(self.max_ratio, int(worst / cost[id(p)])))
            left = min(a[0].nsteps - a[4] for a in p.occupant.values())
            out[id(p)] = min(self.chunk * ratio, left)
        return out

    def warm(self, keys):
        """Create the operators of `keys` ahead of the run (those that fit the budget)."""
        for key in keys:
            self._ensure_op(key)

    def _fits_alone(self, key) -> bool:
        return self.be.estimate_op_bytes(key) + self.be.estimate_pool_bytes(key) <= self.budget

    def _slot_for(self, key):
        """A free slot for a request of `key` (creating the operator and a pool within the
        budget), or None."""
        for pool in self.pools.get(key, []):
            if pool.free:
                return pool
        if not self._ensure_op(key):
            return None
        need = self.be.estimate_pool_bytes(key)
        if not self._evict_for(need):
            return None
        if key not in self.ops:              # evicted while making room for the pool
            return None
        handle, nbytes = self.be.create_pool(self.ops[key][0])
        pool = _Pool(handle, nbytes, self.pool_slots)
        self.pools.setdefault(key, []).append(pool)
        self.used += nbytes
        self.peak_used = max(self.peak_used, self.used)
        return pool

    def run(self, requests: List[Request], progress=None, progress_every: float = 30.0) -> List[Record]:
        """progress(done, total, seconds), if given, is called about every
        `progress_every` seconds of the run."""
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        qi = 0
        waiting: List[Request] = []
        active: List[list] = []                    # [request, key, pool, slot, steps done]
        records: Dict[int, Record] = {}
        t0 = self.clock()
        now = lambda: self.clock() - t0
        ndone = [0]
        next_report = progress_every

        def finish(rec, u=None, energy=None, error=None):
            rec.done = now()
            rec.u, rec.energy, rec.error = u, energy, error
            ndone[0] += 1

        try:
            while qi < len(pending) or waiting or active:
                t = now()
                if progress is not None and t >= next_report:
                    progress(ndone[0], len(pending), t)
                    next_report = t + progress_every
                while qi < len(pending) and pending[qi].arrival <= t:
                    waiting.append(pending[qi])
                    qi += 1
                # admit in arrival order while slots and memory allow (no overtaking)
                while waiting and len(active) < self.max_slots:
                    r = waiting[0]
                    key = op_key(r)
                    if not self._fits_alone(key):
                        waiting.pop(0)
                        records[r.rid] = Record(r.rid, r.arrival, now(), math.nan, r.nsteps, r.N, r.kind, r.dtype)
                        finish(records[r.rid], error="rejected: operator and pool exceed the HBM budget")
                        continue
                    pool = self._slot_for(key)
                    if pool is None:
                        break
                    waiting.pop(0)
                    rec = Record(r.rid, r.arrival, now(), math.nan, r.nsteps, r.N, r.kind, r.dtype)
                    records[r.rid] = rec
                    self.ops.move_to_end(key)
                    hist, result = self.be.start(self.ops[key][0], r)
                    if hist is None and result is None:        # start-up steps non-finite
                        finish(rec, error="non-finite trajectory in its start-up steps")
                        continue
                    if result is not None:
                        finish(rec, u=result[0], energy=result[1])
                        continue
                    slot = pool.free.pop(0)
                    self.be.set_slot(pool.handle, slot, hist)
                    entry = [r, key, pool, slot, RAMP]
                    pool.occupant[slot] = entry
                    self.ops[key][2] += 1
                    active.append(entry)
                if not active:
                    if qi < len(pending):
                        self.sleep(max(0.0, pending[qi].arrival - now()))
                        continue
                    if waiting:
                        raise RuntimeError("a waiting request can never be admitted")
                    break
                self.batches.append(len(active))
                keyed = [(key, p) for key, plist in self.pools.items() for p in plist if p.occupant]
                stepped = [p for _, p in keyed]
                step_pools = getattr(self.be, "step_pools", None)
                if step_pools is not None:
                    counts = self._round(keyed)
                    failed = bool(step_pools([(p.handle, counts[id(p)]) for p in stepped]))
                else:
                    n = min(self.chunk, min(a[0].nsteps - a[4] for a in active))
                    counts = {id(p): n for p in stepped}
                    failed = not self.be.step([p.handle for p in stepped], n)
                for a in active:
                    a[4] += counts[id(a[2])]
                retire = []
                if failed:
                    # end the requests whose trajectories became non-finite, clear their slots
                    for pool in stepped:
                        ok = self.be.slot_finite(pool.handle)
                        bad = [b for b in pool.occupant if not ok[b]]
                        for b in bad:
                            retire.append((pool.occupant[b], "non-finite trajectory"))
                        for b in range(len(ok)):
                            if not ok[b] and b not in pool.occupant:
                                self.be.set_slot(pool.handle, b, None)
                for a in active:
                    if a[4] >= a[0].nsteps and all(a is not x for x, _ in retire):
                        retire.append((a, None))
                by_pool: Dict[int, list] = {}
                for a, err in retire:
                    by_pool.setdefault(id(a[2]), []).append((a, err))
                for items in by_pool.values():
                    pool = items[0][0][2]
                    res = self.be.slot_results(pool.handle, [a[3] for a, err in items if err is None])
                    for q, (a, err) in enumerate(items):
                        r, key, _, slot, _ = a
                        rec = records[r.rid]
                        if err is None:
                            finish(rec, u=res[slot][0], energy=res[slot][1])
                        else:
                            finish(rec, error=err)
                        last = q == len(items) - 1
                        self.be.set_slot(pool.handle, slot, None, clear_health=failed and last)
                        del pool.occupant[slot]
                        pool.free.append(slot)
                        self.ops[key][2] -= 1
                gone = {id(a) for a, _ in retire}
                active = [a for a in active if id(a) not in gone]
                # pools grow their energy logs with the steps: re-read their sizes
                for pool in stepped:
                    nb = self.be.pool_bytes(pool.handle)
                    self.used += nb - pool.bytes
                    pool.bytes = nb
                self.peak_used = max(self.peak_used, self.used)
        finally:
            t_end = now()
            for a in active:
                rec = records[a[0].rid]
                if rec.error is None and math.isnan(rec.done):
                    rec.done, rec.error = t_end, "aborted"
            for r in waiting + pending[qi:]:
                if r.rid not in records:
                    records[r.rid] = Record(r.rid, r.arrival, t_end, t_end, r.nsteps, r.N, r.kind, r.dtype,
                                            error="not admitted")
        return [records[r.rid] for r in requests]

    def close(self):
        for key, plist in self.pools.items():
            for pool in plist:
                self.be.destroy_pool(pool.handle)
        self.pools.clear()
        for key in list(self.ops.keys()):
            self.be.destroy_op(self.ops[key][0])
        self.ops.clear()
        self.used = 0


def summarize(records: List[Record], wall: float) -> dict:
    ok = [r for r in records if r.error is None]
    lat = np.array([r.latency for r in ok]) if ok else np.array([math.nan])
    steps = sum(r.nsteps for r in ok)
    return {
        "requests": len(records),
        "completed": len(ok),
        "failed": len(records) - len(ok),
        "trajectory_steps": int(steps),
        "wall_s": wall,
        "throughput_traj_steps_per_s": steps / wall if wall > 0 else float("nan"),
        "requests_per_s": len(ok) / wall if wall > 0 else float("nan"),
        "latency_p50_s": float(np.percentile(lat, 50)),
        "latency_p99_s": float(np.percentile(lat, 99)),
        "latency_max_s": float(np.max(lat)),
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


def at_rate(requests: List[Request], rate: float, rng_seed: int = 0) -> List[Request]:
    """The same requests with fresh exponential inter-arrival times at `rate` per second
    (arrival order kept)."""
    g = np.random.default_rng(rng_seed)
    t = 0.0
    out = []
    for r in requests:
        t += g.exponential(1.0 / rate)
        out.append(dataclasses.replace(r, arrival=t))
    return out
