"""Tile autotuner for the contraction kernels.

For a context and a batch size it times every launch variant of the kernels that
batch uses (rom_set_tile / rom_tile_count: 0 = single-trajectory dense stream,
1 = batched dense contraction, 2 = CP projections, 3 = CP scatter), keeps the fastest, and
caches the choice in a JSON table keyed by (kernel, N, R, B, dtype) so later contexts
of the same shape start from it (apply()).  Timing is whole BDF steps on a scratch
state, synchronized on the device, best of `reps`.
"""
from __future__ import annotations

import json
import os
import time
from typing import Dict, Optional

import numpy as np

from . import binding as rb

DEFAULT_CACHE = os.environ.get("ROM_TILE_CACHE",
                               os.path.join(os.path.dirname(os.path.abspath(__file__)), "tiles.json"))

KIND_NAMES = {0: "dense1", 1: "dense_batched", 2: "cp_proj", 3: "cp_scatter"}


def kinds_for(dense: bool, batch: int):
    if batch == 1:
        return [0] if dense else []
    return [1] if dense else [2, 3]


def key(kind: int, N: int, R: int, B: int, dtype: str) -> str:
    return f"{KIND_NAMES[kind]}:N{N}:R{R}:B{B}:{dtype}"


def load(path: str = DEFAULT_CACHE) -> Dict[str, int]:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def save(table: Dict[str, int], path: str = DEFAULT_CACHE):
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time_steps(rom: rb.Rom, u0: np.ndarray, steps: int, reps: int) -> float:
    import torch
    st = rom.state(u0)
    try:
        st.step(2)                      # warm: allocations, first launches
        best = float("inf")
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            st.step(steps)
            best = min(best, (time.perf_counter() - t) / steps)
        return best
    finally:
        st.close()


def tune(rom: rb.Rom, u0: np.ndarray, *, dense: bool, R: int = 0, steps: int = 20, reps: int = 3,
         table: Optional[Dict[str, int]] = None) -> Dict[str, dict]:
    """Tune the kernels a batch of u0.shape[0] trajectories uses; returns
    {key: {"best": idx, "seconds_per_step": [...]}} and fills `table` if given."""
    u0 = np.atleast_2d(u0)
    B = u0.shape[0]
    out = {}
    for kind in kinds_for(dense, B):
        times = []
        for v in range(rb.rom_tile_count(kind)):
            rb.rom_set_tile(rom.handle, kind, v)
            times.append(_time_steps(rom, u0, steps, reps))
        best = int(np.argmin(times))
        rb.rom_set_tile(rom.handle, kind, best)
        k = key(kind, rom.N, R, B, rom.dtype)
        out[k] = {"best": best, "seconds_per_step": times}
        if table is not None:
            table[k] = best
    return out


def apply(rom: rb.Rom, batch: int, *, dense: bool, R: int = 0, table: Optional[Dict[str, int]] = None) -> int:
    """Set the cached tile of every kernel this batch uses; returns how many were set."""
    table = load() if table is None else table
    n = 0
    for kind in kinds_for(dense, batch):
        k = key(kind, rom.N, R, batch, rom.dtype)
        if k in table:
            rb.rom_set_tile(rom.handle, kind, int(table[k]))
            n += 1
    return n


def main(argv=None):
    """Tune the named workloads' batched kernels and store the table:
    python -m paper_2311_03694_amd.tune [--out tiles.json] [--quick]"""
    import argparse

    import romsynth
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_CACHE)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--reps", type=int, default=2)
    args = ap.parse_args(argv)
    table = load(args.out)
    report = {}
    p3 = romsynth.make_config(3)
    p2 = romsynth.make_config(2, R=400)
    jobs = []
    for dt in ("fp32", "bf16", "fp64"):
        jobs.append((p3, True, dt, 1, 0))
    for B in (16, 64):
        for dt in ("fp32", "bf16"):
            jobs.append((p3, True, dt, B, 0))
            jobs.append((p3, False, dt, B, p3.R))
    for dt in ("bf16", "bf16x3", "fp32"):
        jobs.append((p2, True, dt, 256, 0))
    jobs.append((p2, False, "fp32", 256, 400))
    for p, dense, dt, B, R in jobs:
        u0 = romsynth.initial_u(p.N, range(B), cfg=3)
        rom = rb.Rom.from_problem(p, dense=dense, dtype=dt, max_batch=B)
        res = tune(rom, u0, dense=dense, R=R, steps=args.steps, reps=args.reps, table=table)
        for k, v in res.items():
            print(f"{k}: best {v['best']}  " + " ".join(f"{1e6 * x:.0f}" for x in v["seconds_per_step"]),
                  flush=True)
        report.update(res)
        rom.close()
        save(table, args.out)
    return report


if __name__ == "__main__":
    main()
