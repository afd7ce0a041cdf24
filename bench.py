#!/usr/bin/env python3
"""Benchmark: online ROM steps on one MI355X, CP-ROM vs dense G-ROM at N = 1000.

Headline workload (synthetic, seeded): N = 1000 modes, dense advection tensor built
from a skew-preserving CP of rank 2000 (1000 skew pairs, weights 1/p, unit Gaussian
factors) plus 1e-7 skew Gaussian noise; stiffness A = diag(k^2) plus an SPD perturbation
of spectral norm 0.1; nu = dt = 5e-4; BDF3/EXT3 with the 1-2-3 start-up ramp.  The
CP-ROM uses the rank-2000 factors, the G-ROM the dense tensor, both with FP32
contractions and FP64 state updates, one trajectory.

One timed step = one BDF3/EXT3 step of the trajectory batch (contraction, FP64 right-hand
side, FP64 Helmholtz solve, energy, health flag).  `value` is CP-ROM
trajectory-steps/s; the dense G-ROM is timed the same way in the same run.  Inputs sit
in HBM before a timed region opens; each region is bracketed by device
synchronization and timed with HIP events on the library's stream.

Also in the one JSON line:
  dense / speedup_cp_vs_dense   the G-ROM beside it
  roofline      dense contraction kernel (HBM-bound): algorithmic bytes N^3*4 per launch
                over its event-timed average duration, against 8 TB/s
  roofline_cp   one CP step through the per-step kernels (resident runs off): N R + 1.5 R N
                operator words and the FP64 Hinv_3 (8 N^2 bytes) against 8 TB/s
  resident      the headline's own path: the CP step with its operator resident in LDS
                (k_cp_resident), its step time and the streaming bandwidth it equals
  cp_evaluation CP projections + Hadamard-scatter alone (2.5NR*4 bytes per launch in the
                pair form of skew-paired factors, 3NR*4 in the general form)
  cp_general    the same CP-ROM with the general-form projections (kernel knob 4 = 0)
  batched       N = 1000 with B = 16 and 64 trajectories (MFMA kernels), FP32 and BF16
  config2       N = 400, B = 256, the dense Khatri-Rao MFMA GEMM (BF16, BF16x3, FP32)
                and CP rank 400, with TFLOP/s against the dense MFMA peaks
  svd           the SVD-ROM (Sec. 4.4) at N = 1000 with SVD ranks 100 and 250 (compression
                N/R = 10 and 4), FP32, one trajectory: steps/s and the streaming bandwidth
  full          the full form of the reduced system (dense SPD mass matrix, zeroth-mode
                terms) at the headline size, CP rank 2000 FP32, against the plain step
  als           CP-ALS sweeps (rom_cp_als) at N = 200, R = 400, FP64: ms per sweep; ALS-skew
                (rom_cp_als_skew) with 200 column pairs and 3 subiterations
  multi         uneven N and mixed formats: CP states at N = 100..1000 in FP32, BF16X3 and
                BF16 with SPD or diagonal stiffness, a dense state and a batch of 16, stepped
                together (rom_step_multi) and one after the other
  serving       a config-4 request stream (a stated fraction, shorter step counts by default)
                through the continuous-batching loop: saturation throughput, then p50/p99
                latency at 0.5, 0.8 and 0.95 of the saturation request rate
  model_error   the CP-ROM's distance from the G-ROM (Sec. 4.1: errors relative to the
                G-ROM) at CP ranks 500, 1000, 2000 over 1000 steps, GPU FP32 trajectories
  rel_err       every section: sampled GPU trajectories against the FP64 oracle of the
                same operator (the oracle leg runs after all GPU timing)
  cpu_baseline  the FP64 oracle (plain C) on a bounded sample of steps, on all host cores
                of one GPU's host share (results identical to one thread) and on one
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ROM steps/s×trajectories at N=1000: CP vs dense G-ROM, rel err ≤1e-5 vs FP64"
HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"bf16": 2500.0, "bf16x3": 2500.0, "fp32": 157.3, "fp64": 78.6}
ELEM_BYTES = {"fp64": 8, "fp32": 4, "bf16": 2, "bf16x3": 4}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--dtype", default="fp32", choices=["fp32", "fp64", "bf16", "bf16x3"])
    ap.add_argument("--R", type=int, default=2000)
    ap.add_argument("--dense-steps", type=int, default=None,
                    help="timed steps of the dense G-ROM (default: min(steps, 2000))")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="target length of the oracle sample (CPU baseline)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle legs (profiling runs)")
    ap.add_argument("--no-extra", action="store_true", help="headline only (no batched/config2/serving)")
    ap.add_argument("--section", default="all", choices=["all", "headline", "batched", "config2", "svd", "full", "als", "multi", "serving"],
                    help="run one section only (profiling); the JSON line then holds that section")
    ap.add_argument("--kernel-reps", type=int, default=50)
    ap.add_argument("--serving-requests", type=int, default=60,
                    help="requests of the serving stream (config 4 has 10,000)")
    ap.add_argument("--serving-max-steps", type=int, default=10000,
                    help="largest step count of a serving request (config 4: 100,000)")
    ap.add_argument("--no-resident", action="store_true",
                    help="step CP states through the per-step kernels only (counter runs)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain 1 GiB device copy (HBM counter calibration)")
    return ap.parse_args()


CSRC = os.path.join(ROOT, "paper_2311_03694_amd", "csrc")
# the sources each profiled kernel is compiled from (its counter record is valid only
# while their combined hash is unchanged)
KERNEL_SOURCES = {
    "dense_gemv": ["k_dense1.hip", "kdot.h", "kcommon.h", "rom_dev.h"],
    "kr": ["k_kr.hip", "kmfma.h", "kcommon.h", "rom_dev.h"],
}


def sources_sha(kernel):
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[kernel]:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _traffic(name, kernel):
    """HBM bytes per launch from committed rocprofv3 counter runs, if the kernel's
    sources have not changed since they were taken; else None."""
    path = os.path.join(ROOT, "profiles", f"{name}_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("sources_sha256") != sources_sha(kernel):
        return None
    return rec.get("hbm_bytes_per_launch")


class Timer:
    """Events on the library's stream around enqueued work, bracketed by device syncs."""

    def __init__(self, torch, stream):
        self.torch, self.stream = torch, stream

    def __call__(self, fn):
        torch = self.torch
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(self.stream)
        fn()
        e1.record(self.stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3


ORC_THREADS = max(1, min(16, os.cpu_count() or 1))     # the host share of one GPU


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


class Checks:
    """GPU results kept for the oracle leg: each entry names a section, the operator, the
    initial coefficients, the number of steps and the GPU's final coefficients (and
    energy log)."""

    def __init__(self):
        self.items = []
        self.fns = []

    def add_fn(self, section, fn):
        """A check the oracle leg evaluates by calling fn(oracle) -> {label: errors}."""
        self.fns.append((section, fn))

    def add(self, section, label, prob, ops, u0, nsteps, u_gpu, E_gpu=None, full=None, dtype="fp32"):
        self.items.append(dict(section=section, label=label, N=prob[0], nu=prob[1], dt=prob[2], A=prob[3],
                               ops=ops, u0=np.array(u0, dtype=np.float64), nsteps=int(nsteps),
                               u_gpu=np.array(u_gpu, dtype=np.float64),
                               E_gpu=None if E_gpu is None else np.array(E_gpu, dtype=np.float64),
                               full=full, dtype=dtype))


TOL = {"fp64": 1e-12, "fp32": 1e-5, "bf16x3": 1e-5, "bf16": 1e-3}


def run_checks(checks, orc, log):
    """The oracle leg of the accuracy report: {section: {label: errors}}.  Oracle runs of
    the same operator, start and length are shared."""
    out = {}
    cache = {}
    for c in checks.items:
        key = (id(c["ops"]), id(c["full"]), c["u0"].tobytes(), c["nsteps"])
        if key not in cache:
            t = time.perf_counter()
            with orc.threads(ORC_THREADS):
                r = orc.run(c["N"], c["nu"], c["dt"], c["A"], c["nsteps"], u0=c["u0"], **c["ops"], **(c["full"] or {}))
            cache[key] = r
            log(f"oracle: {c['section']} {c['label']} ({c['nsteps']} steps, {time.perf_counter() - t:.1f}s)")
        r = cache[key]
        ref = r["u_hist"][0]
        e = dict(steps=c["nsteps"], traj=float(np.linalg.norm(c["u_gpu"] - ref) / np.linalg.norm(ref)),
                 tol=TOL[c["dtype"]])
        if c["E_gpu"] is not None:
            e["energy"] = float(np.max(np.abs(c["E_gpu"] - r["E"]) / r["E"]))
        out.setdefault(c["section"], {})[c["label"]] = e
    for section, fn in checks.fns:
        out.setdefault(section, {}).update(fn(orc))
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: this library has no multi-GPU path "
              f"(requested --gpus {args.gpus}); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2311_03694_amd as rg
    import romsynth
    from paper_2311_03694_amd import tune

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    timer = Timer(torch, stream)
    N, R, dt = 1000, args.R, args.dtype
    K, W = args.steps, args.warmup
    Kd = args.dense_steps if args.dense_steps is not None else min(K, 2000)
    log = lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True)

    t0 = time.time()
    log(f"generating N={N} workload")
    p = romsynth.make_config(3, R=R, batch=1, dense=args.section in ("all", "headline", "batched"))
    log(f"generated in {time.time() - t0:.1f}s")

    if args.calib_copy:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        torch.cuda.synchronize()
        b2 = a.clone()
        torch.cuda.synchronize()
        log(f"calibration copy of {a.numel() * 4} bytes done")
        del a, b2

    def make(dense, dtype=dt, batch=1):
        rom = rg.Rom.from_problem(p, dense=dense, dtype=dtype, max_batch=batch, stream=stream)
        if args.no_resident and not dense:
            rom.set_tile(5, 0)
        return rom

    def step_rate(rom, u0, nsteps, warm):
        s = rom.state(u0)
        s.prepare(warm + nsteps)    # capture the timed call's graphs (runs no step)
        s.prepare(nsteps)
        s.step(warm)
        t = timer(lambda: s.step_async(nsteps))
        s.sync()
        return s, t

    def kernel_avg(rom, u, reps):
        """Average duration of the contraction kernels alone: HIP events around `reps`
        back-to-back launches on the library's stream (rom_nonlinear_timed)."""
        ud = torch.tensor(np.atleast_2d(u), dtype=torch.float64, device=dev)
        yd = torch.empty_like(ud)
        B = ud.shape[0]
        rg.rom_nonlinear(rom.handle, B, ud, yd)
        torch.cuda.synchronize()
        return rg.rom_nonlinear_timed(rom.handle, B, ud, yd, reps) * 1e-6

    sec = args.section
    checks = Checks()
    prob = (N, p.nu, p.dt, p.A)
    ops_dense = dict(C=p.C)
    ops_cp = dict(lam=p.lam, Af=p.Af, Bf=p.Bf, Cf=p.Cf)
    result = {"metric": METRIC, "value": None, "unit": "trajectory-steps/s", "n_gpus": 1,
              "section": sec}
    if sec in ("all", "headline"):
        # ---------------- headline: CP-ROM and dense G-ROM, one trajectory
        log("CP-ROM")
        rom_cp = make(False)
        cp_form = rg.rom_query(rom_cp.handle, None, 7)       # skew column pairs in use
        s_cp, t_cp = step_rate(rom_cp, p.u0, K, W)
        cp_kernel = kernel_avg(rom_cp, p.u0, args.kernel_reps * 10)
        log(f"CP {K} steps in {t_cp:.3f}s (pair layout {cp_form})")
        t_gen = None
        if cp_form:
            rg.rom_set_tile(rom_cp.handle, 4, 0)
            s_gen, t_gen = step_rate(rom_cp, p.u0, K, W)
            s_gen.close()
            rg.rom_set_tile(rom_cp.handle, 4, -1)
            log(f"CP general form {K} steps in {t_gen:.3f}s")
        # the same steps through the per-step kernels (resident runs off): the streaming
        # path that the HBM roofline of a CP step applies to
        res_blocks = s_cp.resident_blocks
        rg.rom_set_tile(rom_cp.handle, 5, 0)
        s_ps, t_ps = step_rate(rom_cp, p.u0, K, W)
        s_ps.close()
        rg.rom_set_tile(rom_cp.handle, 5, 0 if args.no_resident else -1)
        log(f"CP per-step kernels {K} steps in {t_ps:.3f}s (resident blocks {res_blocks})")
        log("dense G-ROM")
        rom_d = make(True)
        s_d, t_d = step_rate(rom_d, p.u0, Kd, min(W, 20))
        d_kernel = kernel_avg(rom_d, p.u0, args.kernel_reps)
        log(f"dense {Kd} steps in {t_d:.3f}s")

        es = ELEM_BYTES[dt]
        cp_rate = K / t_cp
        d_rate = Kd / t_d
        d_bytes = float(N) ** 3 * es
        # one CP step with a dense stiffness: the scatter reads Af [N][R]; the Helmholtz
        # kernel reads Hinv_k [N][N] (FP64) and the projection operator [B|C]^T Hinv_k,
        # 1.5R rows in the pair form (2R in the general form) of N values
        cp_step_bytes = N * R * es + 8.0 * N * N + (1.5 if cp_form else 2.0) * R * N * es
        cp_bytes = (2.5 if cp_form else 3.0) * N * R * es
        s_chk = rom_d.state(p.u0)
        s_chk.step(3)
        checks.add("headline", "dense", prob, ops_dense, p.u0[0], 3, s_chk.u(), E_gpu=s_chk.energy()[1][:, 0], dtype=dt)
        s_chk.close()
        # the CP-ROM's distance from the G-ROM (Sec. 4.1): GPU trajectories, u every 100th
        # level over 1000 steps, CP ranks 500, 1000, 2000 against the dense tensor
        log("model error: CP ranks 500, 1000, 2000 against the dense G-ROM, 1000 steps")
        marks = list(range(100, 1001, 100))

        def traj_marks(rom):
            st = rom.state(p.u0)
            out, done = [], 0
            for m in marks:
                st.step(m - done)
                done = m
                out.append(st.u()[0].copy())
            st.close()
            return np.stack(out)

        U_dense = traj_marks(rom_d)
        model = {}
        for Rm in (500, 1000, 2000):
            ops_m = dict(zip(("lam", "Af", "Bf", "Cf"), romsynth.truncate_cp(p.lam, p.Af, p.Bf, p.Cf, Rm)))
            rom_m = rg.Rom(N, p.nu, p.dt, p.A, **ops_m, dtype=dt, stream=stream)
            if args.no_resident:
                rom_m.set_tile(5, 0)
            Um = traj_marks(rom_m)
            rom_m.close()
            model[f"R{Rm}"] = {"max_rel_to_grom": float(np.max(np.linalg.norm(Um - U_dense, axis=1) /
                                                                np.linalg.norm(U_dense, axis=1))),
                               "compression_N2_over_3R": N * N / (3.0 * Rm),
                               "compression_skew_2N2_over_3R": 2.0 * N * N / (3.0 * Rm)}
        result = {
            "metric": METRIC,
            "value": cp_rate,
            "unit": "trajectory-steps/s",
            "n_gpus": 1,
            "steps": K,
            "warmup": W,
            "ms_per_step": t_cp / K * 1e3,
            "higher_is_better": True,
            "scaling": "weak",
            "vs_baseline": None,
            "dtype": dt,
            "data": "synthetic (seeded skew-CP tensor, N=1000, rank 2000, eps 1e-7, SPD stiffness)",
            "config": {"workload": f"N=1000 ROM, CP rank {R} vs dense G-ROM, BDF3/EXT3, one trajectory",
                       "N": N, "R": R, "batch": 1, "nu": p.nu, "dt": p.dt, "stiffness": "diag(k^2)+SPD(0.1)"},
            "dense": {"value": d_rate, "unit": "trajectory-steps/s", "steps": Kd, "ms_per_step": t_d / Kd * 1e3},
            "speedup_cp_vs_dense": cp_rate / d_rate,
            "cp_form": "pair form of skew column pairs (Sec. 3.3)" if cp_form else "general",
            "cp_general": None if t_gen is None else {"value": K / t_gen, "unit": "trajectory-steps/s",
                                                      "ms_per_step": t_gen / K * 1e3},
            "roofline": {"bound": "hbm", "kernel": "k_dense_gemv (dense contraction, one trajectory)",
                         "achieved": d_bytes / d_kernel / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": d_bytes / d_kernel / 1e9 / HBM_PEAK_GBS,
                         "traffic": _traffic(f"dense_gemv_n{N}_{dt}", "dense_gemv"),
                         "avg_launch_us": d_kernel * 1e6, "algorithmic_bytes": d_bytes},
            "roofline_cp": {"bound": "hbm", "kernel": "one CP step through the per-step kernels: k_cp_scatter1 "
                                                      "(right-hand side) + k_helm_proj (Helmholtz apply and next "
                                                      "projections)" + (", pair form" if cp_form else ""),
                            "achieved": cp_step_bytes / (t_ps / K) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": cp_step_bytes / (t_ps / K) / 1e9 / HBM_PEAK_GBS,
                            "avg_step_us": t_ps / K * 1e6, "algorithmic_bytes": cp_step_bytes,
                            "value": K / t_ps},
            "resident": {"kernel": "k_cp_resident (operator rows in LDS for a run of up to 512 steps)",
                         "blocks": res_blocks, "avg_step_us": t_cp / K * 1e6,
                         "hbm_operator_bytes_per_step": 0,
                         "equivalent_stream_GBps": cp_step_bytes / (t_cp / K) / 1e9,
                         "equivalent_stream_frac": cp_step_bytes / (t_cp / K) / 1e9 / HBM_PEAK_GBS,
                         "speedup_vs_per_step": t_ps / t_cp,
                         "note": "the step is bound by its two exchanges between blocks (x: N FP64, w: Rp words), "
                                 "not by memory bandwidth; equivalent_stream is the bandwidth a streaming step "
                                 "would need to match it"},
            "cp_evaluation": {"kernel": "k_cp_proj1 + k_cp_scatter1 (rom_nonlinear)", "avg_launch_us": cp_kernel * 1e6,
                              "algorithmic_bytes": cp_bytes, "hbm_frac": cp_bytes / cp_kernel / 1e9 / HBM_PEAK_GBS},
            "model_error": dict(model, steps=1000, note="max over every 100th level of |u_cp - u_dense| / "
                                                        "|u_dense|, FP32 GPU trajectories"),
        }
        s_cp.close()
        s_d.close()


    if sec == "headline":
        args.no_extra = True
    if not args.no_extra:
        tiles = tune.load()
    if not args.no_extra and sec in ("all", "batched"):
        # ---------------- batched trajectories at N = 1000 (MFMA kernels)
        batched = {}
        for B in (16, 64):
            u0 = romsynth.initial_u(N, range(B), cfg=3)
            for bdt in ("fp32", "bf16"):
                entry = {}
                for dense in (True, False):
                    rom = make(dense, bdt, B)
                    tune.apply(rom, B, dense=dense, R=0 if dense else R, table=tiles)
                    steps = 100 if dense else 1000
                    s, t = step_rate(rom, u0, steps, 5)
                    name = "dense" if dense else "cp"
                    entry[name] = {"traj_steps_per_s": steps * B / t, "us_per_step": t / steps * 1e6}
                    s.close()
                    # accuracy: a fresh batch, sampled trajectories against the oracle
                    nchk = 3 if dense else 200
                    s = rom.state(u0)
                    s.step(nchk)
                    ug = s.get()[0][0]
                    ops = ops_dense if dense else ops_cp
                    for b in (0, B - 1):
                        checks.add("batched", f"B{B}_{bdt}_{name}_traj{b}", prob, ops, u0[b], nchk, ug[b], dtype=bdt)
                    if dense:
                        tk = kernel_avg(rom, u0, 10)
                        fl = 2.0 * N ** 3 * B
                        entry[name]["contraction_us"] = tk * 1e6
                        entry[name]["tflops"] = fl / tk / 1e12
                        entry[name]["mfma_frac"] = fl / tk / 1e12 / MFMA_PEAK_TFLOPS[bdt]
                        entry[name]["hbm_frac"] = N ** 3 * ELEM_BYTES[bdt] / tk / 1e9 / HBM_PEAK_GBS
                    s.close()
                    rom.close()
                entry["speedup_cp_vs_dense"] = entry["cp"]["traj_steps_per_s"] / entry["dense"]["traj_steps_per_s"]
                batched[f"B{B}_{bdt}"] = entry
                log(f"batched B={B} {bdt}: dense {entry['dense']['traj_steps_per_s']:.0f} "
                    f"cp {entry['cp']['traj_steps_per_s']:.0f} traj-steps/s")
        result["batched"] = batched

    if not args.no_extra and sec in ("all", "config2"):
        # ---------------- config 2: N = 400, B = 256
        log("config 2 (N=400, B=256)")
        p2 = romsynth.make_config(2, R=400)
        prob2 = (p2.N, p2.nu, p2.dt, p2.A)
        ops2d = dict(C=p2.C)
        ops2c = dict(lam=p2.lam, Af=p2.Af, Bf=p2.Bf, Cf=p2.Cf)
        c2 = {}
        for bdt in ("bf16", "bf16x3", "fp32"):
            rom = rg.Rom.from_problem(p2, dense=True, dtype=bdt, max_batch=256, stream=stream)
            tune.apply(rom, 256, dense=True, table=tiles)
            s, t = step_rate(rom, p2.u0, 50, 5)
            tk = kernel_avg(rom, p2.u0, 10)
            fl = 2.0 * 400 ** 3 * 256 * (3 if bdt == "bf16x3" else 1)
            c2[f"dense_{bdt}"] = {"traj_steps_per_s": 50 * 256 / t, "us_per_step": t / 50 * 1e6,
                                  "contraction_us": tk * 1e6, "tflops": fl / tk / 1e12,
                                  "mfma_frac": fl / tk / 1e12 / MFMA_PEAK_TFLOPS[bdt]}
            s.close()
            s = rom.state(p2.u0)
            s.step(20)
            ug = s.get()[0][0]
            for b in (0, 255):
                checks.add("config2", f"dense_{bdt}_traj{b}", prob2, ops2d, p2.u0[b], 20, ug[b], dtype=bdt)
            s.close()
            rom.close()
        rom = rg.Rom.from_problem(p2, dense=False, dtype="fp32", max_batch=256, stream=stream)
        tune.apply(rom, 256, dense=False, R=400, table=tiles)
        s, t = step_rate(rom, p2.u0, 500, 20)
        c2["cp_fp32_R400"] = {"traj_steps_per_s": 500 * 256 / t, "us_per_step": t / 500 * 1e6}
        ug = s.get()[0][0]
        for b in (0, 255):
            checks.add("config2", f"cp_fp32_R400_traj{b}", prob2, ops2c, p2.u0[b], 520, ug[b])
        s.close()
        rom.close()
        result["config2"] = c2
        result["roofline_mfma"] = {"bound": "mfma", "kernel": "k_kr (dense Khatri-Rao, X in registers, N=400, B=256, BF16)",
                                   "achieved": c2["dense_bf16"]["tflops"], "peak": MFMA_PEAK_TFLOPS["bf16"],
                                   "unit": "TFLOP/s", "frac": c2["dense_bf16"]["mfma_frac"],
                                   "avg_launch_us": c2["dense_bf16"]["contraction_us"],
                                   "algorithmic_flops": 2.0 * 400 ** 3 * 256,
                                   "traffic": _traffic("kr_dense_n400_b256_bf16", "kr")}

    if not args.no_extra and sec in ("all", "svd"):
        # ---------------- SVD-ROM: U, sigma, V of the mode-3 matricization (seeded random
        # factors of the right shapes; the timing does not depend on their values)
        svd = {}
        A3 = p.A
        for Rs in (100, 250):
            rng = np.random.default_rng(Rs)
            U = rng.standard_normal((N, Rs)) / np.sqrt(N)
            sig = 1.0 / (1.0 + np.arange(Rs))
            V = rng.standard_normal((N, N, Rs)) / N
            rom_s = rg.Rom(N, p.nu, p.dt, A3, svd=(U, sig, V), dtype="fp32", max_batch=1, stream=stream)
            steps = 2000
            s_s, t_s = step_rate(rom_s, p.u0, steps, 20)
            tk = kernel_avg(rom_s, p.u0, 10)
            vbytes = float(N) * N * Rs * 4
            svd[f"R{Rs}"] = {"traj_steps_per_s": steps / t_s, "us_per_step": t_s / steps * 1e6,
                             "contraction_us": tk * 1e6, "compression_N_over_R": N / Rs,
                             "hbm_frac": vbytes / tk / 1e9 / HBM_PEAK_GBS}
            log(f"svd R={Rs}: {steps / t_s:.0f} steps/s, contraction {tk * 1e6:.1f} us")
            s_s.close()
            s_s = rom_s.state(p.u0)
            s_s.step(5)
            checks.add("svd", f"R{Rs}", prob, dict(U=U, sigma=sig, V=V), p.u0[0], 5, s_s.u())
            s_s.close()
            rom_s.close()
        result["svd"] = svd

    if not args.no_extra and sec in ("all", "full"):
        # ---------------- full form of the reduced system at the headline size: dense SPD
        # mass matrix and zeroth-mode terms beside the CP rank-2000 contraction; plain and
        # full contexts stepped in alternation on the same stream
        C1, C2, c0, a0 = romsynth.zeroth_terms(N, seed=1, cfg=3, scale=0.1)
        full_terms = dict(M=romsynth.mass_spd(N, seed=2, cfg=3, norm=0.1), C1=C1, C2=C2, c0=c0, a0=a0)
        core = dict(lam=p.lam, Af=p.Af, Bf=p.Bf, Cf=p.Cf)
        rom_f = rg.Rom(N, p.nu, p.dt, p.A, **core, full=full_terms, dtype="fp32", max_batch=1, stream=stream)
        rom_p = rg.Rom(N, p.nu, p.dt, p.A, **core, dtype="fp32", max_batch=1, stream=stream)
        for r in (rom_f, rom_p):
            tune.apply(r, 1, dense=False, R=R, table=tiles)
        rom_p.set_tile(5, 0)       # the plain step through the same per-step kernels
        s_f, s_p = rom_f.state(p.u0), rom_p.state(p.u0)
        s_f.step(200)
        s_p.step(200)
        nf, tf, tp = 4000, [], []
        for _ in range(3):
            tf.append(timer(lambda: s_f.step_async(nf)))
            s_f.sync()
            tp.append(timer(lambda: s_p.step_async(nf)))
            s_p.sync()
        t_f, t_p = min(tf) / nf, min(tp) / nf
        Np = (N + 7) // 8 * 8
        result["full"] = {"traj_steps_per_s": 1.0 / t_f, "us_per_step": t_f * 1e6, "plain_us_per_step": t_p * 1e6,
                          "plain_path": "per-step kernels (resident runs off), the full form's own path",
                          "extra_us_per_step": (t_f - t_p) * 1e6, "terms_bytes_per_step": 16.0 * N * Np,
                          "config": "N=1000, CP rank 2000 FP32, SPD stiffness, dense SPD mass matrix, "
                                    "zeroth-mode C1, C2, c0, a0 (FP64)"}
        log(f"full form: {1.0 / t_f:.0f} steps/s ({t_f * 1e6:.2f} us/step; plain {t_p * 1e6:.2f})")
        for x in (s_f, s_p):
            x.close()
        s_f = rom_f.state(p.u0)
        s_f.step(200)
        checks.add("full", "B1", prob, core, p.u0[0], 200, s_f.u(), E_gpu=s_f.energy()[1][:, 0], full=full_terms)
        for x in (s_f, rom_f, rom_p):
            x.close()
        # 64 trajectories: the terms as one FP64 product X G^T per step
        Bf = 64
        u0b = romsynth.initial_u(N, range(Bf), cfg=3)
        rom_f = rg.Rom(N, p.nu, p.dt, p.A, **core, full=full_terms, dtype="fp32", max_batch=Bf, stream=stream)
        rom_p = rg.Rom(N, p.nu, p.dt, p.A, **core, dtype="fp32", max_batch=Bf, stream=stream)
        for r in (rom_f, rom_p):
            tune.apply(r, Bf, dense=False, R=R, table=tiles)
        s_f, s_p = rom_f.state(u0b), rom_p.state(u0b)
        s_f.step(20)
        s_p.step(20)
        nb, tf, tp = 1000, [], []
        for _ in range(3):
            tf.append(timer(lambda: s_f.step_async(nb)))
            s_f.sync()
            tp.append(timer(lambda: s_p.step_async(nb)))
            s_p.sync()
        t_f, t_p = min(tf) / nb, min(tp) / nb
        result["full"]["B64"] = {"traj_steps_per_s": Bf / t_f, "us_per_step": t_f * 1e6,
                                 "plain_us_per_step": t_p * 1e6}
        log(f"full form B={Bf}: {Bf / t_f:.0f} traj-steps/s ({t_f * 1e6:.2f} us/step; plain {t_p * 1e6:.2f})")
        for x in (s_f, s_p):
            x.close()
        s_f = rom_f.state(u0b)
        s_f.step(50)
        ug = s_f.get()[0][0]
        for b in (0, Bf - 1):
            checks.add("full", f"B{Bf}_traj{b}", prob, core, u0b[b], 50, ug[b], full=full_terms)
        for x in (s_f, rom_f, rom_p):
            x.close()

    if not args.no_extra and sec in ("all", "als"):
        # ---------------- CP-ALS (offline fit of the CP factors): N = 200, R = 400, FP64,
        # seeded random tensor and initial factors (the timing does not depend on values)
        Na, Ra = 200, 400
        rng = np.random.default_rng(2)
        Xd = torch.tensor(rng.standard_normal((Na, Na, Na)), dtype=torch.float64, device=dev)
        Fd = [torch.tensor(rng.standard_normal((Na, Ra)), dtype=torch.float64, device=dev) for _ in range(3)]
        # a call allocates its workspace, unfolds the tensor and captures one sweep into a
        # graph before replaying it: per sweep = the difference of a 12-sweep and a 2-sweep
        # call over 10; the rest of a call is its set-up
        rg.rom_cp_als(Na, Ra, Xd, *Fd, 1, stream=stream)

        def per_sweep(call):
            t2, t12 = timer(lambda: call(2)), timer(lambda: call(12))
            per = (t12 - t2) / 10
            return per, t2 - 2 * per

        t_als, set_als = per_sweep(lambda k: rg.rom_cp_als(Na, Ra, Xd, *Fd, k, stream=stream))
        fl = 3 * 2.0 * Na ** 3 * Ra
        result["als"] = {"N": Na, "R": Ra, "ms_per_sweep": t_als * 1e3, "call_setup_ms": set_als * 1e3,
                         "mttkrp_flops_per_sweep": fl, "sweep_tflops": fl / t_als / 1e12}
        log(f"cp-als N={Na} R={Ra}: {t_als * 1e3:.2f} ms per sweep, {set_als * 1e3:.2f} ms set-up per call")
        # ALS-skew at the same size: P = 200 column pairs (R = 400), 3 subiterations per
        # sweep (one tied solve and three momentum subiterations), on a skew tensor
        Pa, sub = Ra // 2, 3
        Xs = Xd - Xd.permute(2, 1, 0)
        Fs = [torch.tensor(rng.standard_normal((Na, Pa)), dtype=torch.float64, device=dev) for _ in range(3)]
        rg.rom_cp_als_skew(Na, Pa, Xs, *Fs, 1, sub, stream=stream)
        t_sk, set_sk = per_sweep(lambda k: rg.rom_cp_als_skew(Na, Pa, Xs, *Fs, k, sub, stream=stream))
        fl_sk = (1 + sub - 1) * 2.0 * Na ** 3 * Ra
        result["als"]["skew"] = {"P": Pa, "subiters": sub, "momentum": 0.5, "ms_per_sweep": t_sk * 1e3,
                                 "call_setup_ms": set_sk * 1e3, "tensor_product_flops_per_sweep": fl_sk}
        log(f"als-skew N={Na} P={Pa} subiters={sub}: {t_sk * 1e3:.2f} ms per sweep, {set_sk * 1e3:.2f} ms set-up "
            f"per call")
        del Xd, Fd, Xs, Fs
        # accuracy (oracle leg): 2 sweeps of each at N = 40, R = 24 from seeded factors
        rng = np.random.default_rng(4)
        Xc = rng.standard_normal((40, 40, 40))
        Xc = Xc - Xc.transpose(2, 1, 0)
        F0 = [rng.standard_normal((40, 24)) for _ in range(3)]
        S0 = [rng.standard_normal((40, 12)) for _ in range(3)]
        Xcd = torch.tensor(Xc, dtype=torch.float64, device=dev)
        Fg = [torch.tensor(a, dtype=torch.float64, device=dev) for a in F0]
        Sg = [torch.tensor(a, dtype=torch.float64, device=dev) for a in S0]
        rg.rom_cp_als(40, 24, Xcd, *Fg, 2, stream=stream)
        rg.rom_cp_als_skew(40, 12, Xcd, *Sg, 2, sub, stream=stream)
        Fg = [a.cpu().numpy() for a in Fg]
        Sg = [a.cpu().numpy() for a in Sg]

        def als_err(orc, X=Xc, F0=F0, S0=S0, Fg=Fg, Sg=Sg):
            F, _ = orc.als.cp_als(X, *F0, 2)
            Fs_, _ = orc.als.als_skew(X, *S0, sweeps=2, subiters=sub)
            rel = lambda G, R_: max(float(np.max(np.abs(g - r)) / np.max(np.abs(r))) for g, r in zip(G, R_))
            return {"cp_als_N40_R24_2sweeps": {"factors": rel(Fg, F), "tol": 1e-8},
                    "als_skew_N40_P12_2sweeps": {"factors": rel(Sg, Fs_), "tol": 1e-8}}
        checks.add_fn("als", als_err)

    if not args.no_extra and sec in ("all", "multi"):
        # ---------------- uneven N and mixed formats: grouped launches against the same
        # states one by one.  One-trajectory CP states at N = 100..1000 (R = 2N) in FP32,
        # BF16X3 and BF16 with SPD or diagonal stiffness, a dense FP32 state, and a batch
        # of 16 CP FP32 trajectories at N = 400
        specs = [(100, "cp", "fp32", "spd", 1), (200, "cp", "bf16x3", "diag", 1), (400, "cp", "fp32", "spd", 1),
                 (700, "cp", "bf16", "spd", 1), (1000, "cp", "fp32", "spd", 1), (200, "dense", "fp32", "diag", 1),
                 (400, "cp", "fp32", "spd", 16)]
        roms, sts, pms = [], [], []
        for i_, (Nm, kind, mdt, A_kind, Bm) in enumerate(specs):
            pm = romsynth.make_problem(Nm, pairs=Nm, eps=1e-7, nu=5e-4, dt=5e-4, A=A_kind, cfg=40 + i_, batch=Bm,
                                       dense=kind == "dense", cp=kind == "cp")
            rm = rg.Rom.from_problem(pm, dense=kind == "dense", dtype=mdt, max_batch=Bm, stream=stream)
            if Bm > 1:
                tune.apply(rm, Bm, dense=False, R=2 * Nm, table=tiles)
            pms.append(pm)
            roms.append(rm)
            sts.append(rm.state(pm.u0))
        ch, sh = [r.handle for r in roms], [x.handle for x in sts]
        ntraj = sum(x[4] for x in specs)
        nm = 2000
        rg.rom_step_multi(ch, sh, 20)
        rg.rom_step_multi(ch, sh, nm)                    # tables and graphs of this call length
        t_grp = timer(lambda: rg.rom_step_multi(ch, sh, nm))
        for x in sts:
            x.prepare(nm)
            x.step(20)
        t_sep = timer(lambda: [x.step_async(nm) for x in sts])
        for x in sts:
            x.sync()
        result["multi"] = {"pairs": [dict(N=a, form=b, dtype=c, stiffness=d, batch=e) for a, b, c, d, e in specs],
                           "R": "2N", "trajectories": ntraj,
                           "grouped_traj_steps_per_s": ntraj * nm / t_grp,
                           "separate_traj_steps_per_s": ntraj * nm / t_sep,
                           "grouped_us_per_step": t_grp / nm * 1e6, "separate_us_per_step": t_sep / nm * 1e6,
                           "speedup_grouped": t_sep / t_grp}
        log(f"multi: grouped {ntraj * nm / t_grp:.0f}, separate {ntraj * nm / t_sep:.0f} traj-steps/s")
        for x in sts:
            x.close()
        sts = [rm.state(pm.u0) for rm, pm in zip(roms, pms)]
        rg.rom_step_multi([r.handle for r in roms], [x.handle for x in sts], 200)
        for (Nm, kind, mdt, A_kind, Bm), pm, x in zip(specs, pms, sts):
            ops = dict(C=pm.C) if kind == "dense" else dict(lam=pm.lam, Af=pm.Af, Bf=pm.Bf, Cf=pm.Cf)
            ug = x.get()[0][0]
            for b in sorted({0, Bm - 1}):
                checks.add("multi", f"N{Nm}_{kind}_{mdt}_{A_kind}_B{Bm}_traj{b}", (pm.N, pm.nu, pm.dt, pm.A), ops,
                           pm.u0[b], 200, ug[b], dtype=mdt)
            x.close()
        for r in roms:
            r.close()

    if not args.no_extra and sec in ("all", "serving"):
        # ---------------- serving: a seeded stream of config-4 requests (N in {100, ..., 1000},
        # dense or CP rank 2N by a coin, FP32 or BF16X3, log-uniform step counts, operator seeds
        # 0 and 1), operators created before the runs (their creation time reported apart),
        # pools of 16 slots per operator.  One run with every request arriving at once
        # measures the saturation throughput; runs at 0.5, 0.8 and 0.95 of that request rate
        # (Poisson arrivals) give the latency percentiles per rate.
        import dataclasses as _dc
        from paper_2311_03694_amd.serve import RomBackend, Server, at_rate, op_key, poisson_requests, summarize
        nreq, smax = args.serving_requests, args.serving_max_steps
        log(f"serving: {nreq} requests, steps 1e3..{smax}")
        reqs = poisson_requests(nreq, rate=1.0, Ns=(100, 200, 400, 700, 1000), dense_frac=0.5,
                                dtypes=("fp32", "bf16x3"), steps_range=(1000, smax), seeds=(0, 1), rng_seed=7)
        be = RomBackend(pool_slots=16)             # each operator's context on a stream of its own
        srv = Server(be, hbm_budget=200 << 30, max_slots=256, chunk=500)
        t1 = time.perf_counter()
        srv.warm(sorted({op_key(r) for r in reqs}))
        create_s = time.perf_counter() - t1
        log(f"serving: {len(srv.ops)} operators created in {create_s:.1f}s")
        sat = [_dc.replace(r, arrival=0.0) for r in reqs]
        prog = lambda d, n, t: log(f"serving: {d}/{n} requests done after {t:.0f}s")
        t1 = time.perf_counter()
        recs = srv.run(sat, progress=prog)
        wall = time.perf_counter() - t1
        s_sat = summarize(recs, wall)
        lam_sat = s_sat["completed"] / wall
        log(f"serving saturation: {s_sat['throughput_traj_steps_per_s']:.0f} traj-steps/s, {lam_sat:.2f} req/s")
        rates = {}
        for f in (0.5, 0.8, 0.95):
            rq = at_rate(reqs, f * lam_sat, rng_seed=int(100 * f))
            t1 = time.perf_counter()
            rr = srv.run(rq, progress=prog)
            w = time.perf_counter() - t1
            rates[f"{f:.2f}"] = dict(summarize(rr, w), offered_req_per_s=f * lam_sat)
            log(f"serving at {f:.2f} of saturation: p50 {rates[f'{f:.2f}']['latency_p50_s']:.2f}s "
                f"p99 {rates[f'{f:.2f}']['latency_p99_s']:.2f}s")
        result["serving"] = {
            "stream": f"{nreq} requests ({100.0 * nreq / 10000:.1f}% of the 10,000 of config 4), N in "
                      f"{{100,200,400,700,1000}}, dense or CP rank 2N (coin 0.5), fp32/bf16x3, steps log-uniform "
                      f"[1e3, {smax:.0e}], operator seeds 0/1",
            "operators": len(srv.ops), "operator_create_s": create_s, "pool_slots": 16,
            "saturation": s_sat, "saturation_req_per_s": lam_sat, "rates": rates,
            "peak_hbm_bytes": srv.peak_used,
            "note": "latency = completion minus arrival (operators resident before the runs)"}
        # accuracy: the cheapest requests of the saturation run against the oracle
        sample = sorted(range(len(reqs)), key=lambda q: reqs[q].N * reqs[q].nsteps)[:4]
        for q in sample:
            r, rec = reqs[q], recs[q]
            A = romsynth.stiffness_spd(r.N, r.seed, be.cfg)
            if r.kind == "dense":
                ops = dict(C=be.host_tensor(r.N, r.seed))
            else:
                ops = dict(zip(("lam", "Af", "Bf", "Cf"), romsynth.skew_cp_factors(r.N, r.N, r.seed, be.cfg)))
            checks.add("serving", f"req{r.rid}_N{r.N}_{r.kind}_{r.dtype}", (r.N, be.nu, be.dt, A), ops, be.u0(r),
                       r.nsteps, rec.u, dtype=r.dtype)
        srv.close()

    # ---------------- oracle leg (after all GPU timing): accuracy of every section, and the
    # CPU baseline (the FP64 oracle on the host cores of one GPU's share, and on one)
    if not args.no_cpu:
        import oracle as orc
        if sec in ("all", "headline"):
            orc.set_threads(1)
            t1 = time.perf_counter()
            orc.run(N, p.nu, p.dt, p.A, 20, u0=p.u0[0], **ops_cp)
            per = max((time.perf_counter() - t1) / 20, 1e-6)
            n_cpu = int(max(100, min(20000, args.cpu_seconds / per)))
            log(f"oracle CPU baseline: {n_cpu} CP steps, one thread and {ORC_THREADS}")
            t1 = time.perf_counter()
            r1 = orc.run(N, p.nu, p.dt, p.A, n_cpu, u0=p.u0[0], **ops_cp)
            t_one = time.perf_counter() - t1
            with orc.threads(ORC_THREADS):
                t1 = time.perf_counter()
                rm_ = orc.run(N, p.nu, p.dt, p.A, n_cpu, u0=p.u0[0], **ops_cp)
                t_all = time.perf_counter() - t1
            assert np.array_equal(r1["u_hist"], rm_["u_hist"])
            nd = 3
            t2 = time.perf_counter()
            orc.run(N, p.nu, p.dt, p.A, nd, u0=p.u0[0], C=p.C)
            t_d1 = time.perf_counter() - t2
            with orc.threads(ORC_THREADS):
                t2 = time.perf_counter()
                orc.run(N, p.nu, p.dt, p.A, nd, u0=p.u0[0], C=p.C)
                t_dm = time.perf_counter() - t2
            rom_chk = make(False)
            sg = rom_chk.state(p.u0)
            sg.step(n_cpu)
            checks.add("headline", "cp", prob, ops_cp, p.u0[0], n_cpu, sg.u(), E_gpu=sg.energy()[1][:, 0], dtype=dt)
            sg.close()
            rom_chk.close()
            result["cpu_baseline"] = {
                "value": n_cpu / t_all, "unit": "trajectory-steps/s", "cores": ORC_THREADS, "kind": "oracle",
                "sample": f"{n_cpu} CP-ROM steps (N=1000, R={R}, FP64, incl. its one-time Cholesky) on "
                          f"{ORC_THREADS} host threads (row loops; results identical to one thread); dense G-ROM: "
                          f"{nd} steps",
                "cpu_model": cpu_model(), "host_cpus_visible": os.cpu_count(),
                "single_thread_value": n_cpu / t_one,
                "dense_value": nd / t_dm, "dense_single_thread_value": nd / t_d1}
        errs = run_checks(checks, orc, log)
        worst = {}
        for secname, entries in errs.items():
            tgt = result.setdefault(secname, {}) if secname != "headline" else result
            tgt.setdefault("rel_err", {}).update(entries)
            worst[secname] = max(v.get("traj", v.get("factors", 0.0)) / v["tol"] for v in entries.values())
        result["rel_err_worst_over_tol"] = worst
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
