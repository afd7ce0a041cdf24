"""Seeded synthetic operators for the reduced model  B du/dt = -C(u)u - nu*A*u.

Every array is FP64 numpy, row-major:
  A      [N][N]      stiffness (symmetric positive definite), mass matrix is I
  C      [N][N][N]   advection tensor; C[i][j][k] multiplies u_j*u_k in output row i
                     and is skew in positions 1 and 3: C[i][j][k] = -C[k][j][i]
  lam    [R]         CP weights
  Af,Bf,Cf [N][R]    CP factors for positions 1, 2, 3
  u0     [B][N]      initial coefficients, one row per trajectory

If the environment variable ROMSYNTH_CACHE names a directory, large dense tensors are
saved there once and memory-mapped on later calls (same seeds give the same file).

Random streams come from numpy's PCG64 seeded with SeedSequence([config, stream, seed]);
stream 0 = factors (or the rough tensor S), 1 = tensor noise, 2 = stiffness perturbation,
3 = initial coefficients, 4 = mass matrix and zeroth-mode terms.  The draw order inside a
stream is part of the recipe and documented next to each draw.
"""
from __future__ import annotations

import dataclasses
import os
from typing import Optional

import numpy as np

STREAM_FACTORS = 0
STREAM_NOISE = 1
STREAM_STIFF = 2
STREAM_U0 = 3
STREAM_FULL = 4


def _rng(cfg: int, stream: int, seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([cfg, stream, seed])))


@dataclasses.dataclass
class Problem:
    """One reduced model: operators, time-step parameters and initial states."""
    N: int
    nu: float
    dt: float
    A: np.ndarray
    u0: np.ndarray                      # [B][N]
    nsteps: int
    C: Optional[np.ndarray] = None      # [N][N][N]
    lam: Optional[np.ndarray] = None    # [R]
    Af: Optional[np.ndarray] = None     # [N][R]
    Bf: Optional[np.ndarray] = None
    Cf: Optional[np.ndarray] = None
    name: str = ""

    @property
    def R(self) -> int:
        return 0 if self.lam is None else int(self.lam.shape[0])

    @property
    def batch(self) -> int:
        return int(self.u0.shape[0])


# ----------------------------------------------------------------------------- tensors

def dense_rough(N: int, seed: int = 0, cfg: int = 0) -> np.ndarray:
    """C = S - S^(13) with S[i][j][k] ~ N(0,1) * (i*j*k)^(-1/2), indices 1-based.

    S is drawn as one standard_normal((N, N, N)) call in C order.
    """
    z = _rng(cfg, STREAM_FACTORS, seed).standard_normal((N, N, N))
    idx = np.arange(1, N + 1, dtype=np.float64)
    scale = 1.0 / np.sqrt(idx[:, None, None] * idx[None, :, None] * idx[None, None, :])
    S = z * scale
    return S - S.transpose(2, 1, 0)


def skew_cp_factors(N: int, pairs: int, seed: int = 0, cfg: int = 1):
    """Skew-paired CP factors with R = 2*pairs columns.

    Pair p (1-based) has unit-norm Gaussian vectors a_p, b_p, c_p and weight 1/p.  It
    contributes two columns, (1/p; a_p, b_p, c_p) and (1/p; c_p, b_p, -a_p), placed at
    columns 2(p-1) and 2(p-1)+1, so that the Kruskal tensor is skew in positions 1 and 3
    and truncating to the first 2q columns keeps the q leading pairs.
    Draw order: three standard_normal((N, pairs)) calls, for a, b, c.
    """
    rng = _rng(cfg, STREAM_FACTORS, seed)
    ga = rng.standard_normal((N, pairs))
    gb = rng.standard_normal((N, pairs))
    gc = rng.standard_normal((N, pairs))
    a = ga / np.linalg.norm(ga, axis=0, keepdims=True)
    b = gb / np.linalg.norm(gb, axis=0, keepdims=True)
    c = gc / np.linalg.norm(gc, axis=0, keepdims=True)
    w = 1.0 / np.arange(1, pairs + 1, dtype=np.float64)
    R = 2 * pairs
    lam = np.empty(R)
    Af = np.empty((N, R))
    Bf = np.empty((N, R))
    Cf = np.empty((N, R))
    lam[0::2] = w
    lam[1::2] = w
    Af[:, 0::2] = a
    Af[:, 1::2] = c
    Bf[:, 0::2] = b
    Bf[:, 1::2] = b
    Cf[:, 0::2] = c
    Cf[:, 1::2] = -a
    return lam, Af, Bf, Cf


def _cache_path(tag: str) -> Optional[str]:
    d = os.environ.get("ROMSYNTH_CACHE")
    if not d:
        return None
    os.makedirs(d, exist_ok=True)
    return os.path.join(d, tag + ".npy")


def dense_from_skew_cp(N: int, pairs: int, eps: float, seed: int = 0, cfg: int = 1,
                       out: Optional[np.ndarray] = None) -> np.ndarray:
    """Dense tensor T - T^(13) with T = sum_p (1/p) a_p o b_p o c_p + eps*G.

    The factors are those of skew_cp_factors(N, pairs, seed, cfg).  G is i.i.d. N(0,1),
    drawn slab by slab over the middle index j: slab j is one
    standard_normal((N, N), float32) call giving G[:, j, :].  Because the skew
    transposition swaps positions 1 and 3 only, slab j of the result is T_j - T_j^T.
    """
    cache = _cache_path(f"dense_skewcp_N{N}_P{pairs}_e{eps!r}_s{seed}_c{cfg}") if out is None else None
    if cache and os.path.exists(cache):
        return np.load(cache, mmap_mode="r")
    lam, Af, Bf, Cf = skew_cp_factors(N, pairs, seed, cfg)
    a = Af[:, 0::2]
    b = Bf[:, 0::2]
    c = Cf[:, 0::2]
    w = lam[0::2]
    if out is None:
        out = np.empty((N, N, N))
    rng = _rng(cfg, STREAM_NOISE, seed)
    ct = np.ascontiguousarray(c.T)
    for j in range(N):
        Tj = (a * (w * b[j])) @ ct
        if eps != 0.0:
            Tj += eps * rng.standard_normal((N, N), dtype=np.float32).astype(np.float64)
        out[:, j, :] = Tj - Tj.T
    if cache:
        np.save(cache + ".tmp.npy", out)
        os.replace(cache + ".tmp.npy", cache)
    return out


def truncate_cp(lam, Af, Bf, Cf, R: int):
    """Keep the first R columns (R even keeps whole skew pairs)."""
    return (np.ascontiguousarray(lam[:R]), np.ascontiguousarray(Af[:, :R]),
            np.ascontiguousarray(Bf[:, :R]), np.ascontiguousarray(Cf[:, :R]))


# ----------------------------------------------------------------------------- stiffness, states

def stiffness_diag(N: int) -> np.ndarray:
    """A = diag(k^2), k = 1..N."""
    return np.diag(np.arange(1, N + 1, dtype=np.float64) ** 2)


def stiffness_spd(N: int, seed: int = 0, cfg: int = 3, norm: float = 0.1) -> np.ndarray:
    """A = diag(k^2) + P, P = norm * M / ||M||_2, M = G G^T, G one standard_normal((N, N))."""
    G = _rng(cfg, STREAM_STIFF, seed).standard_normal((N, N))
    M = G @ G.T
    P = norm * M / np.linalg.norm(M, 2)
    A = stiffness_diag(N) + P
    return 0.5 * (A + A.T)


def stiffness_graded(N: int, lo: float, hi: float, seed: int = 0, cfg: int = 3) -> np.ndarray:
    """Dense SPD stiffness with eigenvalues log-spaced over [lo, hi] in a random orthonormal
    basis: A = Q diag(lam) Q^T, Q from the QR factorisation of one standard_normal((N, N))
    draw from stream 2, then symmetrized."""
    G = _rng(cfg, STREAM_STIFF, seed).standard_normal((N, N))
    Q, _ = np.linalg.qr(G)
    lam = np.logspace(np.log10(lo), np.log10(hi), N)
    A = (Q * lam) @ Q.T
    return 0.5 * (A + A.T)


def mass_spd(N: int, seed: int = 0, cfg: int = 3, norm: float = 0.1, diag: bool = False) -> np.ndarray:
    """Mass matrix M = I + P: P = norm * G G^T / ||G G^T||_2 with G one standard_normal((N, N))
    from stream 4, or (diag=True) P = norm * diag(v) with v one uniform(N) draw."""
    g = _rng(cfg, STREAM_FULL, seed)
    if diag:
        return np.eye(N) + norm * np.diag(g.uniform(size=N))
    G = g.standard_normal((N, N))
    S = G @ G.T
    M = np.eye(N) + norm * S / np.linalg.norm(S, 2)
    return 0.5 * (M + M.T)


def zeroth_terms(N: int, seed: int = 0, cfg: int = 3, scale: float = 0.1):
    """Zeroth-mode operators (C1, C2 [N][N+1], c0, a0 [N]), column 0 of C1 and C2 being the
    zeroth mode.  Draws from stream 4 with seed + 1 in this order: C1, C2 (standard_normal,
    (N, N+1) each), a0 (standard_normal(N)); entries times scale / sqrt(N + 1).  Column 0 of
    both matrices is the zeroth mode advecting itself, so c0 is set to column 0 of C1 and
    column 0 of C2 is set equal to it."""
    g = _rng(cfg, STREAM_FULL, seed + 1)
    s = scale / np.sqrt(N + 1.0)
    C1 = g.standard_normal((N, N + 1)) * s
    C2 = g.standard_normal((N, N + 1)) * s
    a0 = g.standard_normal(N) * s
    c0 = C1[:, 0].copy()
    C2[:, 0] = c0
    return C1, C2, c0, a0


def initial_u(N: int, seeds, cfg: int = 0) -> np.ndarray:
    """u0[b][k-1] = z_k * k^(-5/6), z = standard_normal(N) from stream 3 with seed seeds[b]."""
    k = np.arange(1, N + 1, dtype=np.float64)
    rows = [_rng(cfg, STREAM_U0, int(s)).standard_normal(N) * k ** (-5.0 / 6.0) for s in seeds]
    return np.stack(rows, axis=0)


# ----------------------------------------------------------------------------- small integers

def integer_dense(N: int, seed: int = 0, cfg: int = 50, vmax: int = 1) -> np.ndarray:
    """Skew tensor of small integers: C = S - S^(13) with S[i][j][k] uniform in
    {-vmax, ..., vmax} (one integers((N, N, N)) draw), so |C| <= 2 vmax."""
    S = _rng(cfg, STREAM_FACTORS, seed).integers(-vmax, vmax + 1, size=(N, N, N)).astype(np.float64)
    return S - S.transpose(2, 1, 0)


def integer_cp_factors(N: int, R: int, seed: int = 0, cfg: int = 51, vmax: int = 1, skew: bool = True):
    """CP factors of small integers.  skew=True: R/2 column pairs laid out like
    skew_cp_factors (columns (lam_p; a_p, b_p, c_p) and (lam_p; c_p, b_p, -a_p)), so the
    pair form applies; skew=False: independent columns.  Entries uniform in
    {-vmax, ..., vmax}, weights in {1, 2}.  Draw order: a, b, c as integers((N, P)) (P =
    R/2, or R columns each when skew=False), then the weights as integers(P) (or R)."""
    rng = _rng(cfg, STREAM_FACTORS, seed)
    cols = R // 2 if skew else R
    a, b, c = (rng.integers(-vmax, vmax + 1, size=(N, cols)).astype(np.float64) for _ in range(3))
    w = rng.integers(1, 3, size=cols).astype(np.float64)
    if not skew:
        return w, a, b, c
    lam = np.empty(R)
    Af = np.empty((N, R))
    Bf = np.empty((N, R))
    Cf = np.empty((N, R))
    lam[0::2] = w
    lam[1::2] = w
    Af[:, 0::2] = a
    Af[:, 1::2] = c
    Bf[:, 0::2] = b
    Bf[:, 1::2] = b
    Cf[:, 0::2] = c
    Cf[:, 1::2] = -a
    return lam, Af, Bf, Cf


def integer_u(N: int, seeds, cfg: int = 52, vmax: int = 2) -> np.ndarray:
    """Rows of small integer coefficients in {-vmax, ..., vmax}, one integers(N) draw per
    seed from stream 3."""
    return np.stack([_rng(cfg, STREAM_U0, int(s)).integers(-vmax, vmax + 1, size=N).astype(np.float64)
                     for s in seeds], axis=0)


# ----------------------------------------------------------------------------- named workloads

CONFIGS = {
    0: dict(N=32, nu=1e-3, dt=1e-3, nsteps=1000, kind="rough", A="diag", batch=1),
    1: dict(N=400, pairs=400, eps=1e-6, nu=1e-3, dt=1e-3, nsteps=20000, A="diag", batch=1),
    2: dict(N=400, pairs=400, eps=1e-6, nu=1e-3, dt=1e-3, nsteps=5000, A="diag", batch=256,
            tensor_cfg=1, R=400),
    3: dict(N=1000, pairs=1000, eps=1e-7, nu=5e-4, dt=5e-4, nsteps=10000, A="spd", batch=1),
}


def make_problem(N: int, *, pairs: int = 0, eps: float = 0.0, nu: float = 1e-3, dt: float = 1e-3,
                 A: str = "diag", batch: int = 1, nsteps: int = 100, seed: int = 0, cfg: int = 1,
                 dense: bool = True, cp: bool = True, R: Optional[int] = None,
                 u0_seeds=None, kind: str = "cp", name: str = "") -> Problem:
    """General recipe used by the named configurations and by the tests.

    kind "rough": dense_rough tensor (no CP factors).  kind "cp": skew-paired factors with
    `pairs` pairs and, if dense, the matching dense tensor plus eps noise.  R truncates
    the CP factors handed to the problem (default: all 2*pairs columns).
    """
    Amat = stiffness_diag(N) if A == "diag" else stiffness_spd(N, seed, cfg)
    seeds = list(range(batch)) if u0_seeds is None else list(u0_seeds)
    u0 = initial_u(N, seeds, cfg)
    p = Problem(N=N, nu=nu, dt=dt, A=Amat, u0=u0, nsteps=nsteps, name=name)
    if kind == "rough":
        p.C = dense_rough(N, seed, cfg)
        return p
    if cp:
        lam, Af, Bf, Cf = skew_cp_factors(N, pairs, seed, cfg)
        if R is not None:
            lam, Af, Bf, Cf = truncate_cp(lam, Af, Bf, Cf, R)
        p.lam, p.Af, p.Bf, p.Cf = lam, Af, Bf, Cf
    if dense:
        p.C = dense_from_skew_cp(N, pairs, eps, seed, cfg)
    return p


def make_config(i: int, *, dense: bool = True, cp: bool = True, R: Optional[int] = None,
                batch: Optional[int] = None, nsteps: Optional[int] = None) -> Problem:
    """The named workloads (0: N=32 rough dense; 1: N=400; 2: N=400 x 256 trajectories;
    3: N=1000 with SPD stiffness).  Config 2 reuses the config-1 tensor streams and
    draws its initial states from its own stream."""
    c = dict(CONFIGS[i])
    B = batch if batch is not None else c["batch"]
    steps = nsteps if nsteps is not None else c["nsteps"]
    if c.get("kind") == "rough":
        A = stiffness_diag(c["N"])
        u0 = initial_u(c["N"], range(B), cfg=0)
        return Problem(N=c["N"], nu=c["nu"], dt=c["dt"], A=A, u0=u0, nsteps=steps,
                       C=dense_rough(c["N"], 0, 0), name=f"config{i}")
    tcfg = c.get("tensor_cfg", i)
    Rsel = R if R is not None else c.get("R")
    p = make_problem(c["N"], pairs=c["pairs"], eps=c["eps"], nu=c["nu"], dt=c["dt"], A=c["A"],
                     batch=B, nsteps=steps, seed=0, cfg=tcfg, dense=dense, cp=cp, R=Rsel,
                     name=f"config{i}")
    p.u0 = initial_u(c["N"], range(B), cfg=i)
    return p
