"""ctypes binding of the plain-C FP64 oracle (rom_oracle.c).

TEST INFRASTRUCTURE ONLY: argument marshalling for numpy arrays; all arithmetic is in C.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rom_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_d = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.c_int64


def lib_path() -> str:
    return _LIB


def build() -> str:
    """Compile rom_oracle.c with gcc: strict IEEE FP64 (no contraction into FMA)."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           "-std=c99", "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    lib.orc_nonlinear_dense.argtypes = [_i64, _d, _d, _d]
    lib.orc_nonlinear_dense_rows.argtypes = [_i64, _d, _d, _i64, ctypes.POINTER(_i64), _d]
    lib.orc_nonlinear_cp.argtypes = [_i64, _i64, _d, _d, _d, _d, _d, _d]
    lib.orc_nonlinear_cp_skew.argtypes = [_i64, _i64, _d, _d, _d, _d, _d, _d]
    lib.orc_nonlinear_svd.argtypes = [_i64, _i64, _d, _d, _d, _d, _d]
    lib.orc_reconstruct.argtypes = [_i64, _i64, _d, _d, _d, _d, _d]
    lib.orc_cholesky.argtypes = [_i64, _d, _d]
    lib.orc_cholesky.restype = ctypes.c_int
    lib.orc_chol_solve.argtypes = [_i64, _d, _d, _d]
    lib.orc_energy.argtypes = [_i64, _d]
    lib.orc_energy.restype = ctypes.c_double
    lib.orc_run.argtypes = [_i64, ctypes.c_double, ctypes.c_double, _d, _d, _i64, _d, _d, _d,
                            _d, _i64, _d, _d, _i64, _d, _d, ctypes.POINTER(_i64)]
    lib.orc_run.restype = ctypes.c_int
    lib.orc_run_svd.argtypes = [_i64, ctypes.c_double, ctypes.c_double, _d, _i64, _d, _d, _d, _i64, _d, _d,
                                _i64, _d, _d, ctypes.POINTER(_i64)]
    lib.orc_run_svd.restype = ctypes.c_int
    lib.orc_explicit_full.argtypes = [_i64, _d, _i64, _d, _d, _d, _d, _d, _d, _d, _d, _d]
    lib.orc_run_full.argtypes = [_i64, ctypes.c_double, ctypes.c_double, _d, _d, _d, _i64, _d, _d,
                                 _d, _d, _d, _d, _d, _d, _i64, _d, _d, _i64, _d, _d,
                                 ctypes.POINTER(_i64)]
    lib.orc_run_full.restype = ctypes.c_int
    lib.orc_round_f32.argtypes = [_i64, _d, _d]
    lib.orc_round_bf16.argtypes = [_i64, _d, _d]
    lib.orc_split_bf16x3.argtypes = [_i64, _d, _d, _d]
    lib.orc_set_threads.argtypes = [ctypes.c_int]
    lib.orc_set_threads.restype = ctypes.c_int
    lib.orc_get_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def set_threads(n: int) -> int:
    """Host threads for the oracle's row loops (results identical for any count); returns
    the previous count."""
    return int(_load().orc_set_threads(int(n)))


def get_threads() -> int:
    return int(_load().orc_get_threads())


class threads:
    """Context manager: `with oracle.threads(n): ...` runs the oracle's row loops on n threads."""

    def __init__(self, n: int):
        self.n = int(n)

    def __enter__(self):
        self.old = set_threads(self.n)
        return self

    def __exit__(self, *exc):
        set_threads(self.old)


def _c(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a: Optional[np.ndarray]):
    if a is None:
        return ctypes.cast(None, _d)
    return a.ctypes.data_as(_d)


def nonlinear_dense(C, u) -> np.ndarray:
    """y = C(u)u for u of shape [N] or [B][N]."""
    lib = _load()
    C = _c(C)
    u = _c(u)
    N = C.shape[0]
    uu = u.reshape(-1, N)
    y = np.empty_like(uu)
    for b in range(uu.shape[0]):
        ub = np.ascontiguousarray(uu[b])
        yb = np.empty(N)
        lib.orc_nonlinear_dense(N, _p(C), _p(ub), _p(yb))
        y[b] = yb
    return y.reshape(u.shape)


def nonlinear_dense_rows(C, u, rows) -> np.ndarray:
    """y_i for i in rows (u of shape [N])."""
    lib = _load()
    C = np.asarray(C)
    if not (C.dtype == np.float64 and C.flags.c_contiguous):
        C = _c(C)
    u = _c(u)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty(rows.shape[0])
    lib.orc_nonlinear_dense_rows(C.shape[0], _p(C), _p(u), rows.shape[0],
                                 rows.ctypes.data_as(ctypes.POINTER(_i64)), _p(out))
    return out


def nonlinear_cp(lam, Af, Bf, Cf, u) -> np.ndarray:
    lib = _load()
    lam, Af, Bf, Cf, u = map(_c, (lam, Af, Bf, Cf, u))
    N, R = Af.shape
    uu = u.reshape(-1, N)
    y = np.empty_like(uu)
    for b in range(uu.shape[0]):
        ub = np.ascontiguousarray(uu[b])
        yb = np.empty(N)
        lib.orc_nonlinear_cp(N, R, _p(lam), _p(Af), _p(Bf), _p(Cf), _p(ub), _p(yb))
        y[b] = yb
    return y.reshape(u.shape)


def nonlinear_cp_skew(lam, A11, A12, A21, u) -> np.ndarray:
    """y = C(u)u for the skew-symmetry preserving CP form (Sec. 3.3, eq. skew_abc_struct):
    factors [A11 A12], [A21 A21], [A12 -A11] with one weight per column pair; A11, A12,
    A21 are [N][P], lam is [P]."""
    lib = _load()
    lam, A11, A12, A21, u = map(_c, (lam, A11, A12, A21, u))
    N, P = A11.shape
    uu = u.reshape(-1, N)
    y = np.empty_like(uu)
    for b in range(uu.shape[0]):
        ub = np.ascontiguousarray(uu[b])
        yb = np.empty(N)
        lib.orc_nonlinear_cp_skew(N, P, _p(lam), _p(A11), _p(A12), _p(A21), _p(ub), _p(yb))
        y[b] = yb
    return y.reshape(u.shape)


def nonlinear_svd(U, sigma, V, u) -> np.ndarray:
    """y = C(u)u for the SVD form (Sec. 4.4): C[i][j][k] ~ sum_r U[j][r] sigma_r V[i][k][r];
    U [N][R], sigma [R], V [N][N][R]."""
    lib = _load()
    U, sigma, V, u = map(_c, (U, sigma, V, u))
    N, R = U.shape
    uu = u.reshape(-1, N)
    y = np.empty_like(uu)
    for b in range(uu.shape[0]):
        ub = np.ascontiguousarray(uu[b])
        yb = np.empty(N)
        lib.orc_nonlinear_svd(N, R, _p(U), _p(sigma), _p(V), _p(ub), _p(yb))
        y[b] = yb
    return y.reshape(u.shape)


def reconstruct(lam, Af, Bf, Cf) -> np.ndarray:
    lib = _load()
    lam, Af, Bf, Cf = map(_c, (lam, Af, Bf, Cf))
    N, R = Af.shape
    T = np.empty((N, N, N))
    lib.orc_reconstruct(N, R, _p(lam), _p(Af), _p(Bf), _p(Cf), _p(T))
    return T


def cholesky(H):
    lib = _load()
    H = _c(H)
    L = np.empty_like(H)
    rc = lib.orc_cholesky(H.shape[0], _p(H), _p(L))
    if rc != 0:
        raise np.linalg.LinAlgError("matrix is not positive definite")
    return L


def chol_solve(L, b):
    lib = _load()
    L = _c(L)
    b = _c(b)
    x = np.empty_like(b)
    lib.orc_chol_solve(L.shape[0], _p(L), _p(b), _p(x))
    return x


def energy(u) -> float:
    lib = _load()
    u = _c(u)
    return float(lib.orc_energy(u.shape[0], _p(u)))


def explicit_full(u, *, C=None, lam=None, Af=None, Bf=None, Cf=None, C1=None, C2=None, c0=None):
    """g = C(u)u + (C1 + C2) ubar - c0 with ubar = [1, u] (eq. nse_d1, one level);
    C1, C2 [N][N+1], c0 [N], each optional."""
    lib = _load()
    u = _c(u)
    N = u.shape[0]
    g = np.empty(N)
    if C is not None:
        core = (_p(_c(C)), 0, _p(None), _p(None), _p(None), _p(None))
    else:
        lam, Af, Bf, Cf = map(_c, (lam, Af, Bf, Cf))
        core = (_p(None), Af.shape[1], _p(lam), _p(Af), _p(Bf), _p(Cf))
    opt = [None if x is None else _c(x) for x in (C1, C2, c0)]
    lib.orc_explicit_full(N, *core, *[_p(x) for x in opt], _p(u), _p(g))
    return g


def run(N, nu, dt, A, nsteps, *, u0=None, C=None, lam=None, Af=None, Bf=None, Cf=None,
        M=None, C1=None, C2=None, c0=None, a0=None, U=None, sigma=None, V=None,
        step0: int = 0, uh=None, yh=None, traj: bool = False) -> dict:
    """Integrate one trajectory for nsteps BDF3/EXT3 steps (with the BDF1/BDF2 ramp).

    Either u0 (start at step 0) or the history (step0, uh [3][N], yh [2][N]) is given.
    The advection term is the dense tensor C, the CP factors, or the SVD form (U [N][Rs],
    sigma [Rs], V [N][N][Rs]; identity mass matrix, no zeroth-mode terms).
    M (mass matrix, default the identity) and the zeroth-mode terms C1, C2 [N][N+1],
    c0, a0 [N] (default zero) select the full form of eq. nse_d1.
    Returns dict(u_hist, y_hist, step, E [nsteps+1], traj [nsteps+1][N] or None,
    status, first_bad).
    """
    lib = _load()
    A = _c(A)
    if uh is None:
        uh = np.zeros((3, N))
        uh[0] = _c(u0).reshape(N)
        yh = np.zeros((2, N))
    uh = _c(uh).copy()
    yh = _c(yh).copy()
    E = np.empty(nsteps + 1)
    T = np.empty((nsteps + 1, N)) if traj else None
    fb = _i64(-1)
    if U is not None:
        U, sigma, V = map(_c, (U, sigma, V))
        st = lib.orc_run_svd(N, float(nu), float(dt), _p(A), U.shape[1], _p(U), _p(sigma), _p(V), int(step0),
                             _p(uh), _p(yh), int(nsteps), _p(E), _p(T), ctypes.byref(fb))
        return dict(u_hist=uh, y_hist=yh, step=step0 + nsteps, E=E, traj=T, status=int(st),
                    first_bad=int(fb.value))
    if C is not None:
        C = np.asarray(C)
        if not (C.dtype == np.float64 and C.flags.c_contiguous):
            C = _c(C)
        R = 0
        args = (_p(C), 0, _p(None), _p(None), _p(None), _p(None))
    else:
        lam, Af, Bf, Cf = map(_c, (lam, Af, Bf, Cf))
        R = Af.shape[1]
        args = (_p(None), R, _p(lam), _p(Af), _p(Bf), _p(Cf))
    full = [None if x is None else _c(x) for x in (M, C1, C2, c0, a0)]
    if all(x is None for x in full):
        st = lib.orc_run(N, float(nu), float(dt), _p(A), *args, int(step0), _p(uh), _p(yh),
                         int(nsteps), _p(E), _p(T), ctypes.byref(fb))
    else:
        Mp, C1p, C2p, c0p, a0p = [_p(x) for x in full]
        st = lib.orc_run_full(N, float(nu), float(dt), _p(A), Mp, *args, C1p, C2p, c0p, a0p,
                              int(step0), _p(uh), _p(yh), int(nsteps), _p(E), _p(T), ctypes.byref(fb))
    return dict(u_hist=uh, y_hist=yh, step=step0 + nsteps, E=E, traj=T, status=int(st),
                first_bad=int(fb.value))


def round_f32(x) -> np.ndarray:
    lib = _load()
    x = _c(x)
    out = np.empty_like(x)
    lib.orc_round_f32(x.size, _p(x), _p(out))
    return out


def round_bf16(x) -> np.ndarray:
    lib = _load()
    x = _c(x)
    out = np.empty_like(x)
    lib.orc_round_bf16(x.size, _p(x), _p(out))
    return out


def split_bf16x3(x):
    lib = _load()
    x = _c(x)
    hi = np.empty_like(x)
    lo = np.empty_like(x)
    lib.orc_split_bf16x3(x.size, _p(x), _p(hi), _p(lo))
    return hi, lo
