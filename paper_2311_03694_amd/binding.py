"""Thin ctypes binding of librom.so (include/rom.h).

Argument marshalling only: numpy arrays for host buffers, torch tensors (or raw
integers) for device buffers and streams.  Every computation happens in the HIP
kernels of librom.so; there is no fallback, and calls raise if the library is missing.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librom.so")

ROM_OK, ROM_E_INVALID, ROM_E_NOMEM, ROM_E_DEVICE, ROM_E_NONFINITE, ROM_E_UNSUPPORTED = range(6)
DTYPES = {"fp64": 0, "fp32": 1, "bf16": 2, "bf16x3": 3}
STATUS_NAMES = {0: "ROM_OK", 1: "ROM_E_INVALID", 2: "ROM_E_NOMEM", 3: "ROM_E_DEVICE",
                4: "ROM_E_NONFINITE", 5: "ROM_E_UNSUPPORTED"}

# every symbol declared in include/rom.h
EXPORTS = ["rom_create", "rom_destroy", "rom_nonlinear", "rom_nonlinear_noalloc", "rom_nonlinear_timed",
           "rom_state_create",
           "rom_state_destroy",
           "rom_step", "rom_step_async", "rom_step_sync", "rom_step_prepare", "rom_energy", "rom_state_get",
           "rom_state_set", "rom_state_set_slot", "rom_state_u", "rom_step_multi", "rom_query", "rom_set_tile",
           "rom_tile_count", "rom_cp_skew_layout", "rom_create_svd", "rom_create_full", "rom_cp_als", "rom_cp_als_skew",
           "rom_last_error"]

_d = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p
_i64p = ctypes.POINTER(ctypes.c_int64)


class rom_desc(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("R", ctypes.c_int32), ("nu", ctypes.c_double),
                ("dt", ctypes.c_double), ("A", _d), ("C", _d), ("lambda_", _d), ("Af", _d),
                ("Bf", _d), ("Cf", _d), ("dtype", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("stream", _vp)]


class rom_full_terms(ctypes.Structure):
    _fields_ = [("M", _d), ("C1", _d), ("C2", _d), ("c0", _d), ("a0", _d)]


class RomError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class NonFinite(RomError):
    def __init__(self, status, msg, first_bad):
        super().__init__(status, msg)
        self.first_bad = first_bad


_lib = None


def lib():
    """Load librom.so; raises if it has not been built (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"librom.so not found at {LIB_PATH}: build it with "
                           "`python -m paper_2311_03694_amd.build` (hipcc, gfx950)")
    # Load PyTorch's HIP runtime first so that librom.so binds to the same runtime
    # instance (PyTorch ships its own libamdhip64); two instances in one process do not
    # share devices, streams or allocations.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    L.rom_create.argtypes = [ctypes.POINTER(rom_desc), ctypes.POINTER(_vp)]
    L.rom_destroy.argtypes = [_vp]
    L.rom_destroy.restype = None
    L.rom_nonlinear.argtypes = [_vp, ctypes.c_int32, _vp, _vp]
    L.rom_nonlinear_noalloc.argtypes = [_vp, ctypes.c_int32, _vp, _vp]
    L.rom_nonlinear_timed.argtypes = [_vp, ctypes.c_int32, _vp, _vp, ctypes.c_int32, _d]
    L.rom_state_create.argtypes = [_vp, ctypes.c_int32, _d, ctypes.POINTER(_vp)]
    L.rom_state_destroy.argtypes = [_vp]
    L.rom_state_destroy.restype = None
    L.rom_step.argtypes = [_vp, _vp, ctypes.c_int64, _i64p]
    L.rom_step_async.argtypes = [_vp, _vp, ctypes.c_int64]
    L.rom_step_prepare.argtypes = [_vp, _vp, ctypes.c_int64]
    L.rom_step_sync.argtypes = [_vp, _vp, _i64p]
    L.rom_energy.argtypes = [_vp, _vp, _d, _d]
    L.rom_state_get.argtypes = [_vp, _vp, _d, _d, _i64p]
    L.rom_state_set.argtypes = [_vp, _vp, _d, _d, ctypes.c_int64]
    L.rom_state_u.argtypes = [_vp, _vp, _vp]
    L.rom_state_set_slot.argtypes = [_vp, _vp, ctypes.c_int32, _d, _d, ctypes.c_int32]
    L.rom_state_set_slot.restype = ctypes.c_int
    L.rom_step_multi.argtypes = [ctypes.c_int32, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                 ctypes.c_int64, _i64p]
    L.rom_query.argtypes = [_vp, _vp, ctypes.c_int32, _i64p]
    L.rom_set_tile.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32]
    L.rom_tile_count.argtypes = [ctypes.c_int32]
    L.rom_tile_count.restype = ctypes.c_int32
    L.rom_cp_skew_layout.argtypes = [ctypes.c_int32, ctypes.c_int32, _d, _d, _d, _d]
    L.rom_create_svd.argtypes = [ctypes.POINTER(rom_desc), ctypes.c_int32, _d, _d, _d, ctypes.POINTER(_vp)]
    L.rom_create_svd.restype = ctypes.c_int
    L.rom_create_full.argtypes = [ctypes.POINTER(rom_desc), ctypes.POINTER(rom_full_terms), ctypes.POINTER(_vp)]
    L.rom_create_full.restype = ctypes.c_int
    L.rom_cp_als.argtypes = [ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp, _vp, ctypes.c_int32, _vp]
    L.rom_cp_als.restype = ctypes.c_int
    L.rom_cp_als_skew.argtypes = [ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32,
                                  ctypes.c_double, _vp]
    L.rom_cp_als_skew.restype = ctypes.c_int
    L.rom_cp_skew_layout.restype = ctypes.c_int32
    L.rom_last_error.argtypes = []
    L.rom_last_error.restype = ctypes.c_char_p
    for name in ("rom_create", "rom_nonlinear", "rom_nonlinear_noalloc", "rom_nonlinear_timed", "rom_state_create", "rom_step", "rom_step_async",
                 "rom_step_sync", "rom_step_prepare", "rom_energy", "rom_state_get", "rom_state_set", "rom_state_u",
                 "rom_step_multi", "rom_query", "rom_set_tile"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(st: int, first_bad: Optional[int] = None):
    if st == ROM_OK:
        return
    msg = lib().rom_last_error().decode(errors="replace")
    if st == ROM_E_NONFINITE:
        raise NonFinite(st, msg, first_bad)
    raise RomError(st, msg)


def _host(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: Optional[np.ndarray]):
    return ctypes.cast(None, _d) if a is None else a.ctypes.data_as(_d)


def _dev_ptr(x) -> int:
    """Device address of a torch tensor (FP64, contiguous) or a raw integer."""
    if isinstance(x, int):
        return x
    import torch
    if not (x.is_cuda and x.dtype == torch.float64 and x.is_contiguous()):
        raise ValueError("device buffers must be contiguous float64 GPU tensors")
    return x.data_ptr()


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


# ----------------------------------------------------------------------------- the C calls

def rom_create(N, nu, dt, A, *, C=None, lam=None, Af=None, Bf=None, Cf=None, svd=None, full=None,
               dtype="fp32", max_batch=1, stream=None) -> int:
    """Returns the context handle (int).  Host arrays are FP64 numpy-compatible.  svd:
    (U [N][R], sigma [R], V [N][N][R]) for the SVD form (rom_create_svd).  full: a dict
    with any of M, C1, C2, c0, a0 for the full form (rom_create_full)."""
    L = lib()
    keep = []

    def h(a):
        if a is None:
            return _ptr(None)
        arr = np.asarray(a)
        if not (arr.dtype == np.float64 and arr.flags.c_contiguous):
            arr = _host(arr)
        keep.append(arr)
        return _ptr(arr)

    R = 0 if lam is None else int(np.asarray(lam).shape[0])
    d = rom_desc(N=int(N), R=R, nu=float(nu), dt=float(dt), A=h(A), C=h(C), lambda_=h(lam),
                 Af=h(Af), Bf=h(Bf), Cf=h(Cf), dtype=DTYPES[dtype] if isinstance(dtype, str) else int(dtype),
                 max_batch=int(max_batch), stream=_stream_handle(stream))
    out = _vp()
    if svd is not None:
        U, sig, V = svd
        Rs = int(np.asarray(U).shape[1])
        _check(L.rom_create_svd(ctypes.byref(d), Rs, h(U), h(sig), h(V), ctypes.byref(out)))
    elif full is not None:
        unknown = set(full) - {"M", "C1", "C2", "c0", "a0"}
        if unknown:
            raise ValueError(f"unknown full-form terms {sorted(unknown)}")
        f = rom_full_terms(**{k: h(full.get(k)) for k in ("M", "C1", "C2", "c0", "a0")})
        _check(L.rom_create_full(ctypes.byref(d), ctypes.byref(f), ctypes.byref(out)))
    else:
        _check(L.rom_create(ctypes.byref(d), ctypes.byref(out)))
    return out.value


def rom_cp_als(N, R, C_dev, A1_dev, A2_dev, A3_dev, sweeps, stream=None):
    """CP-ALS sweeps on device FP64 tensors (C [N][N][N], factors [N][R], updated in place)."""
    _check(lib().rom_cp_als(int(N), int(R), _dev_ptr(C_dev), _dev_ptr(A1_dev), _dev_ptr(A2_dev),
                            _dev_ptr(A3_dev), int(sweeps), _stream_handle(stream)))


def rom_cp_als_skew(N, P, C_dev, A11_dev, A12_dev, B1_dev, sweeps, subiters, momentum=0.5, stream=None):
    """ALS-skew sweeps on device FP64 tensors (C [N][N][N]; blocks [N][P], updated in place)."""
    _check(lib().rom_cp_als_skew(int(N), int(P), _dev_ptr(C_dev), _dev_ptr(A11_dev), _dev_ptr(A12_dev),
                                 _dev_ptr(B1_dev), int(sweeps), int(subiters), float(momentum),
                                 _stream_handle(stream)))


def rom_destroy(ctx: int):
    lib().rom_destroy(ctx)


def rom_nonlinear(ctx: int, batch: int, u_dev, y_dev):
    _check(lib().rom_nonlinear(ctx, int(batch), _dev_ptr(u_dev), _dev_ptr(y_dev)))


def rom_nonlinear_noalloc(ctx: int, batch: int, u_dev, y_dev):
    """rom_nonlinear with the library's fixed device scratch instead of an allocated workspace."""
    _check(lib().rom_nonlinear_noalloc(ctx, int(batch), _dev_ptr(u_dev), _dev_ptr(y_dev)))


def rom_nonlinear_timed(ctx: int, batch: int, u_dev, y_dev, reps: int) -> float:
    """rom_nonlinear with the contraction kernels launched `reps` times between two events;
    returns their average duration in microseconds."""
    us = ctypes.c_double(0.0)
    _check(lib().rom_nonlinear_timed(ctx, int(batch), _dev_ptr(u_dev), _dev_ptr(y_dev), int(reps),
                                     ctypes.byref(us)))
    return float(us.value)


def rom_state_create(ctx: int, u0) -> int:
    u0 = _host(u0)
    batch = 1 if u0.ndim == 1 else u0.shape[0]
    out = _vp()
    _check(lib().rom_state_create(ctx, batch, _ptr(u0), ctypes.byref(out)))
    return out.value


def rom_state_destroy(st: int):
    lib().rom_state_destroy(st)


def rom_step(ctx: int, st: int, nsteps: int) -> None:
    fb = ctypes.c_int64(-1)
    s = lib().rom_step(ctx, st, int(nsteps), ctypes.byref(fb))
    _check(s, fb.value)


def rom_step_async(ctx: int, st: int, nsteps: int) -> None:
    _check(lib().rom_step_async(ctx, st, int(nsteps)))


def rom_step_prepare(ctx: int, st: int, nsteps: int) -> None:
    _check(lib().rom_step_prepare(ctx, st, int(nsteps)))


def rom_step_sync(ctx: int, st: int) -> None:
    fb = ctypes.c_int64(-1)
    s = lib().rom_step_sync(ctx, st, ctypes.byref(fb))
    _check(s, fb.value)


def rom_query(ctx: Optional[int], st: Optional[int], what: int) -> int:
    v = ctypes.c_int64(0)
    _check(lib().rom_query(ctx, st, int(what), ctypes.byref(v)))
    return int(v.value)


def rom_energy(ctx: int, st: int, log: bool = True):
    B = rom_query(ctx, st, 5)
    steps = rom_query(ctx, st, 6)
    E = np.empty(B)
    Elog = np.empty((steps + 1, B)) if log else None
    _check(lib().rom_energy(ctx, st, _ptr(E), _ptr(Elog)))
    return E, Elog


def rom_state_get(ctx: int, st: int):
    B = rom_query(ctx, st, 5)
    N = rom_query(ctx, None, 2)
    uh = np.empty((3, B, N))
    yh = np.empty((2, B, N))
    step = ctypes.c_int64(0)
    _check(lib().rom_state_get(ctx, st, _ptr(uh), _ptr(yh), ctypes.byref(step)))
    return uh, yh, int(step.value)


def rom_state_set(ctx: int, st: int, u_hist, y_hist, step: int):
    uh = _host(u_hist)
    yh = _host(y_hist)
    _check(lib().rom_state_set(ctx, st, _ptr(uh), _ptr(yh), int(step)))


def rom_state_set_slot(ctx: int, st: int, b: int, u_hist, y_hist, clear_health: bool = False):
    uh = _host(u_hist)
    yh = _host(y_hist)
    _check(lib().rom_state_set_slot(ctx, st, int(b), _ptr(uh), _ptr(yh), 1 if clear_health else 0))


def rom_state_u(ctx: int, st: int, u_dev):
    _check(lib().rom_state_u(ctx, st, _dev_ptr(u_dev)))


def rom_step_multi(ctxs, states, nsteps: int):
    n = len(ctxs)
    ca = (_vp * n)(*ctxs)
    sa = (_vp * n)(*states)
    fb = ctypes.c_int64(-1)
    s = lib().rom_step_multi(n, ca, sa, int(nsteps), ctypes.byref(fb))
    _check(s, fb.value)


def rom_set_tile(ctx: int, kind: int, value: int):
    _check(lib().rom_set_tile(ctx, int(kind), int(value)))


def rom_tile_count(kind: int) -> int:
    return int(lib().rom_tile_count(int(kind)))


def rom_cp_skew_layout(lam, Af, Bf, Cf) -> int:
    """Skew column pairs of CP factors (host only): 0 none, 1 interleaved, 2 blocked."""
    lam, Af, Bf, Cf = (_host(x) for x in (lam, Af, Bf, Cf))
    N, R = Af.shape
    return int(lib().rom_cp_skew_layout(N, R, _ptr(lam), _ptr(Af), _ptr(Bf), _ptr(Cf)))


def rom_last_error() -> str:
    return lib().rom_last_error().decode(errors="replace")


# ----------------------------------------------------------------------------- objects

class Rom:
    """Owning wrapper of a context (rom_create / rom_destroy)."""

    def __init__(self, N, nu, dt, A, *, C=None, lam=None, Af=None, Bf=None, Cf=None, svd=None, full=None,
                 dtype="fp32", max_batch=1, stream=None):
        self.N = int(N)
        self.dtype = dtype
        self.max_batch = int(max_batch)
        self.stream = stream
        self.handle = rom_create(N, nu, dt, A, C=C, lam=lam, Af=Af, Bf=Bf, Cf=Cf, svd=svd, full=full,
                                 dtype=dtype, max_batch=max_batch, stream=stream)

    @classmethod
    def from_problem(cls, p, *, dense=True, dtype="fp32", max_batch=None, stream=None):
        mb = p.batch if max_batch is None else max_batch
        if dense:
            return cls(p.N, p.nu, p.dt, p.A, C=p.C, dtype=dtype, max_batch=mb, stream=stream)
        return cls(p.N, p.nu, p.dt, p.A, lam=p.lam, Af=p.Af, Bf=p.Bf, Cf=p.Cf, dtype=dtype,
                   max_batch=mb, stream=stream)

    def nonlinear(self, u_dev, y_dev=None):
        """y = C(u)u for torch device tensors.  The context works on its own stream, so
        this waits for torch's current stream before the call (u is ready) and for the
        device after it (y is ready for torch); rom_nonlinear is the asynchronous form."""
        import torch
        if y_dev is None:
            y_dev = torch.empty_like(u_dev)
        batch = 1 if u_dev.dim() == 1 else u_dev.shape[0]
        torch.cuda.current_stream().synchronize()
        rom_nonlinear(self.handle, batch, u_dev, y_dev)
        torch.cuda.synchronize()
        return y_dev

    def state(self, u0) -> "RomState":
        return RomState(self, u0)

    def set_tile(self, kind: int, value: int):
        rom_set_tile(self.handle, kind, value)

    def bytes(self) -> int:
        return rom_query(self.handle, None, 0)

    def close(self):
        if getattr(self, "handle", None):
            rom_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class RomState:
    """Owning wrapper of a batch of trajectories (rom_state_create / destroy)."""

    def __init__(self, rom: Rom, u0):
        self.rom = rom
        self.handle = rom_state_create(rom.handle, u0)

    def step(self, nsteps: int):
        rom_step(self.rom.handle, self.handle, nsteps)

    def step_async(self, nsteps: int):
        rom_step_async(self.rom.handle, self.handle, nsteps)

    def prepare(self, nsteps: int):
        rom_step_prepare(self.rom.handle, self.handle, nsteps)

    def sync(self):
        rom_step_sync(self.rom.handle, self.handle)

    def energy(self, log=True):
        return rom_energy(self.rom.handle, self.handle, log)

    def get(self):
        return rom_state_get(self.rom.handle, self.handle)

    def set(self, u_hist, y_hist, step):
        rom_state_set(self.rom.handle, self.handle, u_hist, y_hist, step)

    def set_slot(self, b, u_hist, y_hist, clear_health=False):
        rom_state_set_slot(self.rom.handle, self.handle, b, u_hist, y_hist, clear_health)

    @property
    def step_count(self) -> int:
        return rom_query(self.rom.handle, self.handle, 6)

    @property
    def resident_blocks(self) -> int:
        """Blocks of the resident runs this state's steps take from level 2 on (0: none)."""
        return rom_query(self.rom.handle, self.handle, 11)

    def u(self) -> np.ndarray:
        return self.get()[0][0]

    def bytes(self) -> int:
        return rom_query(self.rom.handle, self.handle, 1)

    def close(self):
        if getattr(self, "handle", None):
            rom_state_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
