"""The C ABI library loads on a host without a GPU, exports every symbol that
include/rom.h declares, and rejects invalid descriptions before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2311_03694_amd as rg
import romsynth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_header_symbols_are_exported():
    hdr = open(os.path.join(ROOT, "include", "rom.h")).read()
    declared = set(re.findall(r"\b(rom_[a-z_0-9]+)\s*\(", hdr))
    assert declared == set(rg.EXPORTS), declared ^ set(rg.EXPORTS)
    L = rg.lib()
    for name in declared:
        assert hasattr(L, name), name


def test_desc_layout_matches_header():
    # rom_desc: int32 N, int32 R, double nu, double dt, 6 pointers, int32 dtype,
    # int32 max_batch, void* stream  (x86-64 / LP64 layout)
    assert ctypes.sizeof(rg.binding.rom_desc) == 4 + 4 + 8 + 8 + 6 * 8 + 4 + 4 + 8
    assert rg.binding.rom_desc.stream.offset == 80


@pytest.mark.parametrize("kw,msg", [
    (dict(N=0), "N must be"),
    (dict(dt=0.0), "dt must be"),
    (dict(dt=float("nan")), "dt must be"),
    (dict(nu=-1.0), "nu must be"),
    (dict(dtype=7), "unknown dtype"),
    (dict(max_batch=0), "max_batch"),
    (dict(C=None), "CP rank"),
    (dict(A=None), "stiffness A"),
])
def test_create_rejects_invalid(kw, msg):
    N = 4
    args = dict(N=N, nu=1e-3, dt=1e-3, A=np.eye(N), C=np.zeros((N, N, N)), dtype="fp32", max_batch=1)
    args.update(kw)
    dt = args.pop("dtype")
    with pytest.raises(rg.RomError) as ei:
        rg.rom_create(args.pop("N"), args.pop("nu"), args.pop("dt"), args.pop("A"), dtype=dt, **args)
    assert ei.value.status == rg.binding.ROM_E_INVALID
    assert msg in str(ei.value)


def test_cp_without_factors_rejected():
    N = 4
    with pytest.raises(rg.RomError) as ei:
        rg.rom_create(N, 1e-3, 1e-3, np.eye(N), lam=np.ones(2), Af=np.ones((N, 2)), dtype="fp32")
    assert "needs lambda" in str(ei.value)


def test_null_handles_rejected():
    with pytest.raises(rg.RomError):
        rg.rom_query(None, None, 0)
    assert rg.rom_tile_count(0) >= 1
    assert rg.rom_tile_count(99) == 0


def test_cp_skew_layout_host_check():
    """Skew column pairs (Sec. 3.3, eq. skew_abc_struct) are recognised exactly on the
    host: the generator's interleaved pairs, the paper's blocks, and nothing else."""
    lam, Af, Bf, Cf = romsynth.skew_cp_factors(9, 5, seed=1, cfg=3)
    assert rg.rom_cp_skew_layout(lam, Af, Bf, Cf) == 1
    perm = np.concatenate([np.arange(0, 10, 2), np.arange(1, 10, 2)])     # pairs -> blocks
    assert rg.rom_cp_skew_layout(lam[perm], Af[:, perm], Bf[:, perm], Cf[:, perm]) == 2
    Cb = Cf.copy()
    Cb[4, 3] = np.nextafter(Cb[4, 3], np.inf)                             # one ulp off
    assert rg.rom_cp_skew_layout(lam, Af, Bf, Cb) == 0
    lb = lam.copy()
    lb[1] *= 2.0
    assert rg.rom_cp_skew_layout(lb, Af, Bf, Cf) == 0
    assert rg.rom_cp_skew_layout(lam[:9], Af[:, :9], Bf[:, :9], Cf[:, :9]) == 0   # odd rank
    rng = np.random.default_rng(0)
    assert rg.rom_cp_skew_layout(*(rng.standard_normal(s) for s in [(6,), (9, 6), (9, 6), (9, 6)])) == 0


@pytest.mark.parametrize("kw,status,msg", [
    (dict(R=0), "ROM_E_INVALID", "SVD rank"),
    (dict(V=None), "ROM_E_INVALID", "needs U, sigma and V"),
    (dict(C=True), "ROM_E_INVALID", "takes no dense tensor"),
    (dict(max_batch=2), "ROM_E_UNSUPPORTED", "one trajectory"),
])
def test_create_svd_rejects_invalid(kw, status, msg):
    """rom_create_svd checks its description before any device work."""
    N, R = 5, kw.get("R", 3)
    U = np.ones((N, max(R, 1)))
    sig = np.ones(max(R, 1))
    V = None if "V" in kw else np.ones((N, N, max(R, 1)))
    C = np.zeros((N, N, N)) if kw.get("C") else None
    A = np.eye(N)
    d = rg.binding.rom_desc(N=N, R=0, nu=1e-3, dt=1e-3, A=rg.binding._ptr(A),
                            C=rg.binding._ptr(C), dtype=1, max_batch=kw.get("max_batch", 1))
    out = ctypes.c_void_p()
    st = rg.lib().rom_create_svd(ctypes.byref(d), R, rg.binding._ptr(U), rg.binding._ptr(sig),
                                 rg.binding._ptr(V), ctypes.byref(out))
    assert st == getattr(rg.binding, status)
    assert msg in rg.rom_last_error()


def test_lds_staging_limit_rejected():
    """One-trajectory kernels stage u in 64 KB of LDS: a BF16 CP context at N = 6000 (two
    images of 6 bytes per mode) is refused before any device work."""
    N, R = 6000, 2
    f = np.ones((N, R))
    with pytest.raises(rg.RomError) as ei:
        rg.rom_create(N, 1e-3, 1e-3, np.eye(1), lam=np.ones(R), Af=f, Bf=f, Cf=f, dtype="bf16")
    assert ei.value.status == rg.binding.ROM_E_UNSUPPORTED
    assert "LDS staging of u" in str(ei.value)


@pytest.mark.parametrize("case,status,msg", [
    ("null_terms", "ROM_E_INVALID", "full terms are NULL"),
    ("asymmetric_mass", "ROM_E_INVALID", "not symmetric"),
    ("too_large", "ROM_E_UNSUPPORTED", "N <= 4096"),
])
def test_create_full_rejects_invalid(case, status, msg):
    """rom_create_full checks its terms before any device work."""
    N = 4100 if case == "too_large" else 6
    R = 1
    A = np.eye(N)
    lam, Af = np.ones(R), np.ones((N, R))
    d = rg.binding.rom_desc(N=N, R=R, nu=1e-3, dt=1e-3, A=rg.binding._ptr(A), lambda_=rg.binding._ptr(lam),
                            Af=rg.binding._ptr(Af), Bf=rg.binding._ptr(Af), Cf=rg.binding._ptr(Af),
                            dtype=1, max_batch=1)
    M = np.eye(N) if N < 100 else None
    if case == "asymmetric_mass":
        M[2, 1] = 0.25
    f = rg.binding.rom_full_terms(M=rg.binding._ptr(M))
    out = ctypes.c_void_p()
    fp = None if case == "null_terms" else ctypes.byref(f)
    st = rg.lib().rom_create_full(ctypes.byref(d), fp, ctypes.byref(out))
    assert st == getattr(rg.binding, status)
    assert msg in rg.rom_last_error()
    assert out.value is None


@pytest.mark.parametrize("args,msg", [
    ((0, 3, 1), "N must be"),
    ((5, 0, 1), "R must be"),
    ((5, 3, -1), "sweeps must be"),
])
def test_cp_als_rejects_invalid(args, msg):
    """rom_cp_als checks its sizes before any device work."""
    N, R, sweeps = args
    st = rg.lib().rom_cp_als(N, R, 1, 1, 1, 1, sweeps, None)
    assert st == rg.binding.ROM_E_INVALID
    assert msg in rg.rom_last_error()


def test_cp_als_rejects_null():
    st = rg.lib().rom_cp_als(5, 3, None, 1, 1, 1, 1, None)
    assert st == rg.binding.ROM_E_INVALID
    assert "NULL" in rg.rom_last_error()


def test_missing_library_fails_loudly(monkeypatch):
    """Without librom.so every call raises: there is no CPU fallback."""
    monkeypatch.setattr(rg.binding, "_lib", None)
    monkeypatch.setattr(rg.binding, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "librom.so"))
    with pytest.raises(RuntimeError, match="librom.so not found"):
        rg.binding.lib()
    with pytest.raises(RuntimeError, match="librom.so not found"):
        rg.rom_last_error()


def test_full_terms_layout_matches_header():
    # rom_full_terms: five pointers M, C1, C2, c0, a0 (LP64)
    assert ctypes.sizeof(rg.binding.rom_full_terms) == 5 * 8
    assert rg.binding.rom_full_terms.a0.offset == 32


def test_als_skew_rejects_arguments():
    """rom_cp_als_skew checks its arguments before touching a device."""
    L = rg.lib()
    for args, msg in [((0, 2, None, None, None, None, 1, 1, 0.5, None), b"N must be"),
                      ((4, 0, None, None, None, None, 1, 1, 0.5, None), b"P must be"),
                      ((4, 2, None, None, None, None, 1, -1, 0.5, None), b"subiters"),
                      ((4, 2, None, None, None, None, 1, 1, 1.0, None), b"momentum"),
                      ((4, 2, None, None, None, None, 1, 1, 0.5, None), b"NULL")]:
        assert L.rom_cp_als_skew(*args) == rg.binding.ROM_E_INVALID
        assert msg in L.rom_last_error()


def test_dense_stiffness_size_limit_refused_on_host():
    """A non-diagonal stiffness is solved through an explicit inverse that stages N doubles
    in LDS: N > 4096 is refused before any device work (here N = 8200 with CP factors in
    FP32, whose own LDS staging of u would still fit)."""
    N, R = 8200, 2
    A = np.zeros((N, N))
    A[0, 1] = A[1, 0] = 0.5
    f = np.zeros((N, R))
    with pytest.raises(rg.RomError) as ei:
        rg.rom_create(N, 1e-3, 1e-3, A, lam=np.ones(R), Af=f, Bf=f, Cf=f, dtype="fp32")
    assert ei.value.status == rg.binding.ROM_E_UNSUPPORTED
    assert "non-diagonal stiffness" in str(ei.value)
