"""The library's host runtime (rom_api.hip) under AddressSanitizer and
UndefinedBehaviorSanitizer on a GPU: every operator form through creation, stepping
(graphs, resident runs, grouped steps), restart, slot replacement, evaluation and
destruction, and CP-ALS / ALS-skew, with the driver's bitwise relations checked.  The
GPU kernels are the regular build's; only host code is instrumented.  The executable
is built beforehand with the library (tests/sanitize/build.py)."""
import os
import subprocess
import sys

import pytest

import importlib.util

_spec = importlib.util.spec_from_file_location(
    "sanitize_build", os.path.join(os.path.dirname(os.path.abspath(__file__)), "sanitize", "build.py"))
sb = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(sb)

pytestmark = pytest.mark.gpu


def test_abi_under_host_sanitizers():
    if not os.path.exists(sb.ABI_EXE):
        pytest.fail(f"{sb.ABI_EXE} is not built (run the package build first)")
    print("[case] abi driver under host ASan/UBSan", flush=True)
    sys.stdout.flush()
    env = dict(os.environ)
    # detect_leaks=0: the HIP runtime's own allocations at exit.  A quarantine of freed
    # memory large enough that nothing is recycled at exit: when the HIP runtime is
    # unloaded, its destructors free memory, and a recycle at that point reaches chunks
    # of ASan's device allocator after the device runtime is gone, which ASan rejects
    # with an internal CHECK (observed in the runtime's __cxa_finalize, after every
    # check of the driver had run).  The larger quarantine catches more use-after-free.
    env["ASAN_OPTIONS"] = "detect_leaks=0:quarantine_size_mb=8192"
    r = subprocess.run([sb.ABI_EXE], capture_output=True, text=True, timeout=240, env=env)
    assert r.returncode == 0, (r.stdout + r.stderr)[-6000:]
    assert "mode=gpu" in r.stdout and "all checks hold" in r.stdout
