"""The oracle and the library's host runtime under AddressSanitizer and
UndefinedBehaviorSanitizer, without a GPU (host code only; GPU code is never
instrumented).  The drivers check relations the code must satisfy, so a run is a
test as well as a memory check; tests/sanitize/ holds them and their build."""
import os
import subprocess

import pytest

import importlib.util

_spec = importlib.util.spec_from_file_location(
    "sanitize_build", os.path.join(os.path.dirname(os.path.abspath(__file__)), "sanitize", "build.py"))
sb = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(sb)


def _run(exe, **env):
    e = dict(os.environ)
    e.update(env)
    return subprocess.run([exe], capture_output=True, text=True, timeout=300, env=e)


def test_oracle_under_sanitizers(tmp_path):
    exe = sb.oracle_driver(str(tmp_path / "oracle_asan"))
    r = _run(exe, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all checks hold" in r.stdout


def test_oracle_driver_has_teeth(tmp_path):
    """A planted mistake in a copy of the oracle (the CP weights dropped) fails the
    driver's CP-against-dense check."""
    src = open(os.path.join(sb.ROOT, "oracle", "rom_oracle.c")).read()
    good = "acc += Af[i * R + r] * (lam[r] * s[r] * t[r]);"
    assert src.count(good) == 1
    bad = tmp_path / "rom_oracle_bad.c"
    bad.write_text(src.replace(good, "acc += Af[i * R + r] * (s[r] * t[r]);"))
    exe = str(tmp_path / "bad")
    subprocess.run(["gcc", "-std=c99", "-O1", "-fopenmp", *sb.CPU_SAN, str(bad),
                    os.path.join(sb.HERE, "oracle_asan.c"), "-o", exe, "-lm"], check=True)
    r = _run(exe, ASAN_OPTIONS="detect_leaks=0")
    assert r.returncode == 1 and "cp equals dense of the reconstruction" in r.stderr


def test_abi_host_checks_under_sanitizers():
    exe = sb.abi_driver()
    r = _run(exe, ASAN_OPTIONS="detect_leaks=1", HIP_VISIBLE_DEVICES="")
    if "mode=gpu" in r.stdout:
        pytest.skip("a GPU is visible: the GPU run is test_gpu_sanitize")
    assert r.returncode == 0, r.stdout + r.stderr
    assert "mode=host" in r.stdout and "all checks hold" in r.stdout
