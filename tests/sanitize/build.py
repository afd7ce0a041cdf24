"""Sanitizer builds (test infrastructure).

* ``oracle_driver(out)``: the FP64 oracle (oracle/rom_oracle.c) with oracle_asan.c, built by
  gcc with AddressSanitizer and UndefinedBehaviorSanitizer.
* ``abi_driver()``: the library's host runtime (rom_api.hip) rebuilt with both sanitizers
  on its host code only, linked with the kernel objects of the regular build and with
  abi_asan.cpp into ``tests/sanitize/bin/abi_asan``.  GPU code is never instrumented.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

BIN = os.path.join(HERE, "bin")
ABI_EXE = os.path.join(BIN, "abi_asan")
CLANG = "/opt/rocm/llvm/bin/clang++"
ROCM_INC = "/opt/rocm/include"
ROCM_LIB = "/opt/rocm/lib"
# Sanitizer options: -Xarch_host keeps each of them off the GPU side of a hipcc line.
HIP_HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
CPU_SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"{cmd[0]} failed:\n{r.stderr[-4000:]}")


def oracle_driver(out: str) -> str:
    """Build the oracle and its driver with both sanitizers into the executable `out`."""
    src = [os.path.join(ROOT, "oracle", "rom_oracle.c"), os.path.join(HERE, "oracle_asan.c")]
    _run(["gcc", "-std=c99", "-O1", "-g", "-Wall", "-fopenmp", "-ffp-contract=off", *CPU_SAN, *src, "-o", out,
          "-lm"])
    return out


def abi_driver(verbose: bool = False) -> str:
    from paper_2311_03694_amd import build as hb

    objs = []
    for src in hb.SOURCES:
        if src == "rom_api.hip":
            continue
        obj = os.path.join(hb.BUILD, os.path.splitext(src)[0] + ".o")
        if not os.path.exists(obj) or os.path.getmtime(obj) < os.path.getmtime(os.path.join(hb.CSRC, src)):
            hb.build()
        objs.append(obj)
    os.makedirs(hb.BUILD, exist_ok=True)
    os.makedirs(BIN, exist_ok=True)
    flags = [f for f in hb.FLAGS if f != "-O3"]
    api_obj = os.path.join(hb.BUILD, "rom_api_asan.o")
    _run([hb.HIPCC, *flags, "-O1", "-g", *HIP_HOST_SAN, "-Wno-unused-result", "-c",
          os.path.join(hb.CSRC, "rom_api.hip"), "-o", api_obj])
    drv_obj = os.path.join(hb.BUILD, "abi_asan.o")
    _run([CLANG, "-std=c++17", "-O1", "-g", *CPU_SAN, "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
          "-I", ROCM_INC, "-c", os.path.join(HERE, "abi_asan.cpp"), "-o", drv_obj])
    tmp = ABI_EXE + ".tmp"
    _run([CLANG, *CPU_SAN, drv_obj, api_obj, *objs, "-L", ROCM_LIB, "-lamdhip64", f"-Wl,-rpath,{ROCM_LIB}",
          "-o", tmp])
    os.replace(tmp, ABI_EXE)
    if verbose:
        print(f"built {ABI_EXE}")
    return ABI_EXE


if __name__ == "__main__":
    abi_driver(verbose=True)
