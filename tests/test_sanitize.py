"""CPU: AddressSanitizer and UndefinedBehaviorSanitizer builds.

* The oracle (plain C, gcc) with a driver that runs every entry point on
  small seeded problems, ties, duplicate rows, K = N, one point, M = 16 and
  rejected arguments, checking invariants that hold for any input.
* The host side of libnsga3 (hipcc, sanitizers on the host code only) with a
  driver that calls what needs no device: version and status strings, the
  workspace-size arithmetic over the whole size range, and every entry point
  with arguments its checks reject before any HIP call.

Any out-of-bounds access, leak or undefined operation fails the run.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
ORACLE = [os.path.join(ROOT, "oracle", f) for f in ("oracle.c", "rvea.c", "hype.c", "variation.c")]
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{cmd[0]} failed ({r.returncode}):\n{r.stdout}\n{r.stderr[-4000:]}"
    return r


def test_oracle_under_asan_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_san")
    _run(["gcc", "-std=c11", "-g", "-O1", "-fopenmp", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-ffp-contract=off",
          os.path.join(HERE, "oracle_driver.c"), *ORACLE, "-o", exe, "-lm"])
    r = _run([exe], env=dict(SAN_ENV, OMP_NUM_THREADS="4"), timeout=300)
    assert "ok" in r.stdout


def test_host_abi_under_asan_ubsan(tmp_path):
    sys.path.insert(0, os.path.join(ROOT, "paper_2503_20286_amd"))
    try:
        import build as nbuild
    finally:
        sys.path.pop(0)
    try:
        hipcc = nbuild.hipcc()
    except RuntimeError:
        pytest.skip("hipcc not found")
    clang = os.path.join(os.path.dirname(os.path.realpath(hipcc)), "..", "llvm", "bin", "clang")
    if not os.path.exists(clang):
        clang = "/opt/rocm/llvm/bin/clang"
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    flags = [f"--offload-arch={nbuild.ARCH}", "-O1", "-g", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", nbuild.INCLUDE, "-I", nbuild.CSRC, *host_san]
    objs, procs = [], []
    for src in nbuild.SOURCES:
        obj = str(tmp_path / src.replace(".hip", ".o"))
        objs.append(obj)
        procs.append((src, subprocess.Popen([hipcc, *flags, "-c", os.path.join(nbuild.CSRC, src),
                                             "-o", obj], stdout=subprocess.PIPE,
                                            stderr=subprocess.STDOUT)))
    for src, p in procs:
        out, _ = p.communicate()
        assert p.returncode == 0, f"{src}:\n{out.decode(errors='replace')[-4000:]}"
    drv = str(tmp_path / "abi_driver.o")
    _run([clang, "-std=c11", "-g", "-O1", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-D__HIP_PLATFORM_AMD__", "-I", nbuild.INCLUDE,
          "-I", "/opt/rocm/include", "-c", os.path.join(HERE, "abi_driver.c"), "-o", drv])
    exe = str(tmp_path / "abi_san")
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(hipcc)))
    _run([clang + "++", "-fsanitize=address,undefined", drv, *objs,
          "-L", os.path.join(rocm, "lib"), "-Wl,-rpath," + os.path.join(rocm, "lib"),
          "-lamdhip64", "-o", exe])
    r = _run([exe], env=SAN_ENV, timeout=300)
    assert "ok" in r.stdout
