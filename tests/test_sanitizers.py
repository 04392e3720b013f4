"""Host-side AddressSanitizer and UndefinedBehaviorSanitizer runs (CPU only):
the oracle (gcc) over every placement at small and ragged sizes, and the
library's host runtime (its planner, tuning table and argument checks,
built with the sanitizers on the host side of hipcc only) without a GPU.
Each driver checks its own results and exits non-zero on a failure; the
sanitizers abort on the first error they find."""
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT = os.path.join(ROOT, "_build", "sanitize")
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, (" ".join(cmd), r.stdout[-3000:], r.stderr[-3000:])
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is not installed")
def test_oracle_under_asan_and_ubsan():
    os.makedirs(OUT, exist_ok=True)
    exe = os.path.join(OUT, "oracle_driver")
    _run(["gcc", "-O1", "-g", "-fopenmp", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
          "-fno-omit-frame-pointer", os.path.join(ROOT, "oracle", "ms_oracle.c"),
          os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"), "-o", exe, "-lm"])
    r = _run([exe], env=SAN_ENV, timeout=600)
    assert "0 bad" in r.stdout and "runtime error" not in r.stderr, (r.stdout, r.stderr[-3000:])


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc"), reason="hipcc is not installed")
def test_host_runtime_under_asan_and_ubsan():
    from paper_1508_03167_amd import build as B

    os.makedirs(OUT, exist_ok=True)
    # the kernels as built for the library (built here if missing); the host
    # runtime again with the sanitizers on its host side
    kernels = []
    for src in B.SOURCES[1:]:
        obj = os.path.join(B.BUILD, os.path.splitext(src)[0] + ".o")
        if not os.path.exists(obj):
            os.makedirs(B.BUILD, exist_ok=True)
            B._compile(src)
        kernels.append(obj)
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    api = os.path.join(OUT, "ms_api.o")
    _run([B.HIPCC, "-O1", "-g", "-std=c++17", f"--offload-arch={B.ARCH}", "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops", *san, "-I", os.path.join(ROOT, "include"), "-c",
          os.path.join(B.CSRC, "ms_api.hip"), "-o", api])
    drv = os.path.join(OUT, "host_driver.o")
    _run(["/opt/rocm/llvm/bin/clang++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"),
          "-c", os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"), "-o", drv])
    exe = os.path.join(OUT, "host_driver")
    _run([B.HIPCC, f"--offload-arch={B.ARCH}", *san, drv, api, *kernels, "-o", exe])
    r = _run([exe], env=SAN_ENV, timeout=600)
    assert "0 bad" in r.stdout and "runtime error" not in r.stderr, (r.stdout, r.stderr[-3000:])
