"""CPU-side code built with the address and undefined-behaviour sanitizers:
the oracle (oracle/oracle.c) driven through every exported entry point by
tests/host/oracle_driver.c, and the library's exchange-fold index arithmetic
(tests/host/twin_index.cpp, host code only).  A memory or undefined-behaviour
error aborts the program, which fails the test.  No GPU is used."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(exe):
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=ENV)
    assert run.returncode == 0, (run.stdout[-2000:], run.stderr[-4000:])
    assert run.stdout.startswith("ok")


def test_oracle_under_sanitizers(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not found")
    exe = tmp_path / "oracle_driver"
    build = subprocess.run(
        ["gcc", "-O1", "-g", "-std=c11", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=all", "-ffp-contract=off", "-frounding-math",
         os.path.join(ROOT, "tests", "host", "oracle_driver.c"),
         os.path.join(ROOT, "oracle", "oracle.c"), "-o", str(exe), "-lm"],
        capture_output=True, text=True)
    assert build.returncode == 0, build.stderr[-2000:]
    _run(exe)


def test_exchange_index_arithmetic_under_sanitizers(tmp_path):
    if not (os.path.exists(HIPCC) or shutil.which(HIPCC)):
        pytest.skip("hipcc not found")
    exe = tmp_path / "twin_index"
    src = tmp_path / "twin_index.hip"
    shutil.copy(os.path.join(ROOT, "tests", "host", "twin_index.cpp"), src)
    # the sanitizers instrument the host code only
    build = subprocess.run(
        [HIPCC, "-O1", "-g", "-std=c++17", "--offload-arch=gfx950",
         "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
         "-I" + os.path.join(ROOT, "include"),
         "-I" + os.path.join(ROOT, "paper_2407_10925_amd", "csrc"), str(src), "-o", str(exe)],
        capture_output=True, text=True)
    assert build.returncode == 0, build.stderr[-2000:]
    _run(exe)
