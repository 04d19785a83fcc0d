"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The library's host-only sources (tbpm_host.cpp: coefficients, sample
average, DOS, moment and response transforms, the patch planner's entry
points; tbpm_bessel.cpp; tbpm_patch.cpp) build with g++ alone, and the
oracle with gcc.  Each is linked with a C driver under tests/sanitize/ that
calls every function on generated inputs and on invalid arguments; any
sanitizer report aborts the driver (-fno-sanitize-recover=all), and leaks
are reported at exit.  No device code is built here: only host compilers run.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2509_26309_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300, **kw)
    assert r.returncode == 0, " ".join(cmd) + "\n" + r.stdout + r.stderr
    return r


@pytest.fixture(scope="module")
def tools():
    if not shutil.which("gcc") or not shutil.which("g++"):
        pytest.skip("gcc / g++ not found")
    return True


def test_host_library_code_under_sanitizers(tools, tmp_path):
    objs = []
    for src in ("tbpm_host.cpp", "tbpm_bessel.cpp", "tbpm_patch.cpp"):
        o = str(tmp_path / (src + ".o"))
        _run(["g++", "-std=c++17", "-Wall", "-Wextra", "-Werror", *SAN, "-I", os.path.join(ROOT, "include"), "-c",
              os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    drv = str(tmp_path / "host_checks.o")
    _run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", *SAN, "-I", os.path.join(ROOT, "include"), "-c",
          os.path.join(ROOT, "tests", "sanitize", "host_checks.c"), "-o", drv])
    exe = str(tmp_path / "host_checks")
    _run(["g++", *SAN, drv, *objs, "-o", exe, "-lm"])
    r = _run([exe], env=ENV)
    assert r.stdout.rstrip().endswith("done"), r.stdout
    assert "runtime error" not in r.stderr


def test_oracle_under_sanitizers(tools, tmp_path):
    exe = str(tmp_path / "oracle_checks")
    _run(["gcc", "-std=c11", "-Wall", "-Wextra", *SAN, "-fopenmp", "-ffp-contract=off",
          os.path.join(ROOT, "tests", "sanitize", "oracle_checks.c"), os.path.join(ROOT, "oracle", "tbpm_oracle.c"),
          "-o", exe, "-lm"])
    r = _run([exe], env=dict(ENV, OMP_NUM_THREADS="2"))
    assert r.stdout.rstrip().endswith("done"), r.stdout
    assert "runtime error" not in r.stderr
