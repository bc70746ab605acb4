"""Host code under sanitizers (CPU): the library's host SELL-C-sigma builder (build.cpp, with its
thread pool) on random CSR matrices under AddressSanitizer + UndefinedBehaviorSanitizer and under
ThreadSanitizer, and the C oracle's routines under AddressSanitizer + UndefinedBehaviorSanitizer.
Each harness (tests/sanitize/) also checks its own invariants and exits non-zero on a failure;
a sanitizer report aborts the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_1507_08101_amd", "csrc")


def _compile(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        if "sanitizer" in r.stderr.lower() and "cannot find" in r.stderr.lower():
            pytest.skip("sanitizer runtime not installed")
        raise AssertionError(r.stderr[-3000:])


def _run(exe, *args):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1",
               TSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe, *args], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "ERROR: " not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    return r.stdout


def _host_builder_cmd(out, sanitizers):
    return ["g++", "-std=c++17", "-O1", "-g", *sanitizers, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
            f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}", os.path.join(SAN, "host_builder_check.cpp"),
            os.path.join(CSRC, "build.cpp"), "-o", out, "-lpthread"]


@pytest.mark.skipif(shutil.which("g++") is None, reason="no g++")
def test_host_builder_asan_ubsan(tmp_path):
    exe = str(tmp_path / "hb_asan")
    _compile(_host_builder_cmd(exe, ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"]))
    assert "cases ok" in _run(exe, "60")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no g++")
def test_host_builder_tsan(tmp_path):
    exe = str(tmp_path / "hb_tsan")
    _compile(_host_builder_cmd(exe, ["-fsanitize=thread"]))
    assert "cases ok" in _run(exe, "15")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")
def test_oracle_asan_ubsan(tmp_path):
    exe = str(tmp_path / "orc_asan")
    _compile(["gcc", "-std=c11", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
              "-fopenmp", "-ffp-contract=off", f"-I{os.path.join(ROOT, 'oracle')}",
              os.path.join(SAN, "oracle_check.c"), os.path.join(ROOT, "oracle", "oracle.c"), "-o", exe, "-lm"])
    assert "calls ok" in _run(exe)
