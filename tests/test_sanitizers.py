"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host code
(CPU only): the FP64 oracle and the library's host-side setup
(paper_1906_06327_amd/csrc/sscn_setup.cpp: validation, coefficients,
windows, pivot tables), each driven through valid and invalid inputs by a
small driver (tests/sanitize/).  Any sanitizer report fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _build_and_run(tmp_path, compiler, srcs, includes, extra):
    exe = str(tmp_path / "driver")
    cmd = [compiler] + SAN + [f"-I{d}" for d in includes] + srcs + ["-o", exe] + extra
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    # verify_asan_link_order=0: the environment may preload a library of its
    # own ahead of the sanitizer runtime
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=240)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    return r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers(tmp_path):
    out = _build_and_run(tmp_path, "gcc",
                         [os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
                          os.path.join(ROOT, "oracle", "sscn_oracle.c")],
                         [os.path.join(ROOT, "oracle")], ["-std=c11", "-fopenmp", "-lm"])
    assert "oracle driver: ok" in out


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_library_setup_under_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_1906_06327_amd", "csrc")
    out = _build_and_run(tmp_path, "g++",
                         [os.path.join(ROOT, "tests", "sanitize", "setup_driver.cpp"),
                          os.path.join(csrc, "sscn_setup.cpp")],
                         [csrc, os.path.join(ROOT, "include")], ["-std=c++17"])
    assert "setup driver: ok" in out
