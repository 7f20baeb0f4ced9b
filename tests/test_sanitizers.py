"""AddressSanitizer + UndefinedBehaviorSanitizer runs of the native host code
(CPU only): the oracle's C layer definitions, and the library's host-only code
(the placement's host layer code and genetic search), each driven by a small
native program on ragged shapes (tests/native/).  The sanitizers abort the
program on any out-of-bounds access, use after free, leak or undefined
behaviour; the test fails on a non-zero exit."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _run(cmd, exe, tmp_path):
    subprocess.run(cmd, check=True, cwd=ROOT)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
               DN_CPU_THREADS="4")
    r = subprocess.run([exe], env=env, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-4000:]
    return r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_check")
    out = _run(["gcc"] + SAN + ["-std=c99", "-o", exe, "tests/native/oracle_check.c", "oracle/oracle.c", "-lm"],
               exe, tmp_path)
    assert "oracle checks ran" in out


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_library_code_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_code_check")
    csrc = "paper_1811_03882_amd/csrc"
    out = _run(["g++"] + SAN + ["-std=c++17", "-march=x86-64-v3", "-pthread", "-I", csrc, "-o", exe,
                                "tests/native/host_code_check.cpp", csrc + "/cpu_layers.cpp", csrc + "/ga.cpp"],
               exe, tmp_path)
    assert "host code checks passed" in out
