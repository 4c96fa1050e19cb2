"""CPU: the library's host code (layout generator, ASCII parser, configuration
validation, reset image, state-image checks) and the oracle, built with
AddressSanitizer and UndefinedBehaviorSanitizer (g++/gcc, no GPU) and run over
valid, hostile and mangled inputs (tests/sanitize/*).  Any memory or
undefined-behaviour error, or a failed check, fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2605_19926_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _build_and_run(tmp_path, compiler, args, name):
    exe = str(tmp_path / name)
    r = subprocess.run([compiler] + SAN + args + ["-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
    return out


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_library_host_code_under_sanitizers(tmp_path):
    out = _build_and_run(tmp_path, "g++", [
        "-std=c++17", "-pthread", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-I/opt/rocm/include",
        os.path.join(ROOT, "tests", "sanitize", "host_checks.cpp"), os.path.join(CSRC, "jx_host.cpp"),
        os.path.join(CSRC, "jx_layout.cpp")], "host_checks")
    assert "host checks: 0 failures" in out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    out = _build_and_run(tmp_path, "gcc", [
        "-std=c11", "-D_DEFAULT_SOURCE", "-I" + os.path.join(ROOT, "oracle"),
        os.path.join(ROOT, "tests", "sanitize", "oracle_checks.c"), os.path.join(ROOT, "oracle", "jx_oracle.c"),
        "-lm"], "oracle_checks")
    assert "oracle checks: 0 failures" in out
