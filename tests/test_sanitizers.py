"""The oracle and the library's host-side code under AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU (no GPU is touched): each driver under
tests/sanitize/ is built with both sanitizers and run; any memory error or
undefined behaviour aborts it.  The library build instruments host code only
(each sanitizer flag behind -Xarch_host)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")


def _run(exe):
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=ENV)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "runtime error" not in out.stderr and "ERROR: AddressSanitizer" not in out.stderr, out.stderr
    return out.stdout


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    subprocess.run(["gcc", "-std=c99", "-O1", "-g", "-ffp-contract=off", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    os.path.join(HERE, "sanitize", "oracle_driver.c"), "-lm", "-o", exe], check=True)
    assert "rc 0" in _run(exe)


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"), reason="no hipcc")
def test_host_validation_under_sanitizers(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    exe = str(tmp_path / "host_validation")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    subprocess.run([hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-ffp-contract=off", *san,
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument",
                    "-Wno-pass-failed", "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_1303_2653_amd", "csrc"),
                    os.path.join(HERE, "sanitize", "host_validation.cpp"),
                    os.path.join(ROOT, "paper_1303_2653_amd", "csrc", "lbdps.hip"), "-o", exe],
                   check=True, capture_output=True)
    assert "0 failures" in _run(exe)
