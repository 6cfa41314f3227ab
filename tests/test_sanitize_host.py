"""The library's host-only code (dense Hermitian eigensolver, quadrature, Cholesky)
built with g++ under AddressSanitizer and UndefinedBehaviorSanitizer, and run on the
sizes and inputs the library meets (tests/sanitize/host_check.cpp). No device."""
import shutil
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent
CSRC = ROOT / "paper_1004_0292_amd" / "csrc"


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_code_under_asan_and_ubsan(tmp_path):
    exe = tmp_path / "host_check"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-DSSCG_NO_TARGET_CLONES", f"-I{CSRC}", str(ROOT / "tests" / "sanitize" / "host_check.cpp"),
           str(CSRC / "dense_host.cpp"), str(CSRC / "quad_host.cpp"), "-o", str(exe)]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert b.returncode == 0, b.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300,
                       env={"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0", "UBSAN_OPTIONS": "print_stacktrace=1"})
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failures" in r.stdout
