"""The exported host code (AMG set-up, restart eigensolvers) built with g++
under AddressSanitizer and UndefinedBehaviorSanitizer and run on a CPU
driver (tests/host_sanitize/driver.cpp): hierarchies of symmetric,
variable-coefficient and nonsymmetric operators, the nonzero bounds of the
fused transfer operators, eigen-decompositions of random matrices, and the
non-convergence status on a NaN input."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1405_0707_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not installed")
def test_host_code_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "host_sanitize")
    build = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-I", CSRC,
             os.path.join(HERE, "host_sanitize", "driver.cpp"),
             os.path.join(CSRC, "amg_host.cpp"), os.path.join(CSRC, "eig_host.cpp"), "-o", exe]
    subprocess.run(build, check=True, capture_output=True, text=True, timeout=300)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    print(run.stdout[-4000:])
    assert run.returncode == 0, run.stdout[-2000:] + run.stderr[-4000:]
    assert "ALL OK" in run.stdout
