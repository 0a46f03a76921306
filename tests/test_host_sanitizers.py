"""The library's host code (paper_1408_2981_amd/csrc/mesh.cpp, operator.cpp:
the grid hierarchy and geometry of Section 4.2 and the assembly of Appendix
A) built with g++ under AddressSanitizer and UndefinedBehaviorSanitizer and
driven through every path by tests/host/host_checks.cpp, which also checks
invariants that hold without the oracle (areas tile the sphere, symmetric
neighbours, children tile their parent, coarse mass conserved, proper
colourings, positive coefficients) and that invalid inputs are refused. Any
sanitizer report ends the program with a non-zero status."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1408_2981_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_code_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_checks")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-ffp-contract=off", "-I", os.path.join(ROOT, "include"),
           os.path.join(HERE, "host", "host_checks.cpp"), os.path.join(CSRC, "mesh.cpp"),
           os.path.join(CSRC, "operator.cpp"), "-o", exe]
    build = subprocess.run(cmd, capture_output=True, text=True)
    assert build.returncode == 0, build.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    print(run.stdout[-2000:])
    assert run.returncode == 0, (run.stdout[-4000:], run.stderr[-4000:])
    assert "host checks passed" in run.stdout
