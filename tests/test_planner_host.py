"""The planner (csrc/perm.cpp) on the CPU: compiled against the HIP runtime
test double with no-op launchers, it must tile every matrix's Gray range
exactly once with aligned chunks and one partial slot per item, keep launch
groups homogeneous and sorted largest first, keep staged matrices apart,
and reuse a cached plan only while inputs and chunk lengths are unchanged
(tests/srvsim/plan_driver.cpp)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SIM = os.path.join(HERE, "srvsim")
CSRC = os.path.join(HERE, "..", "paper_2602_10141_amd", "csrc")


def test_planner_invariants(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "plan_driver")
    src = [os.path.join(SIM, f) for f in ("plan_driver.cpp", "plan_stubs.cpp", "sim_runtime.cpp")] + \
          [os.path.join(CSRC, f) for f in ("perm.cpp", "numth.cpp")]
    r = subprocess.run(["g++", "-std=c++17", "-O2", "-I", SIM, "-I", CSRC, *src, "-o", exe,
                        "-lpthread"], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "0 failures" in r.stdout
