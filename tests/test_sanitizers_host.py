"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The oracle's C library, driven through every entry point by
  tests/sanitize/oracle_main.c.
* The planner (csrc/perm.cpp with the CPU runtime double and no-op
  launchers), through tests/srvsim/plan_driver.cpp.
* The request loop (csrc/server.cpp on the runtime double), a burst, a
  paced stream with cancellations and a failed walk launch.

Each is built with gcc/g++ and -fno-sanitize-recover=all, so any finding
ends the program with a nonzero status."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SIM = os.path.join(HERE, "srvsim")
CSRC = os.path.join(ROOT, "paper_2602_10141_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]

pytestmark = pytest.mark.slow


def _need(tool):
    if shutil.which(tool) is None:
        pytest.skip(f"{tool} not available")


def _run(exe, env=None, timeout=300):
    e = dict(os.environ, ASAN_OPTIONS="abort_on_error=0:exitcode=66",
             UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=67")
    e.update(env or {})
    r = subprocess.run([exe], capture_output=True, text=True, timeout=timeout, env=e)
    assert r.returncode == 0, f"exit {r.returncode}\n{r.stdout[-2000:]}\n{r.stderr[-6000:]}"
    return r.stdout


def _compile(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]


def test_oracle_asan_ubsan(tmp_path):
    _need("gcc")
    exe = str(tmp_path / "oracle_san")
    _compile(["gcc", "-std=c11", "-ffp-contract=off", *SAN, os.path.join(ROOT, "oracle", "ryser.c"),
              os.path.join(HERE, "sanitize", "oracle_main.c"), "-o", exe])
    assert "oracle sanitize ok" in _run(exe)


def test_planner_asan_ubsan(tmp_path):
    _need("g++")
    exe = str(tmp_path / "plan_san")
    src = [os.path.join(SIM, f) for f in ("plan_driver.cpp", "plan_stubs.cpp", "sim_runtime.cpp")] + \
          [os.path.join(CSRC, f) for f in ("perm.cpp", "numth.cpp")]
    _compile(["g++", "-std=c++17", *SAN, "-I", SIM, "-I", CSRC, *src, "-o", exe, "-lpthread"])
    assert "0 failures" in _run(exe, env={"ASAN_OPTIONS": "detect_leaks=0:exitcode=66"})


def test_server_asan_ubsan(tmp_path):
    _need("g++")
    exe = str(tmp_path / "srv_san")
    src = [os.path.join(SIM, f) for f in ("sim_runtime.cpp", "sim_kernels.cpp", "sim_driver.cpp")] + \
          [os.path.join(CSRC, f) for f in ("server.cpp", "numth.cpp")]
    _compile(["g++", "-std=c++17", *SAN, "-I", SIM, "-I", CSRC, *src, "-o", exe, "-lpthread"])
    # the simulated device thread is never joined (the driver leaves with
    # _Exit), so leak checking is off
    for sc in ({"SIM_RATE": "0", "SIM_SEED": "21"},
               {"SIM_RATE": "3000", "SIM_SEED": "22", "SIM_CANCEL_EVERY": "4", "SIM_BUDGET_MB": "40"},
               {"SIM_RATE": "0", "SIM_SEED": "23", "SIM_NS_PER_ITEM": "50", "SIM_FAIL_WALK": "4"}):
        out = _run(exe, env={**sc, "SIM_BIG": "26,28,30", "ASAN_OPTIONS": "detect_leaks=0:exitcode=66"})
        assert "wrong 0 desync 0 bad_slots 0" in out, out
