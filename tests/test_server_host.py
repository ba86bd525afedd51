"""The request loop's host logic (admission, slicing over two streams, event
ordering, counter bookkeeping, cancellation, shutdown) on the CPU: server.cpp
is compiled against a test double of the HIP runtime whose "device" runs the
streams' commands in random interleavings, with kernels that tag partial slots
instead of computing permanents.  Every served result must carry its own
matrix's hash with no stale, skipped or misplaced slot, and nothing may hang."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SIM = os.path.join(HERE, "srvsim")
CSRC = os.path.join(HERE, "..", "paper_2602_10141_amd", "csrc")
SOURCES = [os.path.join(SIM, f) for f in ("sim_runtime.cpp", "sim_kernels.cpp", "sim_driver.cpp")] + \
          [os.path.join(CSRC, f) for f in ("server.cpp", "numth.cpp")]
CLANG = "/opt/rocm/llvm/bin/clang++"


def _build(out, compiler, extra):
    cmd = [compiler, "-std=c++17", "-g", "-I", SIM, "-I", CSRC, *extra, *SOURCES, "-o", out,
           "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    return out


@pytest.fixture(scope="module")
def sim(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    return _build(str(tmp_path_factory.mktemp("srvsim") / "srvsim"), "g++", ["-O2"])


def run(binary, timeout=240, **env):
    e = dict(os.environ)
    e.update({f"SIM_{k.upper()}": str(v) for k, v in env.items()})
    r = subprocess.run([binary], capture_output=True, text=True, timeout=timeout, env=e)
    assert r.returncode == 0, f"exit {r.returncode}\n{r.stdout[-2000:]}\n{r.stderr[-4000:]}"
    return r.stdout


@pytest.mark.parametrize("scenario", [
    dict(rate=0, seed=1),                                   # the whole stream at once
    dict(rate=3000, seed=2, ns_per_item=100),               # paced arrivals, device time
    dict(rate=0, seed=3, budget_mb=40, ns_per_item=50),     # admission waits for memory
    dict(rate=0, seed=4, max_inflight=1, budget_mb=36),     # one request at a time
    dict(rate=0, seed=5, cancel_every=3, budget_mb=40),     # cancellations
    dict(rate=0, seed=6, cancel_every=2, max_inflight=3, slice_us=300),
], ids=["burst", "paced", "budget", "inflight1", "cancel", "cancel_inflight3"])
def test_served_results_intact(sim, scenario):
    out = run(sim, **scenario)
    assert "wrong 0 desync 0 bad_slots 0" in out, out


@pytest.mark.parametrize("scenario", [
    dict(rate=0, seed=11, ns_per_item=100, fail_walk=5),            # a walk launch fails
    dict(rate=0, seed=12, ns_per_item=100, fail_event_sync=4),      # a slice's event reports an error
    dict(rate=3000, seed=13, ns_per_item=100, fail_walk=9),         # paced, mid-stream
    dict(rate=0, seed=14, budget_mb=40, ns_per_item=50, fail_walk=3),   # memory-bound admission
    dict(rate=0, seed=15, cancel_every=3, budget_mb=40, fail_event_sync=7),
], ids=["walk_burst", "event_burst", "walk_paced", "walk_budget", "event_cancel"])
def test_device_errors_fail_only_the_affected_requests(sim, scenario):
    """Fault injection in the runtime double: a failed walk launch or an
    event that reports an error.  The requests with work in the failed slice
    report PERM_EDEVICE; every other request completes with its own result;
    no descriptor slot or arena range is handed to a new request while work
    of the old one is in flight (checked by every walk item and finalize);
    the statistics count each request once."""
    out = run(sim, **scenario)
    assert "wrong 0 desync 0 bad_slots 0" in out, out
    failed = int(out.split("failed ")[-1].split()[0])
    assert failed >= 1, out


def test_repeated_servers_in_one_process(sim):
    out = run(sim, rate=0, seed=7, reps=3, big="26,28,30")
    assert out.count("wrong 0 desync 0 bad_slots 0") == 3, out


@pytest.mark.slow
def test_no_data_races(tmp_path):
    """ThreadSanitizer over a burst, a paced stream and a failed walk launch
    (clang's runtime)."""
    if not os.path.exists(CLANG):
        pytest.skip("clang with ThreadSanitizer not available")
    b = _build(str(tmp_path / "srvsim_tsan"), CLANG, ["-O1", "-fsanitize=thread"])
    for sc in (dict(rate=0, seed=8), dict(rate=2000, seed=9, cancel_every=4, budget_mb=40),
               dict(rate=0, seed=10, ns_per_item=50, fail_walk=4)):
        env = dict(sc, big="26,28,30")
        e = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")
        e.update({f"SIM_{k.upper()}": str(v) for k, v in env.items()})
        r = subprocess.run([b], capture_output=True, text=True, timeout=600, env=e)
        assert r.returncode == 0, r.stderr[-6000:]
