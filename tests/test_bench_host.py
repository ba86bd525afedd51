"""CPU tests of bench.py's contract: one GPU only, a loud failure without a
GPU, and the roofline arithmetic (instruction counts per Glynn term, the
fraction of the FP64 VALU peak, and measured traffic only for the kernel
sources the counters were taken on)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def run_bench(*args, timeout=300):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=timeout,
                          env={**os.environ, "HIP_VISIBLE_DEVICES": os.environ.get("HIP_VISIBLE_DEVICES", "")})


def test_more_than_one_gpu_is_refused():
    r = run_bench("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


@pytest.mark.skipif(os.environ.get("GRAFT_REPO_ROOT") is not None, reason="a GPU box has a GPU")
def test_no_gpu_fails_loudly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    r = run_bench("--workload", "single14")
    assert r.returncode != 0 and r.stdout == ""
    assert "no GPU" in r.stderr


def test_instruction_counts_per_term():
    # c128: 2n flip adds, 4(n-1) complex-product ops, (3 + 4) / 4 per component
    assert bench.ops_per_term("c128", 20) == 40 + 76 + 3.5
    assert bench.ops_per_term("c128", 20, kahan=False) == 40 + 76 + 2.0
    # f64: n adds, n-1 products, (3 + 4) / 4
    assert bench.ops_per_term("f64", 20) == 20 + 19 + 1.75
    # F_p Barrett: n adds, 6 per product, 1 accumulate = 7n - 5
    assert bench.ops_per_term("modp", 28) == 7 * 28 - 5


def test_roofline_fraction_and_peak():
    peak = 256 * 4 * 16 * 2.4e9                       # FP64 VALU lane-ops/s
    ops = peak * 2e-3 * 0.5                           # per launch: half the peak for 2 ms
    r = bench.roofline(ops, walk_ms=20.0, launches=10)
    assert r["bound"] == "alu" and r["peak"] == round(peak / 1e12, 3)
    assert r["frac"] == 0.5 and r["kernel_avg_ms"] == 2.0 and r["launches"] == 10
    f = bench.roofline(ops, walk_ms=2.0, launches=1, flops_ratio=2.0)
    assert f["tflops"] == round(2 * f["achieved"], 3)


def test_measured_traffic_follows_the_kernel_sources(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0123456789abcdef")
    prof = tmp_path / "profiles" / "traffic.txt"
    prof.write_text("source_hash: 0123456789abcdef\nbytes_per_launch: 12345\n")
    assert bench.measured_traffic("traffic.txt") == 12345.0
    prof.write_text("source_hash: 0000000000000000\nbytes_per_launch: 12345\n")
    assert bench.measured_traffic("traffic.txt") is None
    assert bench.measured_traffic("no_such_profile.txt") is None


def test_cpu_baseline_states_the_host_and_its_sample():
    """The oracle baseline names its thread count, the host's CPU count and
    model, and an all-core figure that is labelled as a linear estimate."""
    from paper_2602_10141_amd import ensembles as E
    mats = [(E.ginibre_real(8, E.rng(90, i)), "f64") for i in range(40)]
    r = bench.cpu_baseline_many(mats, None, seconds=0.2, label="test")
    assert r["kind"] == "oracle" and r["unit"] == "perms/s" and r["value"] > 0
    assert r["cores"] == min(bench.HOST_THREADS, os.cpu_count())
    assert r["nproc"] == os.cpu_count() and "cpu_model" in r
    assert r["all_cores_linear_estimate"] == r["value_1thread"] * r["nproc"]
    assert "of the 40 test matrices" in r["sample"]


def test_default_workload_is_the_headline_with_sub_records():
    assert bench.WORKLOADS["default"] is bench.bench_default
    import inspect
    src = inspect.getsource(bench.bench_default)
    for key in ("single_haar_u14_c128", "haar_u20_c128_50000", "haar_o20_f64_50000",
                "ragged_gaussian_10000", "serve_stream_530", "single_matrix_orders_20_36"):
        assert key in src


def test_range_baseline_is_scaled_to_glynn_terms():
    """The single-matrix baseline: disjoint subset ranges on every host
    thread, reported per Glynn term (half a Ryser subset)."""
    from paper_2602_10141_amd import ensembles as E
    r = bench.cpu_baseline_range(E.haar_unitary(20, E.rng(90, 0)), "c128", seconds=0.1)
    assert r["kind"] == "oracle" and r["value"] > 0 and r["cores"] >= 1
    assert r["unit"].startswith("subset-terms/s") and "order 20" in r["sample"]


def test_shard_count_must_divide_the_range():
    """The shard workload cuts [0, 2^(n-1)) into equal Gray ranges; a count
    that does not divide it is refused before any device work."""
    import argparse
    args = argparse.Namespace(shard_n=36, shards=3, no_cpu=True)
    with pytest.raises(SystemExit):
        bench.bench_shard(None, None, args)
