"""Benchmark of the Gray-code Glynn permanent path on one MI355X.

Default workload (one "step" = the whole hot path once): the exact integer
permanent of the Schur matrix S_28 by CRT over the three smallest 31-bit
primes p = 1 (mod 28) -- per prime the residue matrix (g^{jk} mod p) already
resident in HBM, then stage, Gray-code walk over 2^27 Glynn terms, fixed-order
reduction and 2^-(27) scaling on the device, then the Garner lift on the host.
Throughput is Glynn subset-terms per second (2^(n-1) per permanent).  The
same line carries, under "configs", one sub-record per other workload of the
metric: a single 14x14 Haar unitary (latency), 50,000 Haar U(20) and O(20)
in one launch each, 10,000 ragged Gaussian matrices, and the serving stream
(p50/p99 per class at 0.5/0.7/0.9 of saturation); each with the median of
at least five timed launches, the walk kernel's roofline and the oracle's
CPU baseline.

Single workloads (--workload): schur28 (the S_28 line alone), single14 (one
14x14 Haar unitary, c128),
haar20 (50,000 Haar U(20) c128 and 50,000 Haar O(20) f64 in one persistent
launch each), ragged (10,000 GUE/GOE/real and complex Ginibre matrices,
n uniform in 8..24, one fused launch), serve (Poisson-arrival geodesic and
Schur requests through the request loop; p50/p99 latency), schur_odd (exact
perm(S_n) for odd n through checkpointed CRT jobs with a redundant prime),
stats (50,000 Haar U(n) and O(n) permanents per odd n in 7..23 and their
distribution checks), dft (the DFT-geodesic fingerprint r(n)), shard (one
GPU's share of perm(S_36) spread over eight: eight Gray-index ranges through
perm_range, whose partials must add up to the single call's residue), sizes
(one matrix per call at orders 20..36).

Prints one JSON line.  The oracle (CPU Ryser) is timed on a bounded prefix of
the same computation for the "cpu_baseline" field.
"""
import argparse
import json
import math
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "Ryser subset-terms/s (c128, F_p) n=20–36; batched perms/s; served p50/p99"
PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9        # FP64 VALU lane-ops/s: 256 CUs x 4 SIMD16 x 2.4 GHz
PEAK_FP64_FLOPS = 78.6e12                    # FMA counted twice
HOST_THREADS = 16                            # host threads for the oracle baseline (one GPU's CPU share)


def ops_per_term(field: str, n: int, kahan: bool = True) -> float:
    """Algorithmic FP64 VALU instructions per Glynn term (one lane, one step).
    Floats: four consecutive terms are combined as (t0 - t1) + (t2 - t3) (3
    adds) and enter the compensated sum once (4 ops; 1 without Kahan), per
    real component."""
    if field == "c128":        # 2n flip adds + 4(n-1) complex-product ops + group sum
        return 2 * n + 4 * (n - 1) + 2 * ((3 + (4 if kahan else 1)) / 4)
    if field == "f64":         # n flip adds + (n-1) products + group sum
        return n + (n - 1) + (3 + (4 if kahan else 1)) / 4
    # F_p, exact Barrett in binary64: n flip adds + 6 per modular product + 1 accumulate
    return n + 6 * (n - 1) + 1


def sync():
    import torch
    torch.cuda.synchronize()


KERNEL_SOURCES = ["paper_2602_10141_amd/csrc/walk_impl.h", "paper_2602_10141_amd/csrc/walk_common.hip",
                  "paper_2602_10141_amd/csrc/kernels.h"]


def kernel_source_hash():
    """sha256 over the walk kernel's sources (instantiation files excluded)."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(profile):
    """HBM bytes per walk launch from a committed counter summary (FETCH_SIZE
    and WRITE_SIZE passes scaled by a plain copy), or None when the kernel
    sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", profile)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and line.split(":")[0].strip() in ("source_hash", "bytes_per_launch"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_hash") != kernel_source_hash() or "bytes_per_launch" not in vals:
        return None
    return float(vals["bytes_per_launch"])


def flops_per_op(field: str, n: int) -> float:
    """FP64 flops per algorithmic instruction (an FMA counts two) of the walk."""
    if field == "c128":        # 2(n-1) of the 4(n-1) product instructions are FMAs
        return (ops_per_term("c128", n) + 2 * (n - 1)) / ops_per_term("c128", n)
    if field == "f64":
        return 1.0
    return (ops_per_term("modp", n) + 2 * (n - 1) - (n - 1)) / ops_per_term("modp", n)   # 2 FMAs, 1 rint


def roofline(ops_per_launch, walk_ms, launches, traffic=None, flops_ratio=None):
    avg_s = walk_ms / max(launches, 1) * 1e-3
    achieved = ops_per_launch / avg_s / 1e12
    peak = PEAK_LANE_OPS / 1e12
    out = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 3),
           "unit": "Tlane-op/s (FP64 VALU)", "frac": round(achieved / peak, 4),
           "traffic": traffic, "kernel_avg_ms": round(avg_s * 1e3, 4),
           "launches": launches}
    if flops_ratio is not None:
        out["tflops"] = round(achieved * flops_ratio, 3)
        out["tflops_of_78_6"] = round(achieved * flops_ratio / (PEAK_FP64_FLOPS / 1e12), 4)
    return out


# ---------------------------------------------------------------- CPU baseline
def host_info():
    """The host the oracle ran on: logical CPUs, CPUs this process may use,
    and the CPU model (as lscpu prints it, from /proc/cpuinfo)."""
    info = {"nproc": os.cpu_count()}
    try:
        info["affinity_cpus"] = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        pass
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    info["cpu_model"] = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return info


def _with_host(d):
    """Add the host description and an all-core figure: the one-thread rate
    times nproc, i.e. linear scaling, an estimate (the oracle runs on the
    16 threads of one GPU's host share, never on every core of the box)."""
    h = host_info()
    d.update(h)
    if d.get("value_1thread") and h.get("nproc"):
        d["all_cores_linear_estimate"] = d["value_1thread"] * h["nproc"]
    return d


def _threads():
    return min(HOST_THREADS, os.cpu_count() or 1)


def _run_threads(work, count):
    """work(0) .. work(count - 1) on threads of their own; the first
    exception a worker raised is raised here once all have ended."""
    errors = []

    def run(i):
        try:
            work(i)
        except BaseException as e:
            errors.append(e)

    ths = [threading.Thread(target=run, args=(i,)) for i in range(count)]
    for th in ths:
        th.start()
    for th in ths:
        th.join()
    if errors:
        raise errors[0]


def cpu_baseline_schur(n, primes, seconds=12.0):
    """Oracle Ryser mod p on S_n, bounded prefix, all host threads."""
    from oracle import crt, native
    mats = [crt.schur_residues(n, p) for p in primes]
    threads = _threads()
    # calibrate one thread on a short prefix
    t = time.perf_counter()
    native.ryser_modp_prefix(mats[0], primes[0], 1 << 18)
    rate1 = (1 << 18) / (time.perf_counter() - t)
    per_thread = int(min(1 << n, max(1 << 18, rate1 * seconds)))
    done = []

    def work(i):
        native.ryser_modp_prefix(mats[i % len(mats)], primes[i % len(primes)], per_thread)
        done.append(per_thread - 1)

    t = time.perf_counter()
    _run_threads(work, threads)
    dt = time.perf_counter() - t
    ryser_subsets_per_s = sum(done) / dt
    # one permanent = 2^n Ryser subsets on the CPU = 2^(n-1) Glynn terms in the metric
    value = ryser_subsets_per_s / (1 << n) * (1 << (n - 1))
    return _with_host({
        "value": value, "unit": "subset-terms/s (Glynn-term equivalents)", "cores": threads,
        "kind": "oracle", "value_1thread": rate1 / 2,
        "sample": f"oracle Ryser mod p on S_{n}: first {per_thread - 1} of 2^{n} subsets per "
                  f"thread, {threads} threads in {dt:.1f} s; rate scaled to 2^{n - 1} terms "
                  f"per permanent"})


def _oracle_perm(A, field):
    from oracle import native
    return native.ryser_c128(A) if field == "c128" else native.ryser_f64(A)


def cpu_baseline_many(mats, field, seconds=5.0, label=None):
    """The oracle on the matrices of a batch, one whole matrix per host
    thread at a time, threads taking the next matrix of a seeded random order
    until `seconds` have passed; every matrix started is finished and
    counted.  mats: list of (A, field) or arrays of one field."""
    import queue
    mats = [m if isinstance(m, tuple) else (m, field) for m in mats]
    order = np.random.Generator(np.random.PCG64(7)).permutation(len(mats))
    threads = _threads()
    # one thread, a few matrices: the per-core rate
    t = time.perf_counter()
    k1 = 0
    while k1 < len(mats) and (k1 < 2 or time.perf_counter() - t < 0.5):
        _oracle_perm(*mats[order[k1]])
        k1 += 1
    rate1 = k1 / (time.perf_counter() - t)
    q = queue.SimpleQueue()
    for i in order:
        q.put(int(i))
    done = [0] * threads
    t0 = time.perf_counter()

    def work(w):
        while time.perf_counter() - t0 < seconds:
            try:
                i = q.get_nowait()
            except queue.Empty:
                return
            _oracle_perm(*mats[i])
            done[w] += 1

    _run_threads(work, threads)
    dt = time.perf_counter() - t0
    return _with_host({
        "value": sum(done) / dt, "unit": "perms/s", "cores": threads, "kind": "oracle",
        "value_1thread": rate1,
        "sample": f"oracle Ryser on {sum(done)} of the {len(mats)} {label or field} matrices "
                  f"(seeded random order, {threads} threads, {dt:.1f} s)"})


def cpu_baseline_single(A, seconds=2.0):
    """One matrix: the oracle's latency on one thread (median of 5 groups)
    and its throughput with every host thread computing the same matrix."""
    from oracle import native
    t = time.perf_counter()
    native.ryser_c128(A)
    once = time.perf_counter() - t
    per = max(1, int(0.1 / max(once, 1e-9)))
    groups = []
    for _ in range(5):
        t = time.perf_counter()
        for _ in range(per):
            native.ryser_c128(A)
        groups.append((time.perf_counter() - t) / per)
    lat = float(np.median(groups))
    threads = _threads()
    counts = [0] * threads
    t0 = time.perf_counter()

    def work(w):
        while time.perf_counter() - t0 < seconds:
            native.ryser_c128(A)
            counts[w] += 1

    _run_threads(work, threads)
    dt = time.perf_counter() - t0
    return _with_host({
        "value": sum(counts) / dt, "unit": "perms/s", "cores": threads, "kind": "oracle",
        "value_1thread": 1.0 / lat, "us_per_call_1thread": lat * 1e6,
        "sample": f"oracle Ryser on the same matrix: 5 x {per} calls on one thread, then "
                  f"{sum(counts)} calls on {threads} threads in {dt:.1f} s"})


def cpu_baseline_serve(P, reqs, seconds_schur=2.0):
    """The oracle on the serving stream, in the stream's unit (Glynn-term
    equivalents per second), from a sample: 16 geodesic points per order (of
    64), and for each Schur order a Ryser prefix of S_n on every thread.
    The time of the whole stream on the host threads is extrapolated from
    the sample (per-order mean time x count), and stated as such."""
    from oracle import native
    threads = _threads()
    total_s = 0.0
    notes = []
    import concurrent.futures as cf
    for n in range(11, 26, 2):
        pts = [r[0] for r in reqs if r[3] == "geodesic" and r[4] == n][:16]
        t = time.perf_counter()
        with cf.ThreadPoolExecutor(threads) as ex:
            list(ex.map(native.ryser_c128, pts))
        dt = time.perf_counter() - t
        cnt = sum(1 for r in reqs if r[3] == "geodesic" and r[4] == n)
        total_s += dt * cnt / len(pts)
        notes.append(f"n={n}: {len(pts)} pts in {dt:.2f} s")
    for n in sorted({r[4] for r in reqs if r[3] == "schur"}):
        rs = [r for r in reqs if r[3] == "schur" and r[4] == n]
        A, _, p = rs[0][0], rs[0][1], rs[0][2]
        t = time.perf_counter()
        native.ryser_modp_prefix(A, p, 1 << 18)
        rate1 = (1 << 18) / (time.perf_counter() - t)
        per = int(max(1 << 18, rate1 * seconds_schur))
        t = time.perf_counter()
        with cf.ThreadPoolExecutor(threads) as ex:
            list(ex.map(lambda i: native.ryser_modp_prefix(A, p, per), range(threads)))
        dt = time.perf_counter() - t
        rate = threads * (per - 1) / dt                 # Ryser subsets per second
        total_s += len(rs) * (1 << n) / rate
        notes.append(f"S_{n}: {per - 1} subsets x {threads} threads in {dt:.2f} s")
    terms = sum(1 << (r[0].shape[0] - 1) for r in reqs)
    return _with_host({
        "value": terms / total_s, "unit": "subset-terms/s (Glynn-term equivalents)",
        "cores": threads, "kind": "oracle", "extrapolated": True,
        "stream_seconds_estimate": total_s,
        "sample": "oracle on a sample of the serving stream, whole-stream time extrapolated: " +
                  "; ".join(notes)})


def median_launches(fn, reps):
    """fn() `reps` times, each followed by a device synchronisation; the
    wall time of each (seconds)."""
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        sync()
        ts.append(time.perf_counter() - t0)
    return ts


def progress(msg):
    print(msg, file=sys.stderr, flush=True)


# ------------------------------------------------------------------ workloads
def bench_schur(P, ctx, args):
    """S_28 over its three primes; each step is one synchronous perm_crt_int
    (residues back on the host, CRT lift), so a step's host time is its
    duration."""
    import torch
    n = 28
    primes = P.perm_schur_primes(n)
    mats = torch.from_numpy(np.stack([P.perm_schur_residues(n, p) for p in primes])
                            .astype(np.int32)).cuda()
    bound = (n / 2) * math.log2(n)
    flags = P.PERM_MONTGOMERY if args.montgomery else 0
    for _ in range(args.warmup):
        val, res = P.perm_crt_int(ctx, mats, primes, bound, flags=flags)
    sync()
    P.perm_prof_enable(ctx, True)
    P.perm_prof_read(ctx)
    steps_s = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        val, res = P.perm_crt_int(ctx, mats, primes, bound, flags=flags)
        steps_s.append(time.perf_counter() - ts)
    sync()
    dt = time.perf_counter() - t0
    walk_ms, launches = P.perm_prof_read(ctx)
    P.perm_prof_enable(ctx, False)
    assert val == 0 and res == [0] * len(primes), (val, res)   # even n: perm(S_n) = 0
    terms = len(primes) * (1 << (n - 1))
    line = {
        "metric": METRIC, "value": terms * args.steps / dt, "unit": "subset-terms/s",
        "ms_per_step": dt / args.steps * 1e3, "dtype": "f64",
        "median_ms_per_step": float(np.median(steps_s)) * 1e3,
        "config": {"workload": "schur_S28_crt_3primes", "n": n, "primes": primes,
                   "field": ("F_p (32-bit Montgomery walk)" if args.montgomery
                             else "F_p (exact FP64 Barrett walk)") + " + CRT",
                   "terms_per_step": terms, "perm": val},
        # (Montgomery is priced at the Barrett walk's instruction count, so
        # the two fractions compare throughput directly)
        "roofline": roofline(terms * ops_per_term("modp", n), walk_ms, launches,
                             None if args.montgomery else
                             measured_traffic("traffic_walk_modp_n28_schur_S28_crt.txt"),
                             flops_per_op("modp", n)),
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline_schur(n, primes)
    return line


def sub_single14(P, ctx, args, calls=200, groups=5):
    """Config 1: one 14x14 Haar unitary per call, device pointers, result
    left on the device; median per-call time over `groups` groups of
    `calls` back-to-back calls.  Timing events add about 9 us to a call, so
    the kernel duration comes from a second, profiled pass.  Beside it: the
    same call through perm_c128_noalloc, each call waited for before the
    next (isolated latency), and the matrix handed over in host memory with
    the result returned to the host (both copies inside the call)."""
    import torch
    from paper_2602_10141_amd import ensembles as E
    A = E.haar_unitary(14, E.rng(1, 0))
    U = torch.from_numpy(A).cuda()
    for _ in range(20):
        P.perm_c128(ctx, U)
    sync()
    per_call = []
    for _ in range(groups):
        t0 = time.perf_counter()
        for _ in range(calls):
            P.perm_c128(ctx, U)
        sync()
        per_call.append((time.perf_counter() - t0) / calls)
    P.perm_prof_enable(ctx, True)
    P.perm_prof_read(ctx)
    for _ in range(calls):
        P.perm_c128(ctx, U)
    sync()
    walk_ms, launches = P.perm_prof_read(ctx)
    P.perm_prof_enable(ctx, False)
    med = float(np.median(per_call))
    # the same call through perm_c128_noalloc (static scratch, no allocation)
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    na = []
    for _ in range(groups):
        t0 = time.perf_counter()
        for _ in range(calls):
            P.perm_c128_noalloc(ctx, U, out=out)
        sync()
        na.append((time.perf_counter() - t0) / calls)
    # isolated calls: each waited for before the next (result on the device),
    # and from host memory to a Python complex (both copies inside the call)
    iso, host = [], []
    for _ in range(groups):
        t0 = time.perf_counter()
        for _ in range(calls):
            P.perm_c128(ctx, U)
            sync()
        iso.append((time.perf_counter() - t0) / calls)
        t0 = time.perf_counter()
        for _ in range(calls):
            P.perm_c128(ctx, A)
        host.append((time.perf_counter() - t0) / calls)
    rec = {"workload": "haar_unitary_14_c128", "n": 14, "value": 1.0 / med, "unit": "perms/s",
           "us_per_call_median": med * 1e6, "timed": f"{groups} groups of {calls} calls",
           "noalloc_us_per_call_median": float(np.median(na)) * 1e6,
           "isolated_us_per_call_median": float(np.median(iso)) * 1e6,
           "host_buffers_us_per_call_median": float(np.median(host)) * 1e6, "dtype": "c128",
           "roofline": roofline((1 << 13) * ops_per_term("c128", 14), walk_ms, launches, None,
                                flops_per_op("c128", 14))}
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_baseline_single(A)
    return rec


def sub_batch(P, ctx, args, workload, mats, reps=5, cpu_label=None):
    """Configs 3 and 4: one perm_batch of all `mats` ((A, field, p) triples),
    inputs resident in HBM, results left on the device; one warm-up launch,
    then `reps` launches back to back (the host plans launch k + 1 while the
    device runs launch k, as a caller streaming batches would), each timed
    between HIP events on the stream: the median is the value.  The median
    of `reps` synchronised launches (host planning on the critical path) is
    reported beside it."""
    import torch
    items, data = P.pack_matrices(mats)
    d = torch.from_numpy(data).cuda()
    res = torch.zeros((len(mats), 2), dtype=torch.float64, device="cuda")
    fn = lambda: P.perm_batch(ctx, items, d, out=res)    # noqa: E731
    fn()
    sync()
    P.perm_prof_enable(ctx, True)
    P.perm_prof_read(ctx)
    ts = median_launches(fn, max(5, reps))
    walk_ms, launches = P.perm_prof_read(ctx)
    P.perm_prof_enable(ctx, False)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(max(5, reps) + 1)]
    evs[0].record()
    for e in evs[1:]:
        fn()
        e.record()
    sync()
    pipe = [evs[i].elapsed_time(evs[i + 1]) * 1e-3 for i in range(len(evs) - 1)]
    sync_med = float(np.median(ts))
    med = float(np.median(pipe))
    ns = [m[0].shape[0] for m in mats]
    fields = sorted({m[1] for m in mats})
    terms = sum(1 << (k - 1) for k in ns)
    ops = sum((1 << (m[0].shape[0] - 1)) * ops_per_term(m[1], m[0].shape[0]) for m in mats)
    flops = sum((1 << (m[0].shape[0] - 1)) * ops_per_term(m[1], m[0].shape[0]) *
                flops_per_op(m[1], m[0].shape[0]) for m in mats)
    rec = {"workload": workload, "count": len(mats), "value": len(mats) / med, "unit": "perms/s",
           "median_ms": med * 1e3, "timed_launches": len(pipe),
           "launch_ms": [round(t * 1e3, 3) for t in pipe], "terms_per_s": terms / med,
           "sync_median_ms": sync_med * 1e3, "sync_launch_ms": [round(t * 1e3, 3) for t in ts],
           "value_sync": len(mats) / sync_med,
           "dtype": "+".join(fields),
           "roofline": roofline(ops * len(ts) / max(launches, 1), walk_ms, launches, None,
                                flops / ops)}
    if not args.no_compare:
        one = per_matrix_launches(P, ctx, items, d, 2000)
        one["batched_speedup"] = rec["value"] / one["perms_per_s"]
        rec["one_launch_per_matrix"] = one
        t0 = time.perf_counter()
        P.perm_batch(ctx, items, data)
        rec["host_buffers_perms_per_s"] = len(mats) / (time.perf_counter() - t0)
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_baseline_many([(m[0], m[1]) for m in mats], None,
                                                label=cpu_label or workload)
    return rec


def bench_single14(P, ctx, args):
    rec = sub_single14(P, ctx, args)
    return {"metric": METRIC, "value": rec["value"], "unit": "perms/s",
            "ms_per_step": rec["us_per_call_median"] * 1e-3, "dtype": "c128",
            "config": {"workload": rec["workload"], "n": 14}, "roofline": rec["roofline"],
            **({"cpu_baseline": rec["cpu_baseline"]} if "cpu_baseline" in rec else {}),
            "detail": rec}


def haar20_inputs(count):
    from paper_2602_10141_amd import ensembles as E
    U = E.haar_unitary(20, E.rng(3, 0), count=count)
    O = E.haar_orthogonal(20, E.rng(3, 1), count=count)
    return U, O


def bench_haar20(P, ctx, args):
    U, O = haar20_inputs(args.count)
    out = {"c128": sub_batch(P, ctx, args, "haar_unitary_20_c128", [(m, "c128", 0) for m in U]),
           "f64": sub_batch(P, ctx, args, "haar_orthogonal_20_f64", [(m, "f64", 0) for m in O])}
    line = {"metric": METRIC, "value": out["c128"]["value"], "unit": "perms/s",
            "ms_per_step": out["c128"]["median_ms"] + out["f64"]["median_ms"], "dtype": "c128",
            "config": {"workload": "haar20_batched", "count": args.count, "n": 20},
            "roofline": out["c128"]["roofline"], "detail": out}
    if "cpu_baseline" in out["c128"]:
        line["cpu_baseline"] = out["c128"]["cpu_baseline"]
    return line


def per_matrix_launches(P, ctx, items, d, sample):
    """The same matrices through one library call (stage, walk, finalize
    launches) per matrix, device pointers, results left on the device: the
    comparator for the batched form.  The chunk length of each (field, n) is
    first autotuned for a single matrix, so the comparator runs in its own
    best configuration.  Returns perms/s over the first `sample` items and
    the summed walk-kernel time per matrix."""
    import ctypes
    import torch
    sample = min(sample, len(items))
    names = {P.PERM_C128: "c128", P.PERM_F64: "f64"}
    shapes = sorted({(int(it["field"]), int(it["n"])) for it in items[:sample]})
    for f, n in shapes:
        P.perm_autotune(ctx, names[f], n, n, batch=1)
    chunks = {f"{names[f]}{n}": P.perm_tune_get(ctx, names[f], n)[0] for f, n in shapes}
    out = torch.zeros((sample, 2), dtype=torch.float64, device="cuda")
    base, optr = d.data_ptr(), out.data_ptr()
    st = P._stream(None)
    fns = {P.PERM_C128: P.lib().perm_c128, P.PERM_F64: P.lib().perm_f64}

    def run(lo, hi):
        for i in range(lo, hi):
            it = items[i]
            rc = fns[int(it["field"])](ctx.ptr, ctypes.c_void_p(base + int(it["offset"])),
                                       int(it["n"]), ctypes.c_void_p(optr + 16 * i),
                                       P.PERM_DEVICE_PTRS, st)
            if rc != P.PERM_OK:
                raise P.PermError(rc, "per-matrix call failed")

    run(0, min(sample, 64))
    sync()
    # timed without the per-launch events (they add about 9 us per call),
    # walk time from a second, profiled pass
    t0 = time.perf_counter()
    run(0, sample)
    sync()
    dt = time.perf_counter() - t0
    P.perm_prof_enable(ctx, True)
    P.perm_prof_read(ctx)
    run(0, sample)
    sync()
    walk_ms, _ = P.perm_prof_read(ctx)
    P.perm_prof_enable(ctx, False)
    for f, n in shapes:
        P.perm_tune_set(ctx, names[f], n, 0)          # back to the library default
    out = {"perms_per_s": sample / dt, "sample": sample,
           "walk_ms_per_matrix": walk_ms / sample, "wall_ms_per_matrix": dt * 1e3 / sample}
    if len(chunks) <= 4:
        out["log2_chunk"] = chunks
    return out


def ragged_inputs(count, seed=4):
    from paper_2602_10141_amd import ensembles as E
    g = E.rng(seed, 0)
    ns = g.integers(8, 25, size=count)
    kinds = g.integers(0, 4, size=count)
    mats = []
    for n, k in zip(ns, kinds):
        n = int(n)
        if k == 0:
            mats.append((E.gue(n, g), "c128", 0))
        elif k == 1:
            mats.append((E.goe(n, g), "f64", 0))
        elif k == 2:
            mats.append((E.ginibre_real(n, g), "f64", 0))
        else:
            mats.append((E.ginibre_complex(n, g), "c128", 0))
    return mats


def bench_ragged(P, ctx, args):
    rec = sub_batch(P, ctx, args, "ragged_gaussian_n8_24", ragged_inputs(args.count),
                    cpu_label="ragged GUE/GOE/Ginibre")
    line = {"metric": METRIC, "value": rec["value"], "unit": "perms/s",
            "ms_per_step": rec["median_ms"], "dtype": rec["dtype"],
            "config": {"workload": rec["workload"], "count": rec["count"]},
            "roofline": rec["roofline"], "detail": rec}
    if "cpu_baseline" in rec:
        line["cpu_baseline"] = rec["cpu_baseline"]
    return line


def serve_requests(P):
    """512 geodesic points (odd n in 11..25, 64-point t grid, principal branch,
    c128) and 18 Schur residue matrices (n in 32, 34, 36; six primes each)."""
    from paper_2602_10141_amd import ensembles as E
    reqs = []
    for n in range(11, 26, 2):
        for t in E.geodesic_grid(64):
            reqs.append((E.cycle_geodesic(n, t), "c128", 0, "geodesic", n))
    for n in (32, 34, 36):
        k = len(P.perm_schur_primes(n))
        for p in P.perm_schur_primes(n, extra=6 - k):
            reqs.append((P.perm_schur_residues(n, p), "modp", p, "schur", n))
    order = E.rng(5, 0).permutation(len(reqs))
    return [reqs[i] for i in order]


SERVE_FLOAT_CHUNK = 9


def serve_tuning(P, ctx, on=True):
    """Serving favours latency: the geodesic orders get wave items of at most
    64 x 2^9 indices (a walk of about 0.1 ms) through the context's tuning
    table, which perm_batch on the same context then shares, so that served
    and batched results stay bit-identical.  on=False restores the
    defaults."""
    for n in range(11, 26, 2):
        if on:
            c = P.perm_tune_get(ctx, "c128", n)[0]
            P.perm_tune_set(ctx, "c128", n, min(c, SERVE_FLOAT_CHUNK))
        else:
            P.perm_tune_set(ctx, "c128", n, 0)


def _serve_run(P, ctx, reqs, rate, seed, slice_us):
    """Submit reqs with exponential inter-arrival times of mean 1/rate (rate =
    None: all at once); collect results and per-request latencies."""
    import threading as th
    srv = P.Server(ctx, hbm_budget=8 << 30, slice_us=slice_us)
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([260210141, 5, seed])))
    gaps = g.exponential(1.0 / rate, size=len(reqs)) if rate else np.zeros(len(reqs))
    tickets = [None] * len(reqs)
    t0 = time.perf_counter()

    errors = []

    def submitter():
        t = t0
        try:
            for i, (A, f, p, _, _) in enumerate(reqs):
                t += gaps[i]
                d = t - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                tickets[i] = srv.submit(A, f, p)
        except BaseException as e:          # surfaced by the collecting loop
            errors.append(e)

    sub = th.Thread(target=submitter)
    sub.start()
    vals, lats, phases = [None] * len(reqs), [0.0] * len(reqs), [None] * len(reqs)
    try:
        for i in range(len(reqs)):
            while tickets[i] is None:
                if errors:
                    raise RuntimeError(f"submitting request {i} failed") from errors[0]
                time.sleep(0.0002)
            vals[i], phases[i] = srv.wait(tickets[i][0], tickets[i][1], timeout_s=120,
                                          with_times=True)
            lats[i] = phases[i]["latency_us"]
    except BaseException:
        srv.close()
        sub.join()
        raise
    sub.join()
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    # where the latency went: waiting for admission, admitted but not yet in
    # a launched slice, and from the first launch to the result
    st["phases"] = {k: _pcts(np.array([ph[k] for ph in phases]))
                    for k in ("queued_us", "admitted_us", "running_us")}
    return vals, np.array(lats), wall, st


def _pcts(x):
    return {"p50_us": float(np.percentile(x, 50)), "p99_us": float(np.percentile(x, 99)),
            "mean_us": float(np.mean(x)), "count": int(len(x))}


SERVE_EVENT_PAIRS = 16384


def sub_serve(P, ctx, args, loads=(0.5, 0.7, 0.9)):
    """Config 5: the 530-request stream through the request loop, all at
    once (saturation) and with Poisson arrivals at fractions of the
    saturation rate; latency from submit to the result on the host, p50/p99
    per class.  The walk launches of the saturation run are timed with HIP
    events on the server's streams; two slices overlap on the device, so the
    summed launch durations exceed the busy time and the per-launch fraction
    is a lower bound; the whole-job fractions beside it are not."""
    reqs = serve_requests(P)
    serve_tuning(P, ctx)
    try:
        terms = sum(1 << (r[0].shape[0] - 1) for r in reqs)
        ops = sum((1 << (r[0].shape[0] - 1)) * ops_per_term(r[1], r[0].shape[0]) for r in reqs)
        flops = sum((1 << (r[0].shape[0] - 1)) * ops_per_term(r[1], r[0].shape[0]) *
                    flops_per_op(r[1], r[0].shape[0]) for r in reqs)
        slice_us = args.slice_us
        _serve_run(P, ctx, reqs[:40], None, 0, slice_us)                 # warm-up
        P.perm_prof_enable(ctx, SERVE_EVENT_PAIRS)
        P.perm_prof_read(ctx)
        vals, lats, wall, st = _serve_run(P, ctx, reqs, None, 1, slice_us)
        walk_ms, launches = P.perm_prof_read(ctx)
        P.perm_prof_enable(ctx, False)
        sat_rate = len(reqs) / wall
        cls = np.array([r[3] for r in reqs])
        rf = roofline(ops / max(launches, 1), walk_ms, launches, None, flops / ops)
        rf["all_launches_timed"] = launches < SERVE_EVENT_PAIRS
        # whole-job fractions of the peak: every request's algorithmic ops over
        # the time the server had work queued or on the device, and over the
        # wall time from the first submit to the last result
        rf["frac_over_busy_time"] = round(ops / max(st["busy_s"], 1e-9) / PEAK_LANE_OPS, 4)
        rf["frac_over_wall_time"] = round(ops / wall / PEAK_LANE_OPS, 4)
        result = {"saturation": {"wall_s": wall, "requests_per_s": sat_rate,
                                 "terms_per_s": terms / wall, **_pcts(lats),
                                 "slices": st["slices"], "busy_s": st["busy_s"],
                                 "items": st["items"], "rate": st["rate"],
                                 "phases": st["phases"],
                                 "geodesic": _pcts(lats[cls == "geodesic"]),
                                 "schur": _pcts(lats[cls == "schur"])}}
        ref = vals
        for f in loads:
            progress(f"serve: load {f}")
            v, l, w, s2 = _serve_run(P, ctx, reqs, f * sat_rate, 2 + int(f * 10), slice_us)
            assert v == ref, "served results differ between runs"
            result[f"load_{f}"] = {"wall_s": w, "offered_per_s": f * sat_rate, **_pcts(l),
                                   "slices": s2["slices"], "busy_s": s2["busy_s"],
                                   "items": s2["items"], "rate": s2["rate"],
                                   "phases": s2["phases"],
                                   "geodesic": _pcts(l[cls == "geodesic"]),
                                   "schur": _pcts(l[cls == "schur"])}
        # every Schur residue is 0 for even n; geodesic perms are real and |.| <= 1
        for r, v in zip(reqs, ref):
            if r[3] == "schur":
                assert v == 0
            else:
                assert abs(v.imag) < 1e-12 and abs(v) <= 1 + 1e-12
    finally:
        serve_tuning(P, ctx, on=False)
    rec = {"workload": "serve_geodesic_c128_and_schur_modp", "requests": len(reqs),
           "value": terms / wall, "unit": "subset-terms/s", "terms": terms,
           "slice_us": slice_us, "c128_log2_chunk_max": SERVE_FLOAT_CHUNK, "dtype": "c128+f64",
           "roofline": rf, "latency": result}
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_baseline_serve(P, reqs)
    return rec


def bench_serve(P, ctx, args):
    rec = sub_serve(P, ctx, args)
    line = {"metric": METRIC, "value": rec["value"], "unit": "subset-terms/s",
            "ms_per_step": rec["latency"]["saturation"]["wall_s"] * 1e3, "dtype": rec["dtype"],
            "config": {"workload": rec["workload"], "requests": rec["requests"],
                       "terms": rec["terms"], "slice_us": rec["slice_us"],
                       "c128_log2_chunk_max": SERVE_FLOAT_CHUNK},
            "roofline": rec["roofline"], "latency": rec["latency"]}
    if "cpu_baseline" in rec:
        line["cpu_baseline"] = rec["cpu_baseline"]
    return line


def bench_default(P, ctx, args):
    """The headline line: S_28 over three primes is `value`; configs 1, 3,
    4 and 5 and single matrices of orders 20..36 follow as sub-records, each
    with its timing, roofline and oracle baseline."""
    progress("S_28 over three primes")
    line = bench_schur(P, ctx, args)
    cfg = {}
    progress("config 1: one Haar U(14)")
    cfg["single_haar_u14_c128"] = sub_single14(P, ctx, args)
    progress("config 3: 50,000 Haar U(20) and O(20)")
    U, O = haar20_inputs(50000)
    cfg["haar_u20_c128_50000"] = sub_batch(P, ctx, args, "haar_unitary_20_c128",
                                           [(m, "c128", 0) for m in U])
    del U
    cfg["haar_o20_f64_50000"] = sub_batch(P, ctx, args, "haar_orthogonal_20_f64",
                                          [(m, "f64", 0) for m in O])
    del O
    progress("config 4: 10,000 ragged Gaussian matrices")
    cfg["ragged_gaussian_10000"] = sub_batch(P, ctx, args, "ragged_gaussian_n8_24",
                                             ragged_inputs(10000),
                                             cpu_label="ragged GUE/GOE/Ginibre")
    progress("config 5: serving stream")
    cfg["serve_stream_530"] = sub_serve(P, ctx, args)
    progress("single matrices of orders 20..36")
    cfg["single_matrix_orders_20_36"] = sub_sizes(P, ctx, args)
    line["configs"] = cfg
    return line


def bench_copycal(P, ctx, args):
    """A plain device copy of known size: the reference for scaling the
    FETCH_SIZE / WRITE_SIZE counters of a profiled run."""
    import torch
    nbytes = 1 << 30
    x = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    sync()
    t0 = time.perf_counter()
    reps = max(1, args.steps // 20)
    for _ in range(reps):
        y.copy_(x)
    sync()
    dt = (time.perf_counter() - t0) / reps
    return {"metric": "copy bandwidth", "value": 2 * nbytes / dt / 1e9, "unit": "GB/s",
            "ms_per_step": dt * 1e3, "dtype": "f64",
            "config": {"workload": "copy_calibration", "bytes_read": nbytes,
                       "bytes_written": nbytes, "copies": reps}}


def haar_statistics(pu, po, n):
    """Distribution checks of the paper's Sec. 3 and 5 on batched outputs:
    pu = perm of Haar U(n) samples (complex), po = perm of Haar O(n) samples."""
    from scipy import stats
    m2 = np.abs(pu) ** 2
    exact = math.factorial(n) * math.factorial(n - 1) / math.factorial(2 * n - 1)
    u = {"mean_abs2": float(m2.mean()), "exact_mean_abs2": exact,
         "mean_abs2_z": float((m2.mean() - exact) / (m2.std(ddof=1) / math.sqrt(len(m2)))),
         "var_ratio_re_im": float(pu.real.std() / pu.imag.std()),
         "corr_re_im": float(np.corrcoef(pu.real, pu.imag)[0, 1]),
         "ks_p_exp": float(stats.kstest(m2 / m2.mean(), "expon").pvalue),
         "ks_p_phase": float(stats.kstest((np.angle(pu) + np.pi) / (2 * np.pi), "uniform").pvalue),
         "weibull_shape": float(stats.weibull_min.fit(np.abs(pu), floc=0)[0])}
    o = {"var": float(po.var(ddof=1)), "excess_kurtosis": float(stats.kurtosis(po)),
         "mean": float(po.mean())}
    return u, o


def bench_stats(P, ctx, args):
    """Haar U(n) (c128) and O(n) (f64) permanents, 50,000 samples per n for
    odd n in 7..23 as in the paper's Sec. 3-5, one batched launch per
    ensemble and n; throughput per n and the distribution checks."""
    import torch
    from paper_2602_10141_amd import ensembles as E
    count = args.count
    runs, tot_s, tot_perms = [], 0.0, 0
    for n in (7, 11, 13, 17, 19, 23):
        row = {"n": n, "count": count}
        vals = {}
        for name, gen, field, cfg in (("U", E.haar_unitary, "c128", 40), ("O", E.haar_orthogonal, "f64", 41)):
            M = gen(n, E.rng(cfg, n), count=count)
            items, data = P.pack_matrices([(m, field, 0) for m in M])
            d = torch.from_numpy(data).cuda()
            res = torch.zeros((count, 2), dtype=torch.float64, device="cuda")
            P.perm_batch(ctx, items, d, out=res)
            sync()
            P.perm_prof_enable(ctx, True)
            P.perm_prof_read(ctx)
            t0 = time.perf_counter()
            P.perm_batch(ctx, items, d, out=res)
            sync()
            dt = time.perf_counter() - t0
            walk_ms, launches = P.perm_prof_read(ctx)
            P.perm_prof_enable(ctx, False)
            r = res.cpu().numpy()
            vals[name] = r[:, 0] + 1j * r[:, 1] if field == "c128" else r[:, 0]
            terms = count * (1 << (n - 1))
            row[name] = {"perms_per_s": count / dt, "ms": dt * 1e3,
                         "roofline": roofline(terms * ops_per_term(field, n), walk_ms, launches)}
            tot_s += dt
            tot_perms += count
        row["U"]["stats"], row["O"]["stats"] = haar_statistics(vals["U"], vals["O"], n)
        runs.append(row)
    return {"metric": METRIC, "value": tot_perms / tot_s, "unit": "perms/s",
            "ms_per_step": tot_s * 1e3, "dtype": "c128+f64",
            "config": {"workload": "haar_U_O_statistics_n7_23", "count": count},
            "runs": runs}


def cpu_baseline_range(A, field, seconds=5.0):
    """The oracle's Ryser sum over a bounded range of subsets of one matrix,
    split over the host threads (disjoint ranges), scaled to Glynn-term
    equivalents (2^n Ryser subsets per permanent against 2^(n-1) terms)."""
    from oracle import native
    n = A.shape[0]
    threads = _threads()
    t = time.perf_counter()
    native.ryser_float_range(A, 1, 1 + (1 << 16))
    rate1 = (1 << 16) / (time.perf_counter() - t)
    # subsets 1 .. 2^n - 1 (the empty set contributes nothing)
    per_thread = int(min(((1 << n) - 1) // threads, max(1 << 16, rate1 * seconds)))

    def work(i):
        native.ryser_float_range(A, 1 + i * per_thread, 1 + (i + 1) * per_thread)

    t = time.perf_counter()
    _run_threads(work, threads)
    dt = time.perf_counter() - t
    return _with_host({
        "value": per_thread * threads / dt / 2, "unit": "subset-terms/s (Glynn-term equivalents)",
        "cores": threads, "kind": "oracle", "value_1thread": rate1 / 2,
        "sample": f"oracle Ryser ({field}) on one matrix of order {n}: {per_thread} subsets per "
                  f"thread, {threads} threads in {dt:.1f} s; rate scaled to 2^{n - 1} terms "
                  f"per permanent"})


def sub_sizes(P, ctx, args):
    """One matrix per call across the orders of the headline metric: Haar
    U(n) (c128) and O(n) (f64) for n = 20..36 and the Schur matrix S_n mod
    one prime (F_p) for n = 22..36.  Per case: the call's time and terms/s
    and the walk kernel's fraction of the FP64 VALU peak; the record's
    roofline is over all cases (their algorithmic instructions over their
    summed walk time).  Single calls of orders 10..27 use the latency
    partition (shorter wave items, so that one matrix occupies the device);
    from order 28 the batch partition already does."""
    import torch
    from paper_2602_10141_amd import ensembles as E
    cases = ([("c128", n) for n in (20, 22, 24, 26, 28, 30, 32, 34, 36)] +
             [("f64", n) for n in (20, 22, 24, 26, 28, 32, 36)] +
             [("modp", n) for n in (22, 24, 26, 28, 30, 32, 34, 36)])
    rows, tot_terms, tot_s, tot_ops, tot_walk_ms = [], 0, 0.0, 0.0, 0.0
    for field, n in cases:
        if field == "c128":
            A = torch.from_numpy(E.haar_unitary(n, E.rng(50, n))).cuda()
            fn = lambda: P.perm_c128(ctx, A)      # noqa: E731
        elif field == "f64":
            A = torch.from_numpy(E.haar_orthogonal(n, E.rng(51, n))).cuda()
            fn = lambda: P.perm_f64(ctx, A)       # noqa: E731
        else:
            p = P.perm_schur_primes(n)[0]
            A = torch.from_numpy(P.perm_schur_residues(n, p).astype(np.int32)).cuda()
            fn = lambda: P.perm_modp(ctx, A, p)   # noqa: E731
        terms = 1 << (n - 1)
        reps = max(1, int(4e9 / terms))
        fn()
        sync()
        # call time without timing events (they add about 9 us to a call),
        # walk time from a second, profiled pass
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        sync()
        dt = (time.perf_counter() - t0) / reps
        P.perm_prof_enable(ctx, True)
        P.perm_prof_read(ctx)
        for _ in range(max(1, reps // 4)):
            fn()
        sync()
        walk_ms, launches = P.perm_prof_read(ctx)
        P.perm_prof_enable(ctx, False)
        ops = terms * ops_per_term(field, n)
        rows.append({"field": field, "n": n, "ms": dt * 1e3, "terms_per_s": terms / dt,
                     "roofline": roofline(ops, walk_ms, launches)})
        tot_terms += terms
        tot_s += dt
        tot_ops += ops
        tot_walk_ms += walk_ms / max(launches, 1)
    rec = {"workload": "single_matrix_orders_20_36", "value": tot_terms / tot_s,
           "unit": "subset-terms/s", "dtype": "c128+f64", "cases": [f"{f}{n}" for f, n in cases],
           "roofline": roofline(tot_ops / len(cases), tot_walk_ms, len(cases)), "runs": rows}
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_baseline_range(E.haar_unitary(28, E.rng(50, 28)), "c128")
    return rec


def bench_sizes(P, ctx, args):
    rec = sub_sizes(P, ctx, args)
    line = {"metric": METRIC, "value": rec["value"], "unit": "subset-terms/s",
            "ms_per_step": sum(r["ms"] for r in rec["runs"]), "dtype": "c128+f64",
            "config": {"workload": rec["workload"], "cases": rec["cases"]},
            "roofline": rec["roofline"], "runs": rec["runs"]}
    if "cpu_baseline" in rec:
        line["cpu_baseline"] = rec["cpu_baseline"]
    return line


def bench_dft(P, ctx, args):
    """The DFT-geodesic fingerprint (paper Sec. 4.2): perm(gamma(t)) on a
    257-point t grid for odd n in 7..23 and both logarithms of -1, one
    batched launch per branch; r(n) = |perm F_n| / min_t |perm gamma(t)|."""
    import torch
    from paper_2602_10141_amd import ensembles as E
    ns = [7, 9, 11, 13, 15, 17, 19, 21, 23]
    grid = np.linspace(0.0, 1.0, 257)
    runs, tot_s, tot = [], 0.0, 0
    for branch in (1, -1):
        mats = [(E.dft_geodesic(n, t, branch), "c128", 0) for n in ns for t in grid]
        items, data = P.pack_matrices(mats)
        d = torch.from_numpy(data).cuda()
        res = torch.zeros((len(mats), 2), dtype=torch.float64, device="cuda")
        P.perm_batch(ctx, items, d, out=res)
        sync()
        t0 = time.perf_counter()
        P.perm_batch(ctx, items, d, out=res)
        sync()
        tot_s += time.perf_counter() - t0
        tot += len(mats)
        r = res.cpu().numpy()
        v = (r[:, 0] + 1j * r[:, 1]).reshape(len(ns), len(grid))
        for i, n in enumerate(ns):
            a = np.abs(v[i])
            k = int(a.argmin())
            runs.append({"n": n, "branch": branch, "r": float(a[-1] / a[k]), "t_min": float(grid[k]),
                         "abs_perm_F": float(a[-1]), "min_abs_perm": float(a[k]),
                         "perm_half": [float(v[i][128].real), float(v[i][128].imag)]})
    return {"metric": METRIC, "value": tot / tot_s, "unit": "perms/s", "ms_per_step": tot_s * 1e3,
            "dtype": "c128", "config": {"workload": "dft_geodesic_fingerprint", "n": ns,
                                       "grid_points": len(grid), "branches": [1, -1]},
            "runs": runs}


# wall times the paper reports for exact perm(S_n) on its GPU (Sec. 2.3)
PAPER_SCHUR_MINUTES = {37: 4.2, 39: 23.0, 41: 88.0, 43: 424.0}


def bench_schur_odd(P, ctx, args):
    """Exact perm(S_n) for odd n through checkpointed jobs over the smallest
    sufficient primes plus `extra` redundant ones; every k-subset of the
    residues must lift to the same integer (no table of known values is
    used)."""
    import itertools
    ns = [int(x) for x in args.n_list.split(",")]
    runs, tot_terms, tot_s, tot_ops = [], 0, 0.0, 0
    P.perm_prof_enable(ctx, True)
    P.perm_prof_read(ctx)
    for n in ns:
        k = len(P.perm_schur_primes(n))
        primes = P.perm_schur_primes(n, extra=args.extra)
        mats = np.stack([P.perm_schur_residues(n, p) for p in primes])
        bound = (n / 2) * math.log2(n)
        ck = os.path.join(args.checkpoint_dir, f"schur_S{n}.ckpt") if args.checkpoint_dir else None
        t0 = time.perf_counter()
        with P.Job(ctx, mats, primes, bound, checkpoint=ck) as job:
            while True:
                done, total = job.run(seconds=20.0)
                print(f"S_{n}: {done}/{total} pieces, {time.perf_counter() - t0:.1f} s",
                      file=sys.stderr, flush=True)
                if done == total:
                    break
            val, res = job.result()
        dt = time.perf_counter() - t0
        lifts = {P.perm_crt_lift([res[i] for i in sub], [primes[i] for i in sub], bound)
                 for sub in itertools.combinations(range(len(primes)), k)}
        assert lifts == {val}, f"S_{n}: prime subsets disagree"
        if len(primes) > k:
            assert P.perm_crt_check(res, primes, bound) == (val, None), f"S_{n}: a residue is off"
        assert val != 0 and abs(val) <= n ** (n / 2)
        terms = len(primes) * (1 << (n - 1))
        run = {"n": n, "primes": primes, "needed": k, "wall_s": dt, "terms": terms,
               "terms_per_s": terms / dt, "perm": str(val), "residues": res}
        if n in PAPER_SCHUR_MINUTES:
            run["paper_minutes"] = PAPER_SCHUR_MINUTES[n]
        runs.append(run)
        tot_terms += terms
        tot_s += dt
        tot_ops += terms * ops_per_term("modp", n)
    walk_ms, launches = P.perm_prof_read(ctx)
    P.perm_prof_enable(ctx, False)
    return {"metric": METRIC, "value": tot_terms / tot_s, "unit": "subset-terms/s",
            "ms_per_step": tot_s * 1e3, "dtype": "f64",
            "config": {"workload": "schur_odd_exact_crt", "n": ns, "extra_primes": args.extra,
                       "field": "F_p (exact FP64 Barrett walk) + CRT, checkpointed pieces"},
            "roofline": roofline(tot_ops / max(launches, 1), walk_ms, launches, None),
            "runs": runs}


def bench_shard(P, ctx, args):
    """One GPU's share of a permanent spread over G GPUs: perm(S_n) mod its
    first prime, the Gray range [0, 2^(n-1)) cut into G equal ranges, each
    walked through perm_range as GPU g would walk it (the same kernel and
    wave items as the whole walk).  The G ranges run here one after another;
    their unscaled partials must add up, mod p, to the residue of the single
    call.  `value` is one shard's Glynn-term rate (median over the shards)."""
    n, G = args.shard_n, args.shards
    T = 1 << (n - 1)
    if G < 1 or T % G:
        raise SystemExit(f"--shards must divide 2^{n - 1}")
    p = P.perm_schur_primes(n)[0]
    A = P.perm_schur_residues(n, p)
    items, data = P.pack_matrices([(A, "modp", p)])
    P.perm_range(ctx, items[0], data, 0, T // G)              # warm-up
    P.perm_prof_enable(ctx, True)
    P.perm_prof_read(ctx)
    parts, walls = [], []
    for k in range(G):
        t0 = time.perf_counter()
        parts.append(int(P.perm_range(ctx, items[0], data, k * T // G, (k + 1) * T // G)))
        walls.append(time.perf_counter() - t0)
    walk_ms, launches = P.perm_prof_read(ctx)
    P.perm_prof_enable(ctx, False)
    t0 = time.perf_counter()
    whole = P.perm_modp(ctx, A, p)
    whole_s = time.perf_counter() - t0
    combined = sum(parts) % p * pow((p + 1) // 2, n - 1, p) % p
    assert combined == whole, f"shards give {combined}, the single call {whole}"
    med = float(np.median(walls))
    rec = {"metric": METRIC, "value": (T // G) / med, "unit": "subset-terms/s",
           "ms_per_step": med * 1e3, "dtype": "f64",
           "config": {"workload": "schur_shard", "n": n, "shards": G, "prime": p,
                      "terms_per_shard": T // G},
           "roofline": roofline((T // G) * ops_per_term("modp", n), walk_ms, launches, None),
           "shard_ms": [round(w * 1e3, 3) for w in walls], "shard_partials": parts,
           "residue": whole, "single_call_s": whole_s}
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_baseline_schur(n, [p])
    return rec


WORKLOADS = {"default": bench_default, "shard": bench_shard, "dft": bench_dft, "stats": bench_stats, "schur_odd": bench_schur_odd, "copycal": bench_copycal, "serve": bench_serve, "schur28": bench_schur, "single14": bench_single14, "haar20": bench_haar20,
             "ragged": bench_ragged, "sizes": bench_sizes}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="default", choices=sorted(WORKLOADS))
    ap.add_argument("--count", type=int, default=50000)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--slice-us", type=float, default=500.0,
                    help="serve: device time per slice of the request loop")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the one-launch-per-matrix comparator (profiling runs)")
    ap.add_argument("--montgomery", action="store_true",
                    help="schur28: the 32-bit Montgomery F_p walk instead of FP64 Barrett")
    ap.add_argument("--n-list", default="29,31,33,35,37,39",
                    help="schur_odd: odd orders to run")
    ap.add_argument("--extra", type=int, default=1, help="schur_odd: redundant primes")
    ap.add_argument("--shard-n", type=int, default=36, help="shard: order of the Schur matrix")
    ap.add_argument("--shards", type=int, default=8, help="shard: GPUs the permanent is spread over")
    ap.add_argument("--checkpoint-dir", default=None,
                    help="schur_odd: keep (and resume from) checkpoints here")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the path would shard "
              "by Gray-index range or by prime", file=sys.stderr)
        sys.exit(2)
    if args.workload == "ragged" and args.count == 50000:
        args.count = 10000
    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    from paper_2602_10141_amd import perm as P
    ctx = P.Context(0)
    try:
        line = WORKLOADS[args.workload](P, ctx, args)
    finally:
        ctx.close()
    base = {"metric": METRIC, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "data": "synthetic"}
    base.update(line)
    order = ["metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
             "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
             "roofline", "cpu_baseline"]
    out = {k: base[k] for k in order if k in base}
    out.update({k: v for k, v in base.items() if k not in out})
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
