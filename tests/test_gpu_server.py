"""GPU tests of the request loop: results bit-identical to perm_batch alone and
in the mix, admission under small budgets, cancellation, statistics."""
import time

import numpy as np
import pytest

from paper_2602_10141_amd import ensembles as E

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_2602_10141_amd import perm
    return perm


@pytest.fixture(scope="module")
def ctx(P):
    c = P.Context(0)
    yield c
    c.close()


def mixed_requests():
    g = E.rng(20, 0)
    reqs = []
    for n in (11, 13, 15, 17):
        for t in (0.0, 0.25, 0.5, 1.0):
            reqs.append((E.cycle_geodesic(n, t), "c128", 0))
    for n in (0, 1, 2, 6, 9, 14, 20):
        reqs.append((E.ginibre_real(n, g) if n else np.zeros((0, 0)), "f64", 0))
        reqs.append((E.random_residues(n, 1073742209, g), "modp", 1073742209))
    reqs.append((E.gue(19, g), "c128", 0))
    return reqs


def test_results_match_batch_bitwise(P, ctx, oracle_lib):
    reqs = mixed_requests()
    items, data = P.pack_matrices(reqs)
    want = P.batch_values(items, P.perm_batch(ctx, items, data))
    srv = P.Server(ctx, slice_us=500)
    try:
        tickets = [srv.submit(A, f, p) for A, f, p in reqs]
        got = [srv.wait(t, it, timeout_s=60) for t, it in tickets]
        st = srv.stats()
    finally:
        srv.close()
    assert got == want
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["p50_us"] > 0 and st["p99_us"] >= st["p50_us"]
    # geodesic endpoints: perm(I) = perm(C_n) = 1
    for (A, f, p), v in zip(reqs, got):
        if f == "c128" and A.shape[0] in (11, 13) and (np.allclose(A, np.eye(len(A)))):
            assert abs(v - 1) < 1e-14


def test_latency_phases(P, ctx):
    """perm_srv_wait_times: the same results, and the phases of each request's
    latency are non-negative and add up to it; under a budget that admits
    one request at a time, the later requests spend time queued."""
    reqs = mixed_requests()
    items, data = P.pack_matrices(reqs)
    want = P.batch_values(items, P.perm_batch(ctx, items, data))
    srv = P.Server(ctx, max_inflight=1, slice_us=500)
    try:
        tickets = [srv.submit(A, f, p) for A, f, p in reqs]
        got = [srv.wait(t, it, timeout_s=60, with_times=True) for t, it in tickets]
    finally:
        srv.close()
    assert [v for v, _ in got] == want
    for _, ph in got:
        assert min(ph["queued_us"], ph["admitted_us"], ph["running_us"]) >= 0
        assert abs(ph["queued_us"] + ph["admitted_us"] + ph["running_us"] - ph["latency_us"]) \
            <= 1e-6 * max(1.0, ph["latency_us"])
        assert ph["running_us"] > 0
    assert got[-1][1]["queued_us"] > got[0][1]["queued_us"]


def test_alone_equals_in_mix(P, ctx):
    A = E.cycle_geodesic(17, 0.3)
    srv = P.Server(ctx)
    try:
        t, it = srv.submit(A, "c128")
        alone = srv.wait(t, it)
        big = [srv.submit(E.random_residues(24, 2147483647, E.rng(21, i)), "modp", 2147483647)
               for i in range(4)]
        t2, it2 = srv.submit(A, "c128")
        mixed = srv.wait(t2, it2)
        for tk, itk in big:
            srv.wait(tk, itk)
    finally:
        srv.close()
    assert alone == mixed


def test_small_budget_admits_in_turn(P, ctx):
    # room for about two n = 20 requests at a time
    srv = P.Server(ctx, hbm_budget=64 * 1024, max_inflight=2)
    reqs = [(E.ginibre_complex(12, E.rng(22, i)), "c128", 0) for i in range(12)]
    items, data = P.pack_matrices(reqs)
    want = P.batch_values(items, P.perm_batch(ctx, items, data))
    try:
        tickets = [srv.submit(A, f, p) for A, f, p in reqs]
        got = [srv.wait(t, it, timeout_s=60) for t, it in tickets]
    finally:
        srv.close()
    assert got == want


def test_request_larger_than_budget_is_rejected(P, ctx):
    srv = P.Server(ctx, hbm_budget=4096)
    try:
        with pytest.raises(P.PermError) as e:
            srv.submit(E.ginibre_complex(30, E.rng(23, 0)), "c128")
        assert e.value.status == P.PERM_ENOMEM
    finally:
        srv.close()


def test_pending_queue_full(P, ctx):
    srv = P.Server(ctx, max_pending=2, max_inflight=1, hbm_budget=1 << 24)
    try:
        big = srv.submit(E.random_residues(34, 2147483647, E.rng(24, 0)), "modp", 2147483647)
        saw_eagain = False
        subs = []
        for i in range(50):
            try:
                subs.append(srv.submit(E.ginibre_real(8, E.rng(24, i + 1)), "f64"))
            except P.PermError as e:
                assert e.status == P.PERM_EAGAIN
                saw_eagain = True
                break
        assert saw_eagain
        srv.cancel(big[0])
        for t, it in subs:
            srv.wait(t, it, timeout_s=120)
    finally:
        srv.close()


def test_cancel(P, ctx):
    srv = P.Server(ctx, slice_us=1000)
    try:
        big = srv.submit(E.random_residues(38, 2147483647, E.rng(25, 0)), "modp", 2147483647)
        small = srv.submit(E.ginibre_complex(10, E.rng(25, 1)), "c128")
        time.sleep(0.05)
        srv.cancel(big[0])
        with pytest.raises(P.PermError) as e:
            srv.wait(big[0], big[1], timeout_s=60)
        assert e.value.status == P.PERM_ECANCELED
        v = srv.wait(small[0], small[1], timeout_s=60)
        assert v == P.perm_c128(ctx, E.ginibre_complex(10, E.rng(25, 1)),
                                flags=P.PERM_SHARED_PARTITION)
        st = srv.stats()
        assert st["canceled"] >= 1
    finally:
        srv.close()


def test_budget_held_by_inflight_requests(P, ctx):
    """Admission that waits for device memory held by requests whose last items
    are in flight completes those slices first (room for one request)."""
    p = 2147483647
    reqs = [(E.random_residues(30, p, E.rng(26, i)), "modp", p) for i in range(8)]
    items, data = P.pack_matrices(reqs)
    want = P.batch_values(items, P.perm_batch(ctx, items, data))
    srv = P.Server(ctx, hbm_budget=800 * 1024, slice_us=500)
    try:
        tickets = [srv.submit(A, f, q) for A, f, q in reqs]
        got = [srv.wait(t, it, timeout_s=30) for t, it in tickets]
        st = srv.stats()
    finally:
        srv.close()
    assert got == want
    assert st["completed"] == len(reqs)


def test_unknown_ticket(P, ctx):
    srv = P.Server(ctx)
    try:
        with pytest.raises(P.PermError) as e:
            srv.poll(12345, P.make_items([(0, 3, "f64", 0)])[0])
        assert e.value.status == P.PERM_ENOTFOUND
    finally:
        srv.close()


def test_serving_stream_530_matches_batch(P, ctx):
    """All 530 geodesic and Schur requests of the serving workload, submitted
    at once and as a paced stream: every result equals perm_batch's."""
    import bench
    reqs = bench.serve_requests(P)
    mats = [(A, f, p) for A, f, p, _, _ in reqs]
    items, data = P.pack_matrices(mats)
    bench.serve_tuning(P, ctx)
    try:
        want = P.batch_values(items, P.perm_batch(ctx, items, data))
        want2 = P.batch_values(items, P.perm_batch(ctx, items, data))
        assert want == want2
        for rate in (None, 400.0):
            got, _, _, _ = bench._serve_run(P, ctx, reqs, rate, 7, 2000.0)
            bad = [(i, reqs[i][3], reqs[i][4], got[i], want[i]) for i in range(len(reqs))
                   if got[i] != want[i]]
            assert not bad, f"{len(bad)} served results differ, first: {bad[:5]}"
    finally:
        bench.serve_tuning(P, ctx, on=False)
