"""Parity at the benchmark's full sizes, in the launch form bench.py times.

Outputs the oracle cannot finish in seconds are checked on seeded samples
(oracle run one matrix at a time, in threads) and through properties that
hold at any size (|perm U| <= 1, real geodesic permanents, even-n Schur
zeros, range partials against directly evaluated Glynn terms).
"""
import concurrent.futures as cf
import math
import os

import numpy as np
import pytest

from paper_2602_10141_amd import ensembles as E

pytestmark = pytest.mark.gpu
TOL = 1e-10
THREADS = min(16, os.cpu_count() or 1)


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


def scale(A):
    return float(np.prod(np.linalg.norm(A, axis=1)))


def oracle_many(O, mats, fn):
    with cf.ThreadPoolExecutor(THREADS) as ex:
        return list(ex.map(fn, mats))


def run_batch_device(P, ctx, mats):
    import torch
    items, data = P.pack_matrices(mats)
    out = P.perm_batch(ctx, items, torch.from_numpy(data).cuda())
    torch.cuda.synchronize()
    return P.batch_values(items, out)


@pytest.mark.parametrize("kind", ["unitary", "orthogonal"])
def test_haar20_batch_50000(P, ctx, oracle_lib, kind):
    n, count = 20, 50000
    if kind == "unitary":
        M = E.haar_unitary(n, E.rng(3, 0), count=count)
        field, fn = "c128", oracle_lib.native.ryser_c128
    else:
        M = E.haar_orthogonal(n, E.rng(3, 1), count=count)
        field, fn = "f64", oracle_lib.native.ryser_f64
    vals = np.array(run_batch_device(P, ctx, [(m, field, 0) for m in M]))
    assert np.all(np.abs(vals) <= 1 + 1e-12)                       # |perm U| <= 1
    idx = E.rng(3, 9).choice(count, size=500, replace=False)
    want = oracle_many(oracle_lib, [M[i] for i in idx], fn)
    for i, w in zip(idx, want):
        assert abs(vals[i] - w) <= TOL * scale(M[i]), (i, vals[i], w)


def test_ragged_batch_10000(P, ctx, oracle_lib):
    import bench
    mats = bench.ragged_inputs(10000)
    vals = run_batch_device(P, ctx, mats)
    ns = np.array([m[0].shape[0] for m in mats])
    g = E.rng(4, 9)
    idx = []
    for n in range(8, 25):
        cand = np.flatnonzero(ns == n)
        idx.extend(g.choice(cand, size=min(len(cand), 60), replace=False))
    assert len(idx) >= 1000

    def ora(i):
        A, f, _ = mats[i]
        return oracle_lib.native.ryser_c128(A) if f == "c128" else oracle_lib.native.ryser_f64(A)

    want = oracle_many(oracle_lib, idx, ora)
    for i, w in zip(idx, want):
        A, f, _ = mats[i]
        assert abs(vals[i] - w) <= TOL * scale(A), (i, A.shape, vals[i], w)
        if f == "c128" and np.allclose(A, A.conj().T):               # GUE: perm is real
            assert abs(vals[i].imag) <= TOL * scale(A)


def test_serving_geodesic_points_512(P, ctx, oracle_lib):
    reqs = [(E.cycle_geodesic(n, t), "c128", 0) for n in range(11, 26, 2) for t in E.geodesic_grid(64)]
    vals = run_batch_device(P, ctx, reqs)
    grid = E.geodesic_grid(64)
    for k, n in enumerate(range(11, 26, 2)):
        row = vals[64 * k:64 * (k + 1)]
        assert abs(row[0] - 1) < 1e-13 and abs(row[-1] - 1) < 1e-13          # gamma(0) = I, gamma(1) = C_n
        for j in range(64):
            assert abs(row[j].imag) < 1e-13 and abs(row[j]) <= 1 + 1e-12
            assert abs(row[j] - row[63 - j]) < 1e-12                          # t <-> 1 - t
        if n <= 17:
            want = oracle_many(oracle_lib, [reqs[64 * k + j][0] for j in range(64)],
                               oracle_lib.native.ryser_c128)
            for j in range(64):
                assert abs(row[j] - want[j]) <= TOL, (n, grid[j])


@pytest.mark.parametrize("n", [32, 34, 36])
def test_serving_schur_orders_32_to_36(P, ctx, oracle_lib, n):
    import torch
    primes = P.perm_schur_primes(n, extra=6 - len(P.perm_schur_primes(n)))
    assert len(primes) == 6
    mats = np.stack([P.perm_schur_residues(n, p) for p in primes])
    val, res = P.perm_crt_int(ctx, torch.from_numpy(mats.astype(np.int32)).cuda(), primes,
                              (n / 2) * math.log2(n))
    assert res == [0] * 6 and val == 0
    # range partials at this size against directly evaluated Glynn terms
    T = 1 << (n - 1)
    g = E.rng(5, n)
    p = primes[0]
    items, data = P.pack_matrices([(mats[0], "modp", p)])
    for _ in range(3):
        x0 = int(g.integers(0, T - 5000))
        x1 = x0 + int(g.integers(1, 4000))
        assert P.perm_range(ctx, items[0], data, x0, x1) == \
            oracle_lib.native.glynn_range_modp(mats[0], p, x0, x1)
