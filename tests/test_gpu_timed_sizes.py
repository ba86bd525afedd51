"""Parity of the kernels the benchmark times, at the sizes it times them.

* S_28 modulo each of its three CRT primes, through perm_crt_int with device
  pointers (the benchmark's call), FP64 Barrett and 32-bit Montgomery walks,
  against the oracle's full Ryser sum mod p (2^28 subsets on host threads).
* A random residue matrix of order 28 (a nonzero permanent), one call per
  walk, against the same oracle.
* Gray-index windows made of whole wave items of the default partition
  (64 lanes x 2^c indices, c from the context's tuning table) at the start,
  around the middle and at the end of [0, 2^(n-1)): F_p at n = 28, 32, 36
  (both walks), c128 at n = 25, 28, 32 and f64 at n = 28, 32, against Glynn
  terms the oracle evaluates one by one.  These are the items the full-size
  walks run; shorter windows only reach the chunk-end code paths.
* Geodesic points of orders 19..25 from the serving stream, in the batch
  form and partition the serving benchmark uses, against the oracle.
* Whole c128 permanents of orders 25..30 and an f64 one of order 28 in every
  call form, against the oracle's full Ryser sum on host threads.

Floats: |gpu - oracle| <= 1e-10 * prod_i ||row_i||_2 for permanents and
1e-10 * prod_i ||row_i||_2 * sqrt(x1 - x0) for unscaled window sums (a sum of
x1 - x0 terms of that magnitude with independent rounding).  F_p bit-exact.
"""
import math

import numpy as np
import pytest

from paper_2602_10141_amd import ensembles as E

pytestmark = pytest.mark.gpu
TOL = 1e-10


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


def say(msg):
    print(msg, flush=True)


# ------------------------------------------------------------------ S_28
@pytest.fixture(scope="module")
def schur28(P):
    n = 28
    primes = P.perm_schur_primes(n)
    assert len(primes) == 3
    mats = np.stack([P.perm_schur_residues(n, p) for p in primes])
    return n, primes, mats


@pytest.mark.parametrize("i", [0, 1, 2])
def test_schur28_residue_vs_oracle(P, ctx, oracle_lib, schur28, i):
    """The benchmark's step: perm_crt_int over the three residue matrices
    resident on the device; residue i against the oracle's full Ryser sum."""
    import torch
    n, primes, mats = schur28
    say(f"S_28 mod {primes[i]}: oracle on host threads")
    want = oracle_lib.native.ryser_modp_threaded(oracle_lib.crt.schur_residues(n, primes[i]),
                                                 primes[i])
    assert want == 0                                     # even n
    dmats = torch.from_numpy(mats.astype(np.int32)).cuda()
    bound = (n / 2) * math.log2(n)
    for flags in (0, P.PERM_MONTGOMERY):
        say(f"S_28 perm_crt_int flags={flags}")
        val, res = P.perm_crt_int(ctx, dmats, primes, bound, flags=flags)
        assert res[i] == want, (flags, res)
        assert val == 0


@pytest.fixture(scope="module")
def random28(oracle_lib):
    n, p = 28, 1073742209
    A = E.random_residues(n, p, E.rng(60, 28))
    want = oracle_lib.native.ryser_modp_threaded(A, p)
    return A, p, want


@pytest.mark.parametrize("mont", [False, True])
def test_random_residues_n28_full_permanent(P, ctx, random28, mont):
    import torch
    A, p, want = random28
    assert want != 0
    say(f"random n=28 mod {p}, montgomery={mont}")
    flags = P.PERM_MONTGOMERY if mont else 0
    assert P.perm_modp(ctx, A, p, flags=flags) == want                      # host buffers
    out = P.perm_modp(ctx, torch.from_numpy(A.astype(np.int32)).cuda(), p, flags=flags)
    torch.cuda.synchronize()
    assert int(out.cpu()[0]) == want                                         # device pointers


# ------------------------------------------- whole float permanents, n >= 25
@pytest.mark.parametrize("field,n", [("c128", 25), ("c128", 26), ("c128", 28), ("c128", 30),
                                     ("f64", 28)])
def test_whole_float_permanents_large(P, ctx, oracle_lib, field, n):
    """Whole permanents of orders 25..30 (the large-order c128 kernels) in
    all three call forms -- a single call (the latency partition below order
    28), a single call with the batch partition, a batch of two -- against
    the oracle's full Ryser sum on host threads."""
    g = E.rng(64, n)
    A = E.haar_unitary(n, g) if field == "c128" else E.haar_orthogonal(n, g)
    B = E.haar_unitary(n, g) if field == "c128" else E.haar_orthogonal(n, g)
    say(f"{field} n={n}: oracle on host threads")
    want = oracle_lib.native.ryser_float_threaded(A)
    fn = P.perm_c128 if field == "c128" else P.perm_f64
    single = fn(ctx, A)
    shared = fn(ctx, A, flags=P.PERM_SHARED_PARTITION)
    items, data = P.pack_matrices([(A, field, 0), (B, field, 0)])
    batch = P.batch_values(items, P.perm_batch(ctx, items, data))
    tol = TOL * scale(A)
    assert abs(single - want) <= tol, (single, want)
    assert abs(shared - want) <= tol, (shared, want)
    assert batch[0] == shared
    assert abs(want) <= 1 + 1e-12                       # |perm| <= 1 for orthogonal/unitary


# ---------------------------------------------------- whole default items
def windows(P, ctx, field, n, items_per_window):
    """Windows of whole default-size wave items: at the start, straddling
    the middle of [0, 2^(n-1)) and at the end."""
    c = P.perm_tune_get(ctx, field, n)[0]
    W = 64 << c
    T = 1 << (n - 1)
    k = items_per_window
    assert T % W == 0 and 2 * k * W <= T
    return c, W, [(0, k * W), (T // 2 - W, T // 2 - W + k * W), (T - k * W, T)]


@pytest.mark.parametrize("n", [28, 32, 36])
def test_modp_whole_items(P, ctx, oracle_lib, n):
    p = 1073742209 if n == 28 else P.perm_schur_primes(n)[0]
    A = E.random_residues(n, p, E.rng(61, n))
    items, data = P.pack_matrices([(A, "modp", p)])
    c, W, wins = windows(P, ctx, "modp", n, 4 if n < 36 else 2)
    for x0, x1 in wins:
        say(f"F_p n={n} c={c} window [{x0}, {x1})")
        want = oracle_lib.native.glynn_range_threaded(A, x0, x1, "modp", p)
        for flags in (0, P.PERM_MONTGOMERY):
            assert P.perm_range(ctx, items[0], data, x0, x1, flags=flags) == want, (flags, x0)


@pytest.mark.parametrize("n", [32, 34, 36])
def test_schur_serving_orders_whole_items(P, ctx, oracle_lib, n):
    """S_n mod its first prime (the serving stream's Schur requests), one
    whole default item in the middle of the range."""
    p = P.perm_schur_primes(n)[0]
    S = P.perm_schur_residues(n, p)
    items, data = P.pack_matrices([(S, "modp", p)])
    c, W, wins = windows(P, ctx, "modp", n, 1)
    x0, x1 = wins[1]
    say(f"S_{n} window [{x0}, {x1})")
    want = oracle_lib.native.glynn_range_threaded(S, x0, x1, "modp", p)
    assert P.perm_range(ctx, items[0], data, x0, x1) == want


@pytest.mark.parametrize("field,n", [("c128", 25), ("c128", 28), ("c128", 32),
                                     ("f64", 28), ("f64", 32)])
def test_float_whole_items(P, ctx, oracle_lib, field, n):
    g = E.rng(62, n)
    A = E.haar_unitary(n, g) if field == "c128" else E.haar_orthogonal(n, g)
    items, data = P.pack_matrices([(A, field, 0)])
    c, W, wins = windows(P, ctx, field, n, 4)
    for x0, x1 in wins:
        say(f"{field} n={n} c={c} window [{x0}, {x1})")
        want = oracle_lib.native.glynn_range_threaded(A, x0, x1, field)
        got = P.perm_range(ctx, items[0], data, x0, x1)
        assert abs(got - want) <= TOL * scale(A) * math.sqrt(x1 - x0), (x0, got, want)


# ------------------------------------------------ serving geodesic points
def test_geodesic_orders_19_to_25_vs_oracle(P, ctx, oracle_lib):
    """All 512 geodesic points in one batch, with the serving benchmark's
    partition (chunks of at most 2^9 indices for these orders), and a seeded
    sample of the orders 19..25 against the oracle."""
    import concurrent.futures as cf
    import bench
    import torch
    reqs = [(E.cycle_geodesic(n, t), "c128", 0) for n in range(11, 26, 2)
            for t in E.geodesic_grid(64)]
    bench.serve_tuning(P, ctx)
    try:
        items, data = P.pack_matrices(reqs)
        out = P.perm_batch(ctx, items, torch.from_numpy(data).cuda())
        torch.cuda.synchronize()
        vals = P.batch_values(items, out)
    finally:
        bench.serve_tuning(P, ctx, on=False)
    g = E.rng(63, 0)
    idx = []
    for k, n in enumerate(range(11, 26, 2)):
        if n >= 19:
            idx.extend(64 * k + int(j) for j in g.choice(np.arange(1, 63), size=4, replace=False))
    say(f"geodesic oracle on {len(idx)} points")
    with cf.ThreadPoolExecutor(oracle_lib.native.default_threads()) as ex:
        want = list(ex.map(lambda i: oracle_lib.native.ryser_c128(reqs[i][0]), idx))
    for i, w in zip(idx, want):
        assert abs(vals[i] - w) <= TOL * scale(reqs[i][0]), (i, vals[i], w)
