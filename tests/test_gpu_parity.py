"""GPU parity: the HIP path against the oracle, element by element.

Floats: |perm_gpu - perm_oracle| <= 1e-10 * prod_i ||row_i||_2 (complex
modulus for c128).  F_p and CRT: bit-exact.  Sizes are those the oracle
finishes in seconds; they span several wave items and the short-chunk paths.
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


@pytest.fixture(scope="module")
def O(oracle_lib):
    return oracle_lib


def scale(A):
    return max(float(np.prod(np.linalg.norm(A, axis=1))), 1e-300) if len(A) else 1.0


# ----------------------------------------------------------- single matrices
@pytest.mark.parametrize("n", list(range(0, 13)) + [14, 16, 18, 20])
def test_c128_random(P, ctx, O, n):
    A = E.ginibre_complex(n, E.rng(1, n)) if n else np.zeros((0, 0), complex)
    got = P.perm_c128(ctx, A)
    want = O.native.ryser_c128(A) if n else 1.0
    assert abs(got - want) <= TOL * scale(A), (got, want)


@pytest.mark.parametrize("n", list(range(0, 13)) + [15, 17, 21])
def test_f64_random(P, ctx, O, n):
    A = E.ginibre_real(n, E.rng(2, n)) if n else np.zeros((0, 0))
    got = P.perm_f64(ctx, A)
    want = O.native.ryser_f64(A) if n else 1.0
    assert abs(got - want) <= TOL * scale(A), (got, want)


@pytest.mark.parametrize("p", [3, 5, 97, 65537, 1073742209, 2147483647])
@pytest.mark.parametrize("n", [0, 1, 2, 3, 5, 7, 8, 9, 11, 13, 16, 19])
@pytest.mark.parametrize("mont", [False, True])
def test_modp_random(P, ctx, O, n, p, mont):
    A = E.random_residues(n, p, E.rng(3, n * 7 + p % 101)) if n else np.zeros((0, 0), np.uint32)
    got = P.perm_modp(ctx, A, p, flags=P.PERM_MONTGOMERY if mont else 0)
    want = O.native.ryser_modp(A, p) if n else 1 % p
    assert got == want


def test_modp_entries_reduced(P, ctx, O):
    """Entries >= p are taken mod p."""
    p, n = 101, 9
    A = E.random_residues(n, 2 ** 31 - 1, E.rng(4, 0))
    assert P.perm_modp(ctx, A, p) == O.native.ryser_modp(A % p, p)


def test_single_haar_unitary_14(P, ctx, O):
    """Single 14x14 complex128 Haar unitary (QR of CN(0,1) Ginibre, phases folded)."""
    U = E.haar_unitary(14, E.rng(1, 0))
    got = P.perm_c128(ctx, U)
    want = O.native.ryser_c128(U)
    assert abs(got - want) <= TOL * scale(U)
    assert abs(got) <= 1 + 1e-12


def test_device_pointer_path(P, ctx, O):
    import torch
    A = E.ginibre_complex(13, E.rng(5, 0))
    out = P.perm_c128(ctx, torch.from_numpy(A).cuda())
    torch.cuda.synchronize()
    got = complex(*out.cpu().numpy())
    assert abs(got - O.native.ryser_c128(A)) <= TOL * scale(A)
    R = E.random_residues(12, 1073742209, E.rng(5, 1))
    o = P.perm_modp(ctx, torch.from_numpy(R.astype(np.int32)).cuda(), 1073742209)
    torch.cuda.synchronize()
    assert int(o.cpu()[0]) == O.native.ryser_modp(R, 1073742209)


def test_device_outputs_written_in_place(P, ctx, O):
    """A single-matrix device output aligned to its element type is written
    by the kernels directly: exactly 16, 8 or 4 bytes, with the neighbouring
    bytes untouched.  An f64 output 4 bytes off its alignment goes through
    the copy path and holds the same value."""
    import ctypes
    import torch
    L, st = P.lib(), P._stream(None)
    g = E.rng(5, 2)
    A = E.ginibre_complex(12, g)
    B = E.ginibre_real(11, g)
    R = E.random_residues(10, 65537, g)
    dA = torch.from_numpy(A).cuda()
    dB = torch.from_numpy(B).cuda()
    dR = torch.from_numpy(R.astype(np.int32)).cuda()
    buf = torch.full((8,), -7.0, dtype=torch.float64, device="cuda")
    base = buf.data_ptr()
    assert L.perm_c128(ctx.ptr, ctypes.c_void_p(dA.data_ptr()), 12, ctypes.c_void_p(base + 16),
                       P.PERM_DEVICE_PTRS, st) == P.PERM_OK
    assert L.perm_f64(ctx.ptr, ctypes.c_void_p(dB.data_ptr()), 11, ctypes.c_void_p(base + 40),
                      P.PERM_DEVICE_PTRS, st) == P.PERM_OK
    torch.cuda.synchronize()
    h = buf.cpu().numpy()
    assert list(h[[0, 1, 4, 6, 7]]) == [-7.0] * 5
    assert abs(complex(h[2], h[3]) - O.native.ryser_c128(A)) <= TOL * scale(A)
    assert abs(h[5] - O.native.ryser_f64(B)) <= TOL * scale(B)
    ibuf = torch.full((8,), -1, dtype=torch.int32, device="cuda")
    assert L.perm_modp(ctx.ptr, ctypes.c_void_p(dR.data_ptr()), 10, 65537,
                       ctypes.c_void_p(ibuf.data_ptr() + 12), P.PERM_DEVICE_PTRS, st) == P.PERM_OK
    torch.cuda.synchronize()
    hi = ibuf.cpu().numpy()
    assert hi[3] == O.native.ryser_modp(R, 65537)
    assert list(np.delete(hi, 3)) == [-1] * 7
    # misaligned f64 output: copied, same bits as the aligned result
    raw = torch.zeros(32, dtype=torch.uint8, device="cuda")
    assert L.perm_f64(ctx.ptr, ctypes.c_void_p(dB.data_ptr()), 11, ctypes.c_void_p(raw.data_ptr() + 4),
                      P.PERM_DEVICE_PTRS, st) == P.PERM_OK
    torch.cuda.synchronize()
    got = np.frombuffer(raw.cpu().numpy()[4:12].tobytes(), dtype=np.float64)[0]
    assert got == h[5]


def test_kahan_off_still_within_tolerance(P, ctx, O):
    A = E.ginibre_complex(16, E.rng(6, 0))
    got = P.perm_c128(ctx, A, flags=P.PERM_NO_KAHAN)
    assert abs(got - O.native.ryser_c128(A)) <= TOL * scale(A)


def test_repeat_bit_identical(P, ctx):
    A = E.ginibre_complex(18, E.rng(7, 0))
    vals = {P.perm_c128(ctx, A) for _ in range(3)}
    assert len(vals) == 1


# ------------------------------------------------------------------- Schur
@pytest.mark.parametrize("n", [3, 5, 7, 9, 10, 11, 13, 15, 17, 19, 21])
def test_schur_modp(P, ctx, O, n):
    for p in O.crt.primes_1_mod_n(n, 2):
        S_lib = P.perm_schur_residues(n, p)
        S_or = O.crt.schur_residues(n, p)
        assert np.array_equal(S_lib, S_or)
        want = O.native.ryser_modp(S_or, p)
        assert P.perm_modp(ctx, S_lib, p) == want
        if n % 2 == 0:
            assert want == 0


@pytest.mark.parametrize("n", [5, 7, 9, 11, 13, 17, 19])
def test_schur_crt_exact(P, ctx, O, n):
    primes = P.perm_schur_primes(n)
    assert primes == O.crt.primes_for_schur(n)
    mats = np.stack([P.perm_schur_residues(n, p) for p in primes])
    val, res = P.perm_crt_int(ctx, mats, primes, (n / 2) * math.log2(n))
    want_res = [O.native.ryser_modp(m, p) for m, p in zip(mats, primes)]
    assert res == want_res
    assert val == O.crt.crt_lift(want_res, primes)
    if n <= 10:
        assert val == O.crt.schur_perm_exact(n)


def test_crt_factorial_sign(P, ctx, O):
    n = 21
    primes = O.crt.primes_1_mod_n(2, 3)
    J = np.stack([np.ones((n, n), np.uint32)] * 3)
    val, _ = P.perm_crt_int(ctx, J, primes, math.log2(math.factorial(n)) + 1)
    assert val == math.factorial(n)
    Jm = J.copy()
    for i, p in enumerate(primes):
        Jm[i, 0, :] = p - 1
    val, _ = P.perm_crt_int(ctx, Jm, primes, math.log2(math.factorial(n)) + 1)
    assert val == -math.factorial(n)


# ------------------------------------------------------------------- ranges
@pytest.mark.parametrize("field", ["c128", "f64", "modp", "mont"])
def test_range_partials(P, ctx, O, field):
    n = 14
    T = 1 << (n - 1)
    g = E.rng(8, 0)
    if field == "c128":
        A = E.ginibre_complex(n, g)
    elif field == "f64":
        A = E.ginibre_real(n, g)
    else:
        A = E.random_residues(n, 1073742209, g)
    modp = field in ("modp", "mont")
    items, data = P.pack_matrices([(A, "modp" if modp else field, 1073742209 if modp else 0)])
    flags = P.PERM_MONTGOMERY if field == "mont" else 0
    for x0, x1 in [(0, T), (1, 2), (3, 77), (100, 4100), (T - 5, T), (0, 1), (4096, 8192), (7, 7)]:
        got = P.perm_range(ctx, items[0], data, x0, x1, flags=flags)
        if field == "c128":
            want = O.native.glynn_range_c128(A, x0, x1)
            assert abs(got - want) <= TOL * scale(A) * max(1, x1 - x0) ** 0.5
        elif field == "f64":
            want = O.native.glynn_range_f64(A, x0, x1)
            assert abs(got - want) <= TOL * scale(A) * max(1, x1 - x0) ** 0.5
        else:
            assert got == O.native.glynn_range_modp(A, 1073742209, x0, x1)


@pytest.mark.parametrize("field,n", [("c128", 40), ("c128", 48), ("f64", 48), ("modp", 44),
                                     ("modp", 48), ("mont", 41), ("mont", 48)])
def test_range_partials_large_orders(P, ctx, O, field, n):
    """Orders up to the maximum, 48, through Gray-index windows the oracle can
    afford (its Glynn terms cost O(n^2) each): at the start, around the
    middle, at the end of [0, 2^(n-1)) and at an unaligned offset past 2^33,
    each spanning several wave items of the large-order kernels."""
    T = 1 << (n - 1)
    g = E.rng(8, n)
    p = 1073742209
    if field == "c128":
        A = E.ginibre_complex(n, g)
    elif field == "f64":
        A = E.ginibre_real(n, g)
    else:
        A = E.random_residues(n, p, g)
    modp = field in ("modp", "mont")
    items, data = P.pack_matrices([(A, "modp" if modp else field, p if modp else 0)])
    flags = P.PERM_MONTGOMERY if field == "mont" else 0
    for x0, x1 in [(0, 1 << 14), (T // 2 - 3000, T // 2 + 9000), (T - 20000, T),
                   ((1 << 33) + 5, (1 << 33) + 4101)]:
        got = P.perm_range(ctx, items[0], data, x0, x1, flags=flags)
        if field == "c128":
            want = O.native.glynn_range_c128(A, x0, x1)
            assert abs(got - want) <= TOL * scale(A) * (x1 - x0) ** 0.5
        elif field == "f64":
            want = O.native.glynn_range_f64(A, x0, x1)
            assert abs(got - want) <= TOL * scale(A) * (x1 - x0) ** 0.5
        else:
            assert got == O.native.glynn_range_modp(A, p, x0, x1)


@pytest.mark.parametrize("field,n,G", [("modp", 21, 8), ("c128", 20, 4), ("f64", 21, 8),
                                       ("modp", 29, 8)])
def test_range_shards_add_up(P, ctx, O, field, n, G):
    """Spreading one permanent over G GPUs gives GPU g the Gray range
    [g T/G, (g+1) T/G), T = 2^(n-1), through perm_range, at the wave-item
    shape of the whole walk.  Walked here one after another, each shard's
    unscaled partial equals the oracle's direct Glynn sum over its range
    (orders up to 21), and the shards add up to the whole permanent: mod p
    exactly (S_29 against the single call, its oracle being too slow), for
    floats within the tolerance of the oracle's permanent."""
    T = 1 << (n - 1)
    p = 1073742209
    g = E.rng(18, n)
    if field == "modp" and n > 21:
        p = P.perm_schur_primes(n)[0]
        A = P.perm_schur_residues(n, p)
    elif field == "modp":
        A = E.random_residues(n, p, g)
    elif field == "c128":
        A = E.haar_unitary(n, g)
    else:
        A = E.haar_orthogonal(n, g)
    items, data = P.pack_matrices([(A, field, p if field == "modp" else 0)])
    parts = [P.perm_range(ctx, items[0], data, k * T // G, (k + 1) * T // G) for k in range(G)]
    if field == "modp":
        total = sum(int(v) for v in parts) % p
        if n <= 21:
            for k, v in enumerate(parts):
                assert v == O.native.glynn_range_modp(A, p, k * T // G, (k + 1) * T // G)
            want = O.native.ryser_modp(A, p)
        else:
            want = P.perm_modp(ctx, A, p)
        assert total * pow((p + 1) // 2, n - 1, p) % p == want
        return
    rng_fn = O.native.glynn_range_c128 if field == "c128" else O.native.glynn_range_f64
    for k, v in enumerate(parts):
        want = rng_fn(A, k * T // G, (k + 1) * T // G)
        assert abs(v - want) <= TOL * scale(A) * (T // G) ** 0.5
    whole = math.ldexp(1.0, -(n - 1)) * sum(parts)
    want = O.native.ryser_c128(A) if field == "c128" else O.native.ryser_f64(A)
    assert abs(whole - want) <= TOL * scale(A)


def test_range_rejects_bad_bounds(P, ctx):
    items, data = P.pack_matrices([(np.eye(5), "f64", 0)])
    with pytest.raises(P.PermError) as e:
        P.perm_range(ctx, items[0], data, 3, 17)
    assert e.value.status == P.PERM_EINVAL


# -------------------------------------------------------------------- batch
def test_batch_mixed_matches_single_bitwise(P, ctx, O):
    g = E.rng(9, 0)
    mats = []
    for n in [0, 1, 2, 5, 8, 11, 13, 16, 20, 24, 3]:
        mats.append((E.ginibre_complex(n, g) if n else np.zeros((0, 0), complex), "c128", 0))
        mats.append((E.ginibre_real(n, g) if n else np.zeros((0, 0)), "f64", 0))
        mats.append((E.random_residues(n, 65537, g), "modp", 65537))
    items, data = P.pack_matrices(mats)
    out = P.perm_batch(ctx, items, data)
    vals = P.batch_values(items, out)
    for (A, field, p), v in zip(mats, vals):
        n = A.shape[0]
        # a single call with the batch partition has the batch's bits; the
        # default single call (the latency partition from order 10) agrees
        # to within the tolerance
        if field == "c128":
            assert v == P.perm_c128(ctx, A, flags=P.PERM_SHARED_PARTITION)
            assert abs(v - P.perm_c128(ctx, A)) <= TOL * scale(A)
            if n <= 16:
                assert abs(v - (O.native.ryser_c128(A) if n else 1)) <= TOL * scale(A)
        elif field == "f64":
            assert v == P.perm_f64(ctx, A, flags=P.PERM_SHARED_PARTITION)
            assert abs(v - P.perm_f64(ctx, A)) <= TOL * scale(A)
            if n <= 16:
                assert abs(v - (O.native.ryser_f64(A) if n else 1)) <= TOL * scale(A)
        else:
            assert v == P.perm_modp(ctx, A, p)
            if n <= 16:
                assert v == (O.native.ryser_modp(A, p) if n else 1)


@pytest.mark.parametrize("field,n", [("c128", 11), ("c128", 14), ("c128", 15), ("c128", 16),
                                     ("c128", 20), ("c128", 22), ("c128", 24),
                                     ("c128", 26), ("f64", 13), ("f64", 17), ("f64", 20),
                                     ("f64", 24), ("f64", 26), ("f64", 27),
                                     ("modp", 14), ("modp", 20), ("modp", 24)])
def test_latency_partition_single_calls(P, ctx, O, field, n):
    """One matrix of order 10..27 alone would leave most resident waves idle
    at the batch partition, so a single call splits it into more, shorter
    wave items.  The result agrees with the oracle (orders up to 24) and
    with the same matrix in a batch to within the tolerance (bit for bit for
    F_p), and with PERM_SHARED_PARTITION it has the batch's bits."""
    import concurrent.futures as cf
    g = E.rng(15, n)
    p = 1073742209
    if field == "c128":
        A = E.haar_unitary(n, g)
    elif field == "f64":
        A = E.haar_orthogonal(n, g)
    else:
        A = E.random_residues(n, p, g)
    items, data = P.pack_matrices([(A, field, p if field == "modp" else 0)])
    batch = P.batch_values(items, P.perm_batch(ctx, items, data))[0]
    if field == "modp":
        assert P.perm_modp(ctx, A, p) == batch == O.native.ryser_modp_threaded(A, p)
        assert P.perm_modp(ctx, A, p, flags=P.PERM_MONTGOMERY) == batch
        return
    fn = P.perm_c128 if field == "c128" else P.perm_f64
    single = fn(ctx, A)
    assert abs(single - batch) <= TOL * scale(A)
    assert fn(ctx, A, flags=P.PERM_SHARED_PARTITION) == batch
    if n <= 24:
        with cf.ThreadPoolExecutor(1) as ex:
            want = ex.submit(O.native.ryser_c128 if field == "c128" else O.native.ryser_f64, A).result()
        assert abs(single - want) <= TOL * scale(A)
        assert abs(batch - want) <= TOL * scale(A)


def test_batch_device_path_and_bad_item(P, ctx):
    import torch
    mats = [(E.ginibre_complex(10, E.rng(10, i)), "c128", 0) for i in range(5)]
    items, data = P.pack_matrices(mats)
    out = P.perm_batch(ctx, items, torch.from_numpy(data).cuda())
    torch.cuda.synchronize()
    host = P.perm_batch(ctx, items, data)
    assert np.array_equal(out.cpu().numpy(), host)
    items["n"][2] = 60
    with pytest.raises(P.PermError) as e:
        P.perm_batch(ctx, items, data)
    assert e.value.status == P.PERM_EINVAL and "item 2" in str(e.value)


# ------------------------------------------------------- persistent claims
@pytest.mark.parametrize("count", [1, 2, 3, 5, 9, 13, 21, 29, 33])
def test_block_claims_small_grids(P, ctx, O, count):
    """One wave item per matrix (c128, n = 12): 1..33 items launch grids of
    1..9 blocks, so the work counters run in groups of 1, 2, 4 and 8 (the
    largest power of two not above the grid) and a block's last run of four
    items is partly empty.  Every result equals the single-matrix call bit
    for bit and the oracle within tolerance."""
    g = E.rng(12, count)
    mats = [(E.ginibre_complex(12, g), "c128", 0) for _ in range(count)]
    items, data = P.pack_matrices(mats)
    vals = P.batch_values(items, P.perm_batch(ctx, items, data))
    for (A, _, _), v in zip(mats, vals):
        assert v == P.perm_c128(ctx, A, flags=P.PERM_SHARED_PARTITION)
        assert abs(P.perm_c128(ctx, A) - v) <= TOL * scale(A)
        assert abs(v - O.native.ryser_c128(A)) <= TOL * scale(A)


def test_block_staging_small_batches(P, ctx, O):
    """A batch whose one walk is short and covers at most four small
    matrices stages them in every block of the walk instead of in a launch of
    its own.  Its results equal those of the same matrices inside a batch
    that takes the stage launch, bit for bit, and the oracle."""
    p = 1073742209
    g = E.rng(16, 0)
    small = [(E.ginibre_complex(19, g), "c128", 0), (E.ginibre_real(20, g), "f64", 0),
             (E.random_residues(18, p, g), "modp", p)]
    big = small + [(E.ginibre_complex(12, g), "c128", 0) for _ in range(30)]
    items, data = P.pack_matrices(small)
    vals = P.batch_values(items, P.perm_batch(ctx, items, data))
    items_b, data_b = P.pack_matrices(big)
    vals_b = P.batch_values(items_b, P.perm_batch(ctx, items_b, data_b))
    assert vals == vals_b[:3]
    assert abs(vals[0] - O.native.ryser_c128(small[0][0])) <= TOL * scale(small[0][0])
    assert abs(vals[1] - O.native.ryser_f64(small[1][0])) <= TOL * scale(small[1][0])
    assert vals[2] == O.native.ryser_modp(small[2][0], p)


def test_last_block_finalize_back_to_back(P, ctx, O):
    """A single call of order 11..17 walks in 1 to 32 blocks and finalizes in
    the block that finishes last, counted on a device counter whose value
    the host tracks across calls; from order 18 (64 blocks and more) a
    finalize launch follows the walk.  Many such calls of different
    matrices, orders and fields, queued without synchronising and mixed with
    batches and CRT calls that finalize in a launch of their own or in one
    block, each give the bits of the same call made alone, and the oracle's
    result."""
    import torch
    p = 1073742209
    g = E.rng(17, 0)
    cases = []
    for rep in range(3):
        for n in (11, 12, 13, 14, 15, 16, 17, 18):
            cases.append(("c128", E.ginibre_complex(n, g)))
            cases.append(("f64", E.ginibre_real(n, g)))
            cases.append(("modp", E.random_residues(n, p, g)))
    alone = []
    for field, A in cases:
        if field == "c128":
            alone.append(P.perm_c128(ctx, A))
        elif field == "f64":
            alone.append(P.perm_f64(ctx, A))
        else:
            alone.append(P.perm_modp(ctx, A, p))
    dev = [torch.from_numpy(A.astype(np.int32) if f == "modp" else A).cuda() for f, A in cases]
    batch = [(E.ginibre_complex(12, g), "c128", 0) for _ in range(40)]
    items, data = P.pack_matrices(batch)
    torch.cuda.synchronize()
    outs = []
    for i, ((field, A), d) in enumerate(zip(cases, dev)):
        if field == "c128":
            outs.append(P.perm_c128(ctx, d))
        elif field == "f64":
            outs.append(P.perm_f64(ctx, d))
        else:
            outs.append(P.perm_modp(ctx, d, p))
        if i % 10 == 0:
            P.perm_batch(ctx, items, data)
        if i % 25 == 0:             # 3 primes x 2^12 indices: every block stages and finalizes
            m = 13
            J = np.stack([np.ones((m, m), np.uint32)] * 3)
            val, _ = P.perm_crt_int(ctx, J, O.crt.primes_1_mod_n(2, 3),
                                    math.log2(math.factorial(m)) + 1)
            assert val == math.factorial(m)
    torch.cuda.synchronize()
    for (field, A), o, want in zip(cases, outs, alone):
        o = o.cpu().numpy()
        if field == "c128":
            assert complex(o[0], o[1]) == want
            assert abs(want - O.native.ryser_c128(A)) <= TOL * scale(A)
        elif field == "f64":
            assert o[0] == want
            assert abs(want - O.native.ryser_f64(A)) <= TOL * scale(A)
        else:
            assert int(o[0]) == want == O.native.ryser_modp(A, p)


def test_multi_item_claims_tiny_matrices(P, ctx, O):
    """140,000 f64 matrices of order 5 (one 16-lane item each): items far
    outnumber resident waves, so blocks claim several items per wave at a
    time.  All agree with the oracle."""
    g = E.rng(13, 0)
    A5 = g.standard_normal((140000, 5, 5))
    mats = [(a, "f64", 0) for a in A5]
    items, data = P.pack_matrices(mats)
    vals = P.batch_values(items, P.perm_batch(ctx, items, data))
    for a, v in zip(A5, vals):
        assert abs(v - O.native.ryser_f64(a)) <= TOL * scale(a)
