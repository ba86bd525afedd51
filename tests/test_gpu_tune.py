"""Tuning table and autotuner: any partition stays within tolerance (floats)
or bit-exact (F_p); the table round-trips through a file."""
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


def scale(A):
    return float(np.prod(np.linalg.norm(A, axis=1)))


@pytest.mark.parametrize("c", [3, 4, 6, 9, 11])
def test_any_chunk_length_is_correct(P, oracle_lib, c):
    ctx = P.Context(0)
    try:
        n = 18
        P.perm_tune_set(ctx, "c128", n, c)
        P.perm_tune_set(ctx, "f64", n, c)
        P.perm_tune_set(ctx, "modp", n, c)
        A = E.ginibre_complex(n, E.rng(30, c))
        B = E.ginibre_real(n, E.rng(32, c))
        R = E.random_residues(n, 1073742209, E.rng(31, c))
        assert abs(P.perm_c128(ctx, A) - oracle_lib.native.ryser_c128(A)) <= 1e-10 * scale(A)
        assert abs(P.perm_f64(ctx, B) - oracle_lib.native.ryser_f64(B)) <= 1e-10 * scale(B)
        assert P.perm_modp(ctx, R, 1073742209) == oracle_lib.native.ryser_modp(R, 1073742209)
        assert P.perm_tune_get(ctx, "c128", n)[0] == c
    finally:
        ctx.close()


@pytest.mark.parametrize("n", [10, 12, 13, 15])
def test_many_items_per_small_matrix(P, oracle_lib, n):
    """Small orders split over many wave items (c = 3), batch and single."""
    ctx = P.Context(0)
    try:
        for f in ("c128", "f64"):
            P.perm_tune_set(ctx, f, n, 3)
        mats = [(E.ginibre_complex(n, E.rng(33, n + i)), "c128", 0) for i in range(3)] + \
               [(E.ginibre_real(n, E.rng(34, n + i)), "f64", 0) for i in range(3)]
        items, data = P.pack_matrices(mats)
        got = P.batch_values(items, P.perm_batch(ctx, items, data))
        for (A, f, _), v in zip(mats, got):
            want = (oracle_lib.native.ryser_c128 if f == "c128" else oracle_lib.native.ryser_f64)(A)
            assert abs(v - want) <= 1e-10 * scale(A)
            single = P.perm_c128(ctx, A) if f == "c128" else P.perm_f64(ctx, A)
            assert single == v
    finally:
        ctx.close()


def test_autotune_and_roundtrip(P, oracle_lib, tmp_path):
    ctx = P.Context(0)
    try:
        P.perm_autotune(ctx, "f64", 14, 16, batch=64)
        P.perm_autotune(ctx, "modp", 22, 22, batch=1)
        tuned = {n: P.perm_tune_get(ctx, "f64", n) for n in (14, 15, 16)}
        path = tmp_path / "tune.txt"
        P.perm_tune_save(ctx, path)
        A = E.ginibre_real(16, E.rng(32, 0))
        before = P.perm_f64(ctx, A)
        assert abs(before - oracle_lib.native.ryser_f64(A)) <= 1e-10 * scale(A)
    finally:
        ctx.close()
    ctx2 = P.Context(0)
    try:
        P.perm_tune_load(ctx2, path)
        assert {n: P.perm_tune_get(ctx2, "f64", n) for n in (14, 15, 16)} == tuned
        assert P.perm_f64(ctx2, A) == before          # same partition, same bits
        with pytest.raises(P.PermError):
            P.perm_tune_set(ctx2, "modp", 30, 22)        # F_p chunks limited to 2^20
    finally:
        ctx2.close()


def test_repeated_calls_follow_the_table(P):
    """A repeated call reuses its plan only while the chunk lengths it used
    are unchanged: after a table change the next call takes the new
    partition (bit-identical to a fresh context with that table)."""
    A = E.ginibre_complex(17, E.rng(35, 0))
    B = E.ginibre_complex(17, E.rng(35, 1))
    ctx, fresh = P.Context(0), P.Context(0)
    try:
        a0 = P.perm_c128(ctx, A)
        b0 = P.perm_c128(ctx, B)                 # same plan, new data
        assert P.perm_c128(fresh, B) == b0
        for c in (3, 6, 0):
            P.perm_tune_set(ctx, "c128", 17, c)
            P.perm_tune_set(fresh, "c128", 17, c)
            got = P.perm_c128(ctx, A)
            other = P.Context(0)
            try:
                P.perm_tune_set(other, "c128", 17, c)
                assert got == P.perm_c128(other, A)
            finally:
                other.close()
            if c == 0:
                assert got == a0
    finally:
        ctx.close()
        fresh.close()
