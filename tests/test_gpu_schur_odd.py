"""Odd-order Schur permanents beyond the oracle's reach, checked by
redundancy, Galois invariance and range additivity (no table of known values
is used).  n = 15..21 are also checked against the oracle outright."""
import itertools
import math

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


@pytest.mark.parametrize("n", [15, 17, 19, 21])
def test_odd_schur_against_oracle(P, ctx, oracle_lib, n):
    primes = P.perm_schur_primes(n)
    mats = np.stack([P.perm_schur_residues(n, p) for p in primes])
    val, res = P.perm_crt_int(ctx, mats, primes, (n / 2) * math.log2(n))
    want = [oracle_lib.native.ryser_modp(m, p) for m, p in zip(mats, primes)]
    assert res == want
    assert val == oracle_lib.crt.crt_lift(want, primes)
    assert abs(val) <= n ** (n / 2)


@pytest.mark.parametrize("n", [23, 25, 27, 29, 31])
def test_odd_schur_redundant_primes_agree(P, ctx, n):
    k = len(P.perm_schur_primes(n))
    primes = P.perm_schur_primes(n, extra=2)
    mats = np.stack([P.perm_schur_residues(n, p) for p in primes])
    bound = (n / 2) * math.log2(n)
    _, res = P.perm_crt_int(ctx, mats, primes, bound)
    vals = set()
    for sub in itertools.combinations(range(len(primes)), k):
        vals.add(P.perm_crt_lift([res[i] for i in sub], [primes[i] for i in sub], bound))
    assert len(vals) == 1
    v = vals.pop()
    assert v != 0 and abs(v) <= n ** (n / 2)
    # Galois: replacing g by g^a (gcd(a, n) = 1) permutes columns, same residue
    p = primes[0]
    S = mats[0]
    a = next(a for a in range(2, n) if math.gcd(a, n) == 1)
    cols = [(a * k_) % n for k_ in range(n)]
    assert P.perm_modp(ctx, S[:, cols].copy(), p) == res[0]


def test_range_split_reassembles_crt(P, ctx):
    """perm mod p from four perm_range pieces equals perm_modp (n = 27)."""
    n = 27
    p = P.perm_schur_primes(n)[0]
    S = P.perm_schur_residues(n, p)
    items, data = P.pack_matrices([(S, "modp", p)])
    T = 1 << (n - 1)
    cuts = [0, T // 3, T // 2 + 12345, T - 7, T]
    tot = sum(P.perm_range(ctx, items[0], data, a, b) for a, b in zip(cuts, cuts[1:])) % p
    assert tot * pow(2, -(n - 1), p) % p == P.perm_modp(ctx, S, p)
