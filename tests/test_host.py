"""Host-side checks of libperm that need no GPU: the exported C ABI, the
number-theory helpers against the oracle, argument validation."""
import math
import os
import random
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2602_10141_amd", "libperm.so")


@pytest.fixture(scope="module")
def P():
    if not os.path.exists(LIB):
        from paper_2602_10141_amd import build
        build.build(force=False)
    from paper_2602_10141_amd import perm
    perm.lib()
    return perm


def header_functions():
    text = open(os.path.join(ROOT, "include", "perm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(perm_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_function(P):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    declared = header_functions()
    assert len(declared) >= 20
    missing = [f for f in declared if f not in exported]
    assert not missing, missing
    for f in declared:
        getattr(P.lib(), f)           # resolvable through ctypes


def test_item_struct_layout(P):
    assert P.ITEM_DTYPE.itemsize == 24


def test_schur_primes_match_oracle(P, oracle_lib):
    for n in (3, 5, 7, 11, 20, 28, 32, 34, 36, 43, 45):
        assert P.perm_schur_primes(n) == oracle_lib.crt.primes_for_schur(n)
        assert P.perm_schur_primes(n, extra=2) == oracle_lib.crt.primes_for_schur(n, extra=2)


def test_pick_primes_is_schur_primes(P):
    for n in (5, 28, 36):
        assert P.perm_pick_primes(n) == P.perm_schur_primes(n)
        assert P.perm_pick_primes(n, extra=3) == P.perm_schur_primes(n, extra=3)


def test_schur_residues_match_oracle(P, oracle_lib):
    for n in (3, 7, 12, 28, 36):
        for p in oracle_lib.crt.primes_1_mod_n(n, 2):
            assert np.array_equal(P.perm_schur_residues(n, p), oracle_lib.crt.schur_residues(n, p))


def test_crt_lift_matches_textbook(P, oracle_lib):
    g = random.Random(1)
    ps = oracle_lib.crt.primes_1_mod_n(36, 6)
    M = math.prod(ps)
    for k in (1, 2, 3, 6):
        Mk = math.prod(ps[:k])
        for _ in range(100):
            X = g.randrange(-(Mk // 2), Mk // 2 + 1)
            res = [X % p for p in ps[:k]]
            bound = max(0.0, math.log2(Mk) - 1.5)
            assert P.perm_crt_lift(res, ps[:k], bound) == X == oracle_lib.crt.crt_lift(res, ps[:k])
    assert P.perm_crt_lift([0] * 6, ps, 10) == 0
    assert M > 0


@pytest.mark.parametrize("n", [9, 11, 13, 15])
def test_residue_flip_names_the_bad_prime(P, oracle_lib, n):
    """perm(S_n) for odd n over the sufficient primes plus one redundant
    prime, residues from the oracle: consistent residues lift to the exact
    value with no bad prime; one corrupted residue (any of the k + 1, any
    nonzero offset) is named and the value still comes out right; two
    corrupted residues are reported as inconsistent."""
    O = oracle_lib
    primes = P.perm_schur_primes(n, extra=1)
    bound = (n / 2) * math.log2(n)
    res = [O.native.ryser_modp(O.crt.schur_residues(n, p), p) for p in primes]
    want = O.crt.crt_lift(res, primes)
    if n <= 10:
        assert want == O.crt.schur_perm_exact(n)
    assert want != 0
    assert P.perm_crt_check(res, primes, bound) == (want, None)
    g = random.Random(n)
    for j in range(len(primes)):
        for _ in range(3):
            bad = list(res)
            bad[j] = (bad[j] + g.randrange(1, primes[j])) % primes[j]
            assert P.perm_crt_check(bad, primes, bound) == (want, j)
    two = list(res)
    two[0] = (two[0] + 1) % primes[0]
    two[-1] = (two[-1] + 7) % primes[-1]
    with pytest.raises(P.PermError) as e:
        P.perm_crt_check(two, primes, bound)
    assert e.value.status == P.PERM_ERANGE
    with pytest.raises(P.PermError) as e:                 # no redundant prime
        P.perm_crt_check(res[:-1], primes[:-1], bound * 1.9)
    assert e.value.status == P.PERM_ERANGE


def test_crt_lift_rejects_bad_input(P):
    ps = [1073742209, 1073742517]
    with pytest.raises(P.PermError) as e:
        P.perm_crt_lift([1, 2], ps, 61.0)            # 2 primes < 2^62 cannot hold 2^62
    assert e.value.status == P.PERM_ERANGE
    with pytest.raises(P.PermError) as e:
        P.perm_crt_lift([1, 2], [ps[0], ps[0]], 10)
    assert e.value.status == P.PERM_EINVAL
    with pytest.raises(P.PermError) as e:
        P.perm_crt_lift([1, 2], [ps[0], (1 << 30) + 1], 10)       # 2^30 + 1 is composite
    assert e.value.status == P.PERM_EINVAL


def test_schur_residues_reject_bad_prime(P):
    with pytest.raises(P.PermError):
        P.perm_schur_residues(9, 1073742209)     # 1073742209 != 1 mod 9
    with pytest.raises(P.PermError):
        P.perm_schur_residues(5, 15)


def test_context_without_gpu_reports_device_error(P):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(P.PermError) as e:
        P.Context(0)
    assert e.value.status == P.PERM_EDEVICE


def test_strerror(P):
    assert P.perm_strerror(P.PERM_OK) == "ok"
    assert "argument" in P.perm_strerror(P.PERM_EINVAL)
