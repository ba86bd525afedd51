"""Pins of the oracle against what the paper and the mathematics fix.

None of these retypes the oracle's own formula: each compares it with the
definition (brute force, Laplace expansion), a closed form (n!, derangements,
products of diagonals), an invariance, an independent exact route (the Schur
group-ring count) or a value the paper prints (tests/golden/).
"""
import math
import random

import numpy as np
import pytest

from conftest import golden
from paper_2602_10141_amd import ensembles as E


@pytest.fixture(scope="module")
def O(oracle_lib):
    return oracle_lib


def _cplx(n, seed):
    return E.ginibre_complex(n, E.rng(900, seed))


# --------------------------------------------------------------- definition
@pytest.mark.parametrize("n", range(0, 8))
def test_ryser_c128_equals_bruteforce(O, n):
    A = _cplx(n, n)
    want = O.reference.bruteforce(A.tolist()) if n else 1
    got = O.native.ryser_c128(A)
    scale = max(1.0, float(np.prod(np.linalg.norm(A, axis=1)))) if n else 1.0
    assert abs(got - want) <= 1e-13 * scale


@pytest.mark.parametrize("n", range(0, 8))
def test_ryser_f64_equals_bruteforce(O, n):
    A = E.ginibre_real(n, E.rng(901, n))
    want = O.reference.bruteforce(A.tolist()) if n else 1
    got = O.native.ryser_f64(A)
    scale = max(1.0, float(np.prod(np.linalg.norm(A, axis=1)))) if n else 1.0
    assert abs(got - complex(want).real) <= 1e-13 * scale


@pytest.mark.parametrize("p", [2, 3, 5, 7, 97, 65537, 1073742209, 2147483647])
@pytest.mark.parametrize("n", [1, 2, 3, 5, 7])
def test_ryser_modp_equals_bruteforce(O, n, p):
    A = E.random_residues(n, p, E.rng(902, n * 1000 + p % 1000))
    want = O.reference.bruteforce_mod(A.tolist(), p)
    assert O.native.ryser_modp(A, p) == want


def test_ryser_modp_integer_matrix_equals_laplace(O):
    g = random.Random(5)
    for n in (8, 9, 10, 11):
        A = [[g.randrange(-50, 51) for _ in range(n)] for _ in range(n)]
        exact = O.reference.laplace(A)
        for p in (1073742209, 2147483647, 101):
            R = np.array([[a % p for a in row] for row in A], dtype=np.uint32)
            assert O.native.ryser_modp(R, p) == exact % p


def test_two_by_two(O):
    a, b, c, d = 1.5 - 2j, 0.25 + 1j, -3 + 0.5j, 2 - 1j
    assert abs(O.native.ryser_c128(np.array([[a, b], [c, d]])) - (a * d + b * c)) < 1e-14
    assert O.native.ryser_f64(np.array([[2.0, 3.0], [5.0, 7.0]])) == 2 * 7 + 3 * 5
    assert O.native.ryser_modp(np.array([[2, 3], [5, 7]], dtype=np.uint32), 11) == (14 + 15) % 11


# ------------------------------------------------------------- closed forms
@pytest.mark.parametrize("n", range(1, 14))
def test_all_ones_is_factorial(O, n):
    J = np.ones((n, n))
    assert O.native.ryser_f64(J) == math.factorial(n)          # exact below 2^53
    assert O.native.ryser_c128(J.astype(complex)) == math.factorial(n)
    p = 1073742209
    assert O.native.ryser_modp(np.ones((n, n), dtype=np.uint32), p) == math.factorial(n) % p


@pytest.mark.parametrize("n", range(1, 13))
def test_derangements(O, n):
    J = np.ones((n, n)) - np.eye(n)
    want = O.reference.subfactorial(n)
    assert O.native.ryser_f64(J) == want
    p = 2147483647
    assert O.native.ryser_modp(J.astype(np.uint32), p) == want % p


def test_subfactorial_counts_fixed_point_free_permutations(O):
    import itertools
    for n in range(0, 8):
        cnt = sum(all(s[i] != i for i in range(n)) for s in itertools.permutations(range(n)))
        assert O.reference.subfactorial(n) == cnt


@pytest.mark.parametrize("n", [1, 4, 9, 16])
def test_permutation_diagonal_triangular(O, n):
    g = E.rng(903, n)
    perm = g.permutation(n)
    P = np.zeros((n, n))
    P[np.arange(n), perm] = 1.0
    assert O.native.ryser_f64(P) == 1.0
    assert O.native.ryser_modp(P.astype(np.uint32), 7) == 1
    D = np.diag(E.ginibre_complex(n, g)[0])
    want = np.prod(np.diag(D))
    assert abs(O.native.ryser_c128(D) - want) <= 1e-13 * max(1, abs(want))
    T = np.triu(E.ginibre_complex(n, g))
    want = np.prod(np.diag(T))
    scale = float(np.prod(np.linalg.norm(T, axis=1)))
    assert abs(O.native.ryser_c128(T) - want) <= 1e-12 * max(1.0, scale)


# --------------------------------------------------------------- invariances
def test_row_column_permutation_and_transpose(O):
    n = 10
    A = _cplx(n, 77)
    g = E.rng(904, 0)
    base = O.native.ryser_c128(A)
    scale = float(np.prod(np.linalg.norm(A, axis=1)))
    for B in (A[g.permutation(n)], A[:, g.permutation(n)], A.T.copy()):
        assert abs(O.native.ryser_c128(B) - base) <= 1e-12 * scale
    R = E.random_residues(n, 1073742209, g)
    b = O.native.ryser_modp(R, 1073742209)
    assert O.native.ryser_modp(R[g.permutation(n)], 1073742209) == b
    assert O.native.ryser_modp(R[:, g.permutation(n)], 1073742209) == b
    assert O.native.ryser_modp(R.T.copy(), 1073742209) == b


def test_row_scaling_is_multilinear(O):
    n = 9
    A = _cplx(n, 78)
    c = 2.5 - 0.75j
    B = A.copy()
    B[3] *= c
    scale = float(np.prod(np.linalg.norm(B, axis=1)))
    assert abs(O.native.ryser_c128(B) - c * O.native.ryser_c128(A)) <= 1e-12 * scale
    # additivity in one row
    C = A.copy()
    C[0] = _cplx(n, 79)[0]
    S = A.copy()
    S[0] = A[0] + C[0]
    lhs = O.native.ryser_c128(S)
    rhs = O.native.ryser_c128(A) + O.native.ryser_c128(C)
    assert abs(lhs - rhs) <= 1e-12 * float(np.prod(np.linalg.norm(S, axis=1)))


def test_laplace_expansion_row0(O):
    n = 9
    A = _cplx(n, 80)
    tot = 0
    for j in range(n):
        minor = np.delete(np.delete(A, 0, axis=0), j, axis=1)
        tot += A[0, j] * O.native.ryser_c128(minor)
    scale = float(np.prod(np.linalg.norm(A, axis=1)))
    assert abs(O.native.ryser_c128(A) - tot) <= 1e-12 * scale


# ------------------------------------------------ Glynn terms (range checks)
@pytest.mark.parametrize("n", [1, 2, 5, 8, 11])
def test_glynn_full_range_equals_perm(O, n):
    A = _cplx(n, 81 + n)
    full = O.native.glynn_range_c128(A, 0, 1 << (n - 1)) / 2 ** (n - 1)
    scale = float(np.prod(np.linalg.norm(A, axis=1)))
    assert abs(full - O.native.ryser_c128(A)) <= 1e-12 * max(1.0, scale)
    R = A.real.copy()
    assert abs(O.native.glynn_range_f64(R, 0, 1 << (n - 1)) / 2 ** (n - 1)
               - O.native.ryser_f64(R)) <= 1e-12 * max(1.0, scale)
    p = 1073742209
    M = E.random_residues(n, p, E.rng(905, n))
    inv = pow(2 ** (n - 1), -1, p)
    assert O.native.glynn_range_modp(M, p, 0, 1 << (n - 1)) * inv % p == O.native.ryser_modp(M, p)


def test_glynn_ranges_are_additive(O):
    n, p = 12, 2147483647
    M = E.random_residues(n, p, E.rng(906, 0))
    T = 1 << (n - 1)
    cuts = [0, 1, 7, 64, 1000, T]
    parts = [O.native.glynn_range_modp(M, p, a, b) for a, b in zip(cuts, cuts[1:])]
    assert sum(parts) % p == O.native.glynn_range_modp(M, p, 0, T)


# ----------------------------------------------------------------- Kahan
def test_long_double_audit_and_kahan(O):
    """The double walk agrees with the long double walk to ~1e-13 of scale."""
    for n, seed in ((14, 1), (16, 2)):
        A = _cplx(n, 200 + seed)
        ld = O.native.ryser_c128_longdouble(A)
        d = O.native.ryser_c128(A)
        scale = float(np.prod(np.linalg.norm(A, axis=1)))
        assert abs(ld - d) <= 1e-12 * scale


# ---------------------------------------------------------------------- CRT
def test_primality_and_primes_against_sympy(O):
    import sympy
    g = random.Random(3)
    for _ in range(300):
        m = g.randrange(1 << 30, 1 << 31)
        assert O.crt.is_prime(m) == sympy.isprime(m)
    for m in range(0, 2000):
        assert O.crt.is_prime(m) == sympy.isprime(m)
    for n in (5, 7, 28, 36):
        ps = O.crt.primes_1_mod_n(n, 6)
        assert ps == sorted(ps)
        for p in ps:
            assert p % n == 1 and (1 << 30) < p < (1 << 31) and sympy.isprime(p)
        # nothing was skipped: every q = 1 (mod n) below the last one is composite
        q = ps[0] - n
        while q > (1 << 30):
            assert not sympy.isprime(q)
            q -= n


@pytest.mark.parametrize("n,k", [(28, 3), (32, 3), (34, 3), (36, 4), (43, 4), (45, 5)])
def test_prime_counts(O, n, k):
    assert len(O.crt.primes_for_schur(n)) == k


def test_root_of_unity_has_order_n(O):
    from sympy.ntheory import n_order
    for n in (3, 5, 9, 10, 11, 28, 36):
        for p in O.crt.primes_1_mod_n(n, 3):
            assert n_order(O.crt.root_of_unity(n, p), p) == n


def test_crt_lift_against_sympy(O):
    from sympy.ntheory.modular import crt as sympy_crt
    g = random.Random(11)
    ps = O.crt.primes_1_mod_n(36, 5)
    M = math.prod(ps)
    for _ in range(200):
        X = g.randrange(-(M // 2), M // 2 + 1)
        res = [X % p for p in ps]
        assert O.crt.crt_lift(res, ps) == X
        y, _ = sympy_crt(ps, res)
        assert (int(y) - X) % M == 0


def test_cyclotomic_against_sympy(O):
    import sympy
    x = sympy.Symbol("x")
    for n in range(1, 25):
        want = sympy.Poly(sympy.cyclotomic_poly(n, x), x).all_coeffs()[::-1]
        assert O.crt.cyclotomic(n) == [int(c) for c in want]


# -------------------------------------------------------------------- Schur
@pytest.mark.parametrize("n", range(1, 11))
def test_schur_exact_counts_match_complex_perm(O, n):
    """Group-ring count vs the complex permanent of S_n = (e^{2 pi i jk/n})."""
    exact = O.crt.schur_perm_exact(n)
    got = O.native.ryser_c128(E.schur_complex(n))
    assert abs(got - exact) <= 1e-9 * n ** (n / 2)
    assert abs(exact) <= n ** (n / 2)                 # |perm S_n| <= n^{n/2}
    if n % 2 == 0:
        assert exact == 0                              # even n: shift argument


@pytest.mark.parametrize("n", [3, 5, 7, 8, 9, 10, 11, 12])
def test_schur_modp_matches_counts(O, n):
    for p in O.crt.primes_1_mod_n(n, 2):
        S = O.crt.schur_residues(n, p)
        assert O.native.ryser_modp(S, p) == O.crt.schur_perm_mod_p_from_counts(n, p)


@pytest.mark.parametrize("n", [5, 7, 9, 11])
def test_schur_crt_recovers_exact_integer(O, n):
    exact = O.crt.schur_perm_exact(n)
    ps = O.crt.primes_for_schur(n, extra=2)
    res = [O.native.ryser_modp(O.crt.schur_residues(n, p), p) for p in ps]
    k = len(ps) - 2
    assert O.crt.crt_lift(res[:k], ps[:k]) == exact
    assert O.crt.crt_lift(res[2:], ps[2:]) == exact     # another prime set
    assert O.crt.crt_lift(res, ps) == exact             # redundant set


def test_schur_galois_invariance(O):
    for n in (7, 9, 10):
        p = O.crt.primes_1_mod_n(n, 1)[0]
        g = O.crt.root_of_unity(n, p)
        base = O.native.ryser_modp(O.crt.schur_residues(n, p, g), p)
        for a in range(2, n):
            if math.gcd(a, n) == 1:
                assert O.native.ryser_modp(O.crt.schur_residues(n, p, pow(g, a, p)), p) == base


@pytest.mark.parametrize("n", [6, 8, 12])
def test_schur_even_n_is_zero_mod_p(O, n):
    for p in O.crt.primes_1_mod_n(n, 3):
        assert O.native.ryser_modp(O.crt.schur_residues(n, p), p) == 0


def test_schur_28_is_zero_mod_first_prime(O):
    """The benchmark's order: the full 2^28-subset Ryser sum of S_28 mod its
    smallest prime, split over host threads, is 0 (even n)."""
    p = O.crt.primes_1_mod_n(28, 1)[0]
    assert O.native.ryser_modp_threaded(O.crt.schur_residues(28, p), p) == 0


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7])
def test_ryser_modp_ranges_add_up_to_bruteforce(O, n):
    """Random partitions of the subset range [1, 2^n) into Gray-index ranges:
    the range sums (each seeded from its first subset) add up to perm(A) mod p
    from the definition, up to the sign (-1)^n."""
    p = 1073742209
    A = E.random_residues(n, p, E.rng(907, n))
    want = O.reference.bruteforce_mod(A.tolist(), p)
    g = random.Random(n)
    end = 1 << n
    for _ in range(6):
        cuts = sorted({1, end, *(g.randrange(1, end + 1) for _ in range(g.randrange(0, 5)))})
        tot = sum(O.native.ryser_modp_range(A, p, a, b) for a, b in zip(cuts, cuts[1:])) % p
        assert ((p - tot) % p if n % 2 else tot) == want
    assert O.native.ryser_modp_threaded(A, p, threads=3) == want


def test_ryser_modp_threaded_equals_laplace(O):
    g = random.Random(6)
    for n in (10, 13):
        A = [[g.randrange(-40, 41) for _ in range(n)] for _ in range(n)]
        exact = O.reference.laplace(A)
        p = 2147483647
        R = np.array([[a % p for a in row] for row in A], dtype=np.uint32)
        assert O.native.ryser_modp_threaded(R, p, threads=5) == exact % p


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7])
def test_ryser_float_ranges_add_up_to_bruteforce(O, n):
    """Complex and real Ryser sums over random partitions of [1, 2^n), each
    range seeded from its first subset, add up to perm(A) from the
    definition, up to the sign (-1)^n."""
    A = _cplx(n, 910 + n)
    R = A.real.copy()
    scale = max(1.0, float(np.prod(np.linalg.norm(A, axis=1))))
    wc = O.reference.bruteforce(A.tolist())
    wr = O.reference.bruteforce(R.tolist())
    g = random.Random(100 + n)
    end = 1 << n
    sign = -1 if n % 2 else 1
    for _ in range(6):
        cuts = sorted({1, end, *(g.randrange(1, end + 1) for _ in range(g.randrange(0, 5)))})
        zc = sum(O.native.ryser_float_range(A, a, b) for a, b in zip(cuts, cuts[1:]))
        zr = sum(O.native.ryser_float_range(R, a, b) for a, b in zip(cuts, cuts[1:]))
        assert abs(sign * zc - wc) <= 1e-13 * scale
        assert abs(sign * zr - wr) <= 1e-13 * scale
    assert abs(O.native.ryser_float_threaded(A, threads=3) - wc) <= 1e-13 * scale


def test_ryser_float_threaded_matches_the_whole_walk(O):
    for n in (12, 15):
        A = _cplx(n, 920 + n)
        scale = float(np.prod(np.linalg.norm(A, axis=1)))
        assert abs(O.native.ryser_float_threaded(A, threads=5) - O.native.ryser_c128(A)) <= 1e-12 * scale
        R = A.real.copy()
        assert abs(O.native.ryser_float_threaded(R, threads=5) - O.native.ryser_f64(R)) <= 1e-12 * scale


def test_glynn_range_threaded_is_the_plain_range(O):
    n, p = 12, 1073742209
    M = E.random_residues(n, p, E.rng(908, 0))
    A = _cplx(n, 908)
    for x0, x1 in [(0, 1 << 11), (5, 1999), (100, 101)]:
        assert O.native.glynn_range_threaded(M, x0, x1, "modp", p, threads=4) == \
            O.native.glynn_range_modp(M, p, x0, x1)
        whole = O.native.glynn_range_c128(A, x0, x1)
        got = O.native.glynn_range_threaded(A, x0, x1, "c128", threads=4)
        assert abs(got - whole) <= 1e-13 * float(np.prod(np.linalg.norm(A, axis=1))) * (x1 - x0)


def test_crt_factorial_and_sign(O):
    """perm(J_n) = n! and perm(diag(-1,1,..,1) J_n) = -n! through the CRT."""
    n = 21                                   # 21! ~ 2^65.4: three 31-bit primes
    ps = O.crt.primes_1_mod_n(2, 3)          # any odd 31-bit primes
    J = np.ones((n, n), dtype=np.uint32)
    res = [O.native.ryser_modp(J, p) for p in ps]
    assert O.crt.crt_lift(res, ps) == math.factorial(n)
    res_neg = []
    for p in ps:
        Jm = J.copy()
        Jm[0, :] = p - 1
        res_neg.append(O.native.ryser_modp(Jm, p))
    assert O.crt.crt_lift(res_neg, ps) == -math.factorial(n)


# ----------------------------------------------------------------- geodesic
@pytest.mark.parametrize("n", [5, 7, 11, 13])
def test_cycle_geodesic_closed_form_is_exp_t_log(O, n):
    from scipy.linalg import expm, logm
    L = logm(E.cycle_matrix(n).astype(complex))
    for t in (0.0, 0.1, 0.5, 0.77, 1.0):
        G = E.cycle_geodesic(n, t)
        assert np.max(np.abs(G - expm(t * L))) < 1e-12
        assert np.max(np.abs(G @ G.conj().T - np.eye(n))) < 1e-12   # unitary (and real)


def test_geodesic_endpoints_and_symmetry(O):
    for n in (7, 11, 13):
        assert abs(O.native.ryser_c128(E.cycle_geodesic(n, 0.0)) - 1) < 1e-14
        assert abs(O.native.ryser_c128(E.cycle_geodesic(n, 1.0)) - 1) < 1e-14
        for t in E.geodesic_grid(64)[1:8]:
            a = O.native.ryser_c128(E.cycle_geodesic(n, t))
            b = O.native.ryser_c128(E.cycle_geodesic(n, 1 - t))
            assert abs(a.imag) < 1e-15 and abs(a - b) < 1e-13
            assert abs(a) <= 1 + 1e-12


@pytest.mark.parametrize("row", golden("midpoint_table.txt"), ids=lambda r: "n=" + r[0])
def test_midpoint_table(O, row):
    n, printed, ratio = int(row[0]), float(row[1]), float(row[2])
    v = O.native.ryser_c128(E.cycle_geodesic(n, 0.5))
    assert abs(v.imag) <= 1e-14
    assert v.real > 0                                    # principal branch
    # magnitude to the 4 printed significant figures
    assert abs(abs(v) - abs(printed)) <= 0.5e-3 * abs(printed) * 1.0001
    assert abs(abs(v) / (2 * math.exp(-n)) - ratio) <= 0.6e-4
    # the circulant-formula branch carries the printed sign
    w = O.native.ryser_c128(E.cycle_geodesic_circulant(n, 0.5))
    assert abs(w.imag) <= 1e-12 and math.copysign(1, w.real) == math.copysign(1, printed)
    assert abs(abs(w) - abs(v)) <= 1e-12


def test_midpoint_asymptotic_n25(O):
    n = 25
    v = O.native.ryser_c128(E.cycle_geodesic(n, 0.5)).real
    assert abs(v / (2 * math.exp(-n) * (1 + 1 / (3 * n))) - 1) < 2e-3


def _dft_geodesic_by_eigh(n, t, branch):
    """gamma(t) from an orthonormal eigenbasis: H + 2K with H = (F + F^*)/2 and
    K = (F - F^*)/(2i) is Hermitian with eigenvalue 1, -1, 2, -2 on the
    eigenspaces of F for 1, -1, i, -i (F is normal and F^4 = I)."""
    F = E.dft_matrix(n)
    H = (F + F.conj().T) / 2
    K = (F - F.conj().T) / 2j
    mu, V = np.linalg.eigh(H + 2 * K)
    angle = {1: 0.0, -1: branch * np.pi, 2: np.pi / 2, -2: -np.pi / 2}
    ph = np.array([np.exp(1j * t * angle[int(round(m))]) for m in mu])
    return (V * ph) @ V.conj().T


@pytest.mark.parametrize("n", [4, 5, 7, 9, 12])
@pytest.mark.parametrize("branch", [1, -1])
def test_dft_geodesic_construction(O, n, branch):
    F = E.dft_matrix(n)
    assert np.max(np.abs(E.dft_geodesic(n, 0.0, branch) - np.eye(n))) < 1e-13
    assert np.max(np.abs(E.dft_geodesic(n, 1.0, branch) - F)) < 1e-13
    for t in (0.13, 0.5, 0.81):
        G = E.dft_geodesic(n, t, branch)
        assert np.max(np.abs(G @ G.conj().T - np.eye(n))) < 1e-13      # unitary
        assert np.max(np.abs(G - _dft_geodesic_by_eigh(n, t, branch))) < 1e-12
        # one-parameter group: gamma(s) gamma(t) = gamma(s + t)
        assert np.max(np.abs(E.dft_geodesic(n, 0.3, branch) @ G -
                             E.dft_geodesic(n, 0.3 + t, branch))) < 1e-12
    # the two branches differ exactly on the -1 eigenspace
    if n >= 2:
        d = E.dft_geodesic(n, 0.5, 1) - E.dft_geodesic(n, 0.5, -1)
        assert np.max(np.abs(d)) > 0.1


def test_dft_permanent_endpoints(O):
    for n in (3, 5, 6, 7):
        F = E.dft_matrix(n)
        assert abs(O.native.ryser_c128(E.dft_geodesic(n, 0.0)) - 1) < 1e-14
        want = O.reference.bruteforce(F)
        assert abs(O.native.ryser_c128(E.dft_geodesic(n, 1.0)) - want) < 1e-12


def test_branch_phase_relation(O):
    for n in (5, 9):
        for t in (0.2, 0.37, 0.5, 0.9):
            pr = O.native.ryser_c128(E.cycle_geodesic(n, t))
            eq = O.native.ryser_c128(E.cycle_geodesic_circulant(n, t))
            assert abs(eq - np.exp(1j * np.pi * (n - 1) * t) * pr) < 1e-13


# --------------------------------------------------------------- ensembles
def test_gue_permanent_is_real(O):
    for s in range(10):
        H = E.gue(9, E.rng(907, s))
        v = O.native.ryser_c128(H)
        assert abs(v.imag) <= 1e-12 * max(1.0, abs(v.real)) + 1e-12 * np.prod(np.linalg.norm(H, axis=1))


def test_haar_unitary_permanent_bounded(O):
    U = E.haar_unitary(8, E.rng(908, 0), count=200)
    assert np.max(np.abs(U @ np.conj(np.swapaxes(U, 1, 2)) - np.eye(8))) < 1e-13
    vals = O.native.ryser_many(U)
    assert np.all(np.abs(vals) <= 1 + 1e-12)


def test_orthogonal_variance_table_n7(O):
    """Var perm(O), n = 7, against the paper's 7.89e-4 within 5 standard errors."""
    Os = E.haar_orthogonal(7, E.rng(909, 0), count=20000)
    v = O.native.ryser_many(Os)
    var = float(np.var(v))
    k = float(np.mean((v - v.mean()) ** 4) / var ** 2 - 3)
    se = var * math.sqrt((k + 2) / len(v))
    assert abs(var - 7.89e-4) < 5 * se


def test_ginibre_second_moment(O):
    """E |perm G|^2 = n! for i.i.d. CN(0,1) entries, within 5 standard errors."""
    n = 5
    G = E.ginibre_complex(n, E.rng(910, 0), count=40000)
    m2 = np.abs(O.native.ryser_many(G)) ** 2
    se = float(np.std(m2)) / math.sqrt(len(m2))
    assert abs(float(np.mean(m2)) - math.factorial(n)) < 5 * se
