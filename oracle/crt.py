"""Exact integer permanents of the Schur matrix by the Chinese remainder theorem.

Test infrastructure only.  Follows the paper's Sec. 2.1:

* S_n = (w^{jk})_{j,k=0..n-1} with w a primitive n-th root of unity.  For a
  prime p = 1 (mod n) the group (Z/pZ)^* holds a primitive n-th root g, and
  perm(S_n) mod p is the permanent of the integer matrix (g^{jk} mod p).
* |perm(S_n)| <= n^{n/2} (from |perm U| <= 1 for unitary U applied to
  S_n / sqrt(n)), so a product of primes M with M > 2 n^{n/2} determines
  perm(S_n) as the unique integer of the residue class in (-M/2, M/2).

Choices where the paper leaves the details open:

* primes are the smallest p = 1 (mod n) of bit length exactly 31
  (2^30 < p < 2^31), ascending; k is the least count with prod p > 2 n^{n/2},
  tested in integers as (prod p)^2 > 4 n^n;
* g = h^{(p-1)/n} mod p for the smallest h >= 2 whose power has order exactly
  n (g^{n/q} != 1 for every prime q dividing n); any primitive root gives the
  same permanent, since g -> g^a (gcd(a,n) = 1) permutes the columns;
* the lift is the textbook sum X = sum_i r_i M_i (M_i^{-1} mod p_i) mod M,
  then X - M when X > M/2 (M is odd, so there is no tie).

``schur_counts`` is an independent exact route: c_r = #{sigma : sum_j j sigma(j)
= r (mod n)}, counted by a dynamic programme over the set of used columns.
Then perm(S_n) = sum_r c_r w^r, which reduces modulo the n-th cyclotomic
polynomial to a rational integer, and perm(S_n) mod p = sum_r c_r g^r mod p.
"""
import numpy as np


# ------------------------------------------------------------------ primes
def is_prime(m: int) -> bool:
    """Trial division by every odd d <= sqrt(m)."""
    if m < 2:
        return False
    if m % 2 == 0:
        return m == 2
    d = 3
    while d * d <= m:
        if m % d == 0:
            return False
        d += 2
    return True


def prime_factors(m: int):
    out, d = [], 2
    while d * d <= m:
        if m % d == 0:
            out.append(d)
            while m % d == 0:
                m //= d
        d += 1
    if m > 1:
        out.append(m)
    return out


def primes_1_mod_n(n: int, count: int, lo: int = 1 << 30, hi: int = 1 << 31):
    """The ``count`` smallest primes p = 1 (mod n) with lo < p < hi, ascending."""
    out = []
    p = lo + 1
    p += (1 - p) % n            # first p > lo with p = 1 (mod n)
    while len(out) < count:
        if p >= hi:
            raise ValueError("not enough primes in range")
        if p > lo and is_prime(p):
            out.append(p)
        p += n
    return out


def schur_bound_ok(n: int, M: int) -> bool:
    """True when M > 2 n^{n/2}, i.e. M^2 > 4 n^n."""
    return M * M > 4 * n ** n


def primes_for_schur(n: int, extra: int = 0):
    """Least number of 31-bit primes = 1 (mod n) whose product exceeds 2 n^{n/2}."""
    k = 1
    while True:
        ps = primes_1_mod_n(n, k)
        M = 1
        for p in ps:
            M *= p
        if schur_bound_ok(n, M):
            return primes_1_mod_n(n, k + extra)
        k += 1


def root_of_unity(n: int, p: int) -> int:
    """A primitive n-th root of unity mod p (p prime, p = 1 mod n)."""
    if (p - 1) % n:
        raise ValueError("p != 1 (mod n)")
    qs = prime_factors(n) if n > 1 else []
    h = 2
    while True:
        g = pow(h, (p - 1) // n, p)
        if all(pow(g, n // q, p) != 1 for q in qs):
            return g
        h += 1


def schur_residues(n: int, p: int, g: int = None):
    """The n x n matrix (g^{jk} mod p) as uint32."""
    if g is None:
        g = root_of_unity(n, p)
    S = np.zeros((n, n), dtype=np.uint32)
    for j in range(n):
        for k in range(n):
            S[j, k] = pow(g, j * k, p)
    return S


# --------------------------------------------------------------------- CRT
def crt_lift(residues, primes) -> int:
    """The integer X in (-M/2, M/2) with X = r_i (mod p_i), M = prod p_i."""
    M = 1
    for p in primes:
        M *= p
    X = 0
    for r, p in zip(residues, primes):
        Mi = M // p
        X += int(r) * Mi * pow(Mi, -1, p)
    X %= M
    if 2 * X > M:
        X -= M
    return X


# ------------------------------------------------- exact Schur permanents
def schur_counts(n: int):
    """c_r = #{sigma in S_n : sum_j j*sigma(j) = r (mod n)}, r = 0..n-1."""
    if n == 0:
        return np.array([1], dtype=object)
    full = 1 << n
    dp = np.zeros((full, n), dtype=object)
    dp[0, 0] = 1
    for mask in range(full):
        row = bin(mask).count("1")
        if row == n:
            continue
        v = dp[mask]
        if not any(v):
            continue
        for j in range(n):
            if not mask >> j & 1:
                dp[mask | 1 << j] += np.roll(v, (row * j) % n)
    return dp[full - 1]


def _poly_divmod(num, den):
    """Integer polynomial division (den monic), coefficients low degree first."""
    num = list(num)
    q = [0] * max(1, len(num) - len(den) + 1)
    while len(num) >= len(den) and any(num):
        shift = len(num) - len(den)
        c = num[-1]
        q[shift] = c
        for i, d in enumerate(den):
            num[shift + i] -= c * d
        while num and num[-1] == 0:
            num.pop()
    return q, num


def cyclotomic(n: int):
    """Phi_n(x) with integer coefficients, from x^n - 1 = prod_{d | n} Phi_d(x)."""
    poly = [-1] + [0] * (n - 1) + [1]
    for d in range(1, n):
        if n % d == 0:
            poly, rem = _poly_divmod(poly, cyclotomic(d))
            assert not any(rem)
    while poly and poly[-1] == 0:
        poly.pop()
    return poly


def schur_perm_exact(n: int) -> int:
    """perm(S_n) as an integer: sum_r c_r x^r reduced modulo Phi_n(x)."""
    c = [int(v) for v in schur_counts(n)]
    if n <= 1:
        return sum(c)
    _, rem = _poly_divmod(c, cyclotomic(n))
    rem = rem + [0] * (1 - len(rem)) if rem else [0]
    if any(rem[1:]):
        raise AssertionError("sum_r c_r w^r is not a rational integer")
    return rem[0]


def schur_perm_mod_p_from_counts(n: int, p: int, g: int = None) -> int:
    if g is None:
        g = root_of_unity(n, p)
    c = schur_counts(n)
    return sum(int(cr) * pow(g, r, p) for r, cr in enumerate(c)) % p
