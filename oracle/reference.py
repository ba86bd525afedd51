"""The permanent straight from its definition.  Test infrastructure only.

perm(A) = sum_{sigma in S_n} prod_i a_{i,sigma(i)}   (paper, Sec. 1)

``bruteforce`` enumerates S_n (n <= 8 in practice: 40,320 terms).  With
Python ``int`` or ``fractions.Fraction`` entries it is exact; with float or
complex entries each product is formed in double precision and the n! terms
are summed with ``math.fsum`` per real component (correctly rounded sum).

``laplace`` expands along the first row, perm(A) = sum_j a_0j perm(A_0j),
memoised over the set of columns still free, which is the same sum regrouped;
it is exact for integer entries and reaches n = 14 or so.
"""
import itertools
import math
from functools import lru_cache


def _rows(A):
    return [list(r) for r in A]


def bruteforce(A):
    A = _rows(A)
    n = len(A)
    if n == 0:
        return 1
    exact = all(isinstance(v, int) or type(v).__name__ == "Fraction" for r in A for v in r)
    if exact:
        tot = 0
        for s in itertools.permutations(range(n)):
            t = 1
            for i in range(n):
                t *= A[i][s[i]]
            tot += t
        return tot
    re, im = [], []
    for s in itertools.permutations(range(n)):
        t = complex(1.0)
        for i in range(n):
            t *= complex(A[i][s[i]])
        re.append(t.real)
        im.append(t.imag)
    return complex(math.fsum(re), math.fsum(im))


def bruteforce_mod(A, p):
    """perm(A) mod p from the definition with exact integers."""
    return bruteforce([[int(v) for v in r] for r in A]) % p


def laplace(A):
    """Exact first-row Laplace expansion, memoised on the free-column mask."""
    A = [[int(v) for v in r] for r in A]
    n = len(A)

    @lru_cache(maxsize=None)
    def rec(row, free):
        if row == n:
            return 1
        tot = 0
        for j in range(n):
            if free >> j & 1:
                a = A[row][j]
                if a:
                    tot += a * rec(row + 1, free & ~(1 << j))
        return tot

    return rec(0, (1 << n) - 1)


def subfactorial(n):
    """!n, the number of derangements: !0 = 1, !1 = 0, !n = (n-1)(!(n-1) + !(n-2))."""
    a, b = 1, 0
    if n == 0:
        return 1
    for k in range(2, n + 1):
        a, b = b, (k - 1) * (a + b)
    return b
