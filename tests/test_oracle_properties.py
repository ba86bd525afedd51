"""Property-based pins of the oracle (hypothesis): exact integer matrices, so
every identity is checked bit-exactly mod p and against exact integers.

* perm is invariant under row and column permutations and transposition;
* it is linear in each row (a row scaled by c scales perm by c; a row that
  is a sum of two rows gives the sum of the two permanents);
* a block-diagonal matrix has the product of its blocks' permanents;
* Ryser mod p equals the exact integer permanent (Laplace expansion) mod p,
  also when the subset range is split at arbitrary points.
"""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

P1 = 1073742209            # a 31-bit prime
P2 = 2147483647


@pytest.fixture(scope="module")
def O(oracle_lib):
    return oracle_lib


def int_matrix(n, draw_vals):
    return np.array(draw_vals, dtype=np.int64).reshape(n, n)


@st.composite
def square(draw, lo=1, hi=7, vmax=40):
    n = draw(st.integers(lo, hi))
    vals = draw(st.lists(st.integers(-vmax, vmax), min_size=n * n, max_size=n * n))
    return int_matrix(n, vals)


def res(A, p):
    return np.ascontiguousarray(np.mod(A, p).astype(np.uint32))


@settings(max_examples=60, deadline=None)
@given(A=square(), data=st.data())
def test_permutations_and_transpose(O, A, data):
    n = A.shape[0]
    rp = data.draw(st.permutations(range(n)))
    cp = data.draw(st.permutations(range(n)))
    want = O.native.ryser_modp(res(A, P1), P1)
    assert O.native.ryser_modp(res(A[list(rp)], P1), P1) == want
    assert O.native.ryser_modp(res(A[:, list(cp)], P1), P1) == want
    assert O.native.ryser_modp(res(A.T, P1), P1) == want


@settings(max_examples=60, deadline=None)
@given(A=square(), c=st.integers(-50, 50), data=st.data())
def test_linear_in_each_row(O, A, c, data):
    n = A.shape[0]
    i = data.draw(st.integers(0, n - 1))
    other = data.draw(st.lists(st.integers(-40, 40), min_size=n, max_size=n))
    base = O.native.ryser_modp(res(A, P2), P2)
    S = A.copy()
    S[i] *= c
    assert O.native.ryser_modp(res(S, P2), P2) == (c * base) % P2
    B = A.copy()
    B[i] = other
    AB = A.copy()
    AB[i] = A[i] + np.array(other)
    assert O.native.ryser_modp(res(AB, P2), P2) == \
        (base + O.native.ryser_modp(res(B, P2), P2)) % P2


@settings(max_examples=40, deadline=None)
@given(A=square(hi=4), B=square(hi=4))
def test_block_diagonal_is_the_product(O, A, B):
    a, b = A.shape[0], B.shape[0]
    D = np.zeros((a + b, a + b), dtype=np.int64)
    D[:a, :a] = A
    D[a:, a:] = B
    pa = O.native.ryser_modp(res(A, P1), P1)
    pb = O.native.ryser_modp(res(B, P1), P1)
    assert O.native.ryser_modp(res(D, P1), P1) == (pa * pb) % P1


@settings(max_examples=40, deadline=None)
@given(A=square(hi=8, vmax=9), cuts=st.lists(st.floats(0, 1), max_size=4))
def test_ryser_mod_p_is_the_integer_permanent(O, A, cuts):
    n = A.shape[0]
    exact = O.reference.laplace(A.tolist())
    assert O.native.ryser_modp(res(A, P1), P1) == exact % P1
    end = 1 << n
    pts = sorted({1, end, *(1 + int(f * (end - 1)) for f in cuts)})
    tot = sum(O.native.ryser_modp_range(res(A, P1), P1, x0, x1) for x0, x1 in zip(pts, pts[1:]))
    assert ((P1 - tot % P1) % P1 if n % 2 else tot % P1) == exact % P1
