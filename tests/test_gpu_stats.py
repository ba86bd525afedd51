"""Batched Haar permanents at the paper's sizes (50,000 samples per odd n in
7..23): an exact second moment, circular symmetry, and the paper's table of
Var perm(O) and excess kurtosis within sampling error; oracle parity on a
subset of each batch."""
import math

import numpy as np
import pytest
from conftest import golden

from paper_2602_10141_amd import ensembles as E

pytestmark = pytest.mark.gpu
COUNT = 50000


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


def batch(P, ctx, M, field):
    items, data = P.pack_matrices([(m, field, 0) for m in M])
    return np.asarray(P.batch_values(items, P.perm_batch(ctx, items, data)))


def jackknife(x, stat, blocks=50):
    """Statistic of x and its delete-one-block jackknife standard error."""
    b = np.array_split(x, blocks)
    loo = np.array([stat(np.concatenate(b[:i] + b[i + 1:])) for i in range(blocks)])
    return float(stat(x)), float(math.sqrt((blocks - 1) / blocks * ((loo - loo.mean()) ** 2).sum()))


TABLE = {int(r[0]): (float(r[1]), float(r[2])) for r in golden("orthogonal_table.txt")}


@pytest.mark.parametrize("n", [7, 11, 13, 17, 19, 23])
def test_haar_unitary_second_moment_and_symmetry(P, ctx, oracle_lib, n):
    U = E.haar_unitary(n, E.rng(40, n), count=COUNT)
    v = batch(P, ctx, U, "c128")
    a2 = np.abs(v) ** 2
    # E|perm U|^2 = 1/binom(2n-1, n): perm U is the matrix element of the
    # n-th symmetric power of U between the one-particle-per-mode state and
    # itself, and that representation is irreducible of dimension
    # binom(2n-1, n) (Schur orthogonality).
    exact = 1.0 / math.comb(2 * n - 1, n)
    z = (a2.mean() - exact) / (a2.std(ddof=1) / math.sqrt(COUNT))
    assert abs(z) < 5, (a2.mean(), exact, z)
    assert 0.95 < v.real.std() / v.imag.std() < 1.05
    assert abs(np.corrcoef(v.real, v.imag)[0, 1]) < 0.03
    assert abs(v.mean()) < 5 * math.sqrt(exact / COUNT)
    if n <= 19:
        for i in range(0, COUNT, COUNT // 40):
            want = oracle_lib.native.ryser_c128(U[i])
            assert abs(v[i] - want) <= 1e-10 * float(np.prod(np.linalg.norm(U[i], axis=1)))


@pytest.mark.parametrize("n", [7, 11, 13, 17, 19])
def test_haar_orthogonal_matches_paper_table(P, ctx, oracle_lib, n):
    O = E.haar_orthogonal(n, E.rng(41, n), count=COUNT)
    v = batch(P, ctx, O, "f64")
    assert np.all(np.abs(v.imag) == 0)
    v = v.real
    var_t, kurt_t = TABLE[n]
    var, se_var = jackknife(v, lambda x: x.var(ddof=1))
    kurt, se_kurt = jackknife(v, lambda x: ((x - x.mean()) ** 4).mean() / x.var() ** 2 - 3)
    # the table's values are 50,000-sample estimates as well: their standard
    # errors are taken equal to ours (hence sqrt 2), plus rounding to 3 digits
    assert abs(var - var_t) < 5 * math.sqrt(2) * se_var + 0.005 * var_t, (var, var_t, se_var)
    assert abs(kurt - kurt_t) < 5 * math.sqrt(2) * se_kurt + 0.0005, (kurt, kurt_t, se_kurt)
    assert abs(v.mean()) < 5 * math.sqrt(var / COUNT)
    for i in range(0, COUNT, COUNT // 40):
        want = oracle_lib.native.ryser_f64(O[i])
        assert abs(v[i] - want) <= 1e-10 * float(np.prod(np.linalg.norm(O[i], axis=1)))
