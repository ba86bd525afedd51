"""DFT geodesic gamma(t) = exp(t log F_n) (paper Sec. 4.2) through the
batched c128 path: oracle parity along the path for both logarithms of -1,
and the recovery ratio r(n) = |perm F_n| / min_t |perm gamma(t)| equal to
the oracle's."""
import numpy as np
import pytest

from paper_2602_10141_amd import ensembles as E

pytestmark = pytest.mark.gpu
GRID = np.linspace(0.0, 1.0, 129)


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


def path(P, ctx, n, branch):
    mats = [E.dft_geodesic(n, t, branch) for t in GRID]
    items, data = P.pack_matrices([(m, "c128", 0) for m in mats])
    return mats, np.asarray(P.batch_values(items, P.perm_batch(ctx, items, data)))


@pytest.mark.parametrize("n", [7, 9, 11, 13])
@pytest.mark.parametrize("branch", [1, -1])
def test_dft_path_matches_oracle(P, ctx, oracle_lib, n, branch):
    mats, got = path(P, ctx, n, branch)
    want = np.array([oracle_lib.native.ryser_c128(m) for m in mats])
    # unitary matrices: prod of row norms is 1
    assert np.max(np.abs(got - want)) <= 1e-10
    assert abs(got[0] - 1) < 1e-13
    assert np.all(np.abs(got) <= 1 + 1e-12)
    r_gpu = abs(got[-1]) / np.abs(got).min()
    r_cpu = abs(want[-1]) / np.abs(want).min()
    assert abs(r_gpu / r_cpu - 1) < 1e-6
