"""perm_c128_noalloc, the entry point that allocates nothing, against
perm_c128 through the C ABI: same bits (same partition and kernels), and the
oracle within 1e-10 * prod_i ||row_i||_2 where it finishes in seconds.  Two
calls in a row on one stream share the static scratch, the second with a
smaller matrix; sizes beyond the scratch are rejected with an error."""
import ctypes

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


def scale(A):
    return float(np.prod(np.linalg.norm(A, axis=1))) if len(A) else 1.0


def noalloc(P, ctx, dA, out):
    L = P.lib()
    return L.perm_c128_noalloc(ctx.ptr, ctypes.c_void_p(dA.data_ptr()), dA.shape[0],
                               ctypes.c_void_p(out.data_ptr()), P.PERM_DEVICE_PTRS,
                               P._stream(None))


@pytest.mark.parametrize("first,second", [(24, 14), (32, 20), (21, 12), (12, 0), (5, 1)])
def test_two_calls_match_perm_c128(P, ctx, oracle_lib, first, second):
    import torch
    print(f"noalloc n={first} then n={second}", flush=True)
    mats = [E.haar_unitary(n, E.rng(70, n)) if n else np.zeros((0, 0), complex)
            for n in (first, second)]
    dev = [torch.from_numpy(A).cuda() for A in mats]
    outs = [torch.full((2,), -7.0, dtype=torch.float64, device="cuda") for _ in mats]
    for d, o in zip(dev, outs):            # back to back on one stream, no sync between
        assert noalloc(P, ctx, d, o) == P.PERM_OK, P.perm_last_error()
    torch.cuda.synchronize()
    for A, d, o in zip(mats, dev, outs):
        got = o.cpu().numpy()
        ref = P.perm_c128(ctx, d)
        torch.cuda.synchronize()
        assert np.array_equal(got, ref.cpu().numpy()), (A.shape, got, ref)
        n = A.shape[0]
        if n <= 24:
            want = oracle_lib.native.ryser_c128(A) if n else 1.0
            assert abs(complex(got[0], got[1]) - want) <= TOL * scale(A)


def test_binding_and_kahan_flag(P, ctx):
    import torch
    A = torch.from_numpy(E.ginibre_complex(18, E.rng(71, 0))).cuda()
    for flags in (0, P.PERM_NO_KAHAN):
        a = P.perm_c128_noalloc(ctx, A, flags=flags)
        b = P.perm_c128(ctx, A, flags=flags)
        torch.cuda.synchronize()
        assert torch.equal(a, b)


def test_rejects_what_does_not_fit(P, ctx):
    import torch
    L = P.lib()
    A = E.ginibre_complex(8, E.rng(72, 0))
    h = np.ascontiguousarray(A)
    out = np.zeros(2)
    # host pointers
    assert L.perm_c128_noalloc(ctx.ptr, h.ctypes.data, 8, out.ctypes.data, 0, None) == P.PERM_EINVAL
    # order above the static scratch's limit
    d33 = torch.zeros((33, 33), dtype=torch.complex128, device="cuda")
    o = torch.zeros(2, dtype=torch.float64, device="cuda")
    assert noalloc(P, ctx, d33, o) == P.PERM_EINVAL
    assert "outside [0, 32]" in P.perm_last_error()
    # a tuning entry whose partition has more wave items than the scratch holds
    P.perm_tune_set(ctx, "c128", 30, 3)
    try:
        d30 = torch.from_numpy(E.ginibre_complex(30, E.rng(72, 1))).cuda()
        assert noalloc(P, ctx, d30, o) == P.PERM_ENOMEM
        assert "static scratch" in P.perm_last_error()
    finally:
        P.perm_tune_set(ctx, "c128", 30, 0)
    torch.cuda.synchronize()
