"""Stream ordering of device-pointer calls made without an explicit stream.

The binding then passes PyTorch's current stream; on PyTorch's default stream
that is HIP's null stream, and the library runs there.  So a matrix written by
PyTorch work queued earlier on that stream, and a result read by PyTorch work
queued later, need no synchronisation in between.  The inputs here are written
only after tens of milliseconds of other work, so a call that did not wait for
them would read stale memory and fail the bit comparison with the synchronous
host-buffer call of the same matrix (same partition, same kernels)."""
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


def _busy(torch):
    """A chain of dependent 2048^3 products on the current stream."""
    x = torch.randn(2048, 2048, device="cuda", dtype=torch.float32)
    for _ in range(24):
        x = torch.tanh(x @ x * (1.0 / 48))
    return x


def _late_copy(torch, src):
    """src's values in a new tensor written only after the busy work."""
    x = _busy(torch)
    d = torch.zeros_like(src)
    d.add_(src)
    return d, x


def test_single_and_noalloc_ordered_with_default_stream(P, ctx):
    import torch
    A = E.haar_unitary(16, E.rng(41, 0))
    want = P.perm_c128(ctx, A)
    src = torch.from_numpy(A).cuda()
    torch.cuda.synchronize()
    for _ in range(3):
        dA, _x = _late_copy(torch, src)
        out = P.perm_c128(ctx, dA)
        got = (out * 1.0).cpu().numpy()             # a PyTorch op on the result first
        assert got[0] == want.real and got[1] == want.imag
        dB, _y = _late_copy(torch, src)
        out2 = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
        P.perm_c128_noalloc(ctx, dB, out=out2)
        got2 = out2.cpu().numpy()
        assert got2[0] == want.real and got2[1] == want.imag


def test_batch_ordered_with_default_stream(P, ctx):
    import torch
    U = E.haar_unitary(15, E.rng(41, 1), count=64)
    R = [E.random_residues(13, 1073742209, E.rng(41, 2 + i)) for i in range(8)]
    mats = [(m, "c128", 0) for m in U] + [(r, "modp", 1073742209) for r in R]
    items, data = P.pack_matrices(mats)
    want = P.perm_batch(ctx, items, data)
    src = torch.from_numpy(data).cuda()
    torch.cuda.synchronize()
    for _ in range(3):
        d, _x = _late_copy(torch, src)
        out = P.perm_batch(ctx, items, d)
        assert np.array_equal(out.cpu().numpy(), want)


def test_events_on_default_stream_bracket_the_walk(P, ctx):
    """PyTorch events recorded around a call on the default stream measure at
    least the walk kernels the library timed inside them."""
    import torch
    U = E.haar_unitary(18, E.rng(41, 3), count=512)
    items, data = P.pack_matrices([(m, "c128", 0) for m in U])
    d = torch.from_numpy(data).cuda()
    res = torch.zeros((len(U), 2), dtype=torch.float64, device="cuda")
    P.perm_batch(ctx, items, d, out=res)
    torch.cuda.synchronize()
    P.perm_prof_enable(ctx, True)
    try:
        P.perm_prof_read(ctx)
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        evs[0].record()
        for e in evs[1:]:
            P.perm_batch(ctx, items, d, out=res)
            e.record()
        torch.cuda.synchronize()
        walk_ms, launches = P.perm_prof_read(ctx)
    finally:
        P.perm_prof_enable(ctx, False)
    spans = [evs[i].elapsed_time(evs[i + 1]) for i in range(3)]
    assert launches >= 3
    assert sum(spans) >= 0.99 * walk_ms, (spans, walk_ms)
    assert min(spans) >= 0.99 * walk_ms / launches * 0.5, (spans, walk_ms, launches)
