"""Checkpointed CRT jobs: the result equals perm_crt_int's and the oracle's,
does not depend on the piece size, and a run resumed from a truncated (even
torn) checkpoint gives the same bits; foreign or corrupt checkpoints are
refused."""
import math

import numpy as np
import pytest

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


def schur(P, n, extra=0):
    primes = P.perm_schur_primes(n, extra=extra)
    return np.stack([P.perm_schur_residues(n, p) for p in primes]), primes, (n / 2) * math.log2(n)


def test_job_matches_oracle(P, ctx, oracle_lib):
    n = 19
    mats, primes, bound = schur(P, n)
    with P.Job(ctx, mats, primes, bound, piece_log2=12) as job:
        done, total = job.run()
        assert done == total == len(primes) * (1 << (n - 1 - 12))
        val, res = job.result()
    want = [oracle_lib.native.ryser_modp(m, p) for m, p in zip(mats, primes)]
    assert res == want
    assert val == oracle_lib.crt.crt_lift(want, primes)


@pytest.mark.parametrize("piece_log2", [10, 17, 24, 26])
def test_piece_size_does_not_matter(P, ctx, piece_log2):
    n = 27
    mats, primes, bound = schur(P, n, extra=1)
    want = P.perm_crt_int(ctx, mats, primes, bound)
    with P.Job(ctx, mats, primes, bound, piece_log2=piece_log2) as job:
        job.run()
        assert job.result() == want


def test_resume_from_truncated_checkpoint(P, ctx, tmp_path):
    n = 25
    mats, primes, bound = schur(P, n, extra=1)
    path = tmp_path / "s25.ckpt"
    with P.Job(ctx, mats, primes, bound, piece_log2=18, checkpoint=path) as job:
        job.run()
        want = job.result()
    lines = path.read_text().splitlines(keepends=True)
    header, body = lines[0], lines[1:]
    assert len(body) == len(primes) * (1 << (n - 1 - 18))
    cut = tmp_path / "cut.ckpt"
    # a third of the pieces, then a line torn in the middle of a write
    cut.write_text(header + "".join(body[: len(body) // 3]) + body[len(body) // 3][:3])
    with P.Job(ctx, mats, primes, bound, piece_log2=18, checkpoint=cut) as job:
        with pytest.raises(P.PermError) as e:
            job.result()
        assert e.value.status == P.PERM_EAGAIN
        done, total = job.run(seconds=0)        # one batch
        assert done == total
        assert job.result() == want
    # the resumed file is complete again: a third job only reads it
    with P.Job(ctx, mats, primes, bound, piece_log2=18, checkpoint=cut) as job:
        assert job.result() == want


def test_foreign_or_corrupt_checkpoint_refused(P, ctx, tmp_path):
    n = 21
    mats, primes, bound = schur(P, n, extra=1)
    path = tmp_path / "a.ckpt"
    with P.Job(ctx, mats, primes, bound, piece_log2=14, checkpoint=path) as job:
        job.run()
    # other primes, other piece size: not this job's file
    mats2, primes2, _ = schur(P, n, extra=2)
    for args in ((mats2, primes2, bound, 14), (mats, primes, bound, 15)):
        with pytest.raises(P.PermError) as e:
            P.Job(ctx, *args[:3], piece_log2=args[3], checkpoint=path)
        assert e.value.status == P.PERM_EINVAL
    lines = path.read_text().splitlines(keepends=True)
    i, j, v = lines[1].split()
    bad_value = lines + [f"{i} {j} {(int(v) + 1) % primes[int(i)]}\n"]
    bad_index = lines + [f"{len(primes)} 0 1\n"]
    for k, body in enumerate((bad_value, bad_index)):
        f = tmp_path / f"bad{k}.ckpt"
        f.write_text("".join(body))
        with pytest.raises(P.PermError) as e:
            P.Job(ctx, mats, primes, bound, piece_log2=14, checkpoint=f)
        assert e.value.status == P.PERM_EINVAL


def test_job_argument_errors(P, ctx):
    mats, primes, bound = schur(P, 15)
    with pytest.raises(P.PermError):
        P.Job(ctx, mats, primes, bound, piece_log2=9)          # below 10
    with pytest.raises(P.PermError):
        P.Job(ctx, mats, primes, bound, piece_log2=15)         # above n - 1
    with pytest.raises(ValueError):
        P.Job(ctx, mats, primes[:1], bound)                   # k != number of matrices
    with pytest.raises(P.PermError) as e:
        P.Job(ctx, mats[:1], primes[:1], bound)               # one prime is not enough
    assert e.value.status == P.PERM_ERANGE
