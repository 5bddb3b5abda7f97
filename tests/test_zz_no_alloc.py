"""pss_run_noalloc (no allocation, workspace in one fixed device array per
GPU) against pss_run with the same C, on the GPU: two calls in a row, the
second with a smaller input, both equal to pss_run's results; plus the
oracle on a small case and the size limits."""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1606_04669_amd import binding
    return binding


@pytest.fixture(scope="module")
def ctx(B):
    c = B.Context(0)
    yield c
    c.close()


def dev(items):
    import torch
    a = np.ascontiguousarray(np.asarray(items, dtype=np.uint32))
    return torch.from_numpy(a.view(np.int32)).to("cuda")


def noalloc(B, d, k, chunks, cap):
    import torch
    out = torch.zeros(cap * 24, dtype=torch.uint8, device="cuda")
    nout = torch.zeros(1, dtype=torch.int32, device="cuda")
    used = B.pss_run_noalloc(d, k, out, nout, chunks=chunks)
    torch.cuda.synchronize()
    q = int(nout.cpu().numpy().view(np.uint32)[0])
    assert q != 0xFFFFFFFF, "a block failed"
    return B.entries_from_bytes(out.cpu().numpy(), min(q, cap)), q, used


@pytest.mark.parametrize("k,n1,n2,chunks", [(100, 1 << 22, 1 << 18, 0), (2000, 1 << 22, 300000, 0),
                                            (500, 1 << 21, 70001, 37), (4000, 1 << 21, 50000, 9)])
def test_noalloc_equals_pss_run_twice(B, ctx, k, n1, n2, chunks):
    a = W.plain_large(1.2, 7, n1).generate()
    b = W.plain_large(0.8, 8, n2).generate()
    for items in (a, b):
        d = dev(items)
        say("noalloc k=%d n=%d chunks=%d" % (k, len(items), chunks))
        got, q, used = noalloc(B, d, k, chunks, k)
        want, used2 = B.pss_run(ctx, d, k=k, chunks=used)
        assert used2 == used and (chunks == 0 or used == chunks)
        assert q == len(want)
        assert B.to_tuples(got) == B.to_tuples(want)


def test_noalloc_equals_oracle_and_truncates(B):
    items = W.plain(seed=5).generate()
    d = dev(items)
    got, q, used = noalloc(B, d, 100, 64, 100)
    want = O.run(items, 100, 64)
    assert used == 64 and B.to_tuples(got) == O.to_tuples(want)
    got3, q3, _ = noalloc(B, d, 100, 64, 3)  # only cap entries are written; q is the full count
    assert q3 == len(want) and B.to_tuples(got3) == O.to_tuples(want[:3])


def test_noalloc_limits(B):
    import torch
    d = dev(np.arange(1000, dtype=np.uint32))
    out = torch.zeros(24 * 10, dtype=torch.uint8, device="cuda")
    nout = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(B.PssError) as e:
        B.pss_run_noalloc(d, 1001, out, nout)  # k > n
    assert e.value.code == B.PSS_ERANGE
    with pytest.raises(B.PssError) as e:
        B.pss_run_noalloc(d, 50, out, nout, chunks=1 << 21)  # workspace beyond the array
    assert e.value.code == B.PSS_ERANGE
    assert B.noalloc_scratch_bytes() == 128 << 20
