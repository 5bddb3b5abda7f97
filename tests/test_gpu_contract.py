"""The all-or-nothing contract of updates and merges, on the GPU.

A failed call leaves a summary's entries and its stream length N as they
were: a call that runs out of its context's device-memory budget fails
before queueing anything, and a fold whose block-tree root carries a block
kernel's failure mark (injected through the library's test hook, so that no
kernel is made to fail) leaves the summary untouched on the device and makes
the next query report PSS_EDEVICE once.  Expected values come only from the
oracle.
"""
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


def top(B, s):
    ent, n = B.pss_query(s, B.PSS_Q_TOPK, cap=s.k)
    return B.to_tuples(ent), n


@pytest.mark.parametrize("k", [100, 2000, 6000])
def test_failed_block_fold_leaves_summary_unchanged(B, ctx, k):
    a = W.plain(seed=11, n=1 << 16).generate()
    b = W.plain(seed=12, n=1 << 15).generate()
    say("failed-fold contract k=%d" % k)
    s = B.pss_create(ctx, k)
    ref = O.Summary(k)
    B.pss_update(s, dev(a), chunks=8)
    ref.update(a, 8)
    before = top(B, s)
    assert before == (ref.as_tuples(), len(a))
    B.pss_test_fold_failed_block(s, 12345)
    with pytest.raises(B.PssError) as ei:
        B.pss_query(s, B.PSS_Q_TOPK, cap=k)
    assert ei.value.code == B.PSS_EDEVICE
    # reported once; the summary and N are those before the failed fold
    assert top(B, s) == before
    ent, n = B.pss_query(s, B.PSS_Q_MAJORITY)
    assert n == len(a) and B.to_tuples(ent) == O.to_tuples(ref.query_majority())
    # later updates and merges continue from the unchanged summary
    B.pss_update(s, dev(b), chunks=5)
    ref.update(b, 5)
    assert top(B, s) == (ref.as_tuples(), len(a) + len(b))
    t = B.pss_create(ctx, k)
    B.pss_update(t, dev(a[:1000]), chunks=2)
    B.pss_test_fold_failed_block(t, 777)
    B.pss_merge(s, t)  # t is as before its failed fold
    ref.merge(O.Summary(k).update(a[:1000], 2))
    assert top(B, s) == (ref.as_tuples(), len(a) + len(b) + 1000)
    with pytest.raises(B.PssError):
        B.pss_query(t, B.PSS_Q_TOPK, cap=k)
    t.close()
    s.close()


def test_budget_enomem_leaves_summary_unchanged(B):
    a = W.plain(seed=13, n=1 << 16).generate()
    big = W.plain(seed=14, n=1 << 18).generate()
    k = 300
    c = B.Context(0)
    s = B.pss_create(c, k)
    ref = O.Summary(k)
    B.pss_update(s, dev(a), chunks=4)
    ref.update(a, 4)
    before = top(B, s)
    c.set_budget(1)  # no workspace may grow from here on
    with pytest.raises(B.PssError) as ei:
        B.pss_update(s, dev(big), chunks=256)
    assert ei.value.code == B.PSS_ENOMEM
    assert top(B, s) == before == (ref.as_tuples(), len(a))
    # within the workspace already held, calls still run
    B.pss_update(s, dev(big[:5000]), chunks=4)
    ref.update(big[:5000], 4)
    assert top(B, s) == (ref.as_tuples(), len(a) + 5000)
    c.set_budget(0)
    B.pss_update(s, dev(big), chunks=256)
    ref.update(big, 256)
    assert top(B, s) == (ref.as_tuples(), len(a) + 5000 + len(big))
    s.close()
    c.close()


def test_merge_adds_stream_lengths_on_device(B, ctx):
    k = 50
    x = W.plain(seed=15, n=30000).generate()
    s, t = B.pss_create(ctx, k), B.pss_create(ctx, k)
    B.pss_update(s, dev(x[:10000]), chunks=3)
    B.pss_update(t, dev(x[10000:]), chunks=6)
    B.pss_merge(s, t)  # queued behind both updates; N(t) is read on the device
    B.pss_merge(s, t)
    ref = O.Summary(k).update(x[:10000], 3)
    rt = O.Summary(k).update(x[10000:], 6)
    ref.merge(rt)
    ref.merge(rt)
    assert top(B, s) == (ref.as_tuples(), 10000 + 2 * 20000)
    s.close()
    t.close()
