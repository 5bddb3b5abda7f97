"""GPU parity on streams whose ids all share the same buckets of the block
kernel's hash table.

The block kernel keeps each counter in one of two 8-slot buckets chosen by
hashing the item id (three above k = 1024), with a 64-slot stash for items
whose buckets are full.  Ids picked so that the buckets of every one of them
are the same two (three) overflow them and the stash under the kernel's
first hash functions; the kernel must then run the block again with other
hash functions (the table only indexes the counters, so the summary is the
same).  Expected values come only from the oracle.
"""
import functools
import sys

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

M32 = 0xFFFFFFFF


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def choices(k):
    # buckets per item: three for the LDS classes above k = 1024
    return 3 if 1024 < k <= 4096 else 2


def nbuckets(k):
    # hash slots per counter x16: 30 up to k = 1024, 21 with three choices;
    # at least 256 slots; 8-slot buckets (the block layout's sizing)
    want = max(256, (k * (30 if k <= 1024 else 21) + 15) // 16)
    return (want + 7) // 8


def buckets(x, nb):
    """The two buckets of ids x (numpy uint64 array) under the first
    attempt's hash functions."""
    b1 = (((x * 0x9E3779B1) & M32) * nb) >> 32
    h = (x * 0x85EBCA77) & M32
    h = ((h << 15) | (h >> 17)) & M32
    b2 = (((h * 0xC2B2AE3D) & M32) * nb) >> 32
    b2 = np.where(b2 != b1, b2, np.where(b1 + 1 == nb, 0, b1 + 1))
    return b1, b2


def third(x, nb, b1, b2):
    """The third bucket of ids x under the first attempt's hash functions:
    a third multiplicative hash, stepped past b1 and b2."""
    h = (x * 0x27D4EB2F) & M32
    h = ((h << 9) | (h >> 23)) & M32
    b = (((h * 0xC2B2AE3D) & M32) * nb) >> 32
    for _ in range(2):
        step = (b == b1) | (b == b2)
        b = np.where(step, np.where(b + 1 == nb, 0, b + 1), b)
    return b


@functools.lru_cache(maxsize=None)
def _colliding(k):
    nb = nbuckets(k)
    nch = choices(k)
    out = []
    base = 0
    while len(out) < 400:
        x = np.arange(base, base + (1 << 22), dtype=np.uint64)
        x = x[((((x * 0x9E3779B1) & M32) * nb) >> 32) < nch]  # first bucket, before the others
        b1, b2 = buckets(x, nb)
        sel = (b1 < nch) & (b2 < nch)
        x, b1, b2 = x[sel], b1[sel], b2[sel]
        if nch == 3:
            x = x[third(x, nb, b1, b2) < 3]
        out.extend(x.tolist())
        base += 1 << 22
    return tuple(out[:400])


def colliding_ids(k, count):
    """ids whose buckets are all among the first choices(k) buckets"""
    assert count <= 400
    return np.array(_colliding(k)[:count], dtype=np.uint32)


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


@pytest.mark.parametrize("k", [100, 300, 1500])
def test_colliding_ids_host_check(k):
    # the ids really share their buckets (and there are more of them than
    # those buckets and the stash hold)
    ids = colliding_ids(k, 150).astype(np.uint64)
    nb = nbuckets(k)
    b1, b2 = buckets(ids, nb)
    got = set(np.unique(np.concatenate([b1, b2])).tolist())
    if choices(k) == 3:
        got |= set(np.unique(third(ids, nb, b1, b2)).tolist())
        assert got == {0, 1, 2}
    else:
        assert got == {0, 1}
    assert len(np.unique(ids)) == 150 > 8 * choices(k) + 64


@pytest.mark.parametrize("k,distinct,n,chunks", [(100, 150, 30000, 3), (100, 400, 50000, 1), (300, 400, 60000, 2),
                                                 (1500, 150, 60000, 1), (1500, 300, 90000, 2)])
def test_colliding_ids_equal_oracle(B, ctx, k, distinct, n, chunks):
    ids = colliding_ids(k, distinct)
    rng = np.random.default_rng(k * 1000 + distinct)
    # a round-robin pass (every id live at once), then random draws with a
    # heavy head so that some counts exceed n/k
    rr = np.tile(ids, n // (2 * distinct) + 1)[: n // 2]
    head = ids[rng.zipf(1.3, size=n - n // 2).clip(1, distinct) - 1]
    items = np.concatenate([rr, head]).astype(np.uint32)
    say("colliding ids: k=%d distinct=%d n=%d C=%d" % (k, distinct, n, chunks))
    got, used = B.pss_run(ctx, dev(items), k=k, chunks=chunks)
    assert used == chunks
    assert B.to_tuples(got) == O.to_tuples(O.run(items, k, chunks))
    blocks = B.pss_block_summaries(ctx, dev(items), k, chunks, list(range(chunks)))
    ref = O.chunk_summaries(items, k, chunks)
    for c in range(chunks):
        ent, mn = blocks[c]
        assert sorted(B.to_tuples(ent)) == sorted(O.to_tuples(ref[c].entries)), c
        assert mn == ref[c].m, c
