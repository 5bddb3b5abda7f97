"""GPU parity on streams whose ids all share one bucket pair of the block
kernel's hash table.

The block kernel keeps each counter in one of two 8-slot buckets chosen by
hashing the item id, with a 64-slot stash for items whose buckets are full.
Ids picked so that both buckets of every one of them are the same pair
overflow that pair and the stash under the kernel's first hash functions;
the kernel must then run the block again with other hash functions (the
table only indexes the counters, so the summary is the same).  Expected
values come only from the oracle.
"""
import sys

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

M32 = 0xFFFFFFFF


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def nbuckets(k):
    # hash slots per counter x16: 32 up to k = 1024, 26 above; at least 256
    # slots; 8-slot buckets (the block layout's sizing)
    want = max(256, (k * (32 if k <= 1024 else 26) + 15) // 16)
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


def colliding_ids(k, count, pair=(0, 1)):
    nb = nbuckets(k)
    out = []
    base = 0
    while len(out) < count:
        x = np.arange(base, base + (1 << 22), dtype=np.uint64)
        b1, b2 = buckets(x, nb)
        sel = ((b1 == pair[0]) & (b2 == pair[1])) | ((b1 == pair[1]) & (b2 == pair[0]))
        out.extend(x[sel].tolist())
        base += 1 << 22
    return np.array(out[:count], dtype=np.uint32)


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


def test_colliding_ids_host_check():
    # the ids really share one pair (and there are more than 16 + 64 of them)
    ids = colliding_ids(100, 150)
    b1, b2 = buckets(ids.astype(np.uint64), nbuckets(100))
    assert set(np.unique(np.concatenate([b1, b2])).tolist()) == {0, 1}
    assert len(np.unique(ids)) == 150


@pytest.mark.parametrize("k,distinct,n,chunks", [(100, 150, 30000, 3), (100, 400, 50000, 1), (300, 400, 60000, 2)])
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
