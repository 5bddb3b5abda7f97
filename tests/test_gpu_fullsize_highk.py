"""GPU parity at the high-k benchmark size, in the launch configuration the
benchmark times: n = 2^31 uint32 items (Zipf 1.1 over 2^32 hashed ids, and
the adversarial round-robin stream with a 5% planted item), k in
{10^4, 5 x 10^4}, the chunk count the planner picks.  Block state, COMBINE
arrays and the report live in device memory at these k.

* sampled blocks (first, last and one seeded random) are compared with the
  oracle's summaries of the same blocks, bit for bit;
* the final summary is checked for properties that hold at any size (counts
  at least errors, counts summing to at most n, minimum at most n / k, the
  majority report equal to the top entries above the threshold) and, on the
  adversarial stream, for the planted item (5% of the stream, far above
  n / k, so every correct summary reports it).
"""
import random
import sys
import zlib

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

N = 1 << 31


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


STREAMS = [("zipf1.1", lambda: W.plain_highk(1, N)), ("adversarial", lambda: W.plain_highk_adversarial(1, N))]


@pytest.mark.parametrize("name,make", STREAMS, ids=[s[0] for s in STREAMS])
def test_high_k_full_size_sampled_blocks_and_invariants(B, ctx, name, make):
    import torch
    items = make().generate()
    d = torch.from_numpy(items.view(np.int32)).to("cuda")
    rng = random.Random(zlib.crc32(name.encode()))
    for k in (10000, 50000):
        C = ctx.plan_chunks(N, k)
        sel = sorted({0, C - 1, rng.randrange(C)})
        say("%s k=%d C=%d blocks %s" % (name, k, C, sel))
        got = B.pss_block_summaries(ctx, d, k, C, sel)
        ref = O.chunk_summaries(items, k, C, which=sel)
        for i, c in enumerate(sel):
            ent, mn = got[i]
            assert sorted(B.to_tuples(ent)) == sorted(O.to_tuples(ref[c].entries)), (name, k, c)
            assert mn == ref[c].m, (name, k, c)
        s = B.Summary(ctx, k)
        used = B.pss_update(s, d, chunks=C)
        assert used == C
        top, n = B.pss_query(s, B.PSS_Q_TOPK, cap=k)
        assert n == N
        cnt = top["count"].astype(np.uint64)
        err = top["error"].astype(np.uint64)
        assert np.all(cnt >= err)
        assert int(cnt.sum()) <= N
        assert len(np.unique(top["item"])) == len(top)
        if len(top) == k:
            assert int(cnt[-1]) <= N // k
        maj, _ = B.pss_query(s, B.PSS_Q_MAJORITY)
        want = [t for t in B.to_tuples(top) if t[1] * k > N]
        assert B.to_tuples(maj) == want
        if name == "adversarial":
            planted = W.adversarial_planted_id(1)
            assert planted in [t[0] for t in want]
        s.close()
    del d
    torch.cuda.empty_cache()
