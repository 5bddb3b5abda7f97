"""GPU parity at full size, in the launch configuration the benchmark times.

The plain-large streams (n = 2^30 uint32 items; Zipf 0.8, 1.2, 1.8 over 2^32
hashed ids and a uniform control) with k in {500, 2000} and the chunk count
the planner picks.  The oracle cannot afford all of them, so:

* sampled blocks (first, middle, last, and one seeded random) of every case
  are compared with the oracle's summaries of the same blocks, bit for bit;
* every case's final summary is checked for properties that hold at any
  size (counts at least errors, counts summing to at most n, minimum at most
  n / k, the majority report equal to the top entries above the threshold);
* three cases (Zipf 1.2 with k = 500; Zipf 0.8 and Zipf 1.8 with k = 2000)
  are compared with the oracle end to end; the oracle's chunk summaries run
  on several host threads (the same sequential function per chunk), its tree
  on one.
"""
import os
import random
import sys
import zlib

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

N = 1 << 30


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


STREAMS = [("zipf0.8", lambda: W.plain_large(0.8, 1, N)), ("zipf1.2", lambda: W.plain_large(1.2, 1, N)),
           ("zipf1.8", lambda: W.plain_large(1.8, 1, N)), ("uniform", lambda: W.plain_large_uniform(1, N))]


@pytest.mark.parametrize("name,make", STREAMS, ids=[s[0] for s in STREAMS])
def test_full_size_sampled_blocks_and_invariants(B, ctx, name, make):
    import torch
    items = make().generate()
    d = torch.from_numpy(items.view(np.int32)).to("cuda")
    rng = random.Random(zlib.crc32(name.encode()))
    for k in (500, 2000):
        C = ctx.plan_chunks(N, k)
        sel = sorted({0, C // 2, C - 1, rng.randrange(C)})
        say("%s k=%d C=%d blocks %s" % (name, k, C, sel))
        got = B.pss_block_summaries(ctx, d, k, C, sel)
        ref = O.chunk_summaries(items, k, C, which=sel)
        for i, c in enumerate(sel):
            ent, mn = got[i]
            assert sorted(B.to_tuples(ent)) == sorted(O.to_tuples(ref[c].entries)), (name, k, c)
            assert mn == ref[c].m, (name, k, c)
        # the whole path at this size: invariants of the final summary
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
            assert int(cnt[-1]) <= N // k  # the minimum of a full summary
        maj, _ = B.pss_query(s, B.PSS_Q_MAJORITY)
        want = [t for t in B.to_tuples(top) if t[1] * k > N]
        assert B.to_tuples(maj) == want
        s.close()
    del d
    torch.cuda.empty_cache()


THREADS = max(1, min(16, os.cpu_count() or 1))


@pytest.mark.parametrize("alpha,k", [(1.2, 500), (0.8, 2000), (1.8, 2000)])
def test_full_size_end_to_end_against_the_oracle(B, ctx, alpha, k):
    import torch
    items = W.plain_large(alpha, 1, N).generate()
    d = torch.from_numpy(items.view(np.int32)).to("cuda")
    C = ctx.plan_chunks(N, k)
    say("zipf%.1f k=%d C=%d: GPU" % (alpha, k, C))
    got, used = B.pss_run(ctx, d, k=k, chunks=C)
    assert used == C
    say("oracle over 2^30 items on %d threads" % THREADS)
    want = O.run_threads(items, k, C, THREADS)
    assert B.to_tuples(got) == O.to_tuples(want)
    assert len(want) >= 1
    del d
    torch.cuda.empty_cache()
