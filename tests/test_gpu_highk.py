"""GPU parity for k beyond LDS, bit-exact against the oracle.

Above the largest k whose block state fits one workgroup's LDS, the block
kernel keeps its hash, counters and minimum-level list in a device-memory slab
per block; COMBINE and the report switch to device-memory scratch at their own
limits.  The method (Section 3, Algorithms 1 and 2) is unchanged, so every
result must equal the oracle's exactly, on both sides of each limit.
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


def whole(B, ctx, items, k, C):
    s = B.Summary(ctx, k)
    B.pss_update(s, dev(items), chunks=C)
    ent, n = B.pss_query(s, B.PSS_Q_TOPK, cap=k)
    s.close()
    return B.to_tuples(ent), n


def test_limits(ctx):
    say("max_k", ctx.max_k, "max_lds_k", ctx.max_lds_k)
    assert ctx.max_k == 1 << 20
    assert 2000 <= ctx.max_lds_k < 10000


def test_both_sides_of_the_lds_limit(B, ctx):
    items = W.zipf_hashed(1 << 20, 1.1, 1 << 32, seed=5)
    kl = ctx.max_lds_k
    for k in (kl, kl + 1):
        say("lds limit k=%d C=3" % k)
        got, n = whole(B, ctx, items, k, 3)
        assert n == len(items)
        assert got == O.summary(items, k, 3).as_tuples(), k


def test_combine_scratch_between_limits(B, ctx):
    # k=4000: block state in LDS, COMBINE arrays in device memory;
    # k=6000: block state and COMBINE in device memory; the report in LDS
    items = W.zipf_hashed(1 << 21, 0.9, 1 << 32, seed=6)
    for k, C in [(4000, 9), (6000, 5)]:
        say("mid k=%d C=%d" % (k, C))
        got, _ = whole(B, ctx, items, k, C)
        assert got == O.summary(items, k, C).as_tuples(), k


def test_high_k_block_summaries(B, ctx):
    items = W.zipf_hashed(1 << 22, 1.1, 1 << 32, seed=11)
    for k, C in [(10000, 4), (50000, 3)]:
        say("blocks k=%d C=%d" % (k, C))
        blocks = B.pss_block_summaries(ctx, dev(items), k, C, list(range(C)))
        ref = O.chunk_summaries(items, k, C)
        for c in range(C):
            ent, mn = blocks[c]
            assert sorted(B.to_tuples(ent)) == sorted(O.to_tuples(ref[c].entries)), (k, c)
            assert mn == ref[c].m, (k, c)


def test_high_k_summary_and_report(B, ctx):
    items = W.zipf_hashed(1 << 22, 1.1, 1 << 32, seed=12)
    for k, C in [(10000, 16), (50000, 5)]:
        say("high-k summary k=%d C=%d" % (k, C))
        got, n = whole(B, ctx, items, k, C)
        assert n == len(items)
        assert got == O.summary(items, k, C).as_tuples(), k
        rep, used = B.pss_run(ctx, dev(items), k=k, chunks=C)
        assert used == C
        want = O.run(items, k, C)
        assert B.to_tuples(rep) == O.to_tuples(want), k
        assert len(want) > 100


def test_high_k_adversarial_planted_item(B, ctx):
    # round-robin distinct ids with a 5% planted item: every window evicts
    seed = 2
    items = W.adversarial(1 << 22, seed)
    planted = W.adversarial_planted_id(seed)
    for k, C in [(10000, 8), (50000, 2)]:
        say("adversarial k=%d C=%d" % (k, C))
        rep, _ = B.pss_run(ctx, dev(items), k=k, chunks=C)
        want = O.run(items, k, C)
        assert B.to_tuples(rep) == O.to_tuples(want), k
        assert planted in [int(e["item"]) for e in want]


def test_high_k_update_merge(B, ctx):
    k = 12000
    a = W.zipf_hashed(300000, 1.2, 1 << 32, seed=21)
    b = W.zipf_hashed(500000, 0.9, 1 << 32, seed=22)
    s, t = B.Summary(ctx, k), B.Summary(ctx, k)
    rs, rt = O.Summary(k), O.Summary(k)
    B.pss_update(s, dev(a), chunks=3)
    rs.update(a, 3)
    B.pss_update(t, dev(b), chunks=6)
    rt.update(b, 6)
    B.pss_update(s, dev(b[:70001]), chunks=2)
    rs.update(b[:70001], 2)
    B.pss_merge(s, t)
    rs.merge(rt)
    got, n = B.pss_query(s, B.PSS_Q_TOPK, cap=k)
    assert n == rs.n
    assert B.to_tuples(got) == rs.as_tuples()
    got, _ = B.pss_query(s, B.PSS_Q_MAJORITY)
    assert B.to_tuples(got) == O.to_tuples(rs.query_majority())
    s.close()
    t.close()


def test_high_k_combine_levels_reuse_scratch_slabs(B, ctx):
    # k = 10^4 COMBINEs do not fit LDS: each tree level runs at most two
    # workgroups per CU, each reusing one scratch slab for several pairs.
    # 1200 blocks give 600 pairs at the first level, more than the slabs.
    import os
    items = W.zipf_hashed(1 << 24, 1.1, 1 << 32, seed=31)
    k, C = 10000, 1200
    say("high-k tree with slab reuse: k=%d C=%d" % (k, C))
    got, n = whole(B, ctx, items, k, C)
    assert n == len(items)
    threads = max(1, min(16, os.cpu_count() or 1))
    assert got == O.summary_threads(items, k, C, threads).as_tuples()
    rep, used = B.pss_run(ctx, dev(items), k=k, chunks=C)
    assert used == C
    assert B.to_tuples(rep) == O.to_tuples(O.run_threads(items, k, C, threads))
