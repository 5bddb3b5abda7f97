"""GPU parity of the Frequent (Misra-Gries) path against its oracle,
bit-exact: block summaries (entries and D), the merged summary, the report,
on the hand-worked examples, seeded Zipf, uniform and adversarial streams,
random small cases with ragged blocks and C > n, ids that overflow their
buckets (two or three per item), and full size with the planner's C."""
import json
import os
import random
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


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


def pairs(entries):
    return [(int(e["item"]), int(e["count"])) for e in entries]


def check_all(B, ctx, items, k, C):
    d = dev(items)
    blocks = B.pss_frequent_block_summaries(ctx, d, k, C, list(range(C)))
    ref = O.frequent_chunk_summaries(items, k, C)
    for c in range(C):
        ent, dc = blocks[c]
        assert sorted(pairs(ent)) == sorted(pairs(ref[c].entries)), (k, C, c)
        assert dc == ref[c].d, (k, C, c)
    whole, dd, used = B.pss_frequent_run(ctx, d, k=k, chunks=C, kind=B.PSS_Q_TOPK, cap=k)
    want = O.frequent_summary(items, k, C)
    assert used == C
    assert pairs(whole) == want.as_pairs() and dd == want.d, (k, C)
    rep, dr, _ = B.pss_frequent_run(ctx, d, k=k, chunks=C)
    assert pairs(rep) == pairs(O.frequent_run(items, k, C)) and dr == want.d, (k, C)


def test_limits(B, ctx):
    say("frequent_max_k", ctx.frequent_max_k)
    assert ctx.frequent_max_k >= 4096
    with pytest.raises(B.PssError) as e:
        B.pss_frequent_run(ctx, dev(np.arange(100, dtype=np.uint32)), k=ctx.frequent_max_k + 1)
    assert e.value.code == B.PSS_ERANGE


def test_worked_examples(B, ctx):
    for case in json.load(open(os.path.join(HERE, "golden", "frequent_examples.json")))["cases"]:
        items = np.array(case["items"], dtype=np.uint32)
        whole, d, _ = B.pss_frequent_run(ctx, dev(items), k=case["k"], chunks=case["chunks"], kind=B.PSS_Q_TOPK)
        assert pairs(whole) == [tuple(x) for x in case["summary"]], case["name"]
        assert d == case["d"], case["name"]
        rep, _, _ = B.pss_frequent_run(ctx, dev(items), k=case["k"], chunks=case["chunks"])
        assert pairs(rep) == [tuple(x) for x in case["reported"]], case["name"]


def test_zipf_uniform_adversarial(B, ctx):
    streams = [("plain", W.plain(seed=4, n=1 << 20).generate()),
               ("zipf0.9", W.zipf_hashed(1 << 20, 0.9, 1 << 32, seed=5)),
               ("uniform", W.uniform(1 << 20, 6)),
               ("adversarial", W.adversarial(1 << 20, 7, d=1 << 14))]
    for name, items in streams:
        for k, C in [(2, 16), (100, 64), (500, 7), (2000, 33), (4096, 3)]:
            say("frequent %s k=%d C=%d" % (name, k, C))
            check_all(B, ctx, items, k, C)


def test_random_small_cases(B, ctx):
    rng = random.Random(2024)
    for t in range(60):
        n = rng.randrange(2, 20000)
        univ = rng.choice([3, 50, 1000, 1 << 32])
        items = np.array([rng.randrange(univ) for _ in range(n)], dtype=np.uint32)
        if rng.random() < 0.3:
            items[rng.randrange(n)] = 0xFFFFFFFF
        k = rng.randrange(2, min(n, 3000) + 1)
        C = rng.choice([1, 2, 5, 64, n + 3])
        check_all(B, ctx, items, k, C)


@pytest.mark.parametrize("k,distinct,chunks", [(100, 300, 3), (1500, 60, 2), (1500, 300, 1)])
def test_colliding_ids(B, ctx, k, distinct, chunks):
    # ids whose buckets are all among the first two (k = 100) or three
    # (k = 1500) of the table: they fill them and the stash, and past that the
    # block retries under other hash functions
    from test_gpu_collisions import colliding_ids
    ids = colliding_ids(k, distinct)
    rng = np.random.default_rng(3)
    items = np.concatenate([np.tile(ids, 40), ids[rng.zipf(1.3, 20000).clip(1, distinct) - 1]]).astype(np.uint32)
    say("frequent colliding ids k=%d distinct=%d n=%d" % (k, distinct, len(items)))
    check_all(B, ctx, items, k, chunks)


def test_planted_majority_k2(B, ctx):
    items = W.uniform(300001, 8)
    items[::2] = 1234567  # 150001 of 300001: a strict majority
    rep, d, _ = B.pss_frequent_run(ctx, dev(items), k=2, chunks=8)
    assert pairs(rep) == pairs(O.frequent_run(items, 2, 8))
    assert [p[0] for p in pairs(rep)] == [1234567]


def test_full_size_end_to_end(B, ctx):
    import torch
    n = 1 << 30
    items = W.plain_large(1.1, 1, n).generate()
    d = torch.from_numpy(items.view(np.int32)).to("cuda")
    threads = max(1, min(16, os.cpu_count() or 1))
    for k in (500, 2000):
        C = ctx.frequent_plan_chunks(n, k)
        say("frequent full size k=%d C=%d" % (k, C))
        whole, dd, used = B.pss_frequent_run(ctx, d, k=k, chunks=C, kind=B.PSS_Q_TOPK)
        want = O.frequent_summary_threads(items, k, C, threads)
        assert pairs(whole) == want.as_pairs() and dd == want.d
        rep, _, _ = B.pss_frequent_run(ctx, d, k=k, chunks=C)
        want.n = n
        assert pairs(rep) == pairs(want.report())
    del d
    torch.cuda.empty_cache()
