"""GPU parity: the HIP path through the C-ABI against the CPU oracle, bit-exact.

Every comparison is on items, counts and errors.  Inputs are seeded synthetic
streams from ``workloads``; expected values come only from ``oracle``.
"""
import random
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


def summary_tuples(B, s):
    ent, n = B.pss_query(s, B.PSS_Q_TOPK, cap=s.k)
    return B.to_tuples(ent), n


def test_device_limits(ctx):
    say("max_k", ctx.max_k)
    assert ctx.max_k >= 2000


def test_plain_small_config_bit_exact(B, ctx):
    # 2^20 items, Zipf 1.5 over 2^20 permuted ids, k=100, 64 chunks
    items = W.plain(seed=1).generate()
    say("plain n=2^20 k=100 C=64")
    got, used = B.pss_run(ctx, dev(items), k=100, chunks=64)
    assert used == 64
    want = O.run(items, 100, 64)
    assert B.to_tuples(got) == O.to_tuples(want)
    assert len(want) >= 5


def test_plain_small_config_block_summaries(B, ctx):
    items = W.plain(seed=2).generate()
    k, C = 100, 64
    blocks = B.pss_block_summaries(ctx, dev(items), k, C, list(range(C)))
    ref = O.chunk_summaries(items, k, C)
    for c in range(C):
        ent, mn = blocks[c]
        assert sorted(B.to_tuples(ent)) == sorted(O.to_tuples(ref[c].entries)), c
        assert mn == ref[c].m, c


def test_whole_summary_equals_oracle_summary(B, ctx):
    items = W.plain(seed=3).generate()
    for k, C in [(100, 64), (37, 1), (512, 7), (2000, 33)]:
        say("summary k=%d C=%d" % (k, C))
        s = B.Summary(ctx, k)
        B.pss_update(s, dev(items), chunks=C)
        got, n = summary_tuples(B, s)
        ref = O.summary(items, k, C)
        assert n == len(items)
        assert got == ref.as_tuples(), (k, C)
        s.close()


@pytest.mark.parametrize("k,n,C", [(64, 65471, 1), (64, 65472, 1), (64, 130942, 2),
                                   (4096, 4190207, 1), (4096, 4190208, 1)])
def test_error_packing_bounds(B, ctx, k, n, C):
    # errors ride in the count words while blocks hold fewer than 2^22 items
    # and floor(block / k), the largest error, is at most 1022: blocks of
    # 1023 k - 1 items pack, 1023 k do not (with k <= 4096 in LDS this bound
    # comes before the count bound).  A long run of one id (counts up to
    # half the block) and a uniform tail (errors at their largest).
    rng = np.random.default_rng(k + n + C)
    items = np.concatenate([np.full(n // 2, 12345, dtype=np.uint32),
                            rng.integers(0, 1 << 32, n - n // 2, dtype=np.uint64).astype(np.uint32)])
    say("error packing k=%d n=%d C=%d" % (k, n, C))
    blocks = B.pss_block_summaries(ctx, dev(items), k, C, list(range(C)))
    ref = O.chunk_summaries(items, k, C)
    for c in range(C):
        ent, mn = blocks[c]
        assert sorted(B.to_tuples(ent)) == sorted(O.to_tuples(ref[c].entries)), (k, n, C, c)
        assert mn == ref[c].m, (k, n, C, c)
    got, _ = B.pss_run(ctx, dev(items), k=k, chunks=C)
    assert B.to_tuples(got) == O.to_tuples(O.run(items, k, C))


@pytest.mark.parametrize("k,every", [(500, 733), (2000, 4001)])
def test_largest_id_in_large_levels(B, ctx, k, every):
    # the level sort compares ids alone and pads a lane's registers with the
    # largest key; the id 0xFFFFFFFF, rarer than the minimum count grows in a
    # uniform stream, is evicted and reinstalled over and over and keeps
    # landing in levels of hundreds of counters
    rng = np.random.default_rng(k)
    n = 400000
    items = rng.integers(0, 0xFFFFFFFF, n, dtype=np.uint64).astype(np.uint32)
    items[::every] = 0xFFFFFFFF
    for C in (1, 3):
        say("largest id k=%d C=%d" % (k, C))
        blocks = B.pss_block_summaries(ctx, dev(items), k, C, list(range(C)))
        ref = O.chunk_summaries(items, k, C)
        for c in range(C):
            ent, mn = blocks[c]
            assert sorted(B.to_tuples(ent)) == sorted(O.to_tuples(ref[c].entries)), (k, C, c)
            assert mn == ref[c].m, (k, C, c)
        got, _ = B.pss_run(ctx, dev(items), k=k, chunks=C)
        assert B.to_tuples(got) == O.to_tuples(O.run(items, k, C))


def _rand_stream(rng, n):
    kind = rng.choice(["few", "zipf", "uniform", "same", "edge", "roundrobin"])
    if kind == "few":
        ids = [rng.randrange(1 << 32) for _ in range(rng.randint(1, 6))]
        return [rng.choice(ids) for _ in range(n)]
    if kind == "zipf":
        univ = rng.choice([10, 100, 5000, 1 << 20])
        a = rng.uniform(0.5, 2.0)
        r = W.zipf_ranks(n, a, univ, rng.randrange(1 << 60))
        key = rng.randrange(1 << 32)
        return [W.fmix32((int(x) - 1) ^ key) for x in r] if n <= 20000 else None
    if kind == "uniform":
        return [rng.randrange(1 << 32) for _ in range(n)]
    if kind == "same":
        return [rng.choice([0, 0xFFFFFFFF, 17])] * n
    if kind == "edge":
        return [rng.choice([0, 0xFFFFFFFF, 1, 0xFFFFFFFE]) for _ in range(n)]
    d = rng.randint(1, 300)
    return [(i % d) * 2654435761 % (1 << 32) for i in range(n)]


def test_random_small_cases_bit_exact(B, ctx):
    rng = random.Random(1234)
    for t in range(120):
        n = rng.choice([2, 3, 63, 64, 65, 511, 512, 513, 1000, 4097, 20000])
        items = _rand_stream(rng, n)
        if items is None:
            continue
        k = rng.randint(2, min(n, 600))
        C = rng.choice([1, 2, 3, 5, 17, 64, n, n + 3])
        say("case", t, "n", n, "k", k, "C", C)
        got, used = B.pss_run(ctx, dev(items), k=k, chunks=C)
        assert used == C
        assert B.to_tuples(got) == O.to_tuples(O.run(items, k, C)), (t, n, k, C)
        s = B.Summary(ctx, k)
        B.pss_update(s, dev(items), chunks=C)
        assert summary_tuples(B, s)[0] == O.summary(items, k, C).as_tuples(), (t, n, k, C)
        s.close()


def test_unaligned_device_pointer_and_ragged_tail(B, ctx):
    import torch
    items = W.zipf_hashed(100_003, 1.1, 1 << 32, seed=9)
    base = torch.from_numpy(np.concatenate([[7], items]).astype(np.uint32).view(np.int32)).to("cuda")
    view = base[1:]  # 4-byte aligned but not 16-byte aligned
    assert view.data_ptr() % 16 != 0
    for k, C in [(50, 13), (300, 1), (1000, 101)]:
        say("unaligned k=%d C=%d" % (k, C))
        got, _ = B.pss_run(ctx, view, k=k, chunks=C)
        assert B.to_tuples(got) == O.to_tuples(O.run(items, k, C))


def test_zipf_hashed_medium_all_ks(B, ctx):
    for alpha in (0.8, 1.2, 1.8):
        items = W.zipf_hashed(1 << 22, alpha, 1 << 32, seed=5)
        for k in (500, 2000):
            C = ctx.plan_chunks(len(items), k)
            say("zipf a=%g n=2^22 k=%d C=%d" % (alpha, k, C))
            got, used = B.pss_run(ctx, dev(items), k=k, chunks=0)
            assert used == C
            assert B.to_tuples(got) == O.to_tuples(O.run(items, k, C)), (alpha, k)


def test_uniform_and_adversarial_medium(B, ctx):
    u = W.uniform(1 << 21, seed=3)
    got, used = B.pss_run(ctx, dev(u), k=2000, chunks=16)
    assert B.to_tuples(got) == O.to_tuples(O.run(u, 2000, 16))
    a = W.adversarial(1 << 21, seed=4, d=1 << 14)
    got, _ = B.pss_run(ctx, dev(a), k=1000, chunks=8)
    want = O.run(a, 1000, 8)
    assert B.to_tuples(got) == O.to_tuples(want)
    assert W.adversarial_planted_id(4, d=1 << 14) in [int(e["item"]) for e in want]


def test_skewed_ids_level_sort_fallback(B, ctx):
    # levels whose ids share all bits but the top one and the low 12: the
    # digit sort finds an oversized bucket and the level is sorted by the
    # fallback network (state in LDS, k in two register classes)
    a = W.skewed_ids(1 << 18, seed=5)
    for k, C in ((700, 4), (1500, 2)):
        say("skewed ids n=2^18 k=%d C=%d" % (k, C))
        got = B.pss_block_summaries(ctx, dev(a), k, C, list(range(C)))
        ref = O.chunk_summaries(a, k, C)
        for c in range(C):
            ent, mn = got[c]
            assert sorted(B.to_tuples(ent)) == sorted(O.to_tuples(ref[c].entries)), (k, c)
            assert mn == ref[c].m, (k, c)
        run, _ = B.pss_run(ctx, dev(a), k=k, chunks=C)
        assert B.to_tuples(run) == O.to_tuples(O.run(a, k, C)), k


def test_errors_and_truncation(B, ctx):
    items = dev([1, 2, 3, 1, 1, 1, 2, 2])
    with pytest.raises(B.PssError) as e:
        B.pss_run(ctx, items, k=1)
    assert e.value.code == B.PSS_ERANGE
    with pytest.raises(B.PssError) as e:
        B.pss_run(ctx, items, k=9)
    assert e.value.code == B.PSS_ERANGE
    with pytest.raises(B.PssError) as e:
        B.Summary(ctx, 1)
    assert e.value.code == B.PSS_EINVAL
    # two items qualify (count*3 > 8: 1 x4, 2 x3); cap=1 truncates and reports 2
    with pytest.raises(B.PssError) as e:
        B.pss_run(ctx, items, k=3, chunks=1, cap=1)
    assert e.value.code == B.PSS_ETRUNC and e.value.required == 2
    got, _ = B.pss_run(ctx, items, k=3, chunks=1, cap=2)
    assert B.to_tuples(got) == O.to_tuples(O.run([1, 2, 3, 1, 1, 1, 2, 2], 3, 1))
    a, b = B.Summary(ctx, 10), B.Summary(ctx, 11)
    with pytest.raises(B.PssError) as e:
        B.pss_merge(a, b)
    assert e.value.code == B.PSS_EINVAL
    with pytest.raises(B.PssError) as e:
        B.pss_merge(a, a)
    assert e.value.code == B.PSS_EINVAL
    # stream lengths reach 2^32 - 128 at most (the top count values are the
    # kernel's window tags); the bound is checked before any device work
    for n in ((1 << 32) - 128, 1 << 32):
        with pytest.raises(B.PssError) as e:
            B.pss_update(a, items, chunks=1, n=n)
        assert e.value.code == B.PSS_ERANGE, n
    assert B.last_device_error()[0] == 0


def test_update_merge_query_sequence(B, ctx):
    rng = random.Random(77)
    k = 64
    s = B.Summary(ctx, k)
    t = B.Summary(ctx, k)
    ref_s, ref_t = O.Summary(k), O.Summary(k)
    for i in range(6):
        n = rng.choice([1, 100, 5000, 70000])
        items = W.zipf_hashed(n, 1.3, 1 << 32, seed=100 + i)
        C = rng.choice([1, 3, 16])
        tgt, ref = (s, ref_s) if i % 2 == 0 else (t, ref_t)
        B.pss_update(tgt, dev(items), chunks=C)
        ref.update(items, C)
        got, n_s = B.pss_query(tgt, B.PSS_Q_MAJORITY)
        assert n_s == ref.n
        assert B.to_tuples(got) == O.to_tuples(ref.query_majority())
        top, _ = B.pss_query(tgt, B.PSS_Q_TOPK, cap=5)
        assert B.to_tuples(top) == O.to_tuples(ref.query_topk(5))
    B.pss_merge(s, t)
    ref_s.merge(ref_t)
    got, n_s = B.pss_query(s, B.PSS_Q_TOPK, cap=k)
    assert n_s == ref_s.n
    assert B.to_tuples(got) == ref_s.as_tuples()


def test_empty_update_is_a_noop(B, ctx):
    import torch
    s = B.Summary(ctx, 5)
    B.pss_update(s, torch.zeros(0, dtype=torch.int32, device="cuda"), chunks=4)
    got, n = B.pss_query(s, B.PSS_Q_TOPK, cap=5)
    assert len(got) == 0 and n == 0


def test_repeat_runs_are_identical(B, ctx):
    items = W.zipf_hashed(1 << 20, 1.2, 1 << 32, seed=8)
    d = dev(items)
    first = B.to_tuples(B.pss_run(ctx, d, k=700, chunks=50)[0])
    for _ in range(3):
        assert B.to_tuples(B.pss_run(ctx, d, k=700, chunks=50)[0]) == first
