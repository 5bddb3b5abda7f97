"""Pins for the CPU oracle: what the paper and the mathematics fix.

Everything here runs on the CPU.  The oracle (oracle/pss_oracle.c) is checked
against hand-worked examples, exact histograms (brute force), the Space
Saving and COMBINE invariants, special cases that reduce to exact counting or
to Moore's majority vote, and a second independent implementation
(oracle/brute.py).  A dropped term, a wrong sign, a swapped minimum or a
wrong tie-break in either implementation fails at least one of these.
"""
import json
import os
import random

import numpy as np
import pytest

import oracle as O
import oracle.brute as B
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_examples.json")


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build(force=False)
    workloads.build(force=False)


def _cases():
    with open(GOLDEN) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c["name"])
def test_worked_examples_c_oracle(case):
    s = O.summary(case["items"], case["k"], case["chunks"])
    assert s.as_tuples() == [tuple(t) for t in case["summary"]]
    assert s.m == case["m"]
    rep = O.run(case["items"], case["k"], case["chunks"])
    assert O.to_tuples(rep) == [tuple(t) for t in case["reported"]]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c["name"])
def test_worked_examples_brute(case):
    s, m = B.summary(case["items"], case["k"], case["chunks"])
    assert B.canonical(s) == [tuple(t) for t in case["summary"]]
    assert m == case["m"]
    assert B.run(case["items"], case["k"], case["chunks"]) == [tuple(t) for t in case["reported"]]


def _random_case(rng):
    n = rng.randint(1, 60)
    k = rng.randint(2, 7)
    univ = rng.randint(1, 14)
    chunks = rng.randint(1, 9)
    # skewed or flat small-universe streams, ids spread over uint32 edges too
    ids = [0, 0xFFFFFFFF, 1, 7, 0x80000000, 12345, 99, 3, 2, 0xFFFFFFFE, 5, 6, 8, 10][:univ]
    if rng.random() < 0.5:
        w = [1.0 / (i + 1) ** 1.3 for i in range(univ)]
    else:
        w = [1.0] * univ
    items = rng.choices(ids, weights=w, k=n)
    return items, k, chunks


def test_c_oracle_equals_independent_python_bit_exact():
    rng = random.Random(2024)
    for _ in range(3000):
        items, k, chunks = _random_case(rng)
        s = O.summary(items, k, chunks)
        bs, bm = B.summary(items, k, chunks)
        assert s.as_tuples() == B.canonical(bs), (items, k, chunks)
        assert s.m == bm
        if k <= len(items):
            assert O.to_tuples(O.run(items, k, chunks)) == B.run(items, k, chunks)


def _check_summary_invariants(items, k, chunks, s):
    """Invariants every reading must satisfy (Section 3 and Algorithm 2)."""
    n = len(items)
    f = B.histogram(items)
    ent = {int(e["item"]): (int(e["count"]), int(e["error"])) for e in s.entries}
    assert len(ent) == len(s.entries) <= k
    for x, (c, e) in ent.items():
        assert c >= f.get(x, 0), "estimate below the true frequency"
        assert c - e <= f.get(x, 0), "guaranteed count above the true frequency"
        assert 0 <= e <= c
    # every unmonitored item occurs at most m times
    for x, fx in f.items():
        if x not in ent:
            assert fx <= s.m
    assert sum(c for c, _ in ent.values()) <= n
    assert s.m * k <= n
    if len(ent) < k:
        assert s.m == 0
    else:
        assert s.m == min(c for c, _ in ent.values())
    # recall: every true k-majority item is reported
    rep = {t[0] for t in O.to_tuples(O.run(items, k, chunks))} if 2 <= k <= n else set()
    for x, fx in f.items():
        if fx * k > n and k <= n:
            assert x in rep, "k-majority item missed"


def test_invariants_against_exact_histograms():
    rng = random.Random(7)
    for _ in range(3000):
        items, k, chunks = _random_case(rng)
        s = O.summary(items, k, chunks)
        _check_summary_invariants(items, k, chunks, s)


def test_chunk_summaries_count_every_item_once():
    rng = random.Random(11)
    for _ in range(500):
        items, k, chunks = _random_case(rng)
        for lo, hi in O.chunk_bounds(len(items), chunks):
            s = O.space_saving(items[lo:hi], k)
            assert int(s.entries["count"].sum()) == hi - lo


def test_partition_matches_block_distribution():
    # floor(n/p) or ceil(n/p) items per block, contiguous, covering [0, n)
    for n in [0, 1, 5, 64, 1000, 2**20 + 3]:
        for chunks in [1, 2, 3, 7, 64, 1000]:
            b = O.chunk_bounds(n, chunks)
            assert b[0][0] == 0 and b[-1][1] == n
            for (lo, hi), (lo2, _) in zip(b, b[1:]):
                assert hi == lo2
            for lo, hi in b:
                assert hi - lo in (n // chunks, -(-n // chunks))


def test_few_distinct_items_is_exact():
    # at most k distinct items: every summary is exact, the report is the
    # exact histogram filtered by f * k > n, all errors 0
    rng = random.Random(3)
    for _ in range(300):
        k = rng.randint(2, 9)
        items = [rng.randrange(k) * 1000003 for _ in range(rng.randint(k, 80))]
        chunks = rng.randint(1, 6)
        f = B.histogram(items)
        want = sorted(((x, c, 0) for x, c in f.items() if c * k > len(items)), key=lambda t: (-t[1], t[2], t[0]))
        assert O.to_tuples(O.run(items, k, chunks)) == want


def test_chunks_at_least_n_makes_every_chunk_exact():
    rng = random.Random(5)
    for _ in range(200):
        items = [rng.randrange(6) for _ in range(rng.randint(2, 30))]
        k = rng.randint(2, len(items))
        chunks = len(items) + rng.randint(0, 4)
        for lo, hi in O.chunk_bounds(len(items), chunks):
            s = O.space_saving(items[lo:hi], k)
            assert s.m == 0 or hi - lo >= k
            assert all(int(e["error"]) == 0 for e in s.entries)


def test_one_chunk_is_sequential_space_saving():
    rng = random.Random(9)
    for _ in range(300):
        items, k, _ = _random_case(rng)
        s = O.summary(items, k, 1)
        ss = O.space_saving(items, k)
        assert s.as_tuples() == ss.as_tuples() and s.m == ss.m


def test_k2_reports_moore_majority():
    rng = random.Random(13)
    for _ in range(500):
        n = rng.randint(2, 50)
        maj = rng.randrange(1 << 32)
        items = [maj if rng.random() < 0.6 else rng.randrange(5) for _ in range(n)]
        rng.shuffle(items)
        bm = B.boyer_moore_majority(items)
        rep = [t[0] for t in O.to_tuples(O.run(items, 2, rng.randint(1, 5)))]
        if bm is not None:
            assert rep == [bm]  # at most one item can exceed n/2
        assert len(rep) <= 1


def test_combine_identity_and_commutativity():
    rng = random.Random(17)
    for _ in range(500):
        items, k, _ = _random_case(rng)
        a = O.space_saving(items, k)
        items2, _, _ = _random_case(rng)
        b = O.space_saving(items2, k)
        empty = O.Summary(k)
        ia = O.combine(a, empty)
        assert ia.as_tuples() == a.as_tuples() and ia.m == a.m
        ab, ba = O.combine(a, b), O.combine(b, a)
        assert ab.as_tuples() == ba.as_tuples() and ab.m == ba.m


def test_combine_is_not_associative_so_the_tree_is_fixed():
    # witness that (S0+S1)+S2 and S0+(S1+S2) can differ: the reduction order
    # is part of the result, hence the fixed level-wise tree
    rng = random.Random(19)
    found = 0
    for _ in range(2000):
        k = rng.randint(2, 4)
        s = [O.space_saving([rng.randrange(8) for _ in range(rng.randint(1, 12))], k) for _ in range(3)]
        left = O.combine(O.combine(s[0], s[1]), s[2])
        right = O.combine(s[0], O.combine(s[1], s[2]))
        if left.as_tuples() != right.as_tuples():
            found += 1
    assert found > 0


def test_tree_shape_pairs_adjacent_and_promotes_odd_tail():
    rng = random.Random(23)
    for _ in range(200):
        k = rng.randint(2, 5)
        count = rng.randint(1, 9)
        sums = [O.space_saving([rng.randrange(10) for _ in range(rng.randint(0, 10))], k) for _ in range(count)]
        level = sums
        while len(level) > 1:
            nxt = [O.combine(level[2 * j], level[2 * j + 1]) for j in range(len(level) // 2)]
            if len(level) % 2:
                nxt.append(level[-1])
            level = nxt
        t = O.tree(sums, k)
        assert t.as_tuples() == level[0].as_tuples() and t.m == level[0].m


def test_update_is_combine_with_batch_summary():
    # an append folds the batch's tree into the live summary: S <- COMBINE(S, B)
    rng = random.Random(29)
    for _ in range(200):
        k = rng.randint(2, 6)
        s = O.Summary(k)
        batches = [[rng.randrange(12) for _ in range(rng.randint(1, 25))] for _ in range(rng.randint(1, 4))]
        ref = None
        for b in batches:
            c = rng.randint(1, 4)
            s.update(b, c)
            bs, bm = B.summary(b, k, c)
            ref = (bs, bm) if ref is None else B.combine(ref[0], ref[1], bs, bm, k)
        assert s.as_tuples() == B.canonical(ref[0]) and s.m == ref[1]
        assert s.n == sum(len(b) for b in batches)


def test_full_range_ids_including_zero_and_max():
    items = [0, 0xFFFFFFFF, 0, 0xFFFFFFFF, 0, 5]
    assert O.to_tuples(O.run(items, 2, 2)) == B.run(items, 2, 2)
    assert O.to_tuples(O.run(items, 3, 1)) == [(0, 3, 0)]


def test_zipf_stream_invariants_at_plain_size():
    # the small plain workload shape (2^20 items, k=100, 64 chunks), with the
    # exact histogram from numpy
    items = workloads.plain(seed=1).generate()
    k, chunks = 100, 64
    s = O.summary(items, k, chunks)
    vals, cnts = np.unique(items, return_counts=True)
    f = dict(zip(vals.tolist(), cnts.tolist()))
    n = len(items)
    for e in s.entries:
        x, c, er = int(e["item"]), int(e["count"]), int(e["error"])
        assert c >= f.get(x, 0) >= c - er
    rep = {int(e["item"]) for e in O.run(items, k, chunks)}
    truth = {x for x, c in f.items() if c * k > n}
    assert truth <= rep and len(truth) >= 5
    assert int(s.entries["count"].sum()) <= n


def test_threaded_chunk_summaries_equal_single_thread():
    # the T-thread form (chunk summaries in parallel, tree on one thread)
    # is the same computation as the single-threaded oracle
    items = workloads.plain(seed=21, n=1 << 17).generate()
    for k, C in [(100, 64), (37, 9), (500, 1), (2000, 33)]:
        a = O.summary(items, k, C)
        b = O.summary_threads(items, k, C, threads=4)
        assert a.as_tuples() == b.as_tuples() and a.m == b.m
        assert O.to_tuples(O.run(items, k, C)) == O.to_tuples(O.run_threads(items, k, C, threads=4))
