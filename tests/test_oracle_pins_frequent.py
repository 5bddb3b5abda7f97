"""Pins of the Frequent (Misra-Gries) oracle against what the definitions
fix: hand-worked examples, an independent pure-Python statement, exact
histograms (f - D <= f^ <= f, D * k <= n, recall of every true k-majority
item), Boyer and Moore's majority vote for k = 2, exact counting with few
distinct items, and the merge's identity and symmetry."""
import json
import os
import random
from collections import Counter

import numpy as np
import pytest

import oracle as O
import oracle.brute as Bru
import workloads

HERE = os.path.dirname(os.path.abspath(__file__))
CASES = json.load(open(os.path.join(HERE, "golden", "frequent_examples.json")))["cases"]


def pairs(entries):
    return sorted(((int(e["item"]), int(e["count"])) for e in entries), key=lambda t: (-t[1], t[0]))


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_worked_examples_c_oracle(case):
    items = np.array(case["items"], dtype=np.uint32)
    s = O.frequent_summary(items, case["k"], case["chunks"])
    assert s.as_pairs() == [tuple(x) for x in case["summary"]]
    assert s.d == case["d"]
    assert pairs(O.frequent_run(items, case["k"], case["chunks"])) == [tuple(x) for x in case["reported"]]


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_worked_examples_brute(case):
    s, d, rep = Bru.frequent_parallel(case["items"], case["k"], case["chunks"])
    assert sorted(s.items(), key=lambda t: (-t[1], t[0])) == [tuple(x) for x in case["summary"]]
    assert d == case["d"]
    assert rep == [tuple(x) for x in case["reported"]]


def test_c_oracle_equals_independent_python():
    rng = random.Random(97)
    for _ in range(2000):
        n = rng.randrange(1, 80)
        univ = rng.choice([2, 3, 5, 9, 30])
        items = [rng.randrange(univ) for _ in range(n)]
        k = rng.randrange(2, 9)
        C = rng.randrange(1, min(n, 8) + 1)
        s, d, rep = Bru.frequent_parallel(items, k, C)
        a = np.array(items, dtype=np.uint32)
        so = O.frequent_summary(a, k, C)
        assert so.as_pairs() == sorted(s.items(), key=lambda t: (-t[1], t[0])), (items, k, C)
        assert so.d == d
        assert pairs(O.frequent_run(a, k, C)) == rep


def test_bounds_against_exact_histograms():
    rng = random.Random(5)
    for _ in range(600):
        n = rng.randrange(1, 400)
        items = [int(x) for x in np.random.default_rng(rng.randrange(1 << 30)).zipf(1.3, n) % 50]
        k = rng.randrange(2, 12)
        C = rng.randrange(1, 9)
        f = Counter(items)
        s = O.frequent_summary(np.array(items, dtype=np.uint32), k, C)
        est = dict(s.as_pairs())
        assert len(est) <= k - 1
        assert s.d * k <= n
        for x, fx in f.items():
            assert fx - s.d <= est.get(x, 0) <= fx, (x, fx, est.get(x), s.d)
        rep = {x for x, _ in pairs(O.frequent_run(np.array(items, dtype=np.uint32), k, C))}
        for x, fx in f.items():
            if fx * k > n:
                assert x in rep  # recall


def boyer_moore(items):
    cand, cnt = None, 0
    for x in items:
        if cnt == 0:
            cand, cnt = x, 1
        elif x == cand:
            cnt += 1
        else:
            cnt -= 1
    return cand, cnt


def test_k2_is_the_majority_vote():
    rng = random.Random(11)
    for _ in range(500):
        items = [rng.randrange(4) for _ in range(rng.randrange(1, 60))]
        s = O.frequent(np.array(items, dtype=np.uint32), 2)
        cand, cnt = boyer_moore(items)
        if cnt == 0:
            assert s.as_pairs() == []
        else:
            assert s.as_pairs() == [(cand, cnt)]


def test_few_distinct_items_is_exact_counting():
    items = workloads.uniform(5000, 3) % np.uint32(7)
    f = Counter(int(x) for x in items)
    for C in (1, 3, 16):
        s = O.frequent_summary(items, 8, C)  # 7 counters for 7 distinct items
        assert s.d == 0
        assert dict(s.as_pairs()) == dict(f)


def test_merge_identity_and_symmetry():
    a = workloads.zipf_hashed(3000, 1.1, 1 << 12, seed=1)
    b = workloads.zipf_hashed(2000, 1.4, 1 << 12, seed=2)
    for k in (2, 5, 40):
        sa, sb = O.frequent(a, k), O.frequent(b, k)
        e = O.FSummary(k)
        assert O.frequent_merge(sa, e).as_pairs() == sa.as_pairs()
        assert O.frequent_merge(e, sa).d == sa.d
        ab, ba = O.frequent_merge(sa, sb), O.frequent_merge(sb, sa)
        assert ab.as_pairs() == ba.as_pairs() and ab.d == ba.d


def test_threaded_form_equals_single_thread():
    items = workloads.zipf_hashed(1 << 16, 1.1, 1 << 32, seed=9)
    for k, C in [(100, 64), (2, 7), (2000, 5)]:
        a, b = O.frequent_summary(items, k, C), O.frequent_summary_threads(items, k, C, 4)
        assert a.as_pairs() == b.as_pairs() and a.d == b.d
