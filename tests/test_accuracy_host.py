"""The accuracy harness's arithmetic on host arrays, against a plain
dictionary count written out here (Section 4's definitions)."""
from collections import Counter

import numpy as np

import oracle as O
import workloads as W
from paper_1606_04669_amd import accuracy as A


def reference_metrics(items, reported, k):
    f = Counter(int(x) for x in items)
    n = len(items)
    true_set = {x for x, c in f.items() if c * k > n}
    rep = [(int(e["item"]), int(e["count"])) for e in reported]
    rel = [abs(c - f[x]) / f[x] for x, c in rep]
    hit = sum(1 for x, _ in rep if x in true_set)
    return {
        "are": sum(rel) / len(rel) if rel else 0.0,
        "precision": hit / len(rep) if rep else 1.0,
        "recall": (sum(1 for x in true_set if x in {r[0] for r in rep}) / len(true_set)) if true_set else 1.0,
        "reported": len(rep),
        "true_majority": len(true_set),
    }


def test_metrics_match_a_plain_count():
    items = W.zipf_hashed(200000, 1.1, 1 << 32, seed=3)
    ex = A.exact_counts_host(items)
    assert int(ex.counts.sum()) == len(items)
    for k, C in [(50, 8), (300, 1), (1000, 16)]:
        rep = O.run(items, k, C)
        got = A.metrics(rep, ex, k)
        want = reference_metrics(items, rep, k)
        for key in want:
            assert abs(got[key] - want[key]) < 1e-12, (k, key, got[key], want[key])
        assert got["recall"] == 1.0  # Space Saving reports every true k-majority item


def test_false_positive_lowers_precision():
    # worked example W2: [9, 4, 7], k = 2 reports 7 with count 2 although f(7) = 1
    items = np.array([9, 4, 7], dtype=np.uint32)
    rep = O.run(items, 2, 1)
    got = A.metrics(rep, A.exact_counts_host(items), 2)
    assert got["reported"] == 1 and got["true_majority"] == 0
    assert got["precision"] == 0.0 and got["recall"] == 1.0
    assert got["are"] == 1.0  # |2 - 1| / 1


def test_frequency_of_absent_items_is_zero():
    ex = A.exact_counts_host(np.array([5, 5, 0, 0xFFFFFFFF], dtype=np.uint32))
    assert ex.frequency(np.array([5, 0, 0xFFFFFFFF, 7, 6], dtype=np.uint32)).tolist() == [2, 1, 1, 0, 0]
    assert ex.majority(2).tolist() == []  # 2 * 2 > 4 is false
    assert ex.majority(3).tolist() == [5]
