"""The seeded input generators: determinism and distribution shape."""
import numpy as np

import workloads as W


def test_generators_are_deterministic_and_thread_independent():
    a = W.zipf_hashed(100_000, 1.2, 1 << 32, seed=3, threads=1)
    b = W.zipf_hashed(100_000, 1.2, 1 << 32, seed=3, threads=7)
    assert np.array_equal(a, b)
    c = W.zipf_hashed(100_000, 1.2, 1 << 32, seed=4, threads=3)
    assert not np.array_equal(a, c)
    assert np.array_equal(W.uniform(5000, 9, threads=1), W.uniform(5000, 9, threads=4))


def test_splitmix_and_fmix_published_values():
    # SplitMix64 seeded with 0: first output 0xE220A8397B1DCDAF (Vigna's reference code)
    assert W.draw(0, 0) == 0xE220A8397B1DCDAF
    # fmix32 is a bijection: no collisions on a block of inputs, and fmix32(0) == 0
    assert W.fmix32(0) == 0
    xs = {W.fmix32(i) for i in range(20000)}
    assert len(xs) == 20000


def test_permutation_is_a_bijection():
    p = W.permutation(1 << 16, key=123)
    assert np.array_equal(np.sort(p), np.arange(1 << 16, dtype=np.uint32))


def test_zipf_rank_frequencies_match_the_law():
    n, s, N = 400_000, 1.5, 1 << 20
    r = W.zipf_ranks(n, s, N, key=77)
    assert r.min() >= 1 and r.max() <= N
    h = np.sum(np.arange(1, N + 1, dtype=np.float64) ** -s)
    for rank in (1, 2, 3, 10):
        p = rank ** -s / h
        got = np.mean(r == rank)
        assert abs(got - p) < 5 * np.sqrt(p * (1 - p) / n), (rank, got, p)


def test_zipf_below_one_covers_a_huge_universe():
    r = W.zipf_ranks(200_000, 0.8, 1 << 32, key=5)
    assert r.max() > (1 << 31) and r.min() == 1


def test_adversarial_stream_structure():
    n = 20 * 5000
    a = W.adversarial(n, seed=2, d=1 << 10)
    planted = W.adversarial_planted_id(2, d=1 << 10)
    assert np.all(a[19::20] == planted)
    rest = np.delete(a, np.arange(19, n, 20))
    assert planted not in set(rest.tolist())
    assert len(np.unique(rest)) == 1 << 10


def test_skewed_ids_structure():
    a = W.skewed_ids(200_000, seed=5)
    assert np.array_equal(a, W.skewed_ids(200_000, seed=5))
    high = (a >> 31) == 1
    assert 0.008 < high.mean() < 0.012  # about 1% carry bit 31
    assert np.all((a & np.uint32(0x7FFFFFFF)) < (1 << 12))  # every other bit above the low 12 is clear
