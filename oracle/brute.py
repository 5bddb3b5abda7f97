"""Second, independent statement of the method in plain Python (tiny inputs).

TEST INFRASTRUCTURE ONLY.  It shares nothing with ``pss_oracle.c`` except the
paper: a dict of counters with a linear scan for the minimum instead of a
hash map plus heap, dict-based COMBINE, and exact histograms.  The tests use
it to cross-check the C oracle bit for bit and to supply exact frequencies.

Same readings as the C oracle: unused counters count 0 (so m = 0 when fewer
than k items are monitored), eviction of the minimum count with the smallest
id, new item gets error 0 / m, Prune keeps (count desc, error asc, item asc),
the fixed tree pairs (2j, 2j+1), chunk c is [floor(cn/C), floor((c+1)n/C)).
"""
from __future__ import annotations

from collections import Counter


def space_saving(items, k):
    """Sequential Space Saving (Section 3): returns ({item: [count, err]}, m)."""
    ctr = {}
    for x in items:
        x = int(x)
        if x in ctr:
            ctr[x][0] += 1
        elif len(ctr) < k:
            ctr[x] = [1, 0]
        else:
            victim = min(ctr, key=lambda y: (ctr[y][0], y))
            m = ctr.pop(victim)[0]
            ctr[x] = [m + 1, m]
    m = min(c for c, _ in ctr.values()) if len(ctr) == k else 0
    return ctr, m


def key(item, count, err):
    return (-count, err, item)


def combine(s1, m1, s2, m2, k):
    """Algorithm 2: ({item: [count, err]}, m) for COMBINE(S1, S2)."""
    cand = {}
    for x, (c, e) in s1.items():
        if x in s2:
            c2, e2 = s2[x]
            cand[x] = [c + c2, e + e2]
        else:
            cand[x] = [c + m2, e + m2]
    for x, (c, e) in s2.items():
        if x not in s1:
            cand[x] = [c + m1, e + m1]
    order = sorted(cand, key=lambda x: key(x, cand[x][0], cand[x][1]))[:k]
    kept = {x: cand[x] for x in order}
    m = cand[order[-1]][0] if len(order) == k else 0
    return kept, m


def chunk_bounds(n, chunks):
    return [((c * n) // chunks, ((c + 1) * n) // chunks) for c in range(chunks)]


def summary(items, k, chunks):
    items = [int(x) for x in items]
    level = []
    for lo, hi in chunk_bounds(len(items), chunks):
        level.append(space_saving(items[lo:hi], k))
    while len(level) > 1:
        nxt = []
        for j in range(len(level) // 2):
            (a, ma), (b, mb) = level[2 * j], level[2 * j + 1]
            nxt.append(combine(a, ma, b, mb, k))
        if len(level) % 2:
            nxt.append(level[-1])
        level = nxt
    return level[0]


def canonical(s):
    return sorted(((x, c, e) for x, (c, e) in s.items()), key=lambda t: key(*t))


def run(items, k, chunks):
    """Reported items (item, count, err) with count * k > n, canonical order."""
    s, _ = summary(items, k, chunks)
    n = len(items)
    return [t for t in canonical(s) if t[1] * k > n]


def histogram(items):
    return Counter(int(x) for x in items)


def boyer_moore_majority(items):
    """Moore's majority vote: the candidate, then a verifying count."""
    cand, cnt = None, 0
    for x in items:
        if cnt == 0:
            cand, cnt = x, 1
        elif x == cand:
            cnt += 1
        else:
            cnt -= 1
    if cand is not None and sum(1 for x in items if x == cand) * 2 > len(items):
        return int(cand)
    return None


# ---------------------------------------------------------------------------
# Frequent (Misra-Gries) for the k-majority problem (k - 1 counters), written
# independently of frequent_oracle.c: a dict, a full pass to decrement, dict
# merge.
# ---------------------------------------------------------------------------

def frequent(items, k):
    """Sequential Frequent: ({item: count}, D) with D the decrement steps."""
    ctr = {}
    d = 0
    for x in items:
        x = int(x)
        if x in ctr:
            ctr[x] += 1
        elif len(ctr) < k - 1:
            ctr[x] = 1
        else:
            d += 1
            ctr = {y: c - 1 for y, c in ctr.items() if c > 1}
    return ctr, d


def frequent_merge(s1, d1, s2, d2, k):
    """Sum the union; beyond k - 1 items subtract the k-th largest count."""
    u = dict(s1)
    for x, c in s2.items():
        u[x] = u.get(x, 0) + c
    cut = 0
    if len(u) > k - 1:
        cut = sorted(u.values(), reverse=True)[k - 1]
    return {x: c - cut for x, c in u.items() if c > cut}, d1 + d2 + cut


def frequent_parallel(items, k, chunks):
    """Chunk summaries, fixed tree, report of (count + D) * k > n."""
    n = len(items)
    nodes = []
    for c in range(chunks):
        lo, hi = c * n // chunks, (c + 1) * n // chunks
        nodes.append(frequent(items[lo:hi], k))
    step = 1
    while step < chunks:
        for a in range(0, chunks - step, 2 * step):
            b = a + step
            nodes[a] = frequent_merge(nodes[a][0], nodes[a][1], nodes[b][0], nodes[b][1], k)
        step *= 2
    s, d = nodes[0]
    rep = sorted(((x, c) for x, c in s.items() if (c + d) * k > n), key=lambda t: (-t[1], t[0]))
    return s, d, rep
