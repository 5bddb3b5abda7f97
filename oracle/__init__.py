"""CPU oracle for Parallel Space Saving -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never does, and the
two share no code.

``pss_oracle.c`` is a plain single-threaded C statement of Algorithm 1
(ParallelSpaceSaving) and Algorithm 2 (COMBINE) of the paper;
``frequent_oracle.c`` states the Frequent (Misra-Gries) summary the paper's
Section 2 names, its merge and the same parallel form.  This module builds
both with gcc and wraps them with ctypes.  ``brute.py`` is a second,
independent pure-Python statement used on tiny inputs.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = [os.path.join(_HERE, "pss_oracle.c"), os.path.join(_HERE, "frequent_oracle.c")]
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

# 24-byte entry: item, reserved, count, error (same layout as the C struct)
ENTRY = np.dtype([("item", "<u4"), ("reserved", "<u4"), ("count", "<u8"), ("error", "<u8")])


def build(force: bool = True) -> str:
    """Compile the oracle sources with gcc into liboracle.so (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-shared", "-fPIC", *_SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        vp = ctypes.c_void_p
        u32, u64 = ctypes.c_uint32, ctypes.c_uint64
        u32p, u64p = ctypes.POINTER(u32), ctypes.POINTER(u64)
        lib.oracle_space_saving.argtypes = [vp, u64, u32, vp, u32p, u64p]
        lib.oracle_combine.argtypes = [vp, u32, u64, vp, u32, u64, u32, vp, u32p, u64p]
        lib.oracle_summary.argtypes = [vp, u64, u32, u32, vp, u32p, u64p]
        lib.oracle_tree.argtypes = [vp, vp, vp, u32, u32]
        lib.oracle_run.argtypes = [vp, u64, u32, u32, vp, u32p]
        lib.oracle_chunk_begin.restype = u64
        lib.oracle_chunk_begin.argtypes = [u64, u32, u32]
        lib.oracle_sort_canonical.argtypes = [vp, u32]
        lib.oracle_prune_threshold.restype = u32
        lib.oracle_prune_threshold.argtypes = [vp, u32, u64, u32]
        lib.oracle_frequent.argtypes = [vp, u64, u32, vp, u32p, u64p]
        lib.oracle_frequent_merge.argtypes = [vp, u32, u64, vp, u32, u64, u32, vp, u32p, u64p]
        lib.oracle_frequent_tree.argtypes = [vp, vp, vp, u32, u32]
        lib.oracle_frequent_summary.argtypes = [vp, u64, u32, u32, vp, u32p, u64p]
        lib.oracle_frequent_report.restype = u32
        lib.oracle_frequent_report.argtypes = [vp, u32, u64, u64, u32]
        lib.oracle_frequent_run.argtypes = [vp, u64, u32, u32, vp, u32p]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _items(items) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(items, dtype=np.uint32))
    return a


class Summary:
    """A summary: entries (ENTRY array, <= k), its minimum m (0 when not
    full), k and the stream length N it covers."""

    def __init__(self, k: int, entries=None, m: int = 0, n: int = 0):
        self.k = int(k)
        self.entries = np.zeros(0, dtype=ENTRY) if entries is None else entries
        self.m = int(m)
        self.n = int(n)

    def canonical(self) -> np.ndarray:
        e = self.entries.copy()
        if len(e):
            _load().oracle_sort_canonical(_ptr(e), len(e))
        return e

    def as_tuples(self):
        return [(int(e["item"]), int(e["count"]), int(e["error"])) for e in self.canonical()]

    def query_majority(self) -> np.ndarray:
        """Entries with count * k > N in canonical order (Algorithm 1, Pruned)."""
        e = self.entries.copy()
        q = _load().oracle_prune_threshold(_ptr(e), len(e), self.n, self.k) if len(e) else 0
        return e[:q]

    def query_topk(self, t: int) -> np.ndarray:
        return self.canonical()[:t]

    # S <- COMBINE(S, tree(batch)); an empty S is COMBINE's identity
    def update(self, items, chunks: int) -> "Summary":
        b = summary(items, self.k, chunks)
        merged = combine(self, b)
        merged.n = self.n + b.n
        self.entries, self.m, self.n = merged.entries, merged.m, merged.n
        return self

    def merge(self, other: "Summary") -> "Summary":
        if other.k != self.k:
            raise ValueError("k mismatch")
        merged = combine(self, other)
        self.entries, self.m, self.n = merged.entries, merged.m, self.n + other.n
        return self


def space_saving(items, k: int) -> Summary:
    """Sequential Space Saving over items with k counters (Section 3)."""
    a = _items(items)
    out = np.zeros(max(k, 1), dtype=ENTRY)
    size, m = ctypes.c_uint32(), ctypes.c_uint64()
    rc = _load().oracle_space_saving(_ptr(a), len(a), k, _ptr(out), ctypes.byref(size), ctypes.byref(m))
    if rc != 0:
        raise RuntimeError("oracle_space_saving: %d" % rc)
    return Summary(k, out[: size.value].copy(), m.value, len(a))


def combine(s1: Summary, s2: Summary) -> Summary:
    """COMBINE(S1, S2) with Prune(k) (Algorithm 2)."""
    k = s1.k
    e1 = np.ascontiguousarray(s1.entries)
    e2 = np.ascontiguousarray(s2.entries)
    out = np.zeros(max(k, 1), dtype=ENTRY)
    nout, mout = ctypes.c_uint32(), ctypes.c_uint64()
    rc = _load().oracle_combine(_ptr(e1), len(e1), s1.m, _ptr(e2), len(e2), s2.m, k, _ptr(out),
                                ctypes.byref(nout), ctypes.byref(mout))
    if rc != 0:
        raise RuntimeError("oracle_combine: %d" % rc)
    return Summary(k, out[: nout.value].copy(), mout.value, s1.n + s2.n)


def chunk_bounds(n: int, chunks: int):
    lib = _load()
    return [(int(lib.oracle_chunk_begin(n, chunks, c)), int(lib.oracle_chunk_begin(n, chunks, c + 1)))
            for c in range(chunks)]


def chunk_summaries(items, k: int, chunks: int, which=None):
    """Space Saving summary of each chunk (or of the chunks listed in which)."""
    a = _items(items)
    bounds = chunk_bounds(len(a), chunks)
    idx = range(chunks) if which is None else which
    return {c: space_saving(a[bounds[c][0]:bounds[c][1]], k) for c in idx}


def tree(summaries, k: int) -> Summary:
    """Fixed binary COMBINE tree over a list of summaries in chunk order."""
    count = len(summaries)
    ent = np.zeros(max(k * count, 1), dtype=ENTRY)
    size = np.zeros(count, dtype=np.uint32)
    mins = np.zeros(count, dtype=np.uint64)
    total = 0
    for i, s in enumerate(summaries):
        ent[i * k: i * k + len(s.entries)] = s.entries
        size[i] = len(s.entries)
        mins[i] = s.m
        total += s.n
    rc = _load().oracle_tree(_ptr(ent), _ptr(size), _ptr(mins), count, k)
    if rc != 0:
        raise RuntimeError("oracle_tree: %d" % rc)
    return Summary(k, ent[: size[0]].copy(), int(mins[0]), total)


def summary(items, k: int, chunks: int) -> Summary:
    """Algorithm 1 up to the reduction: partition, per-chunk summaries, tree."""
    a = _items(items)
    out = np.zeros(max(k, 1), dtype=ENTRY)
    nout, mout = ctypes.c_uint32(), ctypes.c_uint64()
    rc = _load().oracle_summary(_ptr(a), len(a), k, chunks, _ptr(out), ctypes.byref(nout), ctypes.byref(mout))
    if rc != 0:
        raise RuntimeError("oracle_summary: %d" % rc)
    return Summary(k, out[: nout.value].copy(), mout.value, len(a))


def run(items, k: int, chunks: int) -> np.ndarray:
    """ParallelSpaceSaving: the reported k-majority candidates, canonical order."""
    a = _items(items)
    if k < 2 or k > len(a):
        raise ValueError("need 2 <= k <= n")
    out = np.zeros(k, dtype=ENTRY)
    nout = ctypes.c_uint32()
    rc = _load().oracle_run(_ptr(a), len(a), k, chunks, _ptr(out), ctypes.byref(nout))
    if rc != 0:
        raise RuntimeError("oracle_run: %d" % rc)
    return out[: nout.value].copy()


def summary_threads(items, k: int, chunks: int, threads: int) -> Summary:
    """summary() with the chunk summaries computed by `threads` threads (the
    paper's shared-memory form, Section 3: each thread summarises its own
    chunks with the same sequential Space Saving), then the fixed tree on one
    thread.  Equal to summary() by construction: the chunks and the tree are
    the same, only the order in which chunk summaries are computed differs."""
    from concurrent.futures import ThreadPoolExecutor

    a = _items(items)
    bounds = chunk_bounds(len(a), chunks)

    def one(c):
        b0, b1 = bounds[c]
        return space_saving(a[b0:b1], k)

    with ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
        sums = list(ex.map(one, range(chunks)))
    return tree(sums, k)


def run_threads(items, k: int, chunks: int, threads: int) -> np.ndarray:
    """run() on top of summary_threads()."""
    a = _items(items)
    if k < 2 or k > len(a):
        raise ValueError("need 2 <= k <= n")
    s = summary_threads(a, k, chunks, threads)
    s.n = len(a)
    return s.query_majority()


# ---------------------------------------------------------------------------
# Frequent (Misra-Gries) for the k-majority problem (k - 1 counters), its
# merge and the parallel form
# ---------------------------------------------------------------------------

class FSummary:
    """A Frequent summary: entries (item, count; error 0), the number D of
    decrement steps it absorbed (f - D <= count <= f), k and N."""

    def __init__(self, k: int, entries=None, d: int = 0, n: int = 0):
        self.k = int(k)
        self.entries = np.zeros(0, dtype=ENTRY) if entries is None else entries
        self.d = int(d)
        self.n = int(n)

    def as_pairs(self):
        """(item, count) sorted by count descending, item ascending."""
        return sorted(((int(e["item"]), int(e["count"])) for e in self.entries), key=lambda t: (-t[1], t[0]))

    def report(self) -> np.ndarray:
        e = self.entries.copy()
        q = _load().oracle_frequent_report(_ptr(e), len(e), self.d, self.n, self.k) if len(e) else 0
        return e[:q]


def frequent(items, k: int) -> FSummary:
    """Sequential Frequent (Misra-Gries) over items, k - 1 counters."""
    a = _items(items)
    out = np.zeros(max(k, 1), dtype=ENTRY)
    size, d = ctypes.c_uint32(), ctypes.c_uint64()
    rc = _load().oracle_frequent(_ptr(a), len(a), k, _ptr(out), ctypes.byref(size), ctypes.byref(d))
    if rc != 0:
        raise RuntimeError("oracle_frequent: %d" % rc)
    return FSummary(k, out[: size.value].copy(), d.value, len(a))


def frequent_merge(s1: FSummary, s2: FSummary) -> FSummary:
    k = s1.k
    e1, e2 = np.ascontiguousarray(s1.entries), np.ascontiguousarray(s2.entries)
    out = np.zeros(max(len(e1) + len(e2), 1), dtype=ENTRY)
    nout, dout = ctypes.c_uint32(), ctypes.c_uint64()
    rc = _load().oracle_frequent_merge(_ptr(e1), len(e1), s1.d, _ptr(e2), len(e2), s2.d, k, _ptr(out),
                                       ctypes.byref(nout), ctypes.byref(dout))
    if rc != 0:
        raise RuntimeError("oracle_frequent_merge: %d" % rc)
    return FSummary(k, out[: nout.value].copy(), dout.value, s1.n + s2.n)


def frequent_chunk_summaries(items, k: int, chunks: int, which=None):
    a = _items(items)
    bounds = chunk_bounds(len(a), chunks)
    idx = range(chunks) if which is None else which
    return {c: frequent(a[bounds[c][0]:bounds[c][1]], k) for c in idx}


def frequent_tree(summaries, k: int) -> FSummary:
    count = len(summaries)
    ent = np.zeros(max(k * count, 1), dtype=ENTRY)
    size = np.zeros(count, dtype=np.uint32)
    dec = np.zeros(count, dtype=np.uint64)
    total = 0
    for i, s in enumerate(summaries):
        ent[i * k: i * k + len(s.entries)] = s.entries
        size[i] = len(s.entries)
        dec[i] = s.d
        total += s.n
    rc = _load().oracle_frequent_tree(_ptr(ent), _ptr(size), _ptr(dec), count, k)
    if rc != 0:
        raise RuntimeError("oracle_frequent_tree: %d" % rc)
    return FSummary(k, ent[: size[0]].copy(), int(dec[0]), total)


def frequent_summary(items, k: int, chunks: int) -> FSummary:
    a = _items(items)
    out = np.zeros(max(k, 1), dtype=ENTRY)
    nout, dout = ctypes.c_uint32(), ctypes.c_uint64()
    rc = _load().oracle_frequent_summary(_ptr(a), len(a), k, chunks, _ptr(out), ctypes.byref(nout),
                                         ctypes.byref(dout))
    if rc != 0:
        raise RuntimeError("oracle_frequent_summary: %d" % rc)
    return FSummary(k, out[: nout.value].copy(), dout.value, len(a))


def frequent_run(items, k: int, chunks: int) -> np.ndarray:
    """The parallel Frequent report: monitored items with (count + D) * k > n,
    count descending, item ascending."""
    a = _items(items)
    out = np.zeros(max(k, 1), dtype=ENTRY)
    nout = ctypes.c_uint32()
    rc = _load().oracle_frequent_run(_ptr(a), len(a), k, chunks, _ptr(out), ctypes.byref(nout))
    if rc != 0:
        raise RuntimeError("oracle_frequent_run: %d" % rc)
    return out[: nout.value].copy()


def frequent_summary_threads(items, k: int, chunks: int, threads: int) -> FSummary:
    """frequent_summary with the chunk summaries on `threads` threads."""
    from concurrent.futures import ThreadPoolExecutor

    a = _items(items)
    bounds = chunk_bounds(len(a), chunks)
    with ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
        sums = list(ex.map(lambda c: frequent(a[bounds[c][0]:bounds[c][1]], k), range(chunks)))
    return frequent_tree(sums, k)


def to_tuples(entries: np.ndarray):
    return [(int(e["item"]), int(e["count"]), int(e["error"])) for e in entries]
