"""Seeded synthetic item streams shared by the CPU oracle and the GPU library.

Nothing here computes any part of Space Saving or COMBINE: the module only
writes uint32 item streams (Zipf with permuted or hashed ids, uniform,
adversarial) from a counter-based generator, so that the oracle and the GPU
path read byte-identical inputs.  The generator itself is C
(``streamgen.c``), built with gcc into ``libstreamgen.so`` beside it.

The paper's streams are Zipf with skew 1.1 and 1.8 and n in the billions
(Section 4, Table 1); universe, generator and seeds are unstated, so the
recipes below (``plain``, ``plain_large``, ...) are our stand-ins.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "streamgen.c")
_LIB = os.path.join(_HERE, "libstreamgen.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile streamgen.c into libstreamgen.so (host code, gcc)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-pthread", _SRC, "-o", tmp, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u64 = ctypes.c_uint64
        lib.wl_draw.restype = u64
        lib.wl_draw.argtypes = [u64, u64]
        lib.wl_fmix32.restype = ctypes.c_uint32
        lib.wl_fmix32.argtypes = [ctypes.c_uint32]
        lib.wl_permutation.argtypes = [u32p, ctypes.c_uint32, u64]
        lib.wl_zipf_perm.argtypes = [u32p, u64, ctypes.c_double, ctypes.c_uint32, u64, u64, ctypes.c_int]
        lib.wl_zipf_hashed.argtypes = [u32p, u64, ctypes.c_double, u64, u64, ctypes.c_uint32, ctypes.c_int]
        lib.wl_uniform.argtypes = [u32p, u64, u64, ctypes.c_int]
        lib.wl_adversarial.argtypes = [u32p, u64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int]
        lib.wl_zipf_ranks.argtypes = [ctypes.POINTER(ctypes.c_uint64), u64, ctypes.c_double, u64, u64]
        _lib = lib
    return _lib


def _threads(threads: int | None) -> int:
    if threads is not None:
        return max(1, int(threads))
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:  # pragma: no cover
        return max(1, min(16, os.cpu_count() or 1))


def _u32ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def draw(key: int, ctr: int) -> int:
    """The (ctr+1)-th SplitMix64 output for seed ``key`` (64-bit int)."""
    return int(_load().wl_draw(key & (2**64 - 1), ctr & (2**64 - 1)))


def fmix32(h: int) -> int:
    return int(_load().wl_fmix32(h & 0xFFFFFFFF))


def subkey(seed: int, purpose: int) -> int:
    """Independent 64-bit key for one purpose (ranks, ids, ...) of one seed."""
    return draw(0x5EED_0000_0000_0000 ^ seed, purpose)


def permutation(n_univ: int, key: int) -> np.ndarray:
    out = np.empty(n_univ, dtype=np.uint32)
    _load().wl_permutation(_u32ptr(out), n_univ, key)
    return out


def zipf_perm(n: int, alpha: float, n_univ: int, seed: int, threads: int | None = None,
              out: np.ndarray | None = None) -> np.ndarray:
    """n items: Zipf(alpha) ranks over 1..n_univ mapped through a seeded permutation."""
    if n_univ > (1 << 28):
        raise ValueError("permuted ids need n_univ <= 2^28")
    out = np.empty(n, dtype=np.uint32) if out is None else out
    rc = _load().wl_zipf_perm(_u32ptr(out), n, alpha, n_univ, subkey(seed, 1), subkey(seed, 2),
                              _threads(threads))
    if rc != 0:
        raise RuntimeError("wl_zipf_perm failed: %d" % rc)
    return out


def zipf_hashed(n: int, alpha: float, n_univ: int, seed: int, threads: int | None = None,
                out: np.ndarray | None = None) -> np.ndarray:
    """n items: Zipf(alpha) ranks over 1..n_univ (<= 2^32), id = fmix32((r-1) ^ key)."""
    out = np.empty(n, dtype=np.uint32) if out is None else out
    rc = _load().wl_zipf_hashed(_u32ptr(out), n, alpha, n_univ, subkey(seed, 1),
                                subkey(seed, 3) & 0xFFFFFFFF, _threads(threads))
    if rc != 0:
        raise RuntimeError("wl_zipf_hashed failed: %d" % rc)
    return out


def uniform(n: int, seed: int, threads: int | None = None, out: np.ndarray | None = None) -> np.ndarray:
    out = np.empty(n, dtype=np.uint32) if out is None else out
    _load().wl_uniform(_u32ptr(out), n, subkey(seed, 4), _threads(threads))
    return out


def adversarial(n: int, seed: int, d: int = 1 << 20, threads: int | None = None,
                out: np.ndarray | None = None) -> np.ndarray:
    """Round-robin over d hashed ids, planted id at positions i % 20 == 19 (5%)."""
    out = np.empty(n, dtype=np.uint32) if out is None else out
    _load().wl_adversarial(_u32ptr(out), n, d, subkey(seed, 3) & 0xFFFFFFFF, _threads(threads))
    return out


def skewed_ids(n: int, seed: int, low_bits: int = 12, high_share: float = 0.01) -> np.ndarray:
    """Ids below 2^low_bits, a high_share of them with bit 31 set: the ids
    of a level then differ in bit 31 while most share every bit above
    low_bits (a structure that defeats digit bucketing on the top bits)."""
    u = uniform(n, seed)
    flag = uniform(n, seed + 7919)
    out = u & np.uint32((1 << low_bits) - 1)
    out[flag < np.uint32(int(high_share * 2.0 ** 32))] |= np.uint32(1 << 31)
    return out


def adversarial_planted_id(seed: int, d: int = 1 << 20) -> int:
    return fmix32(d ^ (subkey(seed, 3) & 0xFFFFFFFF))


def zipf_ranks(n: int, alpha: float, n_univ: int, key: int) -> np.ndarray:
    out = np.empty(n, dtype=np.uint64)
    _load().wl_zipf_ranks(out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), n, alpha, n_univ, key)
    return out


# ----------------------------------------------------------------------------
# Workload recipes (shapes of the paper's experiments: Zipf skew, long streams, k in the thousands)
# ----------------------------------------------------------------------------

@dataclass(frozen=True)
class Stream:
    name: str
    kind: str          # "zipf_perm" | "zipf_hashed" | "uniform" | "adversarial"
    n: int
    alpha: float = 0.0
    n_univ: int = 0
    seed: int = 1

    def generate(self, threads: int | None = None, out: np.ndarray | None = None) -> np.ndarray:
        if self.kind == "zipf_perm":
            return zipf_perm(self.n, self.alpha, self.n_univ, self.seed, threads, out)
        if self.kind == "zipf_hashed":
            return zipf_hashed(self.n, self.alpha, self.n_univ, self.seed, threads, out)
        if self.kind == "uniform":
            return uniform(self.n, self.seed, threads, out)
        if self.kind == "adversarial":
            return adversarial(self.n, self.seed, threads=threads, out=out)
        raise ValueError(self.kind)


def plain(seed: int = 1, n: int = 1 << 20) -> Stream:
    """Small plain case: Zipf 1.5 over 2^20 permuted ids (k=100, 64 chunks)."""
    return Stream("plain_zipf1.5", "zipf_perm", n, 1.5, 1 << 20, seed)


def plain_large(alpha: float, seed: int = 1, n: int = 1 << 30) -> Stream:
    """Large plain case: Zipf alpha over 2^32 hashed ids (k in {500, 2000})."""
    return Stream("plain_large_zipf%g" % alpha, "zipf_hashed", n, alpha, 1 << 32, seed)


def plain_large_uniform(seed: int = 1, n: int = 1 << 30) -> Stream:
    return Stream("plain_large_uniform", "uniform", n, 0.0, 1 << 32, seed)


def plain_highk(seed: int = 1, n: int = 1 << 31) -> Stream:
    return Stream("plain_highk_zipf1.1", "zipf_hashed", n, 1.1, 1 << 32, seed)


def plain_highk_adversarial(seed: int = 1, n: int = 1 << 31) -> Stream:
    return Stream("plain_highk_adversarial", "adversarial", n, 0.0, 1 << 32, seed)


def batched(seed: int = 1, nstreams: int = 4096, log10_min: float = 3.0, log10_max: float = 7.0,
            k_min: int = 50, k_max: int = 2000):
    """Batched case: nstreams independent streams.  Stream s has length
    floor(10^(log10_min + (log10_max - log10_min) u)), Zipf alpha uniform in
    [0.8, 2.0] over 2^32 hashed ids with its own key, and k uniform in
    {k_min..k_max} (capped at its length).  Returns a list of (Stream, k)."""
    key = subkey(seed, 10)
    out = []
    for s in range(nstreams):
        u1 = (draw(key, 3 * s) >> 11) * 2.0 ** -53
        u2 = (draw(key, 3 * s + 1) >> 11) * 2.0 ** -53
        r3 = draw(key, 3 * s + 2)
        n = int(10.0 ** (log10_min + (log10_max - log10_min) * u1))
        alpha = 0.8 + 1.2 * u2
        k = min(k_min + r3 % (k_max - k_min + 1), n)
        sub = draw(key ^ 0xBA7C4ED, s)  # the stream's own seed
        out.append((Stream("batched_%d" % s, "zipf_hashed", n, alpha, 1 << 32, sub), k))
    return out


def served_append(n: int, alpha: float, summary_key: int, request_seed: int,
                  out: np.ndarray | None = None) -> np.ndarray:
    """Items of one served append: Zipf(alpha) ranks over 2^32 drawn from the
    request's own seed, mapped to ids with the target summary's key, so that
    every append to one summary draws from the same id distribution."""
    out = np.empty(n, dtype=np.uint32) if out is None else out
    rc = _load().wl_zipf_hashed(_u32ptr(out), n, alpha, 1 << 32, subkey(request_seed, 1),
                                summary_key & 0xFFFFFFFF, 1)
    if rc != 0:
        raise RuntimeError("wl_zipf_hashed failed: %d" % rc)
    return out


def served_log(seed: int = 1, nsummaries: int = 10000, nrequests: int = 20000, max_log2: float = 20.0,
               alpha: float = 1.3, append_share: float = 0.9, k_min: int = 100, k_max: int = 1000):
    """Served case: summary ks (uniform in {k_min..k_max}) and a request log.
    Each request targets a uniform summary; with probability append_share it
    is an append of floor(2^(max_log2 u)) items (log-uniform in [1, 2^max_log2])
    of Zipf(alpha) ids with that summary's key, else a query, top or majority
    with equal odds.  Returns (ks, keys, requests) with requests a list of
    ("append", sid, n, request_seed) or ("query", sid, kind)."""
    key = subkey(seed, 20)
    ks = [k_min + draw(key, s) % (k_max - k_min + 1) for s in range(nsummaries)]
    keys = [draw(key ^ 0x5E4, s) for s in range(nsummaries)]
    reqs = []
    rk = subkey(seed, 21)
    for i in range(nrequests):
        r0, r1, r2 = draw(rk, 3 * i), draw(rk, 3 * i + 1), draw(rk, 3 * i + 2)
        sid = r0 % nsummaries
        if (r1 >> 11) * 2.0 ** -53 < append_share:
            n = int(2.0 ** (max_log2 * ((r2 >> 11) * 2.0 ** -53)))
            reqs.append(("append", sid, n, draw(rk ^ 0xA99, i)))
        else:
            reqs.append(("query", sid, int(r2 & 1)))
    return ks, keys, reqs
