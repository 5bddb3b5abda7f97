"""ctypes binding of libpss (include/pss.h): argument marshalling only.

Device buffers and streams come from PyTorch (ROCm): ``d_items`` is a
contiguous int32/uint32 tensor on a HIP device, ``stream`` a
``torch.cuda.Stream`` (default: the current stream).  Every step of the path
runs in the library's HIP kernels; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch  # noqa: F401  -- load torch's HIP runtime before libpss binds to one

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpss.so")

PSS_OK, PSS_EINVAL, PSS_ERANGE, PSS_ENOMEM, PSS_EBUSY, PSS_ETRUNC, PSS_EDEVICE = 0, -1, -2, -3, -4, -5, -6
PSS_Q_MAJORITY, PSS_Q_TOPK = 0, 1

# pss_entry: item u32, reserved u32, count u64, error u64 (24 bytes)
ENTRY_DTYPE = np.dtype([("item", "<u4"), ("reserved", "<u4"), ("count", "<u8"), ("error", "<u8")])


class BatchInfo(ctypes.Structure):
    """pss_batch_info_t"""
    _fields_ = [("nstreams", ctypes.c_uint32), ("nblocks", ctypes.c_uint32), ("nlevels", ctypes.c_uint32),
                ("nclasses", ctypes.c_uint32), ("target_len", ctypes.c_uint64), ("slots_x16", ctypes.c_uint32),
                ("waves_per_group", ctypes.c_uint32), ("tune_candidates", ctypes.c_uint32),
                ("tune_ms", ctypes.c_double), ("report_entries", ctypes.c_uint64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ServerOpts(ctypes.Structure):
    """pss_server_opts"""
    _fields_ = [("hbm_budget", ctypes.c_uint64), ("slots", ctypes.c_uint32), ("max_requests", ctypes.c_uint32),
                ("block_len", ctypes.c_uint64), ("stage_bytes", ctypes.c_uint64)]


class ServerResult(ctypes.Structure):
    """pss_server_result"""
    _fields_ = [("status", ctypes.c_int), ("n_out", ctypes.c_uint32), ("stream_len", ctypes.c_uint64),
                ("chunks_used", ctypes.c_uint32), ("launch", ctypes.c_uint32), ("latency_ms", ctypes.c_double),
                ("queue_ms", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ServerStats(ctypes.Structure):
    """pss_server_stats_t"""
    _fields_ = [("launches", ctypes.c_uint64), ("requests", ctypes.c_uint64), ("items_appended", ctypes.c_uint64),
                ("max_launch_requests", ctypes.c_uint32), ("pending", ctypes.c_uint32), ("status", ctypes.c_int),
                ("stage_ms", ctypes.c_double), ("gpu_ms", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class PssError(RuntimeError):
    def __init__(self, code: int, what: str, required: int | None = None):
        self.code = code
        self.required = required
        super().__init__("%s: %s (%d)" % (what, strerror(code), code))


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libpss.so is not built: run __graft_entry__.build() (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        u32p, u64p = ctypes.POINTER(u32), ctypes.POINTER(u64)
        L.pss_strerror.restype = ctypes.c_char_p
        L.pss_strerror.argtypes = [i32]
        L.pss_last_device_error.restype = i32
        L.pss_last_device_error.argtypes = []
        L.pss_device_error_name.restype = ctypes.c_char_p
        L.pss_device_error_name.argtypes = [i32]
        L.pss_ctx_create.argtypes = [i32, ctypes.POINTER(vp)]
        L.pss_ctx_destroy.argtypes = [vp]
        L.pss_ctx_destroy.restype = None
        L.pss_max_k.restype = u32
        L.pss_max_k.argtypes = [vp]
        L.pss_max_lds_k.restype = u32
        L.pss_max_lds_k.argtypes = [vp]
        L.pss_plan_chunks.restype = u32
        L.pss_plan_chunks.argtypes = [vp, u64, u32]
        L.pss_create.argtypes = [vp, u32, ctypes.POINTER(vp)]
        L.pss_destroy.argtypes = [vp]
        L.pss_destroy.restype = None
        L.pss_update.argtypes = [vp, vp, u64, u32, vp, u32p]
        L.pss_merge.argtypes = [vp, vp, vp]
        L.pss_query.argtypes = [vp, i32, vp, u32, u32p, u64p, vp]
        L.pss_run.argtypes = [vp, vp, u64, u32, u32, vp, u32, u32p, u32p, vp]
        L.pss_block_summaries.argtypes = [vp, vp, u64, u32, u32, u32p, u32, vp, u32p, u64p, vp]
        L.pss_ctx_set_budget.argtypes = [vp, u64]
        L.pss_read_bandwidth.argtypes = [vp, vp, u64, u32, vp, ctypes.POINTER(ctypes.c_double)]
        L.pss_frequent_max_k.restype = u32
        L.pss_frequent_max_k.argtypes = [vp]
        L.pss_frequent_plan_chunks.restype = u32
        L.pss_frequent_plan_chunks.argtypes = [vp, u64, u32]
        L.pss_frequent_run.argtypes = [vp, vp, u64, u32, u32, i32, vp, u32, u32p, u64p, u32p, vp]
        L.pss_frequent_block_summaries.argtypes = [vp, vp, u64, u32, u32, u32p, u32, vp, u32p, u64p, vp]
        L.pss_tune_chunks.argtypes = [vp, vp, u64, u32, vp, u32p, ctypes.POINTER(ctypes.c_double)]
        L.pss_run_noalloc.argtypes = [vp, u64, u32, u32, vp, u32, vp, u32p, vp]
        L.pss_noalloc_scratch_bytes.restype = u64
        L.pss_noalloc_scratch_bytes.argtypes = []
        L.pss_test_fold_failed_block.argtypes = [vp, u64, vp]
        L.pss_batch_max_k.restype = u32
        L.pss_batch_max_k.argtypes = [vp]
        L.pss_batch_create.argtypes = [vp, u32, vp, u64p, u32p, u32p, i32, ctypes.POINTER(vp)]
        L.pss_batch_run.argtypes = [vp, i32, vp, u32p, vp]
        L.pss_batch_info.argtypes = [vp, ctypes.POINTER(BatchInfo)]
        L.pss_batch_destroy.argtypes = [vp]
        L.pss_batch_destroy.restype = None
        L.pss_run_batched.argtypes = [vp, u32, vp, u64p, u32p, u32p, vp, u32p, vp]
        L.pss_server_max_k.restype = u32
        L.pss_server_max_k.argtypes = [vp]
        L.pss_server_create.argtypes = [vp, u32, u32p, ctypes.POINTER(ServerOpts), ctypes.POINTER(vp)]
        L.pss_server_destroy.argtypes = [vp]
        L.pss_server_destroy.restype = None
        L.pss_server_append.argtypes = [vp, u32, vp, u64, u32, u64p]
        L.pss_server_query.argtypes = [vp, u32, i32, u32, u64p]
        L.pss_server_wait.argtypes = [vp, u64, vp, u32, ctypes.POINTER(ServerResult)]
        L.pss_server_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
        L.pss_timing_enable.argtypes = [vp, i32]
        L.pss_phase_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double), u32p, i32]
        for f in ("pss_timing_enable", "pss_phase_times", "pss_ctx_create", "pss_create", "pss_update", "pss_merge",
                  "pss_query", "pss_run", "pss_block_summaries", "pss_batch_create", "pss_batch_run", "pss_batch_info",
                  "pss_run_batched", "pss_server_create", "pss_server_append", "pss_server_query", "pss_server_wait",
                  "pss_server_stats", "pss_ctx_set_budget", "pss_test_fold_failed_block", "pss_tune_chunks", "pss_read_bandwidth", "pss_frequent_run",
                  "pss_frequent_block_summaries", "pss_run_noalloc"):
            getattr(L, f).restype = i32
        _lib = L
    return _lib


def strerror(code: int) -> str:
    return lib().pss_strerror(code).decode()


def last_device_error() -> tuple[int, str]:
    """The HIP error behind this thread's last PSS_EDEVICE from a launch."""
    e = lib().pss_last_device_error()
    return e, lib().pss_device_error_name(e).decode()


def _check(rc: int, what: str, required: int | None = None):
    if rc != PSS_OK:
        if rc == PSS_EDEVICE:
            e, name = last_device_error()
            if e:
                what = "%s [%s]" % (what, name)
        raise PssError(rc, what, required)


def _stream(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _items(d_items):
    if not isinstance(d_items, torch.Tensor):
        raise TypeError("d_items must be a torch tensor on a HIP device")
    if d_items.dtype not in (torch.int32, torch.uint32):
        raise TypeError("d_items must hold 32-bit items (int32 or uint32)")
    if not d_items.is_cuda or not d_items.is_contiguous():
        raise ValueError("d_items must be a contiguous device tensor")
    return ctypes.c_void_p(d_items.data_ptr()), d_items.numel()


class Context:
    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        _check(lib().pss_ctx_create(device, ctypes.byref(h)), "pss_ctx_create")
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            lib().pss_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def max_k(self) -> int:
        return int(lib().pss_max_k(self.handle))

    @property
    def max_lds_k(self) -> int:
        return int(lib().pss_max_lds_k(self.handle))

    @property
    def server_max_k(self) -> int:
        return int(lib().pss_server_max_k(self.handle))

    @property
    def batch_max_k(self) -> int:
        return int(lib().pss_batch_max_k(self.handle))

    def plan_chunks(self, n: int, k: int) -> int:
        return int(lib().pss_plan_chunks(self.handle, n, k))

    def tune_chunks(self, d_items, k: int, stream=None, n: int | None = None):
        """pss_tune_chunks: (chunk count, ms of blocks + tree at that count)."""
        ptr, numel = _items(d_items)
        n = numel if n is None else n
        best, ms = ctypes.c_uint32(), ctypes.c_double()
        _check(lib().pss_tune_chunks(self.handle, ptr, n, k, ctypes.c_void_p(_stream(stream)), ctypes.byref(best),
                                     ctypes.byref(ms)), "pss_tune_chunks")
        return int(best.value), float(ms.value)

    def read_bandwidth(self, d_buf, reps: int = 5, stream=None) -> float:
        """pss_read_bandwidth over a contiguous device tensor: GB/s."""
        if not isinstance(d_buf, torch.Tensor) or not d_buf.is_cuda or not d_buf.is_contiguous():
            raise TypeError("d_buf must be a contiguous device tensor")
        g = ctypes.c_double()
        _check(lib().pss_read_bandwidth(self.handle, ctypes.c_void_p(d_buf.data_ptr()),
                                        d_buf.numel() * d_buf.element_size(), reps,
                                        ctypes.c_void_p(_stream(stream)), ctypes.byref(g)), "pss_read_bandwidth")
        return float(g.value)

    @property
    def frequent_max_k(self) -> int:
        return int(lib().pss_frequent_max_k(self.handle))

    def frequent_plan_chunks(self, n: int, k: int) -> int:
        return int(lib().pss_frequent_plan_chunks(self.handle, n, k))

    def set_budget(self, nbytes: int):
        """Device bytes the context's workspaces may hold in all (0 = no limit)."""
        _check(lib().pss_ctx_set_budget(self.handle, nbytes), "pss_ctx_set_budget")

    def timing(self, enable: bool):
        _check(lib().pss_timing_enable(self.handle, 1 if enable else 0), "pss_timing_enable")

    def phase_times(self, reset: bool = True):
        """(ms[4], launches[4]) for block summaries, tree, fold, report."""
        ms = (ctypes.c_double * 4)()
        nl = (ctypes.c_uint32 * 4)()
        _check(lib().pss_phase_times(self.handle, ms, nl, 1 if reset else 0), "pss_phase_times")
        return list(ms), list(nl)


def pss_ctx_create(device: int = 0) -> Context:
    return Context(device)


def pss_ctx_destroy(ctx: Context):
    ctx.close()


class Summary:
    def __init__(self, ctx: Context, k: int):
        h = ctypes.c_void_p()
        _check(lib().pss_create(ctx.handle, k, ctypes.byref(h)), "pss_create")
        self.handle = h
        self.ctx = ctx
        self.k = k

    def close(self):
        if self.handle:
            lib().pss_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pss_create(ctx: Context, k: int) -> Summary:
    return Summary(ctx, k)


def pss_destroy(s: Summary):
    s.close()


def pss_update(s: Summary, d_items, chunks: int = 0, stream=None, n: int | None = None) -> int:
    """Append d_items[:n] to s; returns the chunk count used."""
    ptr, numel = _items(d_items)
    n = numel if n is None else n
    used = ctypes.c_uint32()
    _check(lib().pss_update(s.handle, ptr, n, chunks, ctypes.c_void_p(_stream(stream)), ctypes.byref(used)),
           "pss_update")
    return int(used.value)


def pss_merge(dst: Summary, src: Summary, stream=None):
    _check(lib().pss_merge(dst.handle, src.handle, ctypes.c_void_p(_stream(stream))), "pss_merge")


def pss_query(s: Summary, kind: int = PSS_Q_MAJORITY, cap: int | None = None, stream=None):
    """Returns (entries as a numpy ENTRY_DTYPE array, stream length N)."""
    cap = s.k if cap is None else cap
    out = np.zeros(max(cap, 1), dtype=ENTRY_DTYPE)
    nout, slen = ctypes.c_uint32(), ctypes.c_uint64()
    rc = lib().pss_query(s.handle, kind, out.ctypes.data_as(ctypes.c_void_p), cap, ctypes.byref(nout),
                         ctypes.byref(slen), ctypes.c_void_p(_stream(stream)))
    _check(rc, "pss_query", int(nout.value))
    return out[: min(int(nout.value), cap)].copy(), int(slen.value)


def pss_run_noalloc(d_items, k: int, d_out, d_nout, chunks: int = 0, stream=None, n: int | None = None) -> int:
    """pss_run without allocation: results stay on the device (d_out: a
    contiguous uint8 tensor of cap * 24 bytes, d_nout: one int32/uint32);
    returns the chunk count used.  Asynchronous on `stream`."""
    ptr, numel = _items(d_items)
    n = numel if n is None else n
    for t in (d_out, d_nout):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
            raise TypeError("d_out and d_nout must be contiguous device tensors")
    if d_out.numel() * d_out.element_size() % ENTRY_DTYPE.itemsize:
        raise ValueError("d_out must hold a whole number of 24-byte entries")
    cap = d_out.numel() * d_out.element_size() // ENTRY_DTYPE.itemsize
    used = ctypes.c_uint32()
    _check(lib().pss_run_noalloc(ptr, n, k, chunks, ctypes.c_void_p(d_out.data_ptr()), cap,
                                 ctypes.c_void_p(d_nout.data_ptr()), ctypes.byref(used),
                                 ctypes.c_void_p(_stream(stream))), "pss_run_noalloc")
    return int(used.value)


def noalloc_scratch_bytes() -> int:
    return int(lib().pss_noalloc_scratch_bytes())


def entries_from_bytes(raw: np.ndarray, count: int) -> np.ndarray:
    """The first `count` entries of a byte array holding pss_entry records."""
    return np.frombuffer(np.ascontiguousarray(raw).tobytes(), dtype=ENTRY_DTYPE)[:count].copy()


def pss_frequent_run(ctx: Context, d_items, k: int, chunks: int = 0, kind: int = PSS_Q_MAJORITY,
                     cap: int | None = None, stream=None, n: int | None = None):
    """Parallel Frequent: (entries, D, chunk count used)."""
    ptr, numel = _items(d_items)
    n = numel if n is None else n
    cap = k if cap is None else cap
    out = np.zeros(max(cap, 1), dtype=ENTRY_DTYPE)
    nout, dec, used = ctypes.c_uint32(), ctypes.c_uint64(), ctypes.c_uint32()
    rc = lib().pss_frequent_run(ctx.handle, ptr, n, k, chunks, kind, out.ctypes.data_as(ctypes.c_void_p), cap,
                                ctypes.byref(nout), ctypes.byref(dec), ctypes.byref(used),
                                ctypes.c_void_p(_stream(stream)))
    _check(rc, "pss_frequent_run", int(nout.value))
    return out[: min(int(nout.value), cap)].copy(), int(dec.value), int(used.value)


def pss_frequent_block_summaries(ctx: Context, d_items, k: int, chunks: int, sel, stream=None,
                                 n: int | None = None):
    """Frequent summaries of the blocks listed in sel: list of (entries, D)."""
    ptr, numel = _items(d_items)
    n = numel if n is None else n
    sel = np.ascontiguousarray(np.asarray(sel, dtype=np.uint32))
    out = np.zeros(max(len(sel) * k, 1), dtype=ENTRY_DTYPE)
    sizes = np.zeros(max(len(sel), 1), dtype=np.uint32)
    decs = np.zeros(max(len(sel), 1), dtype=np.uint64)
    rc = lib().pss_frequent_block_summaries(ctx.handle, ptr, n, k, chunks,
                                            sel.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), len(sel),
                                            out.ctypes.data_as(ctypes.c_void_p),
                                            sizes.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                            decs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                            ctypes.c_void_p(_stream(stream)))
    _check(rc, "pss_frequent_block_summaries")
    return [(out[i * k: i * k + int(sizes[i])].copy(), int(decs[i])) for i in range(len(sel))]


def pss_test_fold_failed_block(s: Summary, n: int, stream=None):
    """Test hook: fold a block summary carrying the failure mark into s."""
    _check(lib().pss_test_fold_failed_block(s.handle, n, ctypes.c_void_p(_stream(stream))),
           "pss_test_fold_failed_block")


def pss_run(ctx: Context, d_items, k: int, chunks: int = 0, cap: int | None = None, stream=None,
            n: int | None = None):
    """Algorithm 1 in one call: (reported entries, chunk count used)."""
    ptr, numel = _items(d_items)
    n = numel if n is None else n
    cap = k if cap is None else cap
    out = np.zeros(max(cap, 1), dtype=ENTRY_DTYPE)
    nout, used = ctypes.c_uint32(), ctypes.c_uint32()
    rc = lib().pss_run(ctx.handle, ptr, n, k, chunks, out.ctypes.data_as(ctypes.c_void_p), cap,
                       ctypes.byref(nout), ctypes.byref(used), ctypes.c_void_p(_stream(stream)))
    _check(rc, "pss_run", int(nout.value))
    return out[: int(nout.value)].copy(), int(used.value)


def pss_block_summaries(ctx: Context, d_items, k: int, chunks: int, sel, stream=None, n: int | None = None):
    """Summaries of the blocks listed in sel: list of (entries, minimum)."""
    ptr, numel = _items(d_items)
    n = numel if n is None else n
    sel = np.ascontiguousarray(np.asarray(sel, dtype=np.uint32))
    out = np.zeros(max(len(sel) * k, 1), dtype=ENTRY_DTYPE)
    sizes = np.zeros(max(len(sel), 1), dtype=np.uint32)
    mins = np.zeros(max(len(sel), 1), dtype=np.uint64)
    rc = lib().pss_block_summaries(ctx.handle, ptr, n, k, chunks,
                                   sel.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), len(sel),
                                   out.ctypes.data_as(ctypes.c_void_p),
                                   sizes.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                   mins.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                   ctypes.c_void_p(_stream(stream)))
    _check(rc, "pss_block_summaries")
    return [(out[i * k: i * k + int(sizes[i])].copy(), int(mins[i])) for i in range(len(sel))]


def _batch_arrays(streams, ks, chunks):
    ptrs, lens = [], []
    for d in streams:
        p, n = _items(d)
        ptrs.append(p.value)
        lens.append(n)
    ns = len(ptrs)
    if len(ks) != ns:
        raise ValueError("one k per stream")
    a_ptr = (ctypes.c_void_p * ns)(*ptrs)
    a_len = np.ascontiguousarray(np.asarray(lens, dtype=np.uint64))
    a_k = np.ascontiguousarray(np.asarray(ks, dtype=np.uint32))
    a_c = np.ascontiguousarray(np.zeros(ns, dtype=np.uint32) if chunks is None else np.asarray(chunks, dtype=np.uint32))
    return ns, a_ptr, a_len, a_k, a_c


def _split_reports(out, counts, ks):
    res, o = [], 0
    for s, k in enumerate(ks):
        res.append(out[o: o + int(counts[s])].copy())
        o += int(k)
    return res


class Batch:
    """pss_batch: the streams (device tensors, kept referenced for the life of
    the batch), their k and, optionally, their chunk counts (None or 0 entries:
    chosen by the autotuner)."""

    def __init__(self, ctx: Context, streams, ks, chunks=None, tune: bool = False):
        self.streams = list(streams)
        ns, a_ptr, a_len, a_k, a_c = _batch_arrays(self.streams, ks, chunks)
        h = ctypes.c_void_p()
        _check(lib().pss_batch_create(ctx.handle, ns, a_ptr, a_len.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                      a_k.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                      a_c.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), 1 if tune else 0,
                                      ctypes.byref(h)), "pss_batch_create")
        self.handle = h
        self.ctx = ctx
        self.ks = [int(k) for k in a_k]
        self.chunks = [int(c) for c in a_c]
        self._out = np.zeros(max(1, int(a_k.sum(dtype=np.uint64))), dtype=ENTRY_DTYPE)
        self._counts = np.zeros(ns, dtype=np.uint32)

    def run(self, eager: bool = False, stream=None):
        """Per-stream reported entries (list of ENTRY_DTYPE arrays)."""
        _check(lib().pss_batch_run(self.handle, 1 if eager else 0, self._out.ctypes.data_as(ctypes.c_void_p),
                                   self._counts.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                   ctypes.c_void_p(_stream(stream))), "pss_batch_run")
        return _split_reports(self._out, self._counts, self.ks)

    def info(self) -> dict:
        i = BatchInfo()
        _check(lib().pss_batch_info(self.handle, ctypes.byref(i)), "pss_batch_info")
        return i.as_dict()

    def close(self):
        if self.handle:
            lib().pss_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pss_batch_create(ctx: Context, streams, ks, chunks=None, tune: bool = False) -> Batch:
    return Batch(ctx, streams, ks, chunks, tune)


def pss_batch_run(b: Batch, eager: bool = False, stream=None):
    return b.run(eager, stream)


def pss_batch_destroy(b: Batch):
    b.close()


def pss_run_batched(ctx: Context, streams, ks, chunks=None, stream=None):
    """One-shot batch: (per-stream reports, chunk counts used)."""
    streams = list(streams)
    ns, a_ptr, a_len, a_k, a_c = _batch_arrays(streams, ks, chunks)
    out = np.zeros(max(1, int(a_k.sum(dtype=np.uint64))), dtype=ENTRY_DTYPE)
    counts = np.zeros(ns, dtype=np.uint32)
    _check(lib().pss_run_batched(ctx.handle, ns, a_ptr, a_len.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                 a_k.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                 a_c.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                 out.ctypes.data_as(ctypes.c_void_p),
                                 counts.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                 ctypes.c_void_p(_stream(stream))), "pss_run_batched")
    return _split_reports(out, counts, [int(k) for k in a_k]), [int(c) for c in a_c]


class Server:
    """pss_server: a pool of device-resident summaries (one per k in ks) served
    by the library's request loop.  Appends take host uint32 arrays, kept
    referenced here until their ticket is waited for."""

    def __init__(self, ctx: Context, ks, hbm_budget: int = 0, slots: int = 0, max_requests: int = 0,
                 block_len: int = 0, stage_bytes: int = 0):
        a_k = np.ascontiguousarray(np.asarray(ks, dtype=np.uint32))
        opts = ServerOpts(hbm_budget, slots, max_requests, block_len, stage_bytes)
        h = ctypes.c_void_p()
        _check(lib().pss_server_create(ctx.handle, len(a_k), a_k.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                       ctypes.byref(opts), ctypes.byref(h)), "pss_server_create")
        self.handle = h
        self.ctx = ctx
        self.ks = [int(k) for k in a_k]
        self._hold = {}

    def append(self, sid: int, items, chunks: int = 0) -> int:
        a = np.ascontiguousarray(np.asarray(items, dtype=np.uint32))
        t = ctypes.c_uint64()
        _check(lib().pss_server_append(self.handle, sid, a.ctypes.data_as(ctypes.c_void_p), len(a), chunks,
                                       ctypes.byref(t)), "pss_server_append")
        self._hold[int(t.value)] = a
        return int(t.value)

    def query(self, sid: int, kind: int = PSS_Q_MAJORITY, cap: int | None = None) -> int:
        t = ctypes.c_uint64()
        cap = self.ks[sid] if cap is None else cap
        _check(lib().pss_server_query(self.handle, sid, kind, cap, ctypes.byref(t)), "pss_server_query")
        return int(t.value)

    def wait(self, ticket: int, cap: int | None = None):
        """(entries, result dict); entries is empty for an append."""
        cap = max(self.ks) if cap is None else cap
        out = np.zeros(max(cap, 1), dtype=ENTRY_DTYPE)
        res = ServerResult()
        rc = lib().pss_server_wait(self.handle, ticket, out.ctypes.data_as(ctypes.c_void_p), cap, ctypes.byref(res))
        self._hold.pop(ticket, None)
        _check(rc, "pss_server_wait", int(res.n_out))
        return out[: min(int(res.n_out), cap)].copy(), res.as_dict()

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().pss_server_stats(self.handle, ctypes.byref(st)), "pss_server_stats")
        return st.as_dict()

    def close(self):
        if self.handle:
            lib().pss_server_destroy(self.handle)
            self.handle = None
            self._hold.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def to_tuples(entries):
    return [(int(e["item"]), int(e["count"]), int(e["error"])) for e in entries]
