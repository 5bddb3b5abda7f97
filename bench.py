#!/usr/bin/env python3
"""Throughput of the Parallel Space Saving hot path on one MI355X.

One step = one pass of the whole path (block summaries -> fixed COMBINE tree
-> fold -> report, Algorithm 1 with Algorithm 2 as the reduction operator)
over every case of the workload.  Default workload "plain-large": four
streams of n = 2^30 uint32 items resident in HBM -- Zipf alpha 0.8, 1.2, 1.8
over 2^32 hashed ids and a uniform control -- each summarised with k = 500
and k = 2000 counters, chunk count picked by the library's planner and
recorded.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
METRIC = "G items/s + % HBM-read roofline (1 GPU); batched/served vs plain; p99 latency"
# HBM traffic of the block kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE runs,
# valid only while the kernel source is the one the counters were taken on
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "chunk_summary_plain_large_traffic.txt")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1606_04669_amd", "csrc", "chunk_summary.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in (KERNEL_SOURCE, os.path.join(os.path.dirname(KERNEL_SOURCE), "pss_layout.h"),
              os.path.join(os.path.dirname(KERNEL_SOURCE), "pss_device.h"),
              os.path.join(os.path.dirname(KERNEL_SOURCE), "pss_table.h")):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload: str, n_log2: int, k: int, split: bool = False):
    """HBM bytes per launch of the block kernel's instance for k, from the
    committed counter runs (split: [read, write]), or None when they were
    taken on another kernel source or workload."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256") != kernel_source_digest():
        return None
    if t.get("workload") != workload or t.get("n_log2") != n_log2:
        return None
    if split:
        return t.get("read_write_bytes_per_launch_by_k", {}).get(str(k))
    return t.get("bytes_per_launch_by_k", {}).get(str(k))


def copy_calibration(log2_elems: int = 28, reps: int = 3):
    """A plain elementwise kernel of known traffic (reads and writes 4 B per
    element) for scaling the HBM byte counters."""
    import torch
    src = torch.arange(1 << log2_elems, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        torch.bitwise_not(src, out=dst)
    torch.cuda.synchronize()
    log("copy calibration: %d launches of bitwise_not over 2^%d int32 (%d bytes read, %d written per launch)"
        % (reps, log2_elems, 4 << log2_elems, 4 << log2_elems))


def workload_cases(name: str, n_log2: int, seed: int):
    import workloads as W
    n = 1 << n_log2
    if name == "plain-large":
        streams = [W.plain_large(0.8, seed, n), W.plain_large(1.2, seed, n), W.plain_large(1.8, seed, n),
                   W.plain_large_uniform(seed, n)]
        ks = [500, 2000]
        return streams, ks
    if name == "plain":
        return [W.plain(seed, n)], [100]
    if name == "plain-highk":
        return [W.plain_highk(seed, n), W.plain_highk_adversarial(seed, n)], [10000, 50000]
    raise SystemExit("unknown workload %s" % name)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads() -> int:
    """Worker threads for the threaded oracle: the CPUs this process may run
    on, at most 16 (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(streams, ks, host, chunks_of, sample_log2: int, threads_sample_log2: int):
    """The oracle on the GPU host's CPU: single-threaded on the first
    2^sample_log2 items of every case, and in its T-thread form (chunk
    summaries on T threads with the same sequential function, the fixed tree
    on one thread: the paper's shared-memory shape) on the first
    2^threads_sample_log2 items."""
    import oracle

    def leg(sample, threads):
        total_items, total_s = 0, 0.0
        for st, a in zip(streams, host):
            for k in ks:
                n = len(a)
                s_n = min(sample, n)
                c = max(1, round(chunks_of[(st.name, k)] * s_n / n))
                t = time.perf_counter()
                if threads == 1:
                    oracle.run(a[:s_n], k, c)
                else:
                    oracle.run_threads(a[:s_n], k, c, threads)
                total_s += time.perf_counter() - t
                total_items += s_n
        return total_items / total_s / 1e9, total_s

    T = host_threads()
    v1, s1 = leg(1 << sample_log2, 1)
    log("cpu baseline: single thread %.4f G items/s" % v1)
    vT, sT = leg(1 << threads_sample_log2, T)
    log("cpu baseline: %d threads %.4f G items/s" % (T, vT))
    ncases = len(streams) * len(ks)
    return {
        "value": round(vT, 4),
        "unit": "G items/s",
        "cores": T,
        "kind": "oracle",
        "sample": "first 2^%d items of each of the %d cases (same k, chunk count scaled to the sample); the C "
                  "oracle with its chunk summaries on %d threads and the fixed tree on one; %.1f s of CPU work"
                  % (threads_sample_log2, ncases, T, sT),
        "cpu_model": cpu_model(),
        "nproc": os.cpu_count(),
        "single_thread": {"value": round(v1, 4), "unit": "G items/s", "cores": 1,
                          "sample": "first 2^%d items of each case, single-threaded C oracle; %.1f s of CPU work"
                                    % (sample_log2, s1)},
    }


def percentile(xs, q):
    xs = sorted(xs)
    return xs[min(len(xs) - 1, int(round(q / 100.0 * (len(xs) - 1))))]


def batched_leg(B, ctx, seed: int, replays: int, nstreams: int):
    """Batched streams in one graph launch vs the same streams through
    per-stream plain calls (same k and C, so the same results)."""
    import numpy as np
    import torch
    import workloads as W
    cases = W.batched(seed, nstreams)
    t = time.perf_counter()
    dev, host_n = [], 0
    for st, _ in cases:
        a = st.generate()
        host_n += len(a)
        dev.append(torch.from_numpy(a.view(np.int32)).to("cuda"))
    ks = [k for _, k in cases]
    torch.cuda.synchronize()
    log("batched: generated %d streams, %d items in %.1fs" % (len(cases), host_n, time.perf_counter() - t))
    stream = torch.cuda.current_stream()
    t = time.perf_counter()
    b = B.Batch(ctx, dev, ks, None)
    create_s = time.perf_counter() - t
    info = b.info()
    log("batched: plan + autotune + capture in %.2fs: %s" % (create_s, info))
    res = b.run(stream=stream)  # warm-up replay
    lat = []
    t0 = time.perf_counter()
    for _ in range(replays):
        tr = time.perf_counter()
        res = b.run(stream=stream)
        lat.append((time.perf_counter() - tr) * 1e3)
    batched_s = time.perf_counter() - t0
    log("batched: %d replays done" % replays)
    # the same streams through the plain path, one call each
    # an untimed pass first (it also allocates the plain path's per-k
    # summaries and workspaces) and checks every stream against the batch
    same = True
    for s in range(len(dev)):
        got, _ = B.pss_run(ctx, dev[s], k=ks[s], chunks=b.chunks[s], stream=stream)
        if same and B.to_tuples(got) != B.to_tuples(res[s]):
            same = False
    plain_lat = []
    t0 = time.perf_counter()
    for s in range(len(dev)):
        tr = time.perf_counter()
        B.pss_run(ctx, dev[s], k=ks[s], chunks=b.chunks[s], stream=stream)
        plain_lat.append((time.perf_counter() - tr) * 1e3)
    plain_s = time.perf_counter() - t0
    log("batched: per-stream plain pass done")
    b.close()
    del dev
    torch.cuda.empty_cache()
    batched_v = host_n * replays / batched_s / 1e9
    plain_v = host_n / plain_s / 1e9
    return {
        "workload": "batched: %d streams, lengths log-uniform in [10^3, 10^7] (total %d items), Zipf alpha "
                    "U[0.8, 2.0] over 2^32 hashed ids, k uniform in {50..2000}; C per stream from the autotuner"
                    % (len(cases), host_n),
        "items": host_n,
        "g_items_per_s": round(batched_v, 3),
        "ms_per_replay_p50": round(percentile(lat, 50), 3),
        "ms_per_replay_p99": round(percentile(lat, 99), 3),
        "replays": replays,
        "plain_per_stream_g_items_per_s": round(plain_v, 3),
        "plain_per_call_ms_p50": round(percentile(plain_lat, 50), 3),
        "plain_per_call_ms_p99": round(percentile(plain_lat, 99), 3),
        "speedup_vs_plain": round(batched_v / plain_v, 3),
        "identical_to_plain": same,
        "plan_autotune_capture_s": round(create_s, 3),
        "tuning": {k: (round(v, 3) if isinstance(v, float) else v) for k, v in info.items()},
    }


def served_leg(B, ctx, seed: int, nrequests: int, loads):
    """Open-loop Poisson arrivals of appends and queries (90:10) on 10^4
    device-resident summaries, at each offered load (requests/s; 0 = all at
    once, saturation), through the library's request loop; then the same log
    through one plain call per request (pss_update / pss_query)."""
    import numpy as np
    import torch
    import workloads as W
    nsum = 10000
    ks, keys, reqs = W.served_log(seed, nsum, nrequests)
    t = time.perf_counter()
    data = [W.served_append(r[2], 1.3, keys[r[1]], r[3]) if r[0] == "append" else None for r in reqs]
    items = sum(len(d) for d in data if d is not None)
    log("served: %d requests, %d appended items, generated in %.1fs" % (len(reqs), items, time.perf_counter() - t))
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0, len(reqs))
    levels = []
    for lam in loads:
        srv = B.Server(ctx, ks)
        arrivals = np.cumsum(gaps) / lam if lam > 0 else np.zeros(len(reqs))
        tickets, sub = [], []
        t0 = time.perf_counter()
        for i, r in enumerate(reqs):
            if lam > 0:
                while time.perf_counter() - t0 < arrivals[i]:
                    pass
            sub.append(time.perf_counter() - t0)
            if r[0] == "append":
                tickets.append(srv.append(r[1], data[i]))
            else:
                tickets.append(srv.query(r[1], B.PSS_Q_MAJORITY if r[2] == 0 else B.PSS_Q_TOPK, cap=ks[r[1]]))
        submit_s = time.perf_counter() - t0
        lat = []
        for tk in tickets:
            _, res = srv.wait(tk)
            lat.append(res["latency_ms"])
        # last completion as the server saw it (submission + latency), not
        # when this loop got round to collecting it
        wall = max(sb + l / 1e3 for sb, l in zip(sub, lat))
        st = srv.stats()
        srv.close()
        levels.append({
            "offered_req_per_s": lam if lam > 0 else "all at t=0",
            "achieved_req_per_s": round(len(reqs) / wall, 1),
            "g_items_per_s": round(items / wall / 1e9, 3),
            "latency_ms_p50": round(percentile(lat, 50), 3),
            "latency_ms_p99": round(percentile(lat, 99), 3),
            "launches": st["launches"],
            "max_requests_per_launch": st["max_launch_requests"],
            "submit_s": round(submit_s, 3),
            "host_staging_ms": round(st["stage_ms"], 1),
            "device_ms": round(st["gpu_ms"], 1),
        })
        log("served: load %s done: %s" % (lam, levels[-1]))
    # the same log through plain calls, one request at a time, items copied
    # from host memory per request as the server does
    summaries = {}
    stream = torch.cuda.current_stream()
    for sid in sorted(set(r[1] for r in reqs)):
        summaries[sid] = B.Summary(ctx, ks[sid])
    plain_lat = []
    t0 = time.perf_counter()
    for i, r in enumerate(reqs):
        tr = time.perf_counter()
        s = summaries[r[1]]
        if r[0] == "append":
            d = torch.from_numpy(data[i].view(np.int32)).to("cuda", non_blocking=False)
            B.pss_update(s, d, stream=stream)
            stream.synchronize()
        else:
            B.pss_query(s, B.PSS_Q_MAJORITY if r[2] == 0 else B.PSS_Q_TOPK, cap=ks[r[1]], stream=stream)
        plain_lat.append((time.perf_counter() - tr) * 1e3)
    plain_wall = time.perf_counter() - t0
    for s in summaries.values():
        s.close()
    best = max(levels, key=lambda x: x["g_items_per_s"])
    return {
        "workload": "served: %d device-resident summaries (k uniform in {100..1000}); %d requests, 90%% appends of "
                    "log-uniform length in [1, 2^20] (Zipf 1.3 over 2^32, per-summary ids), 10%% top/majority "
                    "queries; open-loop Poisson arrivals" % (nsum, len(reqs)),
        "items": items,
        "levels": levels,
        "saturation_g_items_per_s": best["g_items_per_s"],
        "plain_per_request_g_items_per_s": round(items / plain_wall / 1e9, 3),
        "plain_per_request_ms_p50": round(percentile(plain_lat, 50), 3),
        "plain_per_request_ms_p99": round(percentile(plain_lat, 99), 3),
        "speedup_vs_plain": round(best["g_items_per_s"] / (items / plain_wall / 1e9), 3),
    }


def run_cases(B, ctx, streams, dev, ks, chunks_of, steps, warmup, stream):
    """Warm-up, then `steps` timed passes over every (stream, k) case.
    Returns (wall seconds of the timed passes, per-case wall ms lists,
    per-case phase ms sums, per-case launch counts)."""
    import torch
    for i in range(warmup):
        for st, d in zip(streams, dev):
            for k in ks:
                B.pss_run(ctx, d, k=k, chunks=chunks_of[(st.name, k)], stream=stream)
        log("warmup %d done" % i)
    torch.cuda.synchronize()
    ctx.timing(True)
    ctx.phase_times(reset=True)
    wall, phase, nlaunch = {}, {}, {}
    t0 = time.perf_counter()
    for i in range(steps):
        for st, d in zip(streams, dev):
            for k in ks:
                key = (st.name, k)
                tc = time.perf_counter()
                B.pss_run(ctx, d, k=k, chunks=chunks_of[key], stream=stream)  # blocks: its report is on the host
                wall.setdefault(key, []).append((time.perf_counter() - tc) * 1e3)
                ms, nl = ctx.phase_times(reset=True)  # HIP events the library recorded on `stream`
                acc = phase.setdefault(key, [0.0] * 4)
                cnt = nlaunch.setdefault(key, [0] * 4)
                for j in range(4):
                    acc[j] += ms[j]
                    cnt[j] += nl[j]
        log("step %d done" % i)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ctx.timing(False)
    return elapsed, wall, phase, nlaunch


def roofline_of(streams, ks, n_items, phase, nlaunch, peak, measured):
    """Block-kernel read roofline: per case, per k (one kernel instance per
    k class), and for the instance that takes the most GPU time."""
    per_case, per_k = [], {}
    for st in streams:
        for k in ks:
            ms, nl = phase[(st.name, k)][0], max(1, nlaunch[(st.name, k)][0])
            avg = ms / nl
            gbs = 4.0 * n_items / (avg * 1e-3) / 1e9
            per_case.append({"stream": st.name, "k": k, "kernel_ms": round(avg, 4), "achieved_gbs": round(gbs, 1),
                             "frac": round(gbs / peak, 4)})
            t = per_k.setdefault(k, [0.0, 0])
            t[0] += ms
            t[1] += nl
    inst = []
    for k, (ms, nl) in per_k.items():
        avg = ms / max(1, nl)
        gbs = 4.0 * n_items / (avg * 1e-3) / 1e9
        inst.append({"k": k, "gpu_ms": ms, "avg_launch_ms": round(avg, 4), "launches": nl, "achieved": round(gbs, 1)})
    dom = max(inst, key=lambda r: r["gpu_ms"])
    all_ms = sum(r["gpu_ms"] for r in inst)
    all_n = sum(r["launches"] for r in inst)
    blend = 4.0 * n_items / (all_ms / max(1, all_n) * 1e-3) / 1e9
    return dom, inst, per_case, blend


def highk_leg(B, ctx, seed: int, steps: int, warmup: int, tuned: bool):
    """The high-k workload: n = 2^31 (Zipf 1.1 over 2^32 hashed ids and the
    adversarial round-robin stream with a planted 5% item), k in {10^4,
    5 x 10^4}, the chunk count from the tuner (or the planner); block state,
    COMBINE arrays and the report in device memory."""
    import numpy as np
    import torch
    streams, ks = workload_cases("plain-highk", 31, seed)
    dev = []
    n = 0
    for st in streams:
        t = time.perf_counter()
        a = st.generate()
        n = len(a)
        dev.append(torch.from_numpy(a.view(np.int32)).to("cuda"))
        del a
        log("highk: generated %s in %.1fs" % (st.name, time.perf_counter() - t))
    stream = torch.cuda.current_stream()
    chunks_of = {}
    for st, d in zip(streams, dev):
        for k in ks:
            chunks_of[(st.name, k)] = ctx.tune_chunks(d, k, stream=stream)[0] if tuned else ctx.plan_chunks(n, k)
    log("highk chunk counts: %s" % {"%s/k=%d" % key: v for key, v in chunks_of.items()})
    elapsed, wall, phase, nlaunch = run_cases(B, ctx, streams, dev, ks, chunks_of, steps, warmup, stream)
    items = n * len(streams) * len(ks) * steps
    cases = []
    for st in streams:
        for k in ks:
            key = (st.name, k)
            t = sorted(wall[key])
            med = t[len(t) // 2]
            ph = phase[key]
            tot = sum(ph)
            cases.append({"stream": st.name, "k": k, "chunks": chunks_of[key], "ms_median": round(med, 3),
                          "g_items_per_s": round(n / med / 1e6, 3),
                          "reduction_share": round((ph[1] + ph[2]) / tot, 4) if tot else None})
    dom, inst, per_case, _ = roofline_of(streams, ks, n, phase, nlaunch, HBM_PEAK_GBS, None)
    del dev
    torch.cuda.empty_cache()
    return {
        "workload": "plain-highk: n=2^31 per stream, streams=%s, k=%s, chunks from the %s"
                    % ([s.name for s in streams], ks, "tuner (pss_tune_chunks)" if tuned else "planner"),
        "g_items_per_s": round(items / elapsed / 1e9, 3),
        "cases": cases,
        "roofline": {"bound": "hbm", "kernel": "chunk_summary_kernel (state in device memory)",
                     "achieved": dom["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(dom["achieved"] / HBM_PEAK_GBS, 4), "k": dom["k"],
                     "avg_launch_ms": dom["avg_launch_ms"], "launches": dom["launches"]},
    }


def accuracy_leg(B, ctx, streams, dev, seed: int, ks):
    """Section 4's accuracy metrics on the plain-large streams and a Zipf 1.1
    stream of the same length: ARE over the reported items, precision and
    recall against exact counts (device sort); the planner's chunk count."""
    import numpy as np
    import torch
    import workloads as W
    from paper_1606_04669_amd import accuracy as A
    n = dev[0].numel()
    extra = W.plain_large(1.1, seed, n)
    d11 = torch.from_numpy(extra.generate().view(np.int32)).to("cuda")
    out = []
    for st, d in list(zip(streams, dev)) + [(extra, d11)]:
        ex = A.exact_counts_device(d)
        for k in ks:
            C = ctx.plan_chunks(n, k)
            got, _ = B.pss_run(ctx, d, k=k, chunks=C)
            m = A.metrics(got, ex, k)
            if m["recall"] != 1.0:
                raise RuntimeError("recall below 100%% on %s k=%d: %s" % (st.name, k, m))
            m.update({"stream": st.name, "chunks": C, "are": float("%.4g" % m["are"]),
                      "max_rel_error": float("%.4g" % m["max_rel_error"]), "precision": round(m["precision"], 4)})
            out.append(m)
        del ex
        log("accuracy: %s done" % st.name)
    del d11
    torch.cuda.empty_cache()
    return {"metric": "ARE over the reported items (|f - f^| / f), precision, recall vs exact counts",
            "n": n, "cases": out}


def sweep_leg(B, ctx, seed: int, n_log2: int, ks, reps: int):
    """Fractional overhead and accuracy against the chunk count: for Zipf 1.1
    and 1.8 streams, each k and C in {P/4, P, 4P} (P the planner's count):
    wall ms of the whole path, the reduction's share of GPU time (tree and
    fold over all phases: the paper's fractional overhead), and ARE."""
    import numpy as np
    import torch
    import workloads as W
    from paper_1606_04669_amd import accuracy as A
    n = 1 << n_log2
    rows = []
    for alpha in (1.1, 1.8):
        d = torch.from_numpy(W.plain_large(alpha, seed, n).generate().view(np.int32)).to("cuda")
        ex = A.exact_counts_device(d)
        for k in ks:
            P = ctx.plan_chunks(n, k)
            for C in sorted({max(1, P // 4), P, 4 * P}):
                got, _ = B.pss_run(ctx, d, k=k, chunks=C)  # warm-up (allocates)
                ctx.timing(True)
                ctx.phase_times(reset=True)
                wall = []
                for _ in range(reps):
                    t = time.perf_counter()
                    got, _ = B.pss_run(ctx, d, k=k, chunks=C)
                    wall.append((time.perf_counter() - t) * 1e3)
                ms, _nl = ctx.phase_times(reset=True)
                ctx.timing(False)
                tot = sum(ms)
                m = A.metrics(got, ex, k)
                rows.append({"alpha": alpha, "k": k, "chunks": C, "planner": P, "ms": round(sorted(wall)[reps // 2], 3),
                             "block_ms": round(ms[0] / reps, 3), "tree_ms": round(ms[1] / reps, 3),
                             "reduction_share": round((ms[1] + ms[2]) / tot, 4) if tot else None,
                             "are": float("%.4g" % m["are"]), "precision": round(m["precision"], 4),
                             "recall": m["recall"]})
        del d, ex
        torch.cuda.empty_cache()
        log("sweep: alpha %.1f done" % alpha)
    return {"n": n, "rows": rows}


def frequent_leg(B, ctx, streams, dev, ks, steps: int):
    """The Frequent (Misra-Gries) summary in the same pipeline on the same
    streams and k: wall ms per call, G items/s, the block kernel's read
    roofline (HIP events the library records on the launch stream)."""
    import torch
    stream = torch.cuda.current_stream()
    n = dev[0].numel()
    cases = []
    kms = {}
    for st, d in zip(streams, dev):
        for k in ks:
            C = ctx.frequent_plan_chunks(n, k)
            B.pss_frequent_run(ctx, d, k=k, chunks=C, stream=stream)  # warm-up (allocates)
            ctx.timing(True)
            ctx.phase_times(reset=True)
            wall = []
            for _ in range(steps):
                t = time.perf_counter()
                B.pss_frequent_run(ctx, d, k=k, chunks=C, stream=stream)
                wall.append((time.perf_counter() - t) * 1e3)
            ms, nl = ctx.phase_times(reset=True)
            ctx.timing(False)
            med = sorted(wall)[len(wall) // 2]
            kern = ms[0] / max(1, nl[0])
            acc = kms.setdefault(k, [0.0, 0])
            acc[0] += ms[0]
            acc[1] += nl[0]
            cases.append({"stream": st.name, "k": k, "chunks": C, "ms_median": round(med, 3),
                          "g_items_per_s": round(n / med / 1e6, 2), "block_kernel_ms": round(kern, 4),
                          "achieved_gbs": round(4.0 * n / (kern * 1e-3) / 1e9, 1) if kern > 0 else None,
                          "tree_ms": round(ms[1] / max(1, steps), 3)})
    total_items = n * len(cases) * steps
    total_s = sum(c["ms_median"] for c in cases) * steps / 1e3
    dom_k = max(kms, key=lambda k: kms[k][0])
    dom_ms = kms[dom_k][0] / max(1, kms[dom_k][1])
    ach = 4.0 * n / (dom_ms * 1e-3) / 1e9 if dom_ms > 0 else 0.0
    return {"workload": "the plain-large streams and k with the Frequent summary (k - 1 counters), "
                        "the Frequent planner's chunk count",
            "g_items_per_s": round(total_items / total_s / 1e9, 3), "cases": cases,
            "roofline": {"bound": "hbm", "kernel": "frequent_block_kernel, k=%d" % dom_k, "achieved": round(ach, 1),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                         "avg_launch_ms": round(dom_ms, 4)}}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="plain-large", choices=["plain-large", "plain", "plain-highk"])
    ap.add_argument("--n-log2", type=int, default=None)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--chunks", default="tuned", choices=["tuned", "planner"],
                    help="chunk count per case: the library's autotuner (pss_tune_chunks) or its planner")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-log2", type=int, default=25)
    ap.add_argument("--cpu-threads-sample-log2", type=int, default=27)
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-vs-plain leg")
    ap.add_argument("--no-served", action="store_true", help="skip the served leg")
    ap.add_argument("--no-highk", action="store_true", help="skip the high-k leg")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the accuracy leg")
    ap.add_argument("--no-sweep", action="store_true", help="skip the k x chunk-count sweep")
    ap.add_argument("--no-frequent", action="store_true", help="skip the Frequent (Misra-Gries) leg")
    ap.add_argument("--served-requests", type=int, default=4000)
    ap.add_argument("--served-loads", default="2000,10000,40000,0",
                    help="offered loads in requests/s (0: all at once)")
    ap.add_argument("--batched-streams", type=int, default=4096)
    ap.add_argument("--batched-replays", type=int, default=5)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain elementwise kernel of known traffic (for counter runs)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    n_log2 = args.n_log2 if args.n_log2 is not None else {"plain-large": 30, "plain": 20, "plain-highk": 31}[
        args.workload]

    import numpy as np
    import torch
    from paper_1606_04669_amd import binding as B

    if args.copy_calibration:
        copy_calibration()
    streams, ks = workload_cases(args.workload, n_log2, args.seed)
    host, dev = [], []
    for st in streams:
        t = time.perf_counter()
        a = st.generate()
        log("generated %s n=2^%d in %.1fs" % (st.name, n_log2, time.perf_counter() - t))
        host.append(a)
        dev.append(torch.from_numpy(a.view(np.int32)).to("cuda"))
    torch.cuda.synchronize()
    ctx = B.Context(0)
    stream = torch.cuda.current_stream()
    chunks_of, tuned_ms = {}, {}
    for st, a, d in zip(streams, host, dev):
        for k in ks:
            if args.chunks == "tuned":
                c, tms = ctx.tune_chunks(d, k, stream=stream)
                chunks_of[(st.name, k)], tuned_ms[(st.name, k)] = c, tms
            else:
                chunks_of[(st.name, k)] = ctx.plan_chunks(len(a), k)
    if args.chunks == "tuned":
        log("autotuned chunk counts: %s" % {"%s/k=%d" % key: v for key, v in chunks_of.items()})
    read_gbs = ctx.read_bandwidth(dev[0])
    log("read bandwidth over a %d-byte stream: %.1f GB/s" % (dev[0].numel() * 4, read_gbs))

    elapsed, wall, phase, nlaunch = run_cases(B, ctx, streams, dev, ks, chunks_of, args.steps, args.warmup, stream)
    items_per_step = sum(len(a) for a in host) * len(ks)
    value = items_per_step * args.steps / elapsed / 1e9
    n_items = len(host[0])
    dom, inst, per_case, blend = roofline_of(streams, ks, n_items, phase, nlaunch, HBM_PEAK_GBS, read_gbs)
    cases = []
    for st in streams:
        for k in ks:
            key = (st.name, k)
            t = sorted(wall[key])
            med = t[len(t) // 2]
            c = {"stream": st.name, "k": k, "chunks": chunks_of[key], "ms_median": round(med, 3),
                 "g_items_per_s": round(n_items / med / 1e6, 2)}
            if key in tuned_ms:
                c["tuned_blocks_tree_ms"] = round(tuned_ms[key], 3)
            cases.append(c)
    ms = [sum(phase[key][j] for key in phase) for j in range(4)]
    total_ms = sum(ms)
    dom_launch_ms = dom["avg_launch_ms"]
    result = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "G items/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic (seeded Zipf/uniform uint32 streams, resident in HBM)",
        "config": {
            "workload": "%s: n=2^%d per stream, streams=%s, k=%s, chunks %s" % (
                args.workload, n_log2, [s.name for s in streams], ks,
                "from the autotuner (pss_tune_chunks), recorded per case" if args.chunks == "tuned"
                else "from the planner"),
            "n": n_items,
            "cases": cases,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "chunk_summary_kernel, k=%d instance (the most GPU time)" % dom["k"],
            "achieved": dom["achieved"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(dom["achieved"] / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(args.workload, n_log2, dom["k"]),
            "traffic_read_write": measured_traffic(args.workload, n_log2, dom["k"], split=True),
            "avg_launch_ms": dom_launch_ms,
            "launches": dom["launches"],
            "measured_read_gbs": round(read_gbs, 1),
            "frac_of_measured_read": round(dom["achieved"] / read_gbs, 4),
            "by_k": [{"k": r["k"], "achieved": r["achieved"], "frac": round(r["achieved"] / HBM_PEAK_GBS, 4),
                      "avg_launch_ms": r["avg_launch_ms"], "launches": r["launches"]} for r in inst],
            "all_launches_achieved": round(blend, 1),
            "per_case": per_case,
        },
        "phases_ms_per_step": {
            "chunk_summary": round(ms[0] / args.steps, 3),
            "combine_tree": round(ms[1] / args.steps, 3),
            "fold": round(ms[2] / args.steps, 3),
            "report": round(ms[3] / args.steps, 3),
            "reduction_share": round((ms[1] + ms[2]) / total_ms, 4) if total_ms else None,
        },
    }
    if args.workload == "plain-large" and not args.no_frequent:
        result["frequent"] = frequent_leg(B, ctx, streams, dev, ks, 3)
    if args.workload == "plain-large" and not args.no_accuracy:
        result["accuracy"] = accuracy_leg(B, ctx, streams, dev, args.seed, [500, 1000, 2000, 4000, 8000])
    del dev
    torch.cuda.empty_cache()
    if args.workload == "plain-large" and not args.no_sweep:
        result["sweep"] = sweep_leg(B, ctx, args.seed, n_log2, [500, 2000, 8000], 3)
    if args.workload == "plain-large" and not args.no_highk:
        result["highk"] = highk_leg(B, ctx, args.seed, 2, 1, args.chunks == "tuned")
    if not args.no_batched:
        result["batched"] = batched_leg(B, ctx, args.seed, args.batched_replays, args.batched_streams)
    if not args.no_served:
        result["served"] = served_leg(B, ctx, args.seed, args.served_requests,
                                      [float(x) for x in args.served_loads.split(",")])
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on samples")
        result["cpu_baseline"] = cpu_baseline(streams, ks, host, chunks_of, args.cpu_sample_log2,
                                              args.cpu_threads_sample_log2)
    print(json.dumps(result), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
