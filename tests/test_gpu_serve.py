"""GPU parity of the served form: a pool of device-resident summaries fed
by a request loop with continuous batching.

Every append is S <- COMBINE(S, tree(blocks of the append)), N <- N + n, and
every query reports S; requests on one summary take effect in submission
order.  The oracle replays the request log per summary and must agree bit for
bit; the same requests sent alone through the plain calls must too, whatever
else shared their launches.
"""
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


def make_log(seed, nsum, nreq, max_log2):
    ks, keys, reqs = W.served_log(seed, nsum, nreq, max_log2=max_log2)
    log = []
    for r in reqs:
        if r[0] == "append":
            log.append(("append", r[1], W.served_append(r[2], 1.3, keys[r[1]], r[3])))
        else:
            log.append(("query", r[1], r[2]))
    return ks, log


def serve(B, ctx, ks, log, burst, **opts):
    """Submit the log in bursts (waiting for each burst), return per-request
    (entries, result)."""
    srv = B.Server(ctx, ks, **opts)
    out = []
    for i in range(0, len(log), burst):
        tickets = []
        for op in log[i: i + burst]:
            if op[0] == "append":
                tickets.append(srv.append(op[1], op[2]))
            else:
                kind = B.PSS_Q_MAJORITY if op[2] == 0 else B.PSS_Q_TOPK
                tickets.append(srv.query(op[1], kind, cap=ks[op[1]]))
        for t in tickets:
            out.append(srv.wait(t))
    stats = srv.stats()
    srv.close()
    return out, stats


def oracle_replay(ks, log, results):
    ref = [O.Summary(k) for k in ks]
    for op, (ent, res) in zip(log, results):
        sid = op[1]
        if op[0] == "append":
            ref[sid].update(op[2], res["chunks_used"])
            assert res["stream_len"] == ref[sid].n
        else:
            assert res["stream_len"] == ref[sid].n
            if op[2] == 0:
                want = O.to_tuples(ref[sid].query_majority())
            else:
                want = ref[sid].as_tuples()[: ks[sid]]
            got = [(int(e["item"]), int(e["count"]), int(e["error"])) for e in ent]
            assert got == want, (sid, op[2])


def test_server_limits(ctx):
    say("server_max_k", ctx.server_max_k)
    assert ctx.server_max_k >= 1000


def test_served_log_equals_oracle_replay(B, ctx):
    ks, log = make_log(seed=4, nsum=48, nreq=500, max_log2=15.0)
    say("requests", len(log), "appended items", sum(len(op[2]) for op in log if op[0] == "append"))
    results, stats = serve(B, ctx, ks, log, burst=64)
    say("stats", stats)
    assert stats["status"] == 0 and stats["requests"] == sum(1 for op in log if op[0] == "query" or len(op[2]))
    oracle_replay(ks, log, results)


def test_many_launches_in_flight_keep_per_summary_order(B, ctx):
    # few summaries, small launches, three slots: requests on one summary
    # land in different launches that overlap on the device
    ks, log = make_log(seed=5, nsum=6, nreq=300, max_log2=13.0)
    results, stats = serve(B, ctx, ks, log, burst=300, slots=3, max_requests=4)
    say("stats", stats)
    assert stats["launches"] >= 50
    oracle_replay(ks, log, results)


def test_alone_and_in_the_mix_are_identical(B, ctx):
    import torch
    ks, log = make_log(seed=6, nsum=16, nreq=240, max_log2=14.0)
    mixed, _ = serve(B, ctx, ks, log, burst=80)
    for sid in (0, 3, 7):
        s = B.Summary(ctx, ks[sid])
        for op, (ent, res) in zip(log, mixed):
            if op[1] != sid:
                continue
            if op[0] == "append":
                if len(op[2]):
                    d = torch.from_numpy(op[2].view(np.int32)).to("cuda")
                    B.pss_update(s, d, chunks=res["chunks_used"])
            else:
                kind = B.PSS_Q_MAJORITY if op[2] == 0 else B.PSS_Q_TOPK
                alone, n = B.pss_query(s, kind, cap=ks[sid])
                assert n == res["stream_len"]
                assert B.to_tuples(alone) == B.to_tuples(ent), sid
        s.close()


def test_admission_budget_and_limits(B, ctx):
    ks = [500, 700]
    big = W.served_append(1 << 18, 1.3, 77, 1)  # 1 MiB of items
    srv = B.Server(ctx, ks, hbm_budget=3 << 20, slots=2)  # 1.5 MiB per launch: one such append
    with pytest.raises(B.PssError) as e:
        srv.append(0, np.zeros(1 << 20, dtype=np.uint32))  # can never fit a launch
    assert e.value.code == B.PSS_ERANGE
    ref = [O.Summary(k) for k in ks]
    tickets = [(i % 2, srv.append(i % 2, big[: (1 << 18) - 1000 * i])) for i in range(8)]
    for sid, t in tickets:
        _, res = srv.wait(t)
        ref[sid].update(big[: res["stream_len"] - ref[sid].n], res["chunks_used"])
    st = srv.stats()
    say("stats", st)
    assert st["launches"] >= 8
    for sid in (0, 1):
        ent, res = srv.wait(srv.query(sid, B.PSS_Q_TOPK, cap=ks[sid]))
        assert B.to_tuples(ent) == ref[sid].as_tuples()
    # truncation of a majority report to the caller's cap
    t = srv.query(0, B.PSS_Q_MAJORITY)
    with pytest.raises(B.PssError) as e:
        srv.wait(t, cap=1)
    assert e.value.code == B.PSS_ETRUNC
    srv.close()
