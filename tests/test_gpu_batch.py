"""GPU parity of the batched form: many streams, each with its own k and
block count, in one captured graph.

Per stream the batch must give exactly what Algorithm 1 (with Algorithm 2 as
the reduction) gives on that stream alone with the same block count: the
oracle's result, and the plain library call's result, bit for bit.
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


def dev(items):
    import torch
    a = np.ascontiguousarray(np.asarray(items, dtype=np.uint32))
    return torch.from_numpy(a.view(np.int32)).to("cuda")


@pytest.fixture(scope="module")
def small_batch():
    cases = W.batched(seed=3, nstreams=40, log10_min=3.0, log10_max=5.3)
    host = [st.generate() for st, _ in cases]
    ks = [k for _, k in cases]
    # half the block counts fixed by the caller, half left to the autotuner
    chunks = [(1 + s % 9) if s % 2 == 0 else 0 for s in range(len(cases))]
    return host, ks, chunks


def test_batch_limits(ctx):
    say("batch_max_k", ctx.batch_max_k)
    assert ctx.batch_max_k >= 2000


def test_batch_equals_oracle_per_stream(B, ctx, small_batch):
    host, ks, chunks = small_batch
    d = [dev(a) for a in host]
    say("batch of", len(d), "streams, total", sum(len(a) for a in host), "items")
    b = B.Batch(ctx, d, ks, chunks)
    info = b.info()
    say("info", info)
    assert info["nstreams"] == len(d)
    for s, c in enumerate(chunks):
        if c:
            assert b.chunks[s] == c
        assert 1 <= b.chunks[s] <= len(host[s])
    got = b.run()
    for s in range(len(host)):
        want = O.run(host[s], ks[s], b.chunks[s])
        assert B.to_tuples(got[s]) == O.to_tuples(want), (s, ks[s], b.chunks[s])
    b.close()


def test_alone_and_in_the_batch_are_identical(B, ctx, small_batch):
    host, ks, chunks = small_batch
    d = [dev(a) for a in host]
    b = B.Batch(ctx, d, ks, chunks)
    got = b.run()
    for s in range(len(host)):
        alone, used = B.pss_run(ctx, d[s], k=ks[s], chunks=b.chunks[s])
        assert used == b.chunks[s]
        assert B.to_tuples(alone) == B.to_tuples(got[s]), s
    b.close()


def test_graph_replays_match_eager_runs(B, ctx, small_batch):
    import torch
    host, ks, chunks = small_batch
    d = [dev(a) for a in host]
    b = B.Batch(ctx, d, ks, chunks)
    eager = [B.to_tuples(r) for r in b.run(eager=True)]
    for rep in range(4):
        # unrelated eager work and a synchronisation between replays
        x = torch.arange(1 << 20, device="cuda", dtype=torch.int32)
        assert int((x * 2).sum().item()) == (1 << 20) * ((1 << 20) - 1)
        torch.cuda.synchronize()
        g = [B.to_tuples(r) for r in b.run()]
        assert g == eager, rep
    b.close()


def test_tuning_result_neutral_knobs_keeps_results(B, ctx, small_batch):
    host, ks, chunks = small_batch
    d = [dev(a) for a in host]
    fixed = [c if c else 1 + s % 5 for s, c in enumerate(chunks)]
    b0 = B.Batch(ctx, d, ks, fixed, tune=False)
    b1 = B.Batch(ctx, d, ks, fixed, tune=True)
    say("tuned", b1.info())
    assert b0.chunks == fixed and b1.chunks == fixed
    r0 = [B.to_tuples(r) for r in b0.run()]
    r1 = [B.to_tuples(r) for r in b1.run()]
    assert r0 == r1
    b0.close()
    b1.close()


def test_one_shot_and_edge_streams(B, ctx):
    # shortest streams (k = n), one item repeated, full-range ids, C = n
    streams = [np.array([7, 7], dtype=np.uint32), np.full(1000, 0xFFFFFFFF, dtype=np.uint32),
               np.array([0, 0xFFFFFFFF] * 300 + [5] * 400, dtype=np.uint32),
               W.zipf_hashed(5000, 1.2, 1 << 32, seed=9)]
    ks = [2, 50, 3, 2000]
    chunks = [2, 3, 1000, 0]
    got, used = B.pss_run_batched(ctx, [dev(a) for a in streams], ks, chunks)
    for s in range(len(streams)):
        assert B.to_tuples(got[s]) == O.to_tuples(O.run(streams[s], ks[s], used[s])), s


def test_batch_errors(B, ctx):
    a = dev(np.arange(100, dtype=np.uint32))
    with pytest.raises(B.PssError) as e:
        B.Batch(ctx, [a], [101])  # k > n
    assert e.value.code == B.PSS_ERANGE
    with pytest.raises(B.PssError) as e:
        B.Batch(ctx, [a], [1])
    assert e.value.code == B.PSS_EINVAL
    big = dev(np.arange(20000, dtype=np.uint32))
    with pytest.raises(B.PssError) as e:
        B.Batch(ctx, [big], [ctx.batch_max_k + 1])
    assert e.value.code == B.PSS_ERANGE
