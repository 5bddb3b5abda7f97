"""The accuracy harness on the GPU: exact counts from the device sort equal
the host count, and the metrics of the GPU report equal those of the
oracle's report (which is the same report: the two are bit-identical).
Recall is 100% (Space Saving's guarantee); precision is reported, not
asserted."""
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


def test_harness_on_device_equals_host(B):
    import torch
    from paper_1606_04669_amd import accuracy as A
    ctx = B.Context(0)
    items = W.zipf_hashed(1 << 22, 1.1, 1 << 32, seed=41)
    d = torch.from_numpy(items.view(np.int32)).to("cuda")
    exd = A.exact_counts_device(d)
    exh = A.exact_counts_host(items)
    assert np.array_equal(exd.ids, exh.ids) and np.array_equal(exd.counts, exh.counts) and exd.n == exh.n
    for k, C in [(100, 64), (500, 64), (2000, 16)]:
        got, _ = B.pss_run(ctx, d, k=k, chunks=C)
        want = O.run(items, k, C)
        mg, mo = A.metrics(got, exd, k), A.metrics(want, exh, k)
        say("k=%d C=%d" % (k, C), mg)
        assert mg == mo
        assert mg["recall"] == 1.0
    ctx.close()
