"""The entry point that allocates nothing (frnn_query_noalloc): its CSR is
that of frnn_query_batch on the same event, bit for bit, on two calls in a
row (the second with a smaller input, the array keeping the first call's
contents), on an event with rows longer than the stash (fill and long-row
passes in the array) and when the output capacity is too small."""
import numpy as np
import pytest

from gpu_util import dev, say
from paper_2609_31980_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def frnn():
    import torch
    assert torch.cuda.is_available()
    from paper_2609_31980_amd import frnn as f
    return f


def reference(frnn, x, r, K, exclude_self):
    c = frnn.query_batch([x], r, K, exclude_self=exclude_self)[0]
    off, idx, d2 = c.torch()
    c.release()
    return off, idx, d2


def noalloc(frnn, x, r, K, exclude_self, cap):
    import torch
    off = torch.full((x.shape[0] + 1,), -1, dtype=torch.int64, device="cuda")
    idx = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
    d2 = torch.full((cap,), -1.0, dtype=torch.float32, device="cuda")
    nnz = frnn.query_noalloc(x, r, K, off, idx, d2, exclude_self=exclude_self)
    torch.cuda.synchronize()
    return nnz, off, idx[:nnz], d2[:nnz]


def same(a, b, what):
    import torch
    off, idx, d2 = a
    roff, ridx, rd2 = b
    assert torch.equal(off, roff), f"{what}: offsets differ"
    assert torch.equal(idx, ridx), f"{what}: indices differ"
    assert torch.equal(d2.view(torch.int32), rd2.view(torch.int32)), f"{what}: dist2 bits differ"


def test_two_calls_second_smaller(frnn):
    for n, seed in ((120_000, 71), (30_000, 72)):
        x = dev(inputs.tracks(n, 8, seed=seed))
        say(f"no-alloc tracking event N={n}")
        want = reference(frnn, x, 0.1, 256, False)
        nnz, off, idx, d2 = noalloc(frnn, x, 0.1, 256, False, int(want[1].numel()) + 1000)
        assert nnz == want[1].numel()
        same((off, idx, d2), want, f"N={n}")


def test_long_rows_in_the_array(frnn):
    """Dense 12-D clusters with K=1000 and no self pairs: rows longer than
    the stash go through the fill and long-row passes, whose scratch rows
    live in the array too; then a sparse event reuses it."""
    X, _ = inputs.clustered(12000, 0, 12, 0.022, 5)
    r = float(np.float32(0.12))
    for x, K, ex in ((dev(X), 1000, True), (dev(inputs.tracks(8000, 8, seed=73)), 8, False)):
        say(f"no-alloc N={x.shape[0]} D={x.shape[1]} K={K}")
        rr = r if x.shape[1] == 12 else 0.1
        want = reference(frnn, x, rr, K, ex)
        nnz, off, idx, d2 = noalloc(frnn, x, rr, K, ex, int(want[1].numel()))
        same((off, idx, d2), want, f"N={x.shape[0]} K={K}")


def test_capacity_too_small_reports_the_count(frnn):
    x = dev(inputs.tracks(5000, 8, seed=74))
    want = reference(frnn, x, 0.1, 256, False)
    with pytest.raises(frnn.FrnnError) as e:
        noalloc(frnn, x, 0.1, 256, False, 10)
    assert e.value.name == "BUDGET" and e.value.nnz == want[1].numel()
    # the array is left usable
    nnz, off, idx, d2 = noalloc(frnn, x, 0.1, 256, False, int(want[1].numel()))
    same((off, idx, d2), want, "after a refused call")
