"""The synchronous host-array interface (frnn_query_host) against the oracle,
bit for bit, and against the device path."""
import numpy as np
import pytest

import pinlib
from gpu_util import gpu_csr, say
from paper_2609_31980_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def frnn():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2609_31980_amd import frnn as f
    return f


def host(frnn, X, r, K, Q=None, exclude_self=False):
    c = frnn.query_host(X, r, K, queries=Q, exclude_self=exclude_self)
    out = c.numpy()
    c.release()
    return out


def test_host_matches_oracle(orc, frnn):
    w = inputs.c1()
    say("host interface: uniform-4096")
    pinlib.assert_csr_equal(host(frnn, w.points, w.r, 0), pinlib.as_tuple(orc.frnn(w.points, w.r, 0)), "c1")
    pinlib.assert_csr_equal(host(frnn, w.points, w.r, 3, exclude_self=True),
                            pinlib.as_tuple(orc.frnn(w.points, w.r, 3, exclude_self=True)), "c1 K=3 excl")
    X, Q = inputs.clustered(30000, 3000, 12, 0.03, seed=8)
    say("host interface: separate queries d12")
    pinlib.assert_csr_equal(host(frnn, X, inputs.C4_RADIUS, 64, Q=Q),
                            pinlib.as_tuple(orc.frnn(X, inputs.C4_RADIUS, 64, Q=Q)), "clustered K=64")


def test_host_large_event_matches_device_path(frnn):
    """More than one staging chunk (9.6 MB of points) and the device path's CSR."""
    w = inputs.c2()
    say("host interface: tracks-300k")
    a = host(frnn, w.points, w.r, w.K)
    b = gpu_csr(w.points, w.r, w.K)
    pinlib.assert_csr_equal(a, b, "tracks-300k host vs device")


def test_host_edge_cases(frnn):
    X = np.random.default_rng(3).random((100, 3)).astype(np.float32)
    off, idx, d2 = host(frnn, X, 0.2, 0, Q=np.zeros((0, 3), np.float32))
    assert off.tolist() == [0] and len(idx) == 0
    off, idx, d2 = host(frnn, np.zeros((0, 3), np.float32), 0.2, 0)
    assert off.tolist() == [0]
    bad = X.copy()
    bad[7, 1] = np.nan
    with pytest.raises(frnn.FrnnError) as e:
        frnn.query_host(bad, 0.2, 0)
    assert e.value.name == "NONFINITE"
    c = frnn.query_host(X, 0.2, 0, want_dist2=False)
    assert c.dist2 is None and c.nnz > 0
    c.release()
