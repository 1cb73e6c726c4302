"""Helpers for the GPU tests: run the HIP path through the C ABI binding and
compare it with the CPU oracle."""
import sys

import numpy as np

import pinlib


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def gpu_csr(X, r, K=0, Q=None, exclude_self=False, opts=None):
    """Build + query on the GPU; returns host (offsets, indices, dist2)."""
    from paper_2609_31980_amd import frnn
    import torch
    xd = dev(X)
    ix = frnn.build(xd, r, opts)
    c = ix.query(None if Q is None else dev(Q), r, K, exclude_self=exclude_self)
    out = c.numpy()
    c.release()
    ix.close()
    torch.cuda.synchronize()
    return out


def check_full(orc, X, r, K=0, Q=None, exclude_self=False, opts=None, what=""):
    want = orc.frnn(X, r, K, Q=Q, exclude_self=exclude_self)
    got = gpu_csr(X, r, K, Q=Q, exclude_self=exclude_self, opts=opts)
    pinlib.assert_csr_equal(got, pinlib.as_tuple(want), what)
    return want


def check_rows(orc, got, X, r, K, rows, Q=None, self_ids=None, what=""):
    """Compare sampled rows of a GPU CSR with the oracle's rows for them."""
    off, idx, d2 = got
    Qs = (X if Q is None else Q)[rows]
    want = orc.frnn(X, r, K, Q=Qs, self_ids=self_ids)
    for k, i in enumerate(rows):
        a, b = int(off[i]), int(off[i + 1])
        wa, wb = int(want.offsets[k]), int(want.offsets[k + 1])
        assert np.array_equal(idx[a:b], want.indices[wa:wb]), f"{what}: row {i} indices"
        assert np.array_equal(d2[a:b].view(np.uint32), want.dist2[wa:wb].view(np.uint32)), \
            f"{what}: row {i} dist2"
    return want


def check_csr_invariants(got, N, K=0):
    """Properties that hold at any size: offsets monotone from 0, ids in
    range, rows ordered by (dist2, id) strictly, at most K entries."""
    off, idx, d2 = got
    assert off[0] == 0 and np.all(np.diff(off) >= 0)
    assert len(idx) == off[-1]
    if len(idx):
        assert idx.min() >= 0 and idx.max() < N
    if K > 0:
        assert np.diff(off).max(initial=0) <= K
    key = (d2.view(np.uint32).astype(np.uint64) << np.uint64(32)) | idx.astype(np.uint64)
    row = np.repeat(np.arange(len(off) - 1), np.diff(off))
    same = row[1:] == row[:-1]
    assert np.all(key[1:][same] > key[:-1][same]), "rows not strictly ordered by (dist2, id)"
