"""Seeded generators: determinism, shapes and the statistics each workload
is meant to have."""
import numpy as np

from paper_2609_31980_amd import inputs


def test_deterministic_bytes():
    a, b = inputs.tracks(5000, seed=3), inputs.tracks(5000, seed=3)
    assert a.tobytes() == b.tobytes()
    assert inputs.tracks(5000, seed=4).tobytes() != a.tobytes()
    assert inputs.c1().points.tobytes() == inputs.c1().points.tobytes()


def test_c1_shape():
    w = inputs.c1()
    assert w.points.shape == (4096, 3) and w.points.dtype == np.float32
    assert w.points.min() >= 0 and w.points.max() < 1
    assert w.K == 0 and w.queries is None
    assert np.float32(w.r) == np.float32(0.1)


def test_tracks_structure():
    x = inputs.tracks(12000, 8, seed=1, permute=False)
    assert x.dtype == np.float32 and x.shape == (12000, 8)
    # un-noised members of one track sit within a few sigma of each other
    spread = x[:12].std(axis=0)
    assert np.median(spread) < 0.2
    assert np.all(np.abs(x) < 1.2)


def test_c2_shape():
    w = inputs.c2()
    assert w.points.shape == (300_000, 8) and w.K == 256
    assert np.abs(w.points).max() < 1.2


def test_c3_sizes():
    s = inputs.c3_sizes()
    assert len(s) == 64 and s.min() >= 50_000 and s.max() <= 400_000
    assert np.array_equal(s, inputs.c3_sizes())


def test_zipf_sizes():
    rng = np.random.default_rng(0)
    s = inputs.zipf_cluster_sizes(200_000, rng)
    assert s.sum() == 200_000 and s.min() >= 1 and s.max() <= 500
    # P(1) = 1 / zeta_500(1.5) ~ 0.39
    assert 0.35 < np.mean(s == 1) < 0.43


def test_c4_degree_near_100(orc):
    w = inputs.c4()
    assert w.points.shape == (1_000_000, 12) and w.queries.shape == (200_000, 12)
    assert w.K == 64
    s = inputs.subset_rows(len(w.queries), 0.002, 123)
    d = orc.degrees(w.points, w.r, Q=w.queries[s])
    assert 80 < d.mean() < 120


def test_c5_trace():
    tr = inputs.c5_trace(2000, rate=100.0)
    t = np.array([a.t for a in tr])
    n = np.array([a.n for a in tr])
    assert t[0] == 0 and np.all(np.diff(t) >= 0)
    assert 15 < t[-1] < 25                              # 2000 arrivals at 100/s
    assert n.min() >= 10_000 and n.max() <= 500_000
    assert 85_000 < np.median(n) < 115_000
    ev = inputs.c5_event(tr[0])
    assert ev.shape == (tr[0].n, 8)


def test_lattice_edge_case():
    p = inputs.lattice_on_cells(4, 2, 0.1)
    assert p.shape == (48, 2) and p.dtype == np.float32


def test_paper_shaped_degree_near_target(orc):
    """The calibrated spread gives the paper's mean non-self degree (34.16) on
    a sample other than the one used for the calibration."""
    w = inputs.paper_shaped()
    assert w.points.shape == (271_663, 12) and w.points.dtype == np.float32
    assert w.K == 1000 and w.exclude_self and w.queries is None
    assert np.float32(w.r).view(np.uint32) == np.float32(0.12).view(np.uint32)
    s = inputs.subset_rows(len(w.points), 500 / len(w.points), 5)
    d = orc.degrees(w.points, w.r, Q=w.points[s], self_ids=s)
    assert abs(d.mean() - 9_279_672 / 271_663) < 0.15 * 34.16


def test_stored_event_digests_match_the_generators():
    """The oracle digests stored for the multi-event workloads cover every
    event, in order, with the sizes the seeded generators give (the digests
    themselves are written by tests/golden/write_event_hashes.py from the
    oracle alone)."""
    import json
    import os
    g = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    b = json.load(open(os.path.join(g, "batch64_hashes.json")))
    assert [e["event"] for e in b["events"]] == list(range(64))
    assert [e["N"] for e in b["events"]] == inputs.c3_sizes().tolist()
    s = json.load(open(os.path.join(g, "stream40_hashes.json")))
    assert [e["event"] for e in s["events"]] == list(range(40))
    n = [e["N"] for e in s["events"]]
    assert n == [a.n for a in inputs.c5_trace(40, rate=1.0)]
    assert min(n) < 50_000 and max(n) > 200_000          # spans the log-normal range
    for doc in (b, s):
        assert doc["K"] == 256 and doc["self_join"] and not doc["exclude_self"]
        assert all(len(e["sha256"]) == 64 and e["nnz"] <= e["degree_sum"] for e in doc["events"])
