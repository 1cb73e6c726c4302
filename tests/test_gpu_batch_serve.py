"""GPU tests of the batched pipeline, the server, the tuner and the
full-size density workload, all against the CPU oracle or against the
single-event path (which is itself checked against the oracle)."""
import numpy as np
import pytest

import pinlib
from gpu_util import check_csr_invariants, check_rows, dev, gpu_csr, say
from paper_2609_31980_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def frnn():
    import torch
    assert torch.cuda.is_available()
    from paper_2609_31980_amd import frnn as f
    return f


def _np(csr):
    off, idx, d2 = csr.numpy()
    return off, idx, d2


def test_batch_matches_oracle_and_single(orc, frnn):
    sizes = [3000, 0, 1, 12000, 700, 5000]
    evs = [inputs.tracks(n, 8, seed=40 + i) if n else np.zeros((0, 8), np.float32)
           for i, n in enumerate(sizes)]
    say("batch of 6 uneven events")
    outs = frnn.query_batch([dev(e) for e in evs], 0.1, 256)
    for e, (x, o) in enumerate(zip(evs, outs)):
        want = orc.frnn(x, 0.1, 256)
        pinlib.assert_csr_equal(_np(o), pinlib.as_tuple(want), f"batch event {e}")
        if len(x):
            pinlib.assert_csr_equal(_np(o), gpu_csr(x, 0.1, 256), f"batch vs single event {e}")


def test_batch_graph_replay_varies_inputs(orc, frnn):
    """The graph of a capacity class replays for different batches of it."""
    import torch
    og = frnn.default_opts(graphs=1)
    for rep, seed in enumerate((50, 51, 52)):
        sizes = [4000 + 500 * rep, 2500, 6000 - 300 * rep]
        evs = [inputs.tracks(n, 8, seed=seed * 10 + i) for i, n in enumerate(sizes)]
        outs = frnn.query_batch([dev(e) for e in evs], 0.1, 8, opts=og)
        torch.cuda.synchronize()
        for e, (x, o) in enumerate(zip(evs, outs)):
            pinlib.assert_csr_equal(_np(o), pinlib.as_tuple(orc.frnn(x, 0.1, 8)), f"replay {rep} event {e}")


def test_batch_separate_queries_and_exclusion(orc, frnn):
    xs, qs = [], []
    for i in range(4):
        x, q = inputs.clustered(8000 + 1000 * i, 900, 12, 0.03, seed=60 + i)
        xs.append(x)
        qs.append(q)
    outs = frnn.query_batch([dev(x) for x in xs], inputs.C4_RADIUS, 64, queries=[dev(q) for q in qs])
    for e, o in enumerate(outs):
        pinlib.assert_csr_equal(_np(o), pinlib.as_tuple(orc.frnn(xs[e], inputs.C4_RADIUS, 64, Q=qs[e])),
                                f"query batch event {e}")
    evs = [inputs.tracks(3000, 8, seed=70 + i) for i in range(3)]
    outs = frnn.query_batch([dev(e) for e in evs], 0.1, 0, exclude_self=True)
    for e, o in enumerate(outs):
        pinlib.assert_csr_equal(_np(o), pinlib.as_tuple(orc.frnn(evs[e], 0.1, 0, exclude_self=True)),
                                f"exclude-self batch event {e}")


def test_batch_eager_equals_graph(frnn):
    """Graph replay (twice: recorded, then replayed), eager launches (the
    default) and eager launches timed one by one give the same outputs."""
    evs = [inputs.tracks(n, 8, seed=80 + n) for n in (5000, 9000)]
    og = frnn.default_opts(graphs=1)
    a = [_np(o) for o in frnn.query_batch([dev(e) for e in evs], 0.1, 256, opts=og)]
    a2 = [_np(o) for o in frnn.query_batch([dev(e) for e in evs], 0.1, 256, opts=og)]
    b = [_np(o) for o in frnn.query_batch([dev(e) for e in evs], 0.1, 256)]
    frnn.profile_enable(True)
    try:
        c = [_np(o) for o in frnn.query_batch([dev(e) for e in evs], 0.1, 256)]
    finally:
        frnn.profile_enable(False)
        frnn.profile_read()
    for x, x2, y, z in zip(a, a2, b, c):
        pinlib.assert_csr_equal(x, x2, "graph recorded vs replayed")
        pinlib.assert_csr_equal(x, y, "graph vs eager")
        pinlib.assert_csr_equal(x, z, "graph vs timed eager")


def test_batch_rejects_nonfinite(frnn):
    evs = [inputs.tracks(2000, 8, seed=1), inputs.tracks(2000, 8, seed=2)]
    evs[1][7, 3] = np.nan
    with pytest.raises(frnn.FrnnError) as e:
        frnn.query_batch([dev(x) for x in evs], 0.1, 256)
    assert e.value.name == "NONFINITE"
    outs = frnn.query_batch([dev(evs[0])], 0.1, 256)   # the library still works
    assert outs[0].nnz > 0


def test_server_alone_and_in_the_mix(orc, frnn):
    """Each served result equals the same event served alone and the
    oracle, bit for bit."""
    probe = inputs.tracks(7000, 8, seed=90)
    want = orc.frnn(probe, 0.1, 256)
    srv = frnn.Server(8, 0.1, 256, max_batch_events=16, max_inflight=2)
    t = srv.submit(probe)
    alone, tm = srv.wait(t)
    pinlib.assert_csr_equal(_np(alone), pinlib.as_tuple(want), "served alone")
    assert tm["batch_events"] == 1
    others = [inputs.tracks(n, 8, seed=91 + i) for i, n in enumerate([3000, 12000, 500, 8000] * 5)]
    tickets = []
    for i, o in enumerate(others):
        tickets.append(("other", i, srv.submit(o)))
        if i == 9:
            tickets.append(("probe", -1, srv.submit(probe)))
    batches = set()
    for kind, i, t in tickets:
        c, tm = srv.wait(t)
        batches.add(tm["batch_id"])
        if kind == "probe":
            pinlib.assert_csr_equal(_np(c), pinlib.as_tuple(want), "served in the mix")
            mixed = tm["batch_events"]
        elif i % 7 == 0:
            pinlib.assert_csr_equal(_np(c), pinlib.as_tuple(orc.frnn(others[i], 0.1, 256)), f"other {i}")
        c.release()
    say(f"probe was served in a batch of {mixed}; {len(batches)} batches")
    srv.close()


def test_server_budget_admission(frnn):
    ev = inputs.tracks(20000, 8, seed=5)
    # room for about two events at a time (each reserves about 12.8 MB at
    # admission with the default 64-key stash): later ones wait for releases
    srv = frnn.Server(8, 0.1, 256, hbm_budget_bytes=30_000_000, max_batch_events=8, max_inflight=2)
    ts = [srv.submit(ev) for _ in range(6)]
    ref = None
    for t in ts:
        c, tm = srv.wait(t)
        got = _np(c)
        c.release()
        if ref is None:
            ref = got
        pinlib.assert_csr_equal(got, ref, "budgeted run")
        assert tm["batch_events"] <= 3
    with pytest.raises(frnn.FrnnError) as e:
        srv.submit(inputs.tracks(300000, 8, seed=6))
    assert e.value.name == "BUDGET"
    srv.close()


def test_server_memory_within_budget(frnn):
    """The device bytes the server holds (inputs, its workers' contexts and
    unreleased outputs, in the pool's size classes) stay within the budget,
    plus at most one output per batch in flight (the oldest batch may always
    reserve its output); results are still exact and everything is returned
    at the end."""
    budget = 40_000_000
    evs = [inputs.tracks(n, 8, seed=120 + i) for i, n in enumerate([20000, 9000, 26000, 15000] * 3)]
    srv = frnn.Server(8, 0.1, 256, hbm_budget_bytes=budget, max_batch_events=8, max_inflight=2)
    ts = [srv.submit(e) for e in evs]
    out_bytes = []
    batches = {}
    for i, t in enumerate(ts):
        c, tm = srv.wait(t)
        got = _np(c)
        if i % 4 == 0:
            pinlib.assert_csr_equal(got, gpu_csr(evs[i], 0.1, 256), f"budgeted event {i}")
        batches.setdefault(tm["batch_id"], []).append(8 * (len(got[0]) + c.nnz))
        c.release()
    held, peak = srv.memory()
    # one output per batch in flight, with the pool's rounding (at most 1.25x
    # and a 256-byte class) and the long-row scratch block of each output
    largest = max(sum(v) for v in batches.values())
    slack = 2 * (1.25 * largest + 4096 + 512)
    say(f"server memory: peak {peak} of {budget} (+ {slack:.0f} slack), {len(batches)} batches")
    assert peak <= budget + slack
    srv.close()


def test_tuner_candidates_all_exact(frnn):
    x = dev(inputs.tracks(30000, 8, seed=7))
    best, rep = frnn.tune(x, 0.1, 256)
    assert rep["candidates_tried"] >= 10 and rep["candidates_rejected"] == 0
    assert rep["best_ms"] <= rep["default_ms"] * 1.05


def test_out_of_memory_hook(frnn):
    x = dev(inputs.tracks(5000, 8, seed=8))
    ix = frnn.build(x, 0.1)
    frnn.fail_alloc_after(1)
    with pytest.raises(frnn.FrnnError) as e:
        ix.query(None, 0.1, 16)
    frnn.fail_alloc_after(0)
    assert e.value.name == "OOM"
    c = ix.query(None, 0.1, 16)          # recovers
    assert c.nnz > 0


@pytest.mark.timeout(600)
def test_density_workload_full_size(orc, frnn):
    """1M references, 200k queries, D=12, K=64: a seeded 2% of the rows
    against the oracle, and every query's uncapped count."""
    w = inputs.c4()
    say("density workload: GPU")
    import torch
    x, q = dev(w.points), dev(w.queries)
    ix = frnn.build(x, w.r)
    capped = ix.query(q, w.r, w.K).numpy()
    full = ix.query(q, w.r, 0, want_dist2=False).numpy()
    torch.cuda.synchronize()
    check_csr_invariants(capped, len(w.points), w.K)
    rows = inputs.subset_rows(len(w.queries), 0.02, 4)
    say("density workload: oracle rows (2%)")
    check_rows(orc, capped, w.points, w.r, w.K, rows, Q=w.queries, what="density K=64")
    gdeg = np.diff(full[0])
    assert np.array_equal(np.diff(capped[0]), np.minimum(gdeg, w.K))
    say("density workload: oracle counts (all queries)")
    odeg = orc.degrees(w.points, w.r, Q=w.queries)
    assert np.array_equal(gdeg, odeg), "uncapped counts differ"
    say(f"density: mean degree {gdeg.mean():.1f}, rows over K: {(gdeg > w.K).mean():.2f}")


def test_batch_speculative_output_overflow(orc, frnn):
    """A context allocates its next output at a size learned from its previous
    run; a batch of the same class with far more pairs and long rows must
    fall back to an exact-size fill and still match the oracle, in graph
    replay and in eager launches."""
    n, r = 6000, 0.0625
    sparse = inputs.uniform_cube(n, 8, seed=90)
    dense = inputs.tracks(n, 8, track_size=700, sigma=0.002, noise_frac=0.0, seed=91)
    want = {"sparse": pinlib.as_tuple(orc.frnn(sparse, r, 0)), "dense": pinlib.as_tuple(orc.frnn(dense, r, 0))}
    assert len(want["dense"][1]) > 20 * len(want["sparse"][1])
    assert np.diff(want["dense"][0]).max() > 512  # rows sorted in global memory
    for graphs in (1, 0):
        # (adapt off: the sequence must stay in one capacity class's context)
        o_g = frnn.default_opts(graphs=graphs, adapt=0)
        for name in ("sparse", "dense", "dense", "sparse", "dense"):
            x = sparse if name == "sparse" else dense
            say(f"speculative batch {name} graphs={graphs}")
            o = frnn.query_batch([dev(x)], r, 0, opts=o_g)[0]
            pinlib.assert_csr_equal(_np(o), want[name], f"{name} graphs={graphs}")
            o.release()


def test_batch_dense_rows_adapt(orc, frnn):
    """With the default options, a capacity class whose run had long rows
    runs its later batches with the dense-row setting (256-key stash, one
    cell per work item, windows of 16); every run equals the oracle, and
    with adapt = 0 the options stay as given."""
    X, _ = inputs.clustered(12345, 0, 12, 0.022, 5)
    r = float(np.float32(0.12))
    want = pinlib.as_tuple(orc.frnn(X, r, 0, exclude_self=True))
    xd = dev(X)
    seen = []
    for rep in range(3):
        o = frnn.query_batch([xd], r, 0, exclude_self=True)[0]
        pinlib.assert_csr_equal(_np(o), want, f"adapt run {rep}")
        o.release()
        st = frnn.last_stats()
        seen.append((st["adapted"], st["stash_cap"]))
    say(f"dense-row adaptation: {seen}")
    assert seen[1] == (1, 256) and seen[2] == (1, 256)
    o0 = frnn.default_opts(adapt=0)
    for rep in range(2):
        o = frnn.query_batch([xd], r, 0, exclude_self=True, opts=o0)[0]
        pinlib.assert_csr_equal(_np(o), want, f"adapt=0 run {rep}")
        o.release()
        st = frnn.last_stats()
        assert (st["adapted"], st["stash_cap"]) == (0, 64)


def test_batch_long_rows_after_short_run(orc, frnn):
    """A context whose previous run had no row longer than the stash does not
    queue the long-row passes with the short rows; when the next batch of its
    class fits the learned capacity but has long rows, they are filled after
    the counts are read.  Graph replay and eager launches, with a 32-key
    stash."""
    n, r = 6000, 0.0625
    o32 = frnn.default_opts(stash_cap=32)
    o32g = frnn.default_opts(stash_cap=32, graphs=1)
    short = inputs.tracks(n, 8, track_size=20, sigma=0.002, noise_frac=0.0, seed=95)
    rng = np.random.default_rng(96)
    # two clusters of 40: 80 rows of 40 keys, 3,200 long-row keys (within the
    # 4,096-key floor of a context that has seen no long rows)
    mixed = np.concatenate([inputs.tracks(80, 8, track_size=40, sigma=0.002, noise_frac=0.0, seed=97),
                            inputs.uniform_cube(n - 80, 8, seed=98)])
    mixed = np.ascontiguousarray(mixed[rng.permutation(n)])
    want = {"short": pinlib.as_tuple(orc.frnn(short, r, 0)), "mixed": pinlib.as_tuple(orc.frnn(mixed, r, 0))}
    dm = np.diff(want["mixed"][0])
    assert np.diff(want["short"][0]).max() <= 32 < dm.max()
    assert dm[dm > 32].sum() <= 4096
    assert len(want["mixed"][1]) < len(want["short"][1])  # fits the capacity learned from "short"
    for graphs, oo in ((1, o32g), (0, o32)):
        for name in ("short", "mixed", "short", "mixed", "mixed"):
            x = short if name == "short" else mixed
            say(f"long rows after short run: {name} graphs={graphs}")
            o = frnn.query_batch([dev(x)], r, 0, opts=oo)[0]
            pinlib.assert_csr_equal(_np(o), want[name], f"{name} graphs={graphs}")
            o.release()
