"""GPU parity: the HIP path through the C ABI against the CPU oracle, bit for
bit (offsets, indices and dist2 bits; zero tolerance), plus the edge cases."""
import numpy as np
import pytest

import pinlib
from gpu_util import check_csr_invariants, check_full, check_rows, dev, gpu_csr, say
from paper_2609_31980_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def frnn():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2609_31980_amd import frnn as f
    return f


def test_uniform_4096_d3_full(orc, frnn):
    """Plain FRNN, 4,096 uniform points, D=3, r=0.1, no cap (every row)."""
    w = inputs.c1()
    say("uniform-4096-d3 full parity")
    check_full(orc, w.points, w.r, 0, what="uniform-4096")
    check_full(orc, w.points, w.r, 8, what="uniform-4096 K=8")
    check_full(orc, w.points, w.r, 0, exclude_self=True, what="uniform-4096 exclude-self")


def test_golden_cases_on_gpu(frnn):
    for name in ("p1_line.json", "p2_pythagorean.json", "p3_ties.json"):
        g, pts, r = pinlib.load_golden(name)
        for case in g["cases"]:
            K = int(case.get("K", 0))
            ex = bool(case.get("exclude_self", False))
            off, idx, d2 = gpu_csr(pts, r, K, exclude_self=ex)
            rows = [[(int(j), int(b)) for j, b in zip(idx[off[i]:off[i + 1]], d2[off[i]:off[i + 1]].view(np.uint32))]
                    for i in range(len(off) - 1)]
            want = [[(int(j), int(b, 16)) for j, b in row] for row in case["rows"]]
            assert rows == want, f"{name} K={K}"
        if "subnormal" in g:
            sub = g["subnormal"]
            sp = np.array([[int(v, 16) for v in p] for p in sub["points"]], np.uint32).view(np.float32)
            sr = float(np.uint32(int(sub["r"], 16)).view(np.float32))
            off, idx, d2 = gpu_csr(sp, sr, 0)
            rows = [[(int(j), int(b)) for j, b in zip(idx[off[i]:off[i + 1]], d2[off[i]:off[i + 1]].view(np.uint32))]
                    for i in range(len(off) - 1)]
            assert rows == [[(int(j), int(b, 16)) for j, b in row] for row in sub["rows"]], "subnormals"


def test_boundary_ladder_on_gpu(frnn):
    for r, D in ((0.1, 2), (0.12, 3), (0.3125, 5)):
        P, sb, r2b = pinlib.boundary_ladder(r, D)
        off, idx, d2 = gpu_csr(P, r, 0, Q=P[:1])
        got = sorted(zip(idx[off[0]:off[1]].tolist(), d2[off[0]:off[1]].view(np.uint32).tolist()))
        exp = sorted((j, int(sb[j])) for j in range(len(P)) if sb[j] <= r2b)
        assert got == exp, f"boundary ladder r={r} D={D}"


def test_tracks_small_full(orc, frnn):
    """A 20,000-point tracking event (spans many tiles, ragged tail)."""
    X = inputs.tracks(20000, 8, seed=21)
    say("tracks-20k full parity")
    check_full(orc, X, 0.1, 256, what="tracks-20k K=256")
    check_full(orc, X, 0.1, 4, what="tracks-20k K=4")
    check_full(orc, X, 0.1, 0, exclude_self=True, what="tracks-20k exclude-self")


def test_separate_queries_d12(orc, frnn):
    X, Q = inputs.clustered(30000, 3000, 12, 0.03, seed=8)
    say("clustered d12 separate queries")
    check_full(orc, X, inputs.C4_RADIUS, 64, Q=Q, what="clustered K=64")
    check_full(orc, X, inputs.C4_RADIUS, 0, Q=Q, what="clustered uncapped")


@pytest.mark.parametrize("D", [1, 2, 4, 5, 7, 16, 32])
def test_dimensions(orc, frnn, D):
    rng = np.random.default_rng(100 + D)
    X = rng.random((3000, D), dtype=np.float32)
    r = float(np.float32(0.05 * np.sqrt(D)))
    say(f"dimension D={D}")
    check_full(orc, X, r, 0, what=f"D={D}")
    check_full(orc, X, r, 5, what=f"D={D} K=5")


@pytest.mark.parametrize("D", [12, 32])
def test_window_sizes_by_dimension(orc, frnn, D):
    """The window's query rows take LDS in proportion to the window size and
    the row width: windows of 1, 8 and 64 queries at D = 12 and D = 32 (the
    largest row template), with and without self-exclusion."""
    rng = np.random.default_rng(300 + D)
    X = rng.random((3000, D), dtype=np.float32)
    # about 13 neighbours per row, the longest above the 64-key stash at D = 32
    r = float(np.float32({12: 0.74, 32: 1.65}[D]))
    for qpi in (1, 8, 64):
        o = frnn.default_opts(queries_per_item=qpi)
        say(f"D={D} window {qpi}")
        check_full(orc, X, r, 0, opts=o, what=f"D={D} window {qpi}")
        check_full(orc, X, r, 7, exclude_self=True, opts=o, what=f"D={D} window {qpi} K=7 exclude")


def test_empty_and_single(orc, frnn):
    X = np.zeros((1, 3), np.float32)
    check_full(orc, X, 0.1, 0, what="N=1")
    Q = np.zeros((0, 3), np.float32)
    off, idx, d2 = gpu_csr(X, 0.1, 0, Q=Q)
    assert off.tolist() == [0] and len(idx) == 0
    X0 = np.zeros((0, 3), np.float32)
    Qn = np.ones((5, 3), np.float32)
    off, idx, d2 = gpu_csr(X0, 0.1, 0, Q=Qn)
    assert off.tolist() == [0] * 6


def test_identical_points_long_rows(orc, frnn):
    """Every point identical: degree N (> the on-chip row limit), ties by id."""
    X = inputs.identical_points(700, 3)
    say("identical points, long rows")
    check_full(orc, X, 0.01, 0, what="identical uncapped")
    check_full(orc, X, 0.01, 3, what="identical K=3")
    check_full(orc, X, 0.01, 1, exclude_self=True, what="identical K=1 exclude")


def test_forced_long_row_path(orc, frnn):
    """Rows longer than a tiny on-chip cap take the global-memory sort."""
    X = inputs.tracks(8000, 8, seed=3)
    for sc in (0, 8):
        o = frnn.default_opts(row_cap_lds=2, stash_cap=sc)
        check_full(orc, X, 0.1, 0, opts=o, what=f"long path uncapped stash={sc}")
        check_full(orc, X, 0.1, 5, opts=o, what=f"long path K=5 stash={sc}")


def test_lattice_boundaries(orc, frnn):
    """Points exactly on lo + k*h and one ulp either side."""
    P = inputs.lattice_on_cells(7, 3, 0.1)
    check_full(orc, P, 0.1, 0, what="lattice r=h")
    check_full(orc, P, float(np.float32(0.1) * np.float32(1.0000001)), 0, what="lattice r~h")


def test_radius_extremes(orc, frnn):
    rng = np.random.default_rng(4)
    X = rng.random((2000, 3), dtype=np.float32)
    check_full(orc, X, 1e-6, 0, what="tiny radius")
    check_full(orc, X, 0.0, 0, what="zero radius")
    check_full(orc, X, 10.0, 16, what="one cell, kNN")


def test_denormal_differences(orc, frnn):
    rng = np.random.default_rng(5)
    X = (rng.random((500, 3)) * 1e-20).astype(np.float32)
    check_full(orc, X, float(np.float32(3e-21)), 0, what="subnormal squares")


def test_grid_options_same_output(orc, frnn):
    X = inputs.tracks(15000, 8, seed=9)
    want = orc.frnn(X, 0.1, 256)
    for kw in (dict(grid_axes_max=0), dict(grid_axes_max=1), dict(grid_axes_max=5, cells_per_point=16.0),
               dict(cell_multiple=2, grid_axes_max=4), dict(cell_multiple=3, grid_axes_max=3),
               dict(cells_per_item=4), dict(queries_per_item=1), dict(queries_per_item=64),
               dict(persistent=0), dict(blocks_per_cu=1), dict(stash_cap=0), dict(stash_cap=8),
               dict(stash_cap=32), dict(stash_cap=64), dict(stash_cap=128), dict(stash_cap=256),
               dict(stash_cap=0, persistent=0),
               dict(queries_per_item=8, persistent=1),
               dict(queries_per_item=2, cells_per_item=3)):
        got = gpu_csr(X, 0.1, 256, opts=frnn.default_opts(**kw))
        pinlib.assert_csr_equal(got, pinlib.as_tuple(want), f"opts {kw}")


def test_nonfinite_rejected(frnn):
    X = np.zeros((100, 3), np.float32)
    X[17, 2] = np.nan
    with pytest.raises(frnn.FrnnError) as e:
        frnn.build(dev(X), 0.1)
    assert e.value.name == "NONFINITE"
    Xg = np.random.default_rng(0).random((100, 3)).astype(np.float32)
    ix = frnn.build(dev(Xg), 0.1)
    Q = np.ones((5, 3), np.float32)
    Q[3, 0] = np.inf
    with pytest.raises(frnn.FrnnError) as e:
        ix.query(dev(Q), 0.1)
    assert e.value.name == "NONFINITE"


def test_radius_above_index(frnn):
    X = np.random.default_rng(0).random((100, 3)).astype(np.float32)
    ix = frnn.build(dev(X), 0.1)
    with pytest.raises(frnn.FrnnError) as e:
        ix.query(None, 0.2)
    assert e.value.name == "RADIUS"


def test_tracking_event_300k(orc, frnn):
    """The 300,000-point tracking event at full size, every row against the
    oracle's complete CSR (offsets, indices and dist2 bits), through the
    eager build + query calls, through the batched path the benchmark times
    (kernels launched one by one, run twice: the second run sizes its output
    from the first) and through the same path replayed as HIP graphs (run
    twice: recorded, then replayed), plus properties that hold at any
    size."""
    import torch
    w = inputs.c2()
    say("tracks-300k: oracle, all 300,000 rows")
    want = pinlib.as_tuple(orc.frnn(w.points, w.r, w.K))
    say("tracks-300k: GPU, eager API")
    got = gpu_csr(w.points, w.r, w.K)
    check_csr_invariants(got, len(w.points), w.K)
    pinlib.assert_csr_equal(got, want, "tracks-300k eager API")
    xd = dev(w.points)
    for graphs in (0, 1):
        og = frnn.default_opts(graphs=graphs)
        for rep in range(2):
            say(f"tracks-300k: GPU, batched path graphs={graphs} run {rep}")
            c = frnn.query_batch([xd], w.r, w.K, opts=og)[0]
            pinlib.assert_csr_equal(c.numpy(), want, f"tracks-300k batched graphs={graphs} run {rep}")
            c.release()
    torch.cuda.synchronize()
    # K=256 never binds here (max degree ~ 12): the relation is symmetric
    off, idx, d2 = got
    assert np.diff(off).max() < w.K
    i = np.repeat(np.arange(len(off) - 1), np.diff(off))
    fwd = (i.astype(np.int64) << 32) | idx
    rev = (idx.astype(np.int64) << 32) | i
    o1, o2 = np.argsort(fwd), np.argsort(rev)
    assert np.array_equal(fwd[o1], rev[o2]), "self-join adjacency not symmetric"
    assert np.array_equal(d2[o1].view(np.uint32), d2[o2].view(np.uint32)), "dist2 not symmetric"


def test_repeat_runs_identical(frnn):
    X = inputs.tracks(50000, 8, seed=12)
    a = gpu_csr(X, 0.1, 256)
    b = gpu_csr(X, 0.1, 256)
    pinlib.assert_csr_equal(a, b, "two runs")


def test_dense_ball_rows_far_above_k(orc, frnn):
    """Adversarial density: 3,000 points in a ball much smaller than r (rows
    of ~3,000 pairs, far above the on-chip limit) plus a sparse background;
    capped rows must be the first K of the full (dist2, id) order."""
    rng = np.random.default_rng(77)
    ball = (0.5 + 1e-3 * rng.standard_normal((3000, 3))).astype(np.float32)
    bg = rng.random((2000, 3)).astype(np.float32)
    X = np.concatenate([ball, bg])[rng.permutation(5000)]
    say("dense ball")
    for K in (0, 7, 1000):
        check_full(orc, X, 0.05, K, what=f"dense ball K={K}")
    check_full(orc, X, 0.05, 7, exclude_self=True, what="dense ball K=7 exclude-self")


def test_stash_sizes_rows_of_every_length(orc, frnn):
    """Clustered 12-D points with rows of every length class (empty, up to
    8, 16, 32, 64, 128, 256 and up to ~480 keys): each stash size splits them
    differently between the stash rows (lane-sorted up to 16 keys, wave-sorted
    up to the stash size) and the fill pass; all must give the oracle's CSR,
    uncapped and with a cap between the stash sizes, on the single-event and
    the batched path."""
    import torch
    X, _ = inputs.clustered(12000, 0, 12, 0.022, 5)
    r = float(np.float32(0.12))
    want = {K: pinlib.as_tuple(orc.frnn(X, r, K, exclude_self=True)) for K in (1000, 40)}
    deg = np.diff(want[1000][0])
    for lo, hi in ((0, 0), (1, 8), (9, 16), (17, 32), (33, 64), (65, 128), (129, 256), (257, 10**9)):
        assert np.any((deg >= lo) & (deg <= hi)), f"no row of length {lo}..{hi}"
    xd = torch.from_numpy(X).cuda()
    for sc in (0, 8, 16, 32, 64, 128, 256):
        o = frnn.default_opts(stash_cap=sc)
        for K in (1000, 40):
            say(f"stash {sc} K={K}")
            got = gpu_csr(X, r, K, exclude_self=True, opts=o)
            pinlib.assert_csr_equal(got, want[K], f"single stash={sc} K={K}")
            c = frnn.query_batch([xd], r, K, exclude_self=True, opts=o)[0]
            got = c.numpy()
            c.release()
            pinlib.assert_csr_equal(got, want[K], f"batched stash={sc} K={K}")


@pytest.mark.parametrize("D", [3, 8, 12])
def test_unaligned_point_arrays(orc, frnn, D):
    """Point arrays that start off a 16-byte boundary (a view one float into
    its storage) take the scalar row loads and give the same lists, through
    the eager API and the batched path replayed as HIP graphs."""
    import torch
    X = inputs.tracks(5000, D, seed=300 + D)
    Q = inputs.tracks(700, D, seed=400 + D)
    want = pinlib.as_tuple(orc.frnn(X, 0.1, 32))
    want_q = pinlib.as_tuple(orc.frnn(X, 0.1, 32, Q=Q))

    def unaligned(a):
        buf = torch.zeros(a.size + 1, dtype=torch.float32, device="cuda")
        t = buf[1:].view(a.shape)
        t.copy_(torch.from_numpy(a))
        assert t.data_ptr() % 16 != 0 and t.is_contiguous()
        return t

    xd, qd = unaligned(X), unaligned(Q)
    ix = frnn.build(xd, 0.1)
    for qq, w, what in ((None, want, "self"), (qd, want_q, "queries")):
        c = ix.query(qq, 0.1, 32)
        pinlib.assert_csr_equal(c.numpy(), w, f"unaligned D={D} api {what}")
        c.release()
    ix.close()
    og = frnn.default_opts(graphs=1)
    for _ in range(2):  # the second run replays the graphs
        o = frnn.query_batch([xd], 0.1, 32, opts=og)[0]
        pinlib.assert_csr_equal(o.numpy(), want, f"unaligned D={D} batch self")
        o.release()
        o = frnn.query_batch([xd], 0.1, 32, queries=[qd], opts=og)[0]
        pinlib.assert_csr_equal(o.numpy(), want_q, f"unaligned D={D} batch queries")
        o.release()
    torch.cuda.synchronize()
