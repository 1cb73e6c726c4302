"""Pins of the CPU oracle against what the paper and the mathematics fix.

Every check here reaches the answer by a route that shares nothing with the
oracle: hand-derived golden rows, exact rational arithmetic, a float32 NumPy
evaluation, a float64 recomputation inside its rounding band, a sorted-range
search (D = 1), KD-trees, invariances and generator statistics."""
import numpy as np
import pytest

import pinlib
from paper_2609_31980_amd import inputs


@pytest.fixture(scope="module")
def c1():
    return inputs.c1()


def test_r2_reading(orc):
    # fl32(0.1f * 0.1f) = 0x3c23d70b, one ulp above the float32 nearest 0.01
    assert int(orc.r2(0.1).view(np.uint32)) == 0x3C23D70B
    assert int(np.float32(0.01).view(np.uint32)) == 0x3C23D70A
    for r in (0.1, 0.12, 0.3125, 1e-20, 3.0):
        assert pinlib.frac_to_bits(pinlib.exact_r2(r)) == int(orc.r2(r).view(np.uint32))


def test_golden_values_are_exact():
    """The stored golden rows agree with exact rational arithmetic."""
    for name in ("p1_line.json", "p2_pythagorean.json", "p3_ties.json"):
        g, pts, r = pinlib.load_golden(name)
        for case in g["cases"]:
            want = [[(int(j), int(b, 16)) for j, b in row] for row in case["rows"]]
            assert pinlib.exact_rows(pts, r, int(case.get("K", 0)),
                                     exclude_self=bool(case.get("exclude_self", False))) == want


def test_golden_cases(orc):
    pinlib.pin_golden_cases(orc)


def test_boundary_ladder(orc):
    pinlib.pin_boundary_ladder(orc)


def test_exact_small(orc):
    pinlib.pin_exact_small(orc)


def test_numpy_bitwise_c1(orc, c1):
    pinlib.pin_numpy_bitwise(orc, c1.points, c1.r, 0)
    pinlib.pin_numpy_bitwise(orc, c1.points, c1.r, 8)


def test_numpy_bitwise_queries_and_exclusion(orc):
    w = inputs.c2()
    X = w.points[:20000]
    Q = X[:300]
    pinlib.pin_numpy_bitwise(orc, X, w.r, 256, Q=Q)
    pinlib.pin_numpy_bitwise(orc, X, w.r, 0, Q=Q, self_ids=np.arange(300))


def test_numpy_bitwise_d12(orc):
    x, q = inputs.clustered(20000, 300, 12, 0.03, seed=5)
    pinlib.pin_numpy_bitwise(orc, x, inputs.C4_RADIUS, 64, Q=q)


def test_degrees_uniform_cube(orc, c1):
    """Counts only and the CSR's degree field against the NumPy route."""
    pinlib.pin_degrees(orc, c1.points, c1.r, caps=(0, 4, 8))


def test_degrees_tracks_subset_self_ids(orc):
    w = inputs.c2()
    X = w.points[:30000]
    s = inputs.subset_rows(len(X), 0.02, 17)
    pinlib.pin_degrees(orc, X, w.r, Q=X[s], self_ids=s, caps=(0, 4, 256))


def test_degrees_clustered_d12_queries(orc):
    x, q = inputs.clustered(30000, 400, 12, 0.03, seed=8)
    pinlib.pin_degrees(orc, x, inputs.C4_RADIUS, Q=q, caps=(0, 4, 64))


def test_fp64_band_c1(orc, c1):
    flagged = pinlib.pin_fp64_band(orc, c1.points, c1.r)
    assert len(flagged) <= 8


def test_symmetry(orc, c1):
    pinlib.pin_symmetry(orc, c1.points, c1.r)


def test_invariances(orc, c1):
    pinlib.pin_invariances(orc, c1.points, c1.r, 0)
    pinlib.pin_invariances(orc, c1.points, c1.r, 5)


def test_sorted_range_1d(orc):
    pinlib.pin_sorted_range_1d(orc)


def test_kdtree_ball(orc, c1):
    flagged = pinlib.pin_fp64_band(orc, c1.points, c1.r)
    pinlib.pin_kdtree(orc, c1.points, c1.r, flagged)


def test_knn_special_case(orc):
    rng = np.random.default_rng(9)
    X = rng.random((500, 4), dtype=np.float32)
    pinlib.pin_knn(orc, X, 7)


def test_degree_statistics(orc, c1):
    # C1: interior expectation 4096 * (4/3) pi 0.1^3 = 17.2 (boundary lowers it)
    deg = orc.frnn(c1.points, c1.r).degree
    assert 15.5 < deg.mean() < 17.2
    # tracking event: same-track pairs within r with probability
    # P(chi2_8 <= 0.01 / 0.0008) ~ 0.87, so ~ 1 + 0.87 * 11 * 0.9^2 + noise
    w = inputs.c2()
    s = inputs.subset_rows(len(w.points), 0.005, 1)
    d = orc.degrees(w.points, w.r, Q=w.points[s])
    assert 7.5 < d.mean() < 10.0


def test_nonfinite_rejected(orc):
    X = np.zeros((4, 3), np.float32)
    X[2, 1] = np.nan
    import oracle
    with pytest.raises(oracle.OracleError):
        orc.frnn(X, 0.1)
    X[2, 1] = np.inf
    with pytest.raises(oracle.OracleError):
        orc.frnn(X, 0.1)


def test_empty_inputs(orc):
    X = np.zeros((0, 3), np.float32)
    c = orc.frnn(X, 0.1)
    assert c.offsets.tolist() == [0] and c.nnz == 0
    Q = np.zeros((3, 3), np.float32)
    c = orc.frnn(X, 0.1, Q=Q)
    assert c.offsets.tolist() == [0, 0, 0, 0]


def test_thread_count_irrelevant(orc, c1):
    a = orc.frnn(c1.points, c1.r, 0, nthreads=1)
    b = orc.frnn(c1.points, c1.r, 0, nthreads=7)
    pinlib.assert_csr_equal(pinlib.as_tuple(a), pinlib.as_tuple(b), "threads")
