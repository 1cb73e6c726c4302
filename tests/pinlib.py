"""Independent routes to the neighbour relation, used to pin the CPU oracle.

None of these share code with the oracle (a C library) or with the GPU path:

* exact rational arithmetic (`fractions.Fraction`) with an explicit
  round-to-nearest-even to float32, for tiny hand-built cases;
* a float32 NumPy evaluation with one ufunc per rounded operation;
* a float64 recomputation, which the float32 result must match except within
  the forward-error band of a D-term float32 sum;
* a sorted-range search for D = 1 and SciPy KD-trees, different algorithms
  that give the same answer away from the boundary.

Each `pin_*` function raises AssertionError when the oracle object it is given
disagrees; the test suite runs them on the real oracle (all must pass) and on
deliberately broken copies of it (each copy must fail at least one).
"""
from __future__ import annotations

import json
import os
from fractions import Fraction

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

U32 = np.uint32


# ----------------------------------------------------- exact float32 rounding
def f32_to_frac(x) -> Fraction:
    return Fraction(float(np.float32(x)))


def rne32(x: Fraction) -> Fraction:
    """Round a rational to the nearest float32 value, ties to even, with
    gradual underflow (subnormal spacing 2^-149).  Overflow is not handled."""
    if x == 0:
        return Fraction(0)
    sign = -1 if x < 0 else 1
    a = abs(x)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    q = max(e - 23, -149)            # exponent of one unit in the last place
    m = a / Fraction(2) ** q         # significand in units of 2^q
    lo = m.numerator // m.denominator
    rem = m - lo
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and lo % 2 == 1):
        lo += 1
    return sign * Fraction(lo) * Fraction(2) ** q


def frac_to_bits(x: Fraction) -> int:
    v = np.float32(float(x))
    assert Fraction(float(v)) == x, "value is not a float32"
    return int(v.view(U32))


def exact_r2(r) -> Fraction:
    """fl32(r * r) for a float32 r, by exact arithmetic."""
    rf = f32_to_frac(r)
    return rne32(rf * rf)


def exact_dist2(q, x) -> Fraction:
    """The canonical float32 evaluation, every operation rounded explicitly:
    s = +0; per axis t = fl(q_d - x_d), u = fl(t*t), s = fl(s + u)."""
    s = Fraction(0)
    for qd, xd in zip(q, x):
        t = rne32(f32_to_frac(qd) - f32_to_frac(xd))
        u = rne32(t * t)
        s = rne32(s + u)
    return s


def exact_rows(X, r, K=0, Q=None, exclude_self=False):
    """Rows [(j, dist2 bits)] by exact arithmetic; tiny inputs only."""
    Q = X if Q is None else Q
    r2 = exact_r2(r)
    rows = []
    for i, q in enumerate(Q):
        hits = []
        for j, x in enumerate(X):
            if exclude_self and i == j:
                continue
            s = exact_dist2(q, x)
            if s <= r2:
                hits.append((s, j))
        hits.sort()
        if K > 0:
            hits = hits[:K]
        rows.append([(j, frac_to_bits(s)) for s, j in hits])
    return rows


def csr_rows(csr):
    out = []
    for i in range(len(csr.offsets) - 1):
        a, b = int(csr.offsets[i]), int(csr.offsets[i + 1])
        out.append([(int(j), int(v)) for j, v in
                    zip(csr.indices[a:b], csr.dist2[a:b].view(U32))])
    return out


# ------------------------------------------------- float32 NumPy, per axis
def numpy_dist2(Q, X) -> np.ndarray:
    """float32 [M, N] squared distances, one ufunc per rounded operation, axes
    added in order d = 0 .. D-1 (no np.sum: it adds pairwise)."""
    Q = np.asarray(Q, dtype=np.float32)
    X = np.asarray(X, dtype=np.float32)
    s = np.zeros((Q.shape[0], X.shape[0]), dtype=np.float32)
    for d in range(Q.shape[1]):
        t = np.subtract(Q[:, d][:, None], X[:, d][None, :], dtype=np.float32)
        u = np.multiply(t, t, dtype=np.float32)
        s = np.add(s, u, dtype=np.float32)
    return s


def numpy_csr(X, r, K=0, Q=None, self_ids=None):
    """(offsets, indices, dist2) from numpy_dist2; ordering by (s, j)."""
    Qa = X if Q is None else Q
    r32 = np.float32(r)
    r2 = np.multiply(r32, r32, dtype=np.float32)
    offs = [0]
    idx, dd = [], []
    for a in range(0, len(Qa), 512):
        S = numpy_dist2(Qa[a:a + 512], X)
        for k in range(S.shape[0]):
            row = S[k]
            j = np.nonzero(row <= r2)[0]
            if self_ids is not None:
                j = j[j != self_ids[a + k]]
            s = row[j]
            o = np.lexsort((j, s))
            j, s = j[o], s[o]
            if K > 0:
                j, s = j[:K], s[:K]
            idx.append(j.astype(np.int32))
            dd.append(s.astype(np.float32))
            offs.append(offs[-1] + len(j))
    cat = (lambda L, t: np.concatenate(L).astype(t) if L else np.zeros(0, t))
    return np.asarray(offs, np.int64), cat(idx, np.int32), cat(dd, np.float32)


def assert_csr_equal(a, b, what=""):
    """Bitwise equality of two CSRs given as (offsets, indices, dist2)."""
    ao, ai, ad = a
    bo, bi, bd = b
    assert np.array_equal(np.asarray(ao, np.int64), np.asarray(bo, np.int64)), f"{what}: offsets differ"
    assert np.array_equal(np.asarray(ai, np.int32), np.asarray(bi, np.int32)), f"{what}: indices differ"
    assert np.array_equal(np.asarray(ad, np.float32).view(U32),
                          np.asarray(bd, np.float32).view(U32)), f"{what}: dist2 bits differ"


def as_tuple(csr):
    return csr.offsets, csr.indices, csr.dist2


# -------------------------------------------------- golden hand-built cases
def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        g = json.load(f)
    pts = np.array([[np.uint32(int(v, 16)) for v in p] for p in g["points"]], dtype=np.uint32).view(np.float32)
    r = np.uint32(int(g["r"], 16)).view(np.float32)
    return g, pts, float(r)


def golden_rows(g, key="rows"):
    return [[(int(j), int(b, 16)) for j, b in row] for row in g[key]]


# ------------------------------------------------------------------- pins
def pin_golden_cases(o):
    """P1-P3: hand-built cases with exactly derived answers."""
    for name in ("p1_line.json", "p2_pythagorean.json", "p3_ties.json"):
        g, pts, r = load_golden(name)
        for case in g["cases"]:
            K = int(case.get("K", 0))
            ex = bool(case.get("exclude_self", False))
            got = csr_rows(o.frnn(pts, r, K, exclude_self=ex))
            want = [[(int(j), int(b, 16)) for j, b in row] for row in case["rows"]]
            assert got == want, f"{name} K={K} exclude_self={ex}: {got} != {want}"
        if "subnormal" in g:
            sub = g["subnormal"]
            sp = np.array([[int(v, 16) for v in p] for p in sub["points"]], np.uint32).view(np.float32)
            sr = float(np.uint32(int(sub["r"], 16)).view(np.float32))
            want = [[(int(j), int(b, 16)) for j, b in row] for row in sub["rows"]]
            assert csr_rows(o.frnn(sp, sr, 0)) == want, f"{name}: subnormal case"


def pin_exact_small(o, seed=7):
    """Brute force by exact rational arithmetic on tiny random inputs,
    including a query set distinct from the references and self-exclusion."""
    rng = np.random.default_rng(seed)
    for D in (1, 2, 3, 5):
        X = rng.random((14, D), dtype=np.float32) * np.float32(0.5)
        Q = rng.random((6, D), dtype=np.float32) * np.float32(0.5)
        r = float(np.float32(0.21))
        for K in (0, 3):
            assert csr_rows(o.frnn(X, r, K)) == exact_rows(X, r, K), f"self D={D} K={K}"
            assert csr_rows(o.frnn(X, r, K, Q=Q)) == exact_rows(X, r, K, Q=Q), f"Q D={D} K={K}"
        assert csr_rows(o.frnn(X, r, 0, exclude_self=True)) == \
            exact_rows(X, r, 0, exclude_self=True), f"exclude D={D}"
        # counts only: the exact row lengths, with separate queries and
        # with self-exclusion given as explicit ids
        lens = [len(row) for row in exact_rows(X, r, 0, Q=Q)]
        assert o.degrees(X, r, Q=Q).tolist() == lens, f"degrees Q D={D}"
        lens = [len(row) for row in exact_rows(X, r, 0, exclude_self=True)]
        assert o.degrees(X, r, Q=X, self_ids=np.arange(len(X))).tolist() == lens, f"degrees excl D={D}"


def pin_numpy_bitwise(o, X, r, K=0, Q=None, self_ids=None):
    """P7: the float32 per-axis NumPy route gives the same CSR bit for bit."""
    want = numpy_csr(X, r, K, Q=Q, self_ids=self_ids)
    got = o.frnn(X, r, K, Q=Q, self_ids=self_ids)
    assert_csr_equal(as_tuple(got), want, "numpy route")


def numpy_degrees(X, r, Q=None, self_ids=None) -> np.ndarray:
    """Uncapped in-radius counts per query from the float32 per-axis NumPy
    route (numpy_dist2), leaving out self_ids[i] from row i when given."""
    Qa = X if Q is None else Q
    r32 = np.float32(r)
    r2 = np.multiply(r32, r32, dtype=np.float32)
    out = np.zeros(len(Qa), np.int64)
    for a in range(0, len(Qa), 512):
        hit = numpy_dist2(Qa[a:a + 512], X) <= r2
        if self_ids is not None:
            k = np.arange(hit.shape[0])
            sid = np.asarray(self_ids[a:a + 512], np.int64)
            ok = (sid >= 0) & (sid < X.shape[0])
            hit[k[ok], sid[ok]] = False
        out[a:a + 512] = hit.sum(axis=1)
    return out


def pin_degrees(o, X, r, Q=None, self_ids=None, caps=(0, 4)):
    """The counts-only entry point and the CSR's degree field: both equal
    the uncapped row lengths of the independent NumPy route (Eq. 1 counted
    before the K cap), and the CSR's row lengths equal min(degree, K)."""
    want = numpy_degrees(X, r, Q=Q, self_ids=self_ids)
    got = o.degrees(X, r, Q=Q, self_ids=self_ids)
    assert np.array_equal(got, want), "degrees: counts-only path differs"
    for K in caps:
        c = o.frnn(X, r, K, Q=Q, self_ids=self_ids)
        assert np.array_equal(c.degree, want), f"degrees: CSR degree field differs (K={K})"
        lens = np.minimum(want, K) if K > 0 else want
        assert np.array_equal(np.diff(c.offsets), lens), f"degrees: row lengths differ (K={K})"


def pin_fp64_band(o, X, r, Q=None):
    """P6: float64 recomputation.  Membership may differ only where
    |s64 - r^2| is inside the forward-error band of the float32 evaluation,
    and every reported dist2 is within that band of s64."""
    Qa = X if Q is None else Q
    D = X.shape[1]
    got = o.frnn(X, r, 0, Q=Q)
    Qd = Qa.astype(np.float64)
    Xd = X.astype(np.float64)
    rr = float(np.float32(r)) ** 2
    eps = 2.0 ** -24
    band = (D + 4) * eps
    flagged = []
    for a in range(0, len(Qa), 256):
        S64 = np.zeros((min(256, len(Qa) - a), len(X)))
        for d in range(D):
            S64 += (Qd[a:a + 256, d][:, None] - Xd[None, :, d]) ** 2
        for k in range(S64.shape[0]):
            i = a + k
            lo, hi = int(got.offsets[i]), int(got.offsets[i + 1])
            mem32 = np.zeros(len(X), bool)
            mem32[got.indices[lo:hi]] = True
            mem64 = S64[k] <= rr
            dis = np.nonzero(mem32 != mem64)[0]
            for j in dis:
                assert abs(S64[k, j] - rr) <= band * rr + 1e-45, \
                    f"pair ({i},{j}) disagrees outside the rounding band"
                flagged.append((i, int(j)))
            s32 = got.dist2[lo:hi].astype(np.float64)
            s64 = S64[k, got.indices[lo:hi]]
            assert np.all(np.abs(s32 - s64) <= band * s64 + 1e-44), f"row {i}: dist2 off"
    return flagged


def pin_symmetry(o, X, r):
    """P4: in an uncapped self-join s(i,j) and s(j,i) are the same float and
    the adjacency is symmetric."""
    c = o.frnn(X, r, 0)
    i = np.repeat(np.arange(len(X)), np.diff(c.offsets))
    fwd = {(int(a), int(b)): int(v) for a, b, v in zip(i, c.indices, c.dist2.view(U32))}
    for (a, b), v in fwd.items():
        assert fwd.get((b, a)) == v, f"asymmetric pair ({a},{b})"


def pin_invariances(o, X, r, K, seed=3):
    """P5: relabelling the references, scaling everything by 2^k, and
    reflecting one axis leave the rows unchanged (dist2 scales by 4^k)."""
    base = o.frnn(X, r, K)
    rng = np.random.default_rng(seed)
    p = rng.permutation(len(X))
    Xp = X[p]
    cp = o.frnn(Xp, r, K, Q=X)   # queries in the original order
    idx = p[cp.indices]          # permuted slot k holds original point p[k]
    # map back to original ids and re-sort each row by (s, j)
    offs = cp.offsets
    new_i = np.empty_like(cp.indices)
    new_d = np.empty_like(cp.dist2)
    for q in range(len(X)):
        a, b = int(offs[q]), int(offs[q + 1])
        j, s = idx[a:b], cp.dist2[a:b]
        oo = np.lexsort((j, s))
        new_i[a:b], new_d[a:b] = j[oo], s[oo]
    # with a cap, relabelling may change which tied-distance ids survive the
    # cut, so compare uncapped rows only when K binds
    if K <= 0:
        assert_csr_equal(as_tuple(base), (offs, new_i, new_d), "permutation")
    for k in (-3, 5):
        sc = np.float32(2.0 ** k)
        cs = o.frnn(X * sc, float(np.float32(r) * sc), K)
        assert np.array_equal(cs.offsets, base.offsets) and np.array_equal(cs.indices, base.indices), \
            f"scaling by 2^{k} changed the rows"
        assert np.array_equal((base.dist2 * np.float32(4.0 ** k)).view(U32), cs.dist2.view(U32)), \
            f"scaling by 2^{k}: dist2 not scaled exactly"
    Xr = X.copy()
    Xr[:, 0] = -Xr[:, 0]
    assert_csr_equal(as_tuple(base), as_tuple(o.frnn(Xr, r, K)), "reflection")


def pin_sorted_range_1d(o, n=3000, seed=11):
    """P8a: for D = 1, fl32(fl32(q - x)^2) is monotone in x on each side of
    q, so each row is a contiguous range of the sorted points; find it by
    bisection and compare with the brute force."""
    rng = np.random.default_rng(seed)
    X = (rng.random((n, 1), dtype=np.float32) * np.float32(4.0)).astype(np.float32)
    r = float(np.float32(0.01))
    r32 = np.float32(r)
    r2 = np.multiply(r32, r32, dtype=np.float32)
    order = np.argsort(X[:, 0], kind="stable")
    xs = X[order, 0]
    c = o.frnn(X, r, 0)

    def hit(q, x):
        t = np.subtract(q, x, dtype=np.float32)
        return np.multiply(t, t, dtype=np.float32) <= r2

    for i in range(0, n, 7):
        q = X[i, 0]
        c0 = int(np.searchsorted(xs, q))
        lo, hi = 0, c0              # first index whose point is a hit (left side)
        while lo < hi:
            m = (lo + hi) // 2
            if hit(q, xs[m]):
                hi = m
            else:
                lo = m + 1
        a = lo
        lo, hi = c0, n               # first index past the right-side hits
        while lo < hi:
            m = (lo + hi) // 2
            if hit(q, xs[m]):
                lo = m + 1
            else:
                hi = m
        want = set(order[a:lo].tolist())
        got = set(c.row(i)[0].tolist())
        assert got == want, f"D=1 row {i}: sorted-range search differs"


def pin_kdtree(o, X, r, flagged):
    """P8b: SciPy's float64 ball query gives the same sets except the pairs
    the float64 recheck flagged as within the rounding band."""
    from scipy.spatial import cKDTree
    t = cKDTree(X.astype(np.float64))
    c = o.frnn(X, r, 0)
    fl = set(flagged)
    balls = t.query_ball_point(X.astype(np.float64), float(np.float32(r)))
    for i, b in enumerate(balls):
        a = set(b)
        g = set(c.row(i)[0].tolist())
        for j in a ^ g:
            assert (i, j) in fl, f"kd-tree and oracle differ on ({i},{j})"


def pin_knn(o, X, K=5):
    """P8c: with a radius that covers every point, the cap gives exact kNN;
    compare with a KD-tree kNN away from near-ties at the K-th distance."""
    from scipy.spatial import cKDTree
    big = float(np.float32(64.0))
    c = o.frnn(X, big, K)
    t = cKDTree(X.astype(np.float64))
    d64, j64 = t.query(X.astype(np.float64), k=K + 1)
    for i in range(len(X)):
        got = c.row(i)[0].tolist()
        assert len(got) == K
        # skip rows whose K-th and (K+1)-th neighbours are near-tied
        if d64[i, K] - d64[i, K - 1] <= 1e-5 * max(d64[i, K], 1e-30):
            continue
        assert set(got) == set(j64[i, :K].tolist()), f"kNN row {i} differs"


def boundary_ladder(r: float, D: int = 2, per_step: int = 3, seed: int = 5):
    """Points x around the origin whose float32 s(0, x) lands exactly on r2
    and on 1 and 2 ulps either side of it.  Found by a float32 search and
    confirmed by exact arithmetic.  Returns (points, s_bits, r2_bits) with the
    origin as point 0."""
    rng = np.random.default_rng(seed)
    r32 = np.float32(r)
    r2 = exact_r2(r32)
    r2b = frac_to_bits(r2)
    want = {k: [] for k in (-2, -1, 0, 1, 2)}
    pts = [np.zeros(D, np.float32)]
    sbits = [0]
    tries = 0
    while any(len(v) < per_step for v in want.values()) and tries < 20000:
        tries += 1
        x = np.zeros(D, np.float32)
        x[:D - 1] = (rng.random(D - 1) * 0.5 * r).astype(np.float32)
        rest = float(r32) ** 2 - float(np.sum(x[:D - 1].astype(np.float64) ** 2))
        b = np.float32(np.sqrt(max(rest, 0.0)))
        for step in range(-6, 7):
            y = x.copy()
            y[D - 1] = b
            for _ in range(abs(step)):
                y[D - 1] = np.nextafter(y[D - 1], np.float32(np.inf if step > 0 else -np.inf))
            s = exact_dist2(np.zeros(D, np.float32), y)
            k = frac_to_bits(s) - r2b
            if k in want and len(want[k]) < per_step:
                want[k].append(y)
                pts.append(y)
                sbits.append(frac_to_bits(s))
    assert all(len(v) == per_step for v in want.values()), "ladder search failed"
    return np.asarray(pts, np.float32), np.asarray(sbits), r2b


def pin_boundary_ladder(o):
    """Pairs exactly on the boundary and one or two ulps either side: the
    origin's row must hold exactly those with s <= r2, with those s bits."""
    for r, D in ((0.1, 2), (0.12, 3), (0.3125, 5)):
        P, sb, r2b = boundary_ladder(r, D)
        c = o.frnn(P, r, 0, Q=P[:1])
        got = sorted(zip(c.row(0)[0].tolist(), c.row(0)[1].view(U32).tolist()))
        exp = sorted((j, int(sb[j])) for j in range(len(P)) if sb[j] <= r2b)
        assert got == exp, f"boundary ladder r={r} D={D}"
        # the counts-only path decides the same pairs
        assert o.degrees(P, r, Q=P[:1]).tolist() == [len(exp)], f"boundary ladder degrees r={r} D={D}"
        assert c.degree.tolist() == [len(exp)], f"boundary ladder degree field r={r} D={D}"


ALL_FAST_PINS = ("golden", "boundary", "exact", "numpy", "degrees", "fp64", "symmetry", "invariance",
                 "range1d")


def run_fast_pins(o, X):
    """The quick pin set used on broken copies of the oracle; stops at the
    first failure and returns its name, or None when every pin passed."""
    r = float(np.float32(0.1))
    Q = (X[:200] + np.float32(0.01)).astype(np.float32)
    sub = np.arange(3, len(X), 5)     # a query subset whose self ids are not 0..M-1
    steps = {
        "golden": lambda: pin_golden_cases(o),
        "boundary": lambda: pin_boundary_ladder(o),
        "exact": lambda: pin_exact_small(o),
        "numpy": lambda: (pin_numpy_bitwise(o, X, r, 0), pin_numpy_bitwise(o, X, r, 4),
                          pin_numpy_bitwise(o, X, r, 0, Q=Q)),
        "degrees": lambda: (pin_degrees(o, X, r),
                            pin_degrees(o, X, r, Q=X[sub], self_ids=sub),
                            pin_degrees(o, X, r, Q=Q)),
        "fp64": lambda: pin_fp64_band(o, X, r),
        "symmetry": lambda: pin_symmetry(o, X, r),
        "invariance": lambda: pin_invariances(o, X, r, 0),
        "range1d": lambda: pin_sorted_range_1d(o, 800),
    }
    for name in ALL_FAST_PINS:
        try:
            steps[name]()
        except AssertionError:
            return name
    return None
