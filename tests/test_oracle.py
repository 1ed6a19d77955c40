"""Pins for the CPU oracle (no GPU).

The oracle is Andrew's monotone chain on exact integers (``hull_exact.hull``)
and the same chain in C with expansion predicates (``oracle.c_hull``). It is
pinned to things other than itself:
  * an O(n^3) brute-force enumeration of hull edges on tiny inputs;
  * the invariant checker (strict convexity, containment, lowest index per
    position, lexicographic start), which characterises the unique answer;
  * closed forms (parabola, full grid, collinear, coincident, tiny n);
  * hand-derived fixtures in tests/golden/;
  * scipy's Qhull vertex set on general-position inputs (non-authoritative);
  * planted mistakes: mutated copies of the chain must fail these pins.
"""
import glob
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st, HealthCheck

import oracle
from oracle import hull_exact as he
from paper_1501_04706_amd import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def both(xy):
    a = he.hull(xy)
    b = [int(v) for v in oracle.c_hull(xy)]
    assert a == b, f"python oracle {a} != C oracle {b}"
    return a


def load_golden(path):
    pts, hull = [], None
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("hull:"):
            hull = [int(t) for t in line.split(":")[1].split()]
        else:
            x, y = line.split()
            pts.append((float(x), float(y)))
    xy = np.array(pts, dtype=np.float32).reshape(-1, 2)
    # every fixture value must be exact in float32
    assert np.all(xy.astype(np.float64) == np.array(pts, dtype=np.float64).reshape(-1, 2))
    return xy, hull


@pytest.mark.parametrize("path", sorted(glob.glob(os.path.join(GOLDEN, "*.txt"))))
def test_golden(path):
    xy, expect = load_golden(path)
    assert both(xy) == expect
    assert he.brute_force_hull(xy) == expect
    he.check_hull(xy, expect)


def test_degenerate_sizes():
    assert both(np.zeros((0, 2), np.float32)) == []
    assert both(np.array([[3, 4]], np.float32)) == [0]
    assert both(np.array([[1, 1], [0, 0]], np.float32)) == [1, 0]
    assert both(np.array([[1, 1], [1, 1]], np.float32)) == [0]
    assert both(np.array([[0, 0], [1, 0], [0, 1]], np.float32)) == [0, 1, 2]
    assert both(np.array([[0, 0], [0, 1], [1, 0]], np.float32)) == [0, 2, 1]


def test_parabola_closed_form():
    # distinct integers x on y = x^2 (exact in float32 for |x| <= 2048): every
    # point is a vertex, the counter-clockwise order from the leftmost point
    # is ascending x (the lower chain), closed by the chord back.
    rng = np.random.default_rng(1)
    x = rng.permutation(np.arange(-300, 301))[:400]
    xy = np.stack([x, x * x], axis=1).astype(np.float32)
    expect = [int(i) for i in np.argsort(x)]
    assert both(xy) == expect
    he.check_hull(xy, expect)


def test_full_grid_corners():
    k = 9
    g = np.array([(i, j) for j in range(k) for i in range(k)], np.float32)
    idx = lambda i, j: j * k + i
    assert both(g) == [idx(0, 0), idx(k - 1, 0), idx(k - 1, k - 1), idx(0, k - 1)]


def test_all_equal_and_collinear():
    xy = np.full((50, 2), 0.25, np.float32)
    assert both(xy) == [0]
    t = np.linspace(-1, 1, 33).astype(np.float32)
    xy = np.stack([t, 2 * t], axis=1).astype(np.float32)
    xy = xy[np.random.default_rng(3).permutation(len(xy))]
    h = both(xy)
    assert len(h) == 2
    assert tuple(xy[h[0]]) == (-1, -2) and tuple(xy[h[1]]) == (1, 2)


def test_exact_orientation_adversarial():
    # near-collinear triples on a float32 ulp grid (the "classroom example"
    # construction: perturb one point of a collinear triple by a few ulps),
    # tiny/subnormal and huge magnitudes; C expansion sign == exact ints.
    rng = np.random.default_rng(7)
    tri = []
    for _ in range(400):
        a = rng.random(2) * rng.choice([1e-30, 1e-3, 1.0, 1e3, 1e30])
        b = a + rng.standard_normal(2) * rng.choice([1e-38, 1e-5, 1.0, 1e20])
        t = rng.random() * 3 - 1
        c = a + t * (b - a)
        tri.append(np.array([a, b, c], np.float32))
        cc = np.array(c, np.float32)
        for k in range(3):
            cc = np.nextafter(cc, np.float32(np.inf)).astype(np.float32)
            tri.append(np.array([a, b, cc], np.float32))
    tri.append(np.array([[1e-45, 0], [0, 1e-45], [1e-45, 1e-45]], np.float32))
    tri.append(np.array([[3e38, -3e38], [-3e38, 3e38], [1e-45, -1e-45]], np.float32))
    tri = np.stack(tri).astype(np.float32)
    exact = he.orient_sign(tri)
    got = np.array([oracle.c_orient_sign(t[0], t[1], t[2]) for t in tri])
    assert np.array_equal(exact, got)
    # the cases are genuinely degenerate-heavy
    assert np.sum(exact == 0) > 50


def small_float_points():
    coord = st.integers(min_value=-6, max_value=6).map(lambda v: v * 0.5)
    return st.lists(st.tuples(coord, coord), min_size=0, max_size=28)


@settings(max_examples=300, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(small_float_points())
def test_brute_force_small_grid(pts):
    xy = np.array(pts, np.float32).reshape(-1, 2)
    h = both(xy)
    assert h == he.brute_force_hull(xy)
    he.check_hull(xy, h)


@settings(max_examples=150, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(st.integers(0, 2 ** 32 - 1), st.integers(1, 40))
def test_brute_force_ulp_perturbed(seed, n):
    # points within a few ulps of a line: the orientation decisions are all
    # near-degenerate, the regime where inexact predicates go wrong
    rng = np.random.default_rng(seed)
    t = rng.random(n)
    base = np.stack([0.1 + 0.7 * t, 0.3 + 0.45 * t], axis=1).astype(np.float32)
    k = rng.integers(-3, 4, size=(n, 2))
    xy = base.copy()
    for i in range(n):
        for d in range(2):
            for _ in range(abs(int(k[i, d]))):
                xy[i, d] = np.nextafter(xy[i, d], np.float32(np.sign(k[i, d]) * np.inf))
    xy = xy.astype(np.float32)
    h = both(xy)
    assert h == he.brute_force_hull(xy)


@pytest.mark.parametrize("kind", ["square", "disk", "circle", "grid"])
def test_invariants_workloads(kind):
    xy = workloads.make(kind, 3000, 11)
    h = both(xy)
    he.check_hull(xy, h)


def test_scipy_vertex_set_general_position():
    sp = pytest.importorskip("scipy.spatial")
    rng = np.random.default_rng(5)
    for _ in range(5):
        xy = rng.standard_normal((2000, 2)).astype(np.float32)
        h = both(xy)
        qh = sp.ConvexHull(xy.astype(np.float64))
        assert set(h) == set(int(v) for v in qh.vertices)


def test_square_hull_size_band():
    # statistical sanity (Renyi-Sulanke growth), not parity
    xy = workloads.square(100_000, 0)
    h = oracle.c_hull(xy)
    he.check_hull(xy, h)
    assert 15 <= len(h) <= 50
    assert abs(len(h) - he.expected_hull_size_square(100_000)) < 15


def test_c_oracle_matches_python_large():
    for kind, seed in [("square", 0), ("disk", 1), ("circle", 2), ("grid", 3)]:
        xy = workloads.make(kind, 20_000, seed)
        assert he.hull(xy) == [int(v) for v in oracle.c_hull(xy)]


def test_c_oracle_rejects_nonfinite():
    xy = np.array([[0, 0], [1, np.nan]], np.float32)
    with pytest.raises(oracle.OracleError):
        oracle.c_hull(xy)
    with pytest.raises(he.OracleInputError):
        he.hull(xy)


# ---- planted mistakes: each mutant must be caught by a pin ----

def _chain(xy, pop_if, dedup=True, drop_last=True):
    xs, ys = he.exact_ints(xy)
    order = sorted(range(len(xs)), key=lambda i: (xs[i], ys[i], i))
    u = []
    for i in order:
        if dedup and u and (xs[u[-1]], ys[u[-1]]) == (xs[i], ys[i]):
            continue
        u.append(i)
    if len(u) <= 1:
        return u[:1]

    def o(i, j, k):
        return he.orient(xs[i], ys[i], xs[j], ys[j], xs[k], ys[k])
    lo, up = [], []
    for k in u:
        while len(lo) >= 2 and pop_if(o(lo[-2], lo[-1], k)):
            lo.pop()
        lo.append(k)
    for k in reversed(u):
        while len(up) >= 2 and pop_if(o(up[-2], up[-1], k)):
            up.pop()
        up.append(k)
    return lo[:-1] + up[:-1] if drop_last else lo + up


MUTANTS = {
    "keeps collinear (pop only on < 0)": lambda xy: _chain(xy, lambda v: v < 0),
    "wrong sign (pop on >= 0)": lambda xy: _chain(xy, lambda v: v >= 0),
    "no dedup": lambda xy: _chain(xy, lambda v: v <= 0, dedup=False),
    "repeats endpoints": lambda xy: _chain(xy, lambda v: v <= 0, drop_last=False),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistakes_are_caught(name):
    # each mutant must be caught by the brute-force pin and, on its own, by
    # the invariant checker (which is the only pin at large n)
    mutant = MUTANTS[name]
    by_brute = by_check = False
    for path in sorted(glob.glob(os.path.join(GOLDEN, "*.txt"))):
        xy, expect = load_golden(path)
        got = mutant(xy)
        by_brute |= got != he.brute_force_hull(xy)
        try:
            he.check_hull(xy, got)
        except AssertionError:
            by_check = True
    assert by_brute, f"mutant '{name}' passed the brute-force pin"
    assert by_check, f"mutant '{name}' passed check_hull"


# ---- check_hull's own pins: wrong answers that break exactly one of the
# properties defining the hull, each of which check_hull must reject ----

def _square_interior():
    return load_golden(os.path.join(GOLDEN, "square_interior.txt"))


def _rejects(xy, h, what):
    with pytest.raises(AssertionError, match=what):
        he.check_hull(xy, h)


def test_check_hull_accepts_the_answer():
    xy, expect = _square_interior()
    he.check_hull(xy, expect)


def test_check_hull_rejects_a_point_outside():
    # a strictly convex counter-clockwise triangle of input points from the
    # lexicographic minimum, one corner left out: only containment fails
    xy, expect = _square_interior()
    _rejects(xy, [6, 7, 8], "outside edge")
    _rejects(xy, [6, 8, 9], "outside edge")


def test_check_hull_rejects_a_collinear_vertex():
    # the edge midpoint (0.5, 0) (index 2) between (0,0) and (1,0): inside
    # or on every edge, distinct positions, but not strictly convex
    xy, expect = _square_interior()
    _rejects(xy, [6, 2, 7, 8, 9], "strictly convex")


def test_check_hull_rejects_clockwise_order():
    xy, expect = _square_interior()
    _rejects(xy, [6, 9, 8, 7], "strictly convex|outside edge")


def test_check_hull_rejects_a_wrong_start():
    xy, expect = _square_interior()
    _rejects(xy, expect[1:] + expect[:1], "lexicographically smallest")


def test_check_hull_rejects_a_higher_duplicate_index():
    # duplicates.txt: (4,0) at indices 0 and 4; index 4 is not the lowest
    xy, expect = load_golden(os.path.join(GOLDEN, "duplicates.txt"))
    assert expect == [3, 0, 1]
    _rejects(xy, [3, 4, 1], "lowest index")


def test_check_hull_rejects_a_repeated_vertex():
    xy, expect = _square_interior()
    _rejects(xy, expect + [expect[1]], "repeated position")


def test_check_hull_rejects_index_out_of_range():
    xy, expect = _square_interior()
    _rejects(xy, [6, 7, 8, 10], "out of range")


def test_check_hull_rejects_wrong_degenerate_answers():
    xy, expect = load_golden(os.path.join(GOLDEN, "collinear.txt"))
    assert expect == [1, 2]
    _rejects(xy, [1, 0], "lexmax")           # an interior point as the far end
    _rejects(xy, [1], "several distinct positions")
    tri = np.array([[0, 0], [1, 0], [0, 1]], np.float32)
    _rejects(tri, [0, 1], "lexmax|off the line")


@pytest.mark.parametrize("kind", ["square", "disk", "circle", "grid"])
def test_sharded_oracle_equals_one_call(kind):
    # the all-core timing leg: range hulls, then the hull of their union,
    # must give the one-call result exactly (duplicates across ranges too)
    xy = workloads.make(kind, 50_000, 17)
    for threads in (1, 3, 8):
        assert np.array_equal(oracle.c_hull_sharded(xy, threads), oracle.c_hull(xy))
    dup = np.concatenate([xy[:100], xy[:100], xy[:100]])
    assert np.array_equal(oracle.c_hull_sharded(dup, 3), oracle.c_hull(dup))
