"""CPU oracle for the planar convex hull -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import or call anything under ``oracle/``. The library never
does; it shares no code with this package.

What is computed (the plain definition; the paper states the problem in its
introduction, section 1, and builds its GPU method on Andrew's monotone chain
idea in section 3):

    Input p_i = (x_i, y_i), float32, all finite.  Positions are compared by
    value, so -0.0 == +0.0.  The result is the list v_0 .. v_{h-1} of input
    indices such that
      * {p_v} is exactly the set of extreme points (vertices) of conv(p);
        points in the relative interior of a hull edge are not vertices;
      * each v_k is the lowest index among the points at that position;
      * v_0 is the lexicographically smallest position (min x, then min y);
      * the order is counter-clockwise.
    n == 0 -> [];  one distinct position -> [lowest index];
    two or more positions, all collinear -> [lexmin, lexmax].

Exactness: every finite float32 is M * 2**-149 with |M| < 2**277, so scaling
by 2**149 maps the input to Python integers and the orientation determinant
is evaluated without any rounding.

Functions:
  * ``hull``            -- Andrew's monotone chain on the sorted, deduplicated
                           points, exact integer orientation (the oracle).
  * ``brute_force_hull``-- O(n^3) enumeration of hull edges (pin, tiny n).
  * ``check_hull``      -- the invariants that characterise the unique answer.
"""
from __future__ import annotations

import math

import numpy as np

SCALE_EXP = 149  # 2**-149 is the smallest positive float32 (subnormal)


class OracleInputError(ValueError):
    pass


def exact_ints(xy: np.ndarray):
    """float32 (n, 2) -> two lists of Python ints, value * 2**149, exact.

    Scaling a float64 copy of a float32 by 2**149 is exact (a power of two,
    and the largest result 2**277 is far from float64 overflow); the scaled
    values are integers, which ``int`` converts without loss."""
    a = np.asarray(xy, dtype=np.float32).reshape(-1, 2)
    if not np.all(np.isfinite(a)):
        raise OracleInputError("non-finite coordinate")
    s = a.astype(np.float64) * (2.0 ** SCALE_EXP)
    xs = [int(v) for v in s[:, 0]]
    ys = [int(v) for v in s[:, 1]]
    return xs, ys


def orient(ax, ay, bx, by, cx, cy) -> int:
    """(b - a) x (c - a): > 0 if c is left of the directed line a->b."""
    return (bx - ax) * (cy - ay) - (by - ay) * (cx - ax)


def _sign(v: int) -> int:
    return (v > 0) - (v < 0)


def sorted_unique(xs, ys):
    """Indices sorted by (x, y, index); of each run of equal positions only
    the first (lowest index) is kept."""
    order = sorted(range(len(xs)), key=lambda i: (xs[i], ys[i], i))
    uniq = []
    for i in order:
        if uniq and xs[uniq[-1]] == xs[i] and ys[uniq[-1]] == ys[i]:
            continue
        uniq.append(i)
    return uniq


def hull(xy: np.ndarray) -> list:
    """Andrew's monotone chain with exact integer orientation."""
    xs, ys = exact_ints(xy)
    n = len(xs)
    if n == 0:
        return []
    u = sorted_unique(xs, ys)
    if len(u) == 1:
        return [u[0]]

    def o(i, j, k):
        return orient(xs[i], ys[i], xs[j], ys[j], xs[k], ys[k])

    lower = []
    for k in u:
        while len(lower) >= 2 and o(lower[-2], lower[-1], k) <= 0:
            lower.pop()
        lower.append(k)
    upper = []
    for k in reversed(u):
        while len(upper) >= 2 and o(upper[-2], upper[-1], k) <= 0:
            upper.pop()
        upper.append(k)
    return lower[:-1] + upper[:-1]


def brute_force_hull(xy: np.ndarray) -> list:
    """Hull by testing every ordered pair of distinct positions as an edge.

    (i, j) is a counter-clockwise hull edge iff no point is strictly right of
    i->j and every point on the line i-j lies in the closed segment [i, j].
    Each vertex then has exactly one outgoing edge; the list is the walk from
    the lexicographically smallest position. O(n^3) -- tiny inputs only."""
    xs, ys = exact_ints(xy)
    n = len(xs)
    if n == 0:
        return []
    # representatives: lowest index per position
    rep = {}
    for i in range(n):
        rep.setdefault((xs[i], ys[i]), i)
    pts = sorted(rep.values())
    if len(pts) == 1:
        return [pts[0]]
    lexmin = min(pts, key=lambda i: (xs[i], ys[i]))
    lexmax = max(pts, key=lambda i: (xs[i], ys[i]))

    def on_closed_segment(i, j, k):
        dx, dy = xs[j] - xs[i], ys[j] - ys[i]
        t = (xs[k] - xs[i]) * dx + (ys[k] - ys[i]) * dy
        return 0 <= t <= dx * dx + dy * dy

    if all(orient(xs[lexmin], ys[lexmin], xs[lexmax], ys[lexmax], xs[k], ys[k]) == 0 for k in pts):
        return [lexmin, lexmax]
    nxt = {}
    for i in pts:
        for j in pts:
            if i == j:
                continue
            ok = True
            for k in pts:
                s = orient(xs[i], ys[i], xs[j], ys[j], xs[k], ys[k])
                if s < 0 or (s == 0 and not on_closed_segment(i, j, k)):
                    ok = False
                    break
            if ok:
                if i in nxt:
                    raise AssertionError("vertex with two outgoing hull edges")
                nxt[i] = j
    out = [lexmin]
    while True:
        j = nxt[out[-1]]
        if j == lexmin:
            break
        out.append(j)
        if len(out) > len(pts):
            raise AssertionError("hull edge walk does not close")
    if len(out) != len(nxt):
        raise AssertionError("hull edges do not form one cycle")
    return out


def check_hull(xy: np.ndarray, h) -> None:
    """Raise AssertionError unless ``h`` is the hull index list defined above.

    Checks: indices in range; v_0 at the lexicographically smallest position;
    each v_k is the lowest index at its position; positions distinct; for
    h >= 3 every cyclic triple turns strictly left and no input point is
    strictly right of any edge; h == 2 means all points lie on the closed
    segment [lexmin, lexmax]; h == 1 means all points coincide. A convex
    polygon with input points as vertices, no collinear vertices and every
    point inside or on it is the hull, so these checks pin the answer."""
    xs, ys = exact_ints(xy)
    n = len(xs)
    h = [int(v) for v in h]
    if n == 0:
        assert h == [], "empty input must give an empty hull"
        return
    assert 1 <= len(h) <= n
    for v in h:
        assert 0 <= v < n, f"index {v} out of range"
    first = {}
    for i in range(n):
        first.setdefault((xs[i], ys[i]), i)
    for v in h:
        assert first[(xs[v], ys[v])] == v, f"index {v} is not the lowest index at its position"
    pos = [(xs[v], ys[v]) for v in h]
    assert len(set(pos)) == len(pos), "repeated position in hull"
    lm = min(first.keys())
    assert pos[0] == lm, "hull does not start at the lexicographically smallest point"
    if len(h) == 1:
        assert len(first) == 1, "one vertex but several distinct positions"
        return
    if len(h) == 2:
        a, b = h
        assert pos[1] == max(first.keys()), "two-vertex hull must end at lexmax"
        for k in range(n):
            assert orient(xs[a], ys[a], xs[b], ys[b], xs[k], ys[k]) == 0, "point off the line"
        return
    m = len(h)
    for k in range(m):
        a, b, c = h[k], h[(k + 1) % m], h[(k + 2) % m]
        assert orient(xs[a], ys[a], xs[b], ys[b], xs[c], ys[c]) > 0, "hull not strictly convex / not CCW"
    for k in range(m):
        a, b = h[k], h[(k + 1) % m]
        ax, ay, bx, by = xs[a], ys[a], xs[b], ys[b]
        ex, ey = bx - ax, by - ay
        for i in range(n):
            assert ex * (ys[i] - ay) - ey * (xs[i] - ax) >= 0, f"point {i} outside edge {a}->{b}"


def orient_sign(points: np.ndarray) -> np.ndarray:
    """Exact orientation signs for a (k, 3, 2) float32 array of triples."""
    p = np.asarray(points, dtype=np.float32).reshape(-1, 3, 2)
    out = np.empty(len(p), dtype=np.int8)
    for t in range(len(p)):
        xs, ys = exact_ints(p[t])
        out[t] = _sign(orient(xs[0], ys[0], xs[1], ys[1], xs[2], ys[2]))
    return out


def expected_hull_size_square(n: int) -> float:
    """Renyi-Sulanke: the expected vertex count of the hull of n uniform
    points in a square grows as (8/3) ln n + O(1). A statistical sanity
    band only, never a parity check."""
    return 8.0 / 3.0 * math.log(n)
