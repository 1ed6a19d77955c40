"""CPU: the error bounds behind the library's filtered predicates, checked
against exact rational arithmetic.

The kernels decide every side test (paper sections 4.3 and 4.4.3) and every
farthest-point comparison (section 4.4.1) exactly, with three shortcuts
whose soundness rests on derived bounds:

  * the float32 orientation filter: d = fl(fl(dx*a1) - fl(dy*b1)) with the
    certificate es = fl(fl(2^-22 * fl(|P| + |Q|)) + 2^-140): |d| > es must
    imply sign(d) == sign(orient), and |d - orient| <= 2 es must hold (the
    farthest-point interval);
  * the float64 stage: D = fl(t1 - t2) with bound = fl(kD64Rel * fl(|t1| +
    |t2|)): |D - orient| <= bound;
  * the interval comparator: fl(aP - wP) > fl(aQ + wQ) must imply
    area(P) > area(Q), in both precisions.

Each operation is emulated with numpy scalars (IEEE binary32 / binary64,
round to nearest, subnormals kept, as the kernels are built: no
contraction, no flush to zero) in the order the kernels perform it, and
compared with the exact orientation of the float inputs (Fractions). The
inputs are near-degenerate triples (points a few ulps off a line) over
magnitudes from 1e-30 to 1e30, subnormal and mixed-magnitude coordinates,
and pairs of nearly tied farthest-point candidates.
"""
import os
import re
from fractions import Fraction as F

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PRED = os.path.join(ROOT, "paper_1501_04706_amd", "csrc", "sqh_pred.hpp")

F32 = np.float32
F64 = np.float64
FILTER_SCALE = F32(2.0 ** -22)
FILTER_TAU = F32(2.0 ** -140)
D64_REL = F64(4.4453e-16)


def test_constants_match_the_kernel_source():
    text = open(PRED).read()
    assert re.search(r"kFilterScale\s*=\s*0x1p-22f", text)
    assert re.search(r"kFilterTau\s*=\s*0x1p-140f", text)
    assert re.search(r"kD64Rel\s*=\s*4\.4453e-16", text)
    # the float64 constant covers 4 * 2^-53 * (1 + 2^-10)
    assert F(float(D64_REL)) >= 4 * F(2) ** -53 * (1 + F(2) ** -10)


def exact_orient(o, e, p):
    ox, oy, ex, ey, px, py = (F(float(v)) for v in (o[0], o[1], e[0], e[1], p[0], p[1]))
    return (ex - ox) * (py - oy) - (ey - oy) * (px - ox)


def orient32(o, e, p):
    """The kernel's float32 filter, operation by operation."""
    with np.errstate(all="ignore"):
        dx = F32(e[0]) - F32(o[0])
        dy = F32(e[1]) - F32(o[1])
        a1 = F32(p[1]) - F32(o[1])
        b1 = F32(p[0]) - F32(o[0])
        P = dx * a1
        Q = dy * b1
        d = P - Q
        S = abs(P) + abs(Q)
        es = S * FILTER_SCALE + FILTER_TAU
    return F32(d), F32(es)


def orient64(o, e, p):
    """The kernel's float64 stage, operation by operation."""
    a1 = F64(F32(e[0])) - F64(F32(o[0]))
    a2 = F64(F32(p[1])) - F64(F32(o[1]))
    b1 = F64(F32(e[1])) - F64(F32(o[1]))
    b2 = F64(F32(p[0])) - F64(F32(o[0]))
    t1 = a1 * a2
    t2 = b1 * b2
    bound = D64_REL * (abs(t1) + abs(t2))
    return F64(t1 - t2), F64(bound)


def _nudge(v, k):
    v = F32(v)
    for _ in range(abs(int(k))):
        v = np.nextafter(v, F32(np.inf) if k > 0 else F32(-np.inf)).astype(F32)
    return v


def adversarial_triples(seed, count):
    """(o, e, p) float32 triples with p within a few ulps of the line o-e,
    plus subnormal, mixed-magnitude and overflow-range cases."""
    rng = np.random.default_rng(seed)
    out = []
    scales = [1e-30, 1e-12, 1e-3, 1.0, 7.0, 1e3, 1e12, 1e30]
    for _ in range(count):
        s = rng.choice(scales)
        o = (rng.uniform(-1, 1, 2) * s).astype(F32)
        e = (o.astype(F64) + rng.uniform(-1, 1, 2) * s * rng.choice([1e-6, 1e-3, 1.0])).astype(F32)
        t = rng.uniform(-0.5, 1.5)
        p = (o.astype(F64) + t * (e.astype(F64) - o.astype(F64))).astype(F32)
        p = np.array([_nudge(p[0], rng.integers(-4, 5)), _nudge(p[1], rng.integers(-4, 5))], F32)
        out.append((o, e, p))
    tiny = np.float32(1e-45)
    out.append((np.array([0, 0], F32), np.array([tiny, tiny], F32), np.array([2 * tiny, 2 * tiny], F32)))
    out.append((np.array([tiny, 0], F32), np.array([0, tiny], F32), np.array([tiny, tiny], F32)))
    out.append((np.array([1e-20, 1e-20], F32), np.array([3e-20, 2e-20], F32), np.array([5e-20, 3e-20], F32)))
    out.append((np.array([1e30, -1e-30], F32), np.array([-1e30, 1e-30], F32), np.array([1e-38, 1e-38], F32)))
    out.append((np.array([3e38, -3e38], F32), np.array([-3e38, 3e38], F32), np.array([1e-45, -1e-45], F32)))
    out.append((np.array([0.1, 0.1], F32), np.array([0.3, 0.3], F32), np.array([0.2, 0.2], F32)))
    return out


def test_orient32_certificate_and_interval():
    certified = undecided = 0
    for o, e, p in adversarial_triples(11, 3000):
        d, es = orient32(o, e, p)
        exact = exact_orient(o, e, p)
        sign = (exact > 0) - (exact < 0)
        if np.isfinite(d) and np.isfinite(es):
            # the interval the farthest-point comparison uses
            assert abs(F(float(d)) - exact) <= 2 * F(float(es)), (o, e, p)
        with np.errstate(invalid="ignore"):
            ok = bool(abs(d) > es)
        if ok:
            certified += 1
            assert int(d > 0) - int(d < 0) == sign, (o, e, p)
        else:
            undecided += 1
    # both regimes are exercised
    assert certified > 500 and undecided > 500


def test_orient32_overflow_is_never_certified():
    big = F32(3e38)
    o = np.array([-big, -big], F32)
    e = np.array([big, big * F32(0.5)], F32)
    p = np.array([big, -big], F32)
    d, es = orient32(o, e, p)
    with np.errstate(invalid="ignore"):
        assert not bool(abs(d) > es)


def test_orient64_bound_encloses_exact():
    decided = 0
    for o, e, p in adversarial_triples(12, 3000):
        D, bound = orient64(o, e, p)
        exact = exact_orient(o, e, p)
        assert abs(F(float(D)) - exact) <= F(float(bound)), (o, e, p)
        if abs(D) > bound:
            decided += 1
            assert int(D > 0) - int(D < 0) == (exact > 0) - (exact < 0)
    assert decided > 1000


def _pairs(seed, count):
    """An edge and two candidates right of it whose areas nearly tie: Q is
    P moved a few ulps, or moved along a parallel of the edge."""
    rng = np.random.default_rng(seed)
    for _ in range(count):
        s = rng.choice([1e-20, 1e-3, 1.0, 1e4, 1e20])
        o = (rng.uniform(-1, 1, 2) * s).astype(F32)
        e = (o.astype(F64) + rng.uniform(-1, 1, 2) * s).astype(F32)
        nrm = np.array([e[1] - o[1], -(e[0] - o[0])], F64)  # right of o -> e
        t = rng.uniform(0, 1)
        h = rng.uniform(0.01, 1.0)
        p = (o.astype(F64) + t * (e.astype(F64) - o.astype(F64)) + h * nrm).astype(F32)
        r = rng.random()
        if r < 0.4:
            q = np.array([_nudge(p[0], rng.integers(-6, 7)), _nudge(p[1], rng.integers(-6, 7))], F32)
        elif r < 0.7:
            q = (p.astype(F64) + rng.uniform(-0.3, 0.3) * (e.astype(F64) - o.astype(F64))).astype(F32)
        else:
            # slightly nearer or farther: areas differ by a relative 1e-7 .. 1e-3
            dh = h * rng.choice([1e-7, 1e-6, 1e-5, 1e-3]) * rng.choice([-1.0, 1.0])
            q = (p.astype(F64) + dh * nrm).astype(F32)
        yield o, e, p, q


def test_float32_interval_comparator():
    decided = 0
    for o, e, p, q in _pairs(13, 3000):
        dp, ep = orient32(o, e, p)
        dq, eq = orient32(o, e, q)
        if not all(np.isfinite(v) for v in (dp, ep, dq, eq)):
            continue
        # candidates carry a = -d (area, positive right of the edge), w = 2 es
        ap, wp = F32(-dp), F32(F32(2.0) * ep)
        aq, wq = F32(-dq), F32(F32(2.0) * eq)
        area_p, area_q = -exact_orient(o, e, p), -exact_orient(o, e, q)
        if F32(ap - wp) > F32(aq + wq):
            decided += 1
            assert area_p > area_q, (o, e, p, q)
        if F32(aq - wq) > F32(ap + wp):
            decided += 1
            assert area_q > area_p, (o, e, p, q)
    assert decided > 300


def test_float64_interval_comparator():
    decided = 0
    for o, e, p, q in _pairs(14, 3000):
        Dp, bp = orient64(o, e, p)
        Dq, bq = orient64(o, e, q)
        ap, aq = F64(-Dp), F64(-Dq)
        area_p, area_q = -exact_orient(o, e, p), -exact_orient(o, e, q)
        if F64(ap - bp) > F64(aq + bq):
            decided += 1
            assert area_p > area_q, (o, e, p, q)
        if F64(aq - bq) > F64(ap + bp):
            decided += 1
            assert area_q > area_p, (o, e, p, q)
    assert decided > 1000


@pytest.mark.parametrize("scale", [0.0, 2.0 ** -30])
def test_a_weaker_certificate_is_caught(scale):
    # Planted mistakes in the bound (trusting the rounded sign outright, or a
    # relative bound far below the rounding error, without the underflow
    # term) must be caught by the same inputs: some certified sign is wrong.
    caught = False
    for o, e, p in adversarial_triples(11, 3000):
        with np.errstate(all="ignore"):
            dx = F32(e[0]) - F32(o[0])
            dy = F32(e[1]) - F32(o[1])
            P = dx * (F32(p[1]) - F32(o[1]))
            Q = dy * (F32(p[0]) - F32(o[0]))
            d = P - Q
            es = (abs(P) + abs(Q)) * F32(scale)
        exact = exact_orient(o, e, p)
        if np.isfinite(d) and bool(abs(d) > es) and int(d > 0) - int(d < 0) != (exact > 0) - (exact < 0):
            caught = True
            break
    assert caught
