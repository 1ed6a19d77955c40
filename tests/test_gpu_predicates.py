"""GPU unit tests of the hull path's building blocks against exact arithmetic.

The end-to-end parity tests only see a misclassified point if it changes
the hull; these run the device's own orientation filters, exact fallback,
farthest-point order and workgroup scan (through the C-ABI test hooks) on
adversarial cases and check every decision exactly:
- the sign the kernels use equals the exact orientation sign;
- the semi-static filter's value d and bound es: |d - orient| <= 2 es, and
  a certified sign (|d| > es) is the exact sign;
- the static line filter's t and m: |t - orient| < m (the certificate the
  streaming kernels use for |t| > m);
- the farthest-point order (section 4.4.1 with the tie rules of the
  method's readings) is the exact order, antisymmetric;
- the DPP workgroup scan equals numpy's cumulative sums.
"""
import sys
from fractions import Fraction as F

import numpy as np
import pytest

from oracle import hull_exact as he
from paper_1501_04706_amd import sqh

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[case] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "gpu tests need a HIP device"
    return t


def f32(v):
    return np.float32(v)


def orient_cases(rng, n):
    """(n, 6) float32: random triples at many scales, near-collinear triples
    (a point on the line through o and e, rounded, then moved a few ulps),
    degenerate ones (repeated points), and small differences on a large
    offset."""
    out = []
    k = n // 4
    # random, each case at its own scale 2^s, s in [-90, 60]
    s = rng.integers(-90, 61, size=k)
    out.append((rng.standard_normal((k, 6)) * np.exp2(s)[:, None]).astype(np.float32))
    # near-collinear
    o = rng.standard_normal((k, 2)).astype(np.float32)
    e = (o + rng.standard_normal((k, 2)).astype(np.float32) * np.float32(8)).astype(np.float32)
    lam = rng.random(k) * 3 - 1
    p = (o.astype(np.float64) + lam[:, None] * (e.astype(np.float64) - o.astype(np.float64))).astype(np.float32)
    steps = rng.integers(-3, 4, size=(k, 2)).astype(np.int32)
    p = np.nextafter(p, np.where(steps > 0, np.inf, -np.inf).astype(np.float32))
    p = np.where(steps == 0, (o.astype(np.float64) + lam[:, None] * (e - o)).astype(np.float32), p)
    out.append(np.concatenate([o, e, p], 1).astype(np.float32))
    # degenerate: repeated points, axis-parallel edges, integer grid
    g = rng.integers(-4, 5, size=(k, 6)).astype(np.float32)
    g[: k // 3, 4:6] = g[: k // 3, 0:2]
    g[k // 3: 2 * k // 3, 2:4] = g[k // 3: 2 * k // 3, 0:2]
    out.append(g)
    # small differences on a large offset (the line filter stands aside
    # beyond 2^60; here 2^20 .. 2^40)
    off = np.exp2(rng.integers(20, 41, size=n - 3 * k))[:, None]
    d = rng.standard_normal((n - 3 * k, 6))
    out.append((off + d).astype(np.float32))
    return np.concatenate(out, 0).astype(np.float32)


def exact_orient(c):
    ox, oy, ex, ey, px, py = (F(float(v)) for v in c)
    return (ex - ox) * (py - oy) - (ey - oy) * (px - ox)


def sgn(v):
    return (v > 0) - (v < 0)


@pytest.mark.parametrize("fp64", [0, 1])
def test_orientation_filters_and_signs(torch, fp64):
    rng = np.random.default_rng(31)
    cases = orient_cases(rng, 8000)
    n = len(cases)
    say(f"orientation: {n} cases, fp64_only={fp64}")
    dev = torch.device("cuda", 0)
    tri = torch.from_numpy(cases).to(dev)
    sign = torch.empty(n, dtype=torch.int32, device=dev)
    vals = torch.empty((n, 4), dtype=torch.float32, device=dev)
    flags = torch.empty(n, dtype=torch.int32, device=dev)
    assert sqh.sqh_diag_orient(tri, n, fp64, sign, vals, flags) == sqh.SQH_OK
    sign, vals, flags = sign.cpu().numpy(), vals.cpu().numpy(), flags.cpu().numpy()
    want = he.orient_sign(cases.reshape(-1, 3, 2))
    assert np.array_equal(sign, want.astype(np.int32))
    if fp64:
        assert not flags.any()
    else:
        assert flags.sum() > n // 3  # the filter decides most cases
    line_used = 0
    for i in range(n):
        O = exact_orient(cases[i])
        d, es, t, m = (float(v) for v in vals[i])
        if np.isfinite(d) and np.isfinite(es):
            assert abs(F(d) - O) <= 2 * F(es), i
            if flags[i]:
                assert abs(d) > es and sgn(d) == sgn(O), i
        if m >= 0:
            line_used += 1
            assert abs(F(t) - O) < F(m), i
            if abs(t) > m:
                assert sgn(t) == sgn(O), i
    assert line_used > n // 2


def compare_cases(rng, n):
    """(n, 8) float32 and (n, 2) int32: random pairs, pairs of equal area
    (Q = P moved along a direction parallel to the edge, on integer grids),
    pairs at one position with different indices, and near-ties."""
    cs, ids = [], []
    k = n // 4
    a = (rng.standard_normal((k, 8)) * 4).astype(np.float32)
    cs.append(a)
    ids.append(rng.integers(0, 1 << 20, size=(k, 2)))
    # equal areas on a grid: Q = P + j (e - o)
    o = rng.integers(-20, 21, size=(k, 2))
    dvec = rng.integers(-5, 6, size=(k, 2))
    dvec[(dvec == 0).all(1)] = [1, 0]
    p = rng.integers(-40, 41, size=(k, 2))
    j = rng.integers(-3, 4, size=(k, 1))
    j[j == 0] = 1
    cs.append(np.concatenate([o, o + dvec, p, p + j * dvec], 1).astype(np.float32))
    ids.append(rng.integers(0, 1 << 20, size=(k, 2)))
    # the same position, different indices
    b = (rng.standard_normal((k, 8)) * 4).astype(np.float32)
    b[:, 6:8] = b[:, 4:6]
    idb = rng.integers(0, 1 << 20, size=(k, 2))
    idb[idb[:, 0] == idb[:, 1], 1] += 1
    cs.append(b)
    ids.append(idb)
    # near-ties: Q = P moved along the edge direction then a few ulps
    m = n - 3 * k
    c = (rng.standard_normal((m, 8)) * 4).astype(np.float32)
    q = (c[:, 4:6].astype(np.float64) + 0.5 * (c[:, 2:4].astype(np.float64) - c[:, 0:2])).astype(np.float32)
    q = np.nextafter(q, np.where(rng.random((m, 2)) < 0.5, np.inf, -np.inf).astype(np.float32))
    c[:, 6:8] = q
    cs.append(c)
    ids.append(rng.integers(0, 1 << 20, size=(m, 2)))
    ids = np.concatenate(ids, 0).astype(np.int32)
    return np.concatenate(cs, 0).astype(np.float32), ids


def exact_before(c, pid, qid):
    ox, oy, ex, ey, px, py, qx, qy = (F(float(v)) for v in c)
    ap = -((ex - ox) * (py - oy) - (ey - oy) * (px - ox))
    aq = -((ex - ox) * (qy - oy) - (ey - oy) * (qx - ox))
    if ap != aq:
        return ap > aq
    if (px, py) == (qx, qy):
        return pid < qid
    fwd = (ex > ox) or (ex == ox and ey > oy)
    p_first = (px < qx) or (px == qx and py < qy)
    return p_first if fwd else not p_first


@pytest.mark.parametrize("fp64", [0, 1])
def test_farthest_point_order(torch, fp64):
    rng = np.random.default_rng(32)
    cases, ids = compare_cases(rng, 6000)
    n = len(cases)
    say(f"farthest-point order: {n} cases, fp64_only={fp64}")
    dev = torch.device("cuda", 0)
    c = torch.from_numpy(cases).to(dev)
    i = torch.from_numpy(ids).to(dev)
    out = torch.empty(n, dtype=torch.int32, device=dev)
    assert sqh.sqh_diag_compare(c, i, n, fp64, out) == sqh.SQH_OK
    out = out.cpu().numpy()
    ties = 0
    for k in range(n):
        pq = exact_before(cases[k], int(ids[k, 0]), int(ids[k, 1]))
        qp = exact_before(cases[k][[0, 1, 2, 3, 6, 7, 4, 5]], int(ids[k, 1]), int(ids[k, 0]))
        assert pq != qp, k  # distinct candidates: a strict order
        assert (out[k] & 1) == int(pq) and ((out[k] >> 1) & 1) == int(qp), (k, cases[k].tolist(), ids[k])
        ties += exact_orient(cases[k][[0, 1, 2, 3, 4, 5]]) == exact_orient(cases[k][[0, 1, 2, 3, 6, 7]])
    assert ties > n // 4  # the tie rules were exercised


@pytest.mark.parametrize("n", [1, 64, 1000, 1024, 7 * 1024 + 333])
def test_workgroup_scan(torch, n):
    say(f"workgroup scan n={n}")
    rng = np.random.default_rng(n)
    x = rng.integers(-1000, 1001, size=n).astype(np.int32)
    dev = torch.device("cuda", 0)
    runs = (n + 1023) // 1024
    xd = torch.from_numpy(x).to(dev)
    ea = torch.empty(n, dtype=torch.int32, device=dev)
    eb = torch.empty(n, dtype=torch.int32, device=dev)
    tot = torch.empty(2 * runs, dtype=torch.int32, device=dev)
    assert sqh.sqh_diag_scan(xd, n, ea, eb, tot) == sqh.SQH_OK
    ea, eb, tot = ea.cpu().numpy(), eb.cpu().numpy(), tot.cpu().numpy()
    for r in range(runs):
        seg = x[r * 1024:(r + 1) * 1024].astype(np.int64)
        ex = np.concatenate([[0], np.cumsum(seg)[:-1]])
        assert np.array_equal(ea[r * 1024:(r + 1) * 1024], ex), r
        assert np.array_equal(eb[r * 1024:(r + 1) * 1024], np.arange(len(seg))), r
        assert tot[2 * r] == seg.sum() and tot[2 * r + 1] == len(seg)


def test_diag_rejects_bad_arguments(torch):
    assert sqh.sqh_diag_orient(None, 5, 0, None, None, None) == sqh.SQH_EINVAL
    assert sqh.sqh_diag_compare(None, None, -1, 0, None) == sqh.SQH_EINVAL
    assert sqh.sqh_diag_scan(None, 3, None, None, None) == sqh.SQH_EINVAL
