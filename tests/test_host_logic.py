"""CPU: host-side logic around the kernels -- the bench's byte model and its
measured-traffic file, and the error bound behind the pre-filter's line
test (float32 arithmetic emulated exactly, compared with exact
orientation)."""
import json
import os
from fractions import Fraction as F

import numpy as np
import pytest

import bench


def _write_counters(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w") as f:
        f.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for r in rows:
            f.write(",".join(str(v) for v in r) + "\n")


def test_call_bytes_model():
    # seed + split + first read 8 B/pt each, first writes 12 B per survivor,
    # pass k reads its points and writes the next pass's
    st = {"pass_points": [100, 10, 0], "passes": 2, "first_survivors": 100}
    n = 1000
    assert bench.call_bytes(st, n) == 24 * n + 12 * 100 + (12 * 100 + 12 * 10) + (12 * 10 + 0)


def test_launch_bytes_model():
    # streaming path: seed and split read the input, the line-filter first
    # compaction reads it and writes the survivors (the other mode's kernel
    # returns at once), k_spass launches take the passes over more than 6144
    # points in at most 256 segments in order, the passes kernel the rest
    n = 1_000_000
    st = {"pass_points": [400000, 90000, 9000, 500, 20], "pass_segments": [4, 8, 300, 20, 4], "passes": 5,
          "first_survivors": 400000, "line_filter": 1}
    names = ["k_reset", "k_sseed", "k_ssplit", "k_sfirst<line>", "k_sfirst<semistatic>",
             "k_spass", "k_spass", "k_spass", "k_stail", "k_hull<passes>"]
    b = bench.launch_bytes([(x, 0.0) for x in names], st, n)
    p = [12 * (400000 + 90000), 12 * (90000 + 9000), 12 * (9000 + 500), 12 * (500 + 20), 12 * 20]
    assert b == [0, 8 * n, 8 * n, 8 * n + 12 * 400000, 0, p[0], p[1], 0, 0, p[2] + p[3] + p[4]]
    st["line_filter"] = 0
    b = bench.launch_bytes([(x, 0.0) for x in names], st, n)
    assert b[3] == 0 and b[4] == 8 * n + 12 * 400000
    # a call's launches add up to the whole call's bytes
    assert sum(b) == bench.call_bytes(st, n)
    # no passes kernel: the tail takes the rest
    st["pass_segments"] = [4, 8, 20, 20, 4]
    st["pass_points"] = [400000, 90000, 9000, 500, 20]
    b = bench.launch_bytes([(x, 0.0) for x in names[:-1]], st, n)
    assert b[5:8] == [p[0], p[1], p[2]] and b[8] == p[3] + p[4]
    assert sum(b) == bench.call_bytes(st, n)


def test_write_traffic_scales_by_copy(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILE_TRAFFIC", str(tmp_path / "traffic.json"))
    kib = 1024.0
    # two dispatches of the hull kernel, counters split over two instances each
    _write_counters(str(tmp_path / "f"), [
        (1, "void sqh::k_hull<0>(sqh::HullArgs)", "FETCH_SIZE", 300000), (1, "void sqh::k_hull<0>(sqh::HullArgs)",
                                                                         "FETCH_SIZE", 100000),
        (2, "void sqh::k_hull<0>(sqh::HullArgs)", "FETCH_SIZE", 400000),
        (3, "sqh::k_reset(sqh::HullArgs)", "FETCH_SIZE", 999)])
    _write_counters(str(tmp_path / "w"), [
        (1, "void sqh::k_hull<0>(sqh::HullArgs)", "WRITE_SIZE", 50000),
        (2, "void sqh::k_hull<0>(sqh::HullArgs)", "WRITE_SIZE", 70000)])
    # the copy reads and writes 160 MB; its counters read 10 % high
    c = 160_000_000 / kib * 1.1
    _write_counters(str(tmp_path / "cf"), [(7, "__amd_rocclr_copyBuffer", "FETCH_SIZE", c),
                                           (8, "elementwise_uniform", "FETCH_SIZE", 5)])
    _write_counters(str(tmp_path / "cw"), [(7, "__amd_rocclr_copyBuffer", "WRITE_SIZE", c)])
    K = "k_hull<0>"
    rec = bench.write_traffic(K, str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "cf"),
                              str(tmp_path / "cw"))
    assert rec["dispatches"] == 2 and rec["copy_dispatches"] == 1
    assert rec["fetch_kib"] == pytest.approx(400000.0) and rec["write_kib"] == pytest.approx(60000.0)
    assert rec["bytes_per_launch"] == pytest.approx((400000 + 60000) * kib / 1.1, rel=1e-6)
    saved = json.load(open(tmp_path / "traffic.json"))
    assert saved[K]["build"] == bench.library_fingerprint()
    # the bench reads it back only for the same kernel sources
    assert bench.load_traffic(K) == rec["bytes_per_launch"]
    assert bench.load_traffic("k_other") is None
    saved[K]["build"] = "0" * 16
    json.dump(saved, open(tmp_path / "traffic.json", "w"))
    assert bench.load_traffic(K) is None


def _f32(v):
    return np.float32(v)


def _fma32(a, b, c):
    # a*b + c rounded once to float32 (exact rational, then one rounding)
    v = F(float(a)) * F(float(b)) + F(float(c))
    return np.float32(float(v))


def test_prefilter_line_test_bound():
    # The pre-filter discards p when fma(nx, px, fma(ny, py, c)) > m for
    # every edge o -> e, with nx = -dy, ny = dx, dx = fl(ex - ox),
    # dy = fl(ey - oy), c = fl(fl(dy ox) - fl(dx oy)) and
    # m = 2^-19 (|dx| My + |dy| Mx) + 2^-140, Mx, My bounding |x|, |y|.
    # The claimed bound on the rounding is 9 u D (1 + 10 u) + 5 * 2^-150;
    # check it, and that the test never certifies a point that is not
    # strictly left, on points placed within a few ulps of the edge.
    rng = np.random.default_rng(2024)
    u = 2.0 ** -24
    certified = 0
    for trial in range(400):
        scale = float(10.0 ** rng.uniform(-30, 17))
        pts = (rng.uniform(-1, 1, size=(3, 2)) * scale).astype(np.float32)
        o, e = pts[0], pts[1]
        Mx = _f32(np.abs(pts[:, 0]).max())
        My = _f32(np.abs(pts[:, 1]).max())
        dx = _f32(e[0] - o[0])
        dy = _f32(e[1] - o[1])
        c = _f32(_f32(dy * o[0]) - _f32(dx * o[1]))
        m = _f32(_f32(_f32(abs(dx) * My) + _f32(abs(dy) * Mx)) * _f32(2.0 ** -19)) + _f32(2.0 ** -140)
        D = abs(F(float(dx))) * F(float(My)) + abs(F(float(dy))) * F(float(Mx))
        for k in range(12):
            t = rng.uniform(-1, 1)
            p = (o.astype(np.float64) + t * (e.astype(np.float64) - o.astype(np.float64))).astype(np.float32)
            p = (p + rng.integers(-3, 4, size=2) * np.spacing(p) * rng.integers(0, 2 ** 18)).astype(np.float32)
            if abs(p[0]) > Mx or abs(p[1]) > My:
                continue
            tv = _fma32(-dy, p[0], _fma32(dx, p[1], c))
            exact = (F(float(e[0])) - F(float(o[0]))) * (F(float(p[1])) - F(float(o[1]))) - \
                    (F(float(e[1])) - F(float(o[1]))) * (F(float(p[0])) - F(float(o[0])))
            err = abs(F(float(tv)) - exact)
            assert err <= 9 * F(u) * D * (1 + 10 * F(u)) + 5 * F(2) ** -150, (trial, k)
            if tv > m:
                certified += 1
                assert exact > 0, (trial, k)
    assert certified > 100


def test_modes_at_picks_the_workload_rows():
    rows = [{"kind": "square", "n": 20, "mode": "plain", "Mpoints_per_s": 3.0, "kernel": 0.5},
            {"kind": "square", "n": 20, "mode": "sorted", "Mpoints_per_s": 1.0, "kernel": 1.5},
            {"kind": "square", "n": 10, "mode": "plain", "Mpoints_per_s": 9.0, "kernel": 0.1},
            {"kind": "disk", "n": 20, "mode": "plain", "Mpoints_per_s": 2.0, "kernel": 0.7}]
    assert bench.modes_at(rows, "square", 20) == {"plain": {"Mpoints_per_s": 3.0, "ms_kernel": 0.5},
                                                   "sorted": {"Mpoints_per_s": 1.0, "ms_kernel": 1.5}}
    assert bench.modes_at(rows, "circle", 20) == {}
