"""GPU: the sorted-chain variant (the paper's x-sorted layout: one radix sort
after the first split, then passes that only remove points) gives exactly
the oracle's hull, alone and with the pre-filter (through the C ABI)."""
import glob
import os
import sys

import numpy as np
import pytest

import oracle
from oracle import hull_exact as he
from paper_1501_04706_amd import sqh, workloads

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
CONFIGS = {"sorted": sqh.SQH_PREFILTER_NONE, "sorted+octagon": sqh.SQH_PREFILTER_OCTAGON}


def say(msg):
    print(f"[case] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module", params=sorted(CONFIGS))
def H(request):
    import torch
    assert torch.cuda.is_available(), "gpu tests need a HIP device"
    h = sqh.Hull(0)
    h.set_variant(sqh.SQH_VARIANT_SORTED)
    h.set_prefilter(CONFIGS[request.param])
    h.cfg_name = request.param
    yield h
    h.close()


def gpu_hull(H, xy):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(xy, dtype=np.float32).reshape(-1, 2)).to("cuda")
    return [int(v) for v in H.hull(t).cpu().numpy()]


def expect(xy):
    return he.hull(xy) if len(xy) < 3000 else [int(v) for v in oracle.c_hull(xy)]


def check_sort(H):
    # the sort ran on the first compaction's survivors and left them in order
    st = H.stats()
    assert st["sort_violations"] == 0, st["sort_violations"]
    if st["first_survivors"] > 0:
        assert st["sorted_points"] == st["first_survivors"], (st["sorted_points"], st["first_survivors"])
    else:
        assert st["sorted_points"] == -1


def load_golden(path):
    pts, hull = [], None
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("hull:"):
            hull = [int(t) for t in line.split(":")[1].split()]
        else:
            pts.append([float(v) for v in line.split()])
    return np.array(pts, np.float32).reshape(-1, 2), hull


def test_variant_value_checked(H):
    assert sqh.sqh_set_variant(H.ctx, 2) == sqh.SQH_EINVAL
    assert sqh.sqh_set_variant(H.ctx, -1) == sqh.SQH_EINVAL


def test_golden_and_degenerate(H):
    say(f"{H.cfg_name}: golden fixtures and degenerate sets")
    for path in sorted(glob.glob(os.path.join(GOLDEN, "*.txt"))):
        xy, want = load_golden(path)
        assert gpu_hull(H, xy) == want, path
        check_sort(H)
    cases = [
        np.zeros((0, 2), np.float32),
        np.array([[3, 4]], np.float32),
        np.array([[1, 1], [0, 0]], np.float32),
        np.full((5000, 2), 0.5, np.float32),
        np.stack([np.arange(3000), np.arange(3000) * 3], 1).astype(np.float32)[::-1].copy(),
        np.array([[-0.0, 0.0], [0.0, -0.0], [1, 0], [0, 1]], np.float32),
        # many points sharing x (ties in the sort key) on both chains
        np.stack([np.repeat(np.arange(40), 50), np.tile(np.arange(50), 40)], 1).astype(np.float32),
        np.array([[0, 0], [10, 0], [5, 1e-3], [2, 0], [7, 0]], np.float32),
    ]
    for xy in cases:
        assert gpu_hull(H, xy) == he.hull(xy), xy[:6]
        check_sort(H)


def test_small_random_grids(H):
    rng = np.random.default_rng(654)
    say(f"{H.cfg_name}: small random grids")
    for it in range(120):
        n = int(rng.integers(1, 200))
        k = int(rng.integers(1, 9))
        xy = (rng.integers(-k, k + 1, size=(n, 2)) * 0.25).astype(np.float32)
        assert gpu_hull(H, xy) == he.hull(xy), (it, xy.tolist())
        check_sort(H)


@pytest.mark.parametrize("n", [2049, 123457, 1_000_000])
def test_workloads(H, n):
    say(f"{H.cfg_name}: workloads n={n}")
    for kind in ("square", "disk", "circle", "grid"):
        xy = workloads.make(kind, n, n + 11)
        assert gpu_hull(H, xy) == expect(xy), kind
        check_sort(H)


def test_full_size_square_and_disk(H):
    for kind in ("square", "disk"):
        say(f"{H.cfg_name}: {kind} n=20000000")
        xy = workloads.make(kind, 20_000_000, 0)
        assert gpu_hull(H, xy) == expect(xy), kind
        check_sort(H)


def test_fp64_only_same_hull(H):
    say(f"{H.cfg_name}: fp64-only")
    xy = workloads.disk(300_000, 17)
    want = expect(xy)
    H.set_precision(sqh.SQH_FP64_ONLY)
    try:
        assert gpu_hull(H, xy) == want
        check_sort(H)
    finally:
        H.set_precision(sqh.SQH_FP32_FILTER)


def test_graph_replays(H):
    import torch
    say(f"{H.cfg_name}: graph replays")
    xy = workloads.circle(200_000, 23)
    t = torch.from_numpy(xy).cuda()
    want = expect(xy)
    g = H.graph(t)
    try:
        for rep in range(3):
            g.launch()
            out, _ = g.result()
            assert [int(v) for v in out.cpu().numpy()] == want, rep
            assert gpu_hull(H, xy) == want  # eager work between the replays
            torch.cuda.synchronize()
    finally:
        g.close()


def test_non_finite_rejected(H):
    import torch
    say(f"{H.cfg_name}: non-finite coordinate")
    xy = workloads.square(100_000, 4)
    xy[777, 1] = np.nan
    with pytest.raises(sqh.SqhError) as ei:
        H.hull(torch.from_numpy(xy).cuda())
    assert ei.value.code == sqh.SQH_EINVAL
    assert H.stats()["sorted_points"] == -1
    xy = workloads.disk(100_000, 5)
    assert gpu_hull(H, xy) == expect(xy)
    check_sort(H)


def test_batch_of_one_set(H):
    # a batched call on one set takes the same launch chain as sqh_hull
    import torch
    say(f"{H.cfg_name}: batch of one set")
    xy = workloads.disk(250_000, 31)
    off = torch.tensor([0, len(xy)], dtype=torch.int64, device="cuda")
    out, out_off = H.hull_batched(torch.from_numpy(xy).cuda(), off)
    got = [int(v) for v in out[: int(out_off[1])].cpu().numpy()]
    assert got == expect(xy)
    check_sort(H)


def test_autotune_keeps_the_hull(H):
    import torch
    say(f"{H.cfg_name}: autotune")
    xy = workloads.square(500_000, 37)
    t = torch.from_numpy(xy).cuda()
    try:
        text = H.autotune(t, reps=1)
        assert '"log2n": 18' in text, text
        assert gpu_hull(H, xy) == expect(xy)
        check_sort(H)
    finally:
        H.set_tuning('{"entries": []}')
