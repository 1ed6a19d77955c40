"""GPU parity of the streaming path (large single hulls) against the oracle.

Calls on one set of at least 2^16 points run the first phases and the passes
over few large segments as ordinary launches; these cases check that path
against the oracle and against the general path, at the size threshold and
with a ragged tail, in every precision mode, with and without the static line
filter, where the passes kernel takes over, and on its degenerate inputs.
Hull index lists are integer results: the bar is bit-exact equality.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1501_04706_amd import sqh, workloads

pytestmark = pytest.mark.gpu

THRESHOLD = 1 << 16
LARGE = 1 << 20  # several streaming passes before the LDS passes


def say(msg):
    print(f"[case] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def H():
    import torch
    assert torch.cuda.is_available(), "gpu tests need a HIP device"
    h = sqh.Hull(0)
    yield h
    h.close()


def run(H, xy, streaming=True, precision=sqh.SQH_FP32_FILTER):
    import torch
    H.set_streaming(streaming)
    H.set_precision(precision)
    try:
        t = torch.from_numpy(np.ascontiguousarray(xy, dtype=np.float32).reshape(-1, 2)).to("cuda")
        h = [int(v) for v in H.hull(t).cpu().numpy()]
        return h, H.stats()
    finally:
        H.set_streaming(True)
        H.set_precision(sqh.SQH_FP32_FILTER)


@pytest.mark.parametrize("n", [THRESHOLD, THRESHOLD + 12345, LARGE, LARGE + 12345])
@pytest.mark.parametrize("kind", ["square", "disk", "circle", "grid"])
def test_stream_matches_general(H, kind, n):
    say(f"stream vs general: {kind} n={n}")
    xy = workloads.make(kind, n, 11)
    want = [int(v) for v in oracle.c_hull(xy)]
    got, st = run(H, xy)
    assert st["stream_path"] in (1, 2)
    assert got == want
    gen, st = run(H, xy, streaming=False)
    assert st["stream_path"] == 0
    assert gen == want


def test_below_threshold_takes_general_path(H):
    say("n = 2^16 - 1")
    xy = workloads.square(THRESHOLD - 1, 12)
    got, st = run(H, xy)
    assert st["stream_path"] == 0
    assert got == [int(v) for v in oracle.c_hull(xy)]


@pytest.mark.parametrize("mode", [sqh.SQH_FP32_FILTER, sqh.SQH_FP32_SEMISTATIC, sqh.SQH_FP64_ONLY])
def test_stream_precision_modes(H, mode):
    say(f"precision mode {mode}: square n=2000003")
    n = 2_000_003
    xy = workloads.square(n, 13)
    got, st = run(H, xy, precision=mode)
    assert st["stream_path"] in (1, 2)
    assert st["line_filter"] == (1 if mode == sqh.SQH_FP32_FILTER else 0)
    # one test per point in the split, three or four in the first
    # compaction, two per point of each later pass (with room to spare)
    assert 0 < st["orient_evals"] <= 6 * n + 4 * sum(st["pass_points"])
    if mode == sqh.SQH_FP64_ONLY:
        # the first compaction charges three tests per point; a point
        # settled by its first exact test takes fewer
        assert st["orient_exact"] >= 0.99 * st["orient_evals"]
    else:
        assert st["orient_exact"] < 1e-3 * st["orient_evals"]
    assert got == [int(v) for v in oracle.c_hull(xy)]


@pytest.mark.parametrize("case", ["offset", "huge", "tiny", "thin"])
def test_stream_line_filter_domain(H, case):
    # inputs where the static line filter must stand aside (far from the
    # origin compared with the extent; |coordinates| beyond 2^60, with
    # float32 products still in range), where its bound is all underflow
    # margin (coordinates near 2^-90, kept normal), and a thin strip that
    # keeps it
    say(f"line filter domain: {case}")
    xy = workloads.disk(LARGE + 77, 14).astype(np.float64)
    if case == "offset":
        xy += 4096.0
    elif case == "huge":
        xy *= 2.0 ** 62
    elif case == "tiny":
        xy[np.abs(xy) < 2.0 ** -30] = 0.0
        xy *= 2.0 ** -90
    else:
        xy[:, 1] *= 2.0 ** -3
    xy = xy.astype(np.float32)
    got, st = run(H, xy)
    assert st["stream_path"] in (1, 2)
    assert st["line_filter"] == (1 if case in ("tiny", "thin") else 0)
    assert got == [int(v) for v in oracle.c_hull(xy)]


def test_stream_hands_over_to_passes_kernel(H):
    # a jittered circle keeps almost every point: more than 256 segments
    # before the streaming passes finish it
    say("circle n=2000000: passes kernel takes over")
    xy = workloads.circle(2_000_000, 15)
    got, st = run(H, xy)
    assert st["stream_path"] == 2
    assert got == [int(v) for v in oracle.c_hull(xy)]


def test_stream_degenerate(H):
    n = LARGE + 5
    cases = {
        "one position": np.full((n, 2), 0.25, np.float32),
        "two positions": np.where((np.arange(n) % 3 == 0)[:, None], [1.0, 2.0], [-3.0, 0.5]).astype(np.float32),
        "collinear": np.stack([np.arange(n) % 1000, 2 * (np.arange(n) % 1000)], 1).astype(np.float32),
        "vertical": np.stack([np.zeros(n), (np.arange(n) * 7919) % 4096], 1).astype(np.float32),
        "triangle + interior": np.concatenate(
            [workloads.square(n - 3, 16) * 0.5 + 0.25, np.array([[0, 0], [1, 0], [0, 1]], np.float32)]),
    }
    for name, xy in cases.items():
        say(f"degenerate: {name}")
        got, st = run(H, xy)
        assert st["stream_path"] == 1, name
        assert got == [int(v) for v in oracle.c_hull(xy)], name


def test_unaligned_input_takes_general_path(H):
    import torch
    say("input at an 8-byte offset")
    xy = workloads.square(LARGE + 1, 17)
    big = torch.zeros((LARGE + 2, 2), dtype=torch.float32, device="cuda")
    big[1:] = torch.from_numpy(xy).to("cuda")
    view = big[1:]
    assert view.data_ptr() % 16 == 8
    got = [int(v) for v in H.hull(view).cpu().numpy()]
    assert H.stats()["stream_path"] == 0
    assert got == [int(v) for v in oracle.c_hull(xy)]


@pytest.mark.parametrize("mode", [sqh.SQH_FP32_FILTER, sqh.SQH_FP32_SEMISTATIC])
@pytest.mark.parametrize("off", [0.0, 4096.0])
def test_stream_ignores_memory_past_the_end(H, mode, off):
    # the input sits at the start of a larger buffer whose tail holds points
    # far outside its hull: a ragged last tile must never take them in
    import torch
    n = LARGE + 77
    say(f"memory past the end: mode {mode} offset {off}")
    xy = (workloads.disk(n, 18).astype(np.float64) + off).astype(np.float32)
    big = torch.full((n + 16384, 2), off + 1000.0, dtype=torch.float32, device="cuda")
    big[:n] = torch.from_numpy(xy).to("cuda")
    H.set_precision(mode)
    try:
        got = [int(v) for v in H.hull(big[:n]).cpu().numpy()]
        st = H.stats()
    finally:
        H.set_precision(sqh.SQH_FP32_FILTER)
    assert st["stream_path"] in (1, 2)
    assert got == [int(v) for v in oracle.c_hull(xy)]


def test_stream_pass_count_adapts(H):
    # a context enqueues as many streaming passes as the last call of the
    # size class needed (plus one on few workgroups); a call that needs more
    # is finished by the passes kernel, and the next one gets them all
    n = LARGE + 3
    sq = workloads.square(n, 19)
    dk = workloads.disk(n, 19)
    want_sq = [int(v) for v in oracle.c_hull(sq)]
    want_dk = [int(v) for v in oracle.c_hull(dk)]
    for i, (xy, want) in enumerate([(sq, want_sq), (sq, want_sq), (dk, want_dk), (dk, want_dk), (sq, want_sq)]):
        say(f"pass count: call {i}")
        got, st = run(H, xy)
        assert got == want, i
        if i in (1, 3, 4):
            assert st["stream_path"] == 1, i


@pytest.mark.parametrize("n", [0, 1, 5000, THRESHOLD + 99, LARGE + 77])
def test_soa_input_matches_aos(H, n):
    # separate x and y arrays give the same hull as the interleaved input
    import torch
    say(f"structure-of-arrays input n={n}")
    xy = workloads.disk(n, 20)
    x = torch.from_numpy(np.ascontiguousarray(xy[:, 0])).to("cuda")
    y = torch.from_numpy(np.ascontiguousarray(xy[:, 1])).to("cuda")
    got = [int(v) for v in H.hull_soa(x, y).cpu().numpy()]
    assert got == [int(v) for v in oracle.c_hull(xy)]
    if n >= THRESHOLD:
        assert H.stats()["stream_path"] in (1, 2)


def test_soa_input_errors(H):
    import torch
    x = torch.zeros(10, dtype=torch.float32, device="cuda")
    y = torch.zeros(10, dtype=torch.float32, device="cuda")
    y[3] = float("nan")
    with pytest.raises(sqh.SqhError) as e:
        H.hull_soa(x, y)
    assert e.value.code == sqh.SQH_EINVAL
    ws = H.workspace(10, 1)
    out = torch.empty(10, dtype=torch.int32, device="cuda")
    rc, _ = sqh.sqh_hull_soa(H.ctx, x, x, 10, out, 10, ws, 16)
    assert rc == sqh.SQH_ENOMEM
    assert sqh.sqh_workspace_bytes_soa(-1) == 0


@pytest.mark.parametrize("ring", [900, 3000, 6000])
def test_stream_lds_tail_hand_over(H, ring):
    # few hull points around many interior ones: the first compaction leaves
    # about `ring` points, which the LDS passes take; a ring of more than
    # 1024 points outgrows the LDS table (more than 512 segments with more
    # than 1024 points left) and is written back for the passes kernel
    n = THRESHOLD + 1000
    say(f"LDS tail: ring of {ring} in {n}")
    inner = workloads.disk(n - ring, 21) * np.float32(0.5)
    outer = workloads.circle(ring, 22)
    xy = np.ascontiguousarray(np.concatenate([inner, outer], 0).astype(np.float32))
    got, st = run(H, xy)
    assert got == [int(v) for v in oracle.c_hull(xy)]
    assert st["stream_path"] == (1 if ring <= 1024 else 2)
