"""GPU: launch shapes, the autotuner and HIP-graph replays give exactly the
oracle's hulls (through the C ABI)."""
import sys

import numpy as np
import pytest

import oracle
from oracle import hull_exact as he
from paper_1501_04706_amd import sqh, workloads

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[case] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def H():
    import torch
    assert torch.cuda.is_available(), "gpu tests need a HIP device"
    h = sqh.Hull(0)
    yield h
    h.close()


def expect_hull(xy):
    return he.hull(xy) if len(xy) < 3000 else [int(v) for v in oracle.c_hull(xy)]


def make_batch(seed, nsets, hi):
    rng = np.random.default_rng(seed)
    sizes = [int(v) for v in rng.integers(0, hi, size=nsets)]
    sizes[0] = 0
    kinds = ["square", "disk", "circle", "grid"]
    parts = [workloads.make(kinds[i % 4], s, seed * 1000 + i) for i, s in enumerate(sizes)]
    off = np.zeros(nsets + 1, np.int64)
    off[1:] = np.cumsum(sizes)
    return parts, off, np.concatenate(parts, 0).astype(np.float32)


def check_batched(out, out_off, parts):
    out = out.cpu().numpy()
    out_off = out_off.cpu().numpy()
    for s, p in enumerate(parts):
        got = [int(v) for v in out[out_off[s]:out_off[s + 1]]]
        assert got == expect_hull(p), s


@pytest.mark.parametrize("grid_frac,tail", [(1.0, 0), (0.5, 1 << 14), (0.25, 1 << 18), (0.125, 1 << 30)])
def test_launch_shapes_same_hull(H, grid_frac, tail):
    import torch
    H.set_tuning('{"entries": []}')
    assert H.tuning() == '{"entries": []}'
    # more workgroups than can be resident at once is rejected
    with pytest.raises(sqh.SqhError):
        H.set_tuning('{"entries": [{"log2n": 20, "grid": 100000, "tail": 0}]}')
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    grid = max(1, int(cus * grid_frac))
    say(f"launch shape grid={grid} tail={tail}")
    # "stream": 0 keeps the single hulls on the persistent kernel, whose shape this sets
    H.set_tuning('{"entries": [{"log2n": 20, "grid": %d, "tail": %d, "stream": 0}]}' % (grid, tail))
    for kind, n in (("square", 1_000_000), ("circle", 200_000), ("grid", 300_000), ("disk", 5000)):
        xy = workloads.make(kind, n, 11)
        got = [int(v) for v in H.hull(torch.from_numpy(xy).cuda()).cpu().numpy()]
        assert got == expect_hull(xy), (kind, grid, tail)
    parts, off, xy = make_batch(5, 40, 20_000)
    out, out_off = H.hull_batched(torch.from_numpy(xy).cuda(), torch.from_numpy(off).cuda())
    check_batched(out, out_off, parts)
    H.set_tuning('{"entries": []}')


def test_tuning_text_rejected(H):
    say("tuning text validation")
    for bad in ['', '{}', '{"entries": [{"log2n": 3}]}', '{"entries": [{"log2n": 3, "grid": 0, "tail": 1}]}',
                '{"entries": [{"log2n": 3, "grid": 1, "tail": -1}]}', '{"entries": [{"log2n": 3, "grid": 1',
                '{"entries": [], "engine_grid": 0}', '{"entries": [], "engine_grid": 100000}',
                '{"entries": [{"log2n": 3, "grid": 1, "tail": 1, "stream": 2}]}',
                '{"entries": [{"log2n": 3, "grid": 1, "tail": 1, "sgrid": 5000}]}']:
        assert sqh.sqh_set_tuning(H.ctx, bad) == sqh.SQH_EINVAL, bad
    assert H.tuning() == '{"entries": []}'
    H.set_tuning('{"entries": [], "engine_grid": 17}')
    assert H.tuning() == '{"entries": [], "engine_grid": 17}'
    H.set_tuning('{"entries": []}')
    assert H.tuning() == '{"entries": []}'


@pytest.mark.parametrize("sgrid", [1024, 512, 256, 64])
def test_streaming_shapes_same_hull(H, sgrid):
    import torch
    say(f"streaming kernels on {sgrid} workgroups")
    H.set_tuning('{"entries": [{"log2n": 20, "grid": 1, "tail": 0, "stream": 1, "sgrid": %d}]}' % sgrid)
    for kind, n in (("square", 1_000_003), ("disk", 300_001), ("circle", 200_000), ("grid", 300_000)):
        xy = workloads.make(kind, n, 12)
        got = [int(v) for v in H.hull(torch.from_numpy(xy).cuda()).cpu().numpy()]
        assert got == expect_hull(xy), (kind, sgrid)
        assert H.stats()["stream_path"] in (1, 2)
    H.set_tuning('{"entries": []}')


def test_autotune_then_same_hull(H):
    import torch
    say("autotune square 1M")
    xy = workloads.square(1_000_000, 3)
    t = torch.from_numpy(xy).cuda()
    text = H.autotune(t, reps=1)
    assert '"log2n": 19' in text and '"stream": ' in text and '"sgrid": ' in text, text
    H.set_tuning(text)  # round trip
    assert H.tuning() == text
    got = [int(v) for v in H.hull(t).cpu().numpy()]
    assert got == expect_hull(xy)
    say("autotune batched")
    parts, off, bxy = make_batch(6, 64, 80_000)
    text2 = H.autotune(torch.from_numpy(bxy).cuda(), torch.from_numpy(off).cuda(), reps=1)
    assert text2.count("log2n") == 2, text2
    out, out_off = H.hull_batched(torch.from_numpy(bxy).cuda(), torch.from_numpy(off).cuda())
    check_batched(out, out_off, parts)
    H.set_tuning('{"entries": []}')


def test_graph_replays_match_eager(H):
    import torch
    say("graph replays")
    parts, off, xy = make_batch(8, 96, 40_000)
    xy_d = torch.from_numpy(xy).cuda()
    off_d = torch.from_numpy(off).cuda()
    eager, eager_off = H.hull_batched(xy_d, off_d)
    eager = eager.clone()
    eager_off = eager_off.clone()
    check_batched(eager, eager_off, parts)
    g = H.graph(xy_d, off_d)
    try:
        for rep in range(4):
            g.launch()
            out, out_off = g.result()
            assert torch.equal(out_off, eager_off), rep
            assert torch.equal(out, eager), rep
            # the program's own eager work between replays
            e2, _ = H.hull_batched(xy_d, off_d)
            assert torch.equal(e2, eager)
            torch.cuda.synchronize()
        # refill the same buffers with other points of the same sizes
        parts2 = []
        for s in range(len(parts)):
            n = int(off[s + 1] - off[s])
            parts2.append(workloads.make("disk" if s % 2 else "circle", n, 900 + s))
        xy2 = np.concatenate(parts2, 0).astype(np.float32)
        xy_d.copy_(torch.from_numpy(xy2))
        for rep in range(2):
            g.launch()
            out, out_off = g.result()
            check_batched(out, out_off, parts2)
    finally:
        g.close()


def test_graph_single_hull(H):
    import torch
    say("graph single hull")
    xy = workloads.circle(300_000, 21)
    t = torch.from_numpy(xy).cuda()
    g = H.graph(t)
    try:
        expect = expect_hull(xy)
        for rep in range(3):
            g.launch()
            out, _ = g.result()
            assert [int(v) for v in out.cpu().numpy()] == expect, rep
    finally:
        g.close()
