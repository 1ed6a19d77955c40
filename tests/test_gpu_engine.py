"""GPU: the continuous-batching engine returns, for every request, exactly
the oracle's hull -- alone, and mixed with requests admitted before and after
it while their segments are resident (through the C ABI)."""
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


def requests(seed, count, lo, hi):
    rng = np.random.default_rng(seed)
    kinds = ["square", "disk", "circle", "grid"]
    out = []
    for i in range(count):
        n = int(np.floor(np.exp(rng.uniform(np.log(lo), np.log(hi)))))
        out.append(workloads.make(kinds[i % 4], n, seed * 10_000 + i))
    return out


def drain(E, results, max_passes):
    E.step(max_passes)
    while True:
        r = E.poll()
        if r is None:
            return
        tag, hull = r
        assert tag not in results
        results[tag] = hull


def test_engine_alone_equals_oracle(H):
    say("engine: one request at a time")
    E = H.engine(1 << 21, 64)
    try:
        for i, xy in enumerate(requests(1, 12, 5, 200_000)):
            results = {}
            assert E.admit(xy, i)
            for _ in range(200):
                drain(E, results, 3)
                if i in results:
                    break
            assert [int(v) for v in results[i]] == expect_hull(xy), i
            st = E.status()
            assert st["resident"] == 0 and st["staged"] == 0 and st["free_slots"] == E.slots
    finally:
        E.close()


@pytest.mark.parametrize("max_passes,engine_grid", [(1, 0), (2, 64), (5, 128)])
def test_engine_mix_staggered(H, max_passes, engine_grid):
    # new requests join every step while older ones still have segments
    say(f"engine: staggered mix, {max_passes} passes per step, engine grid {engine_grid}")
    reqs = requests(2 + max_passes, 60, 3, 150_000)
    if engine_grid:
        H.set_tuning('{"entries": [], "engine_grid": %d}' % engine_grid)
    E = H.engine(1 << 21, 256)
    try:
        results = {}
        pending = list(range(len(reqs)))
        steps = 0
        overlapped = 0
        while pending or len(results) < len(reqs):
            # admit up to three new requests per step, as room allows
            for _ in range(3):
                if pending and E.admit(reqs[pending[0]], pending[0]):
                    pending.pop(0)
            st = E.status()
            if st["resident"] > 0 and st["staged"] > 0:
                overlapped += 1
            drain(E, results, max_passes)
            steps += 1
            assert steps < 5000
        assert overlapped > 0, "no step mixed new and resident requests"
        for i, xy in enumerate(reqs):
            assert [int(v) for v in results[i]] == expect_hull(xy), i
        assert E.status()["free_slots"] == E.slots
    finally:
        E.close()
        H.set_tuning('{"entries": []}')


def test_engine_admission_by_footprint(H):
    say("engine: admission by footprint")
    E = H.engine(1 << 18, 16)  # 262144 slots
    try:
        big = workloads.circle(200_000, 5)
        small = workloads.square(100_000, 6)
        assert E.admit(big, 0)
        assert not E.admit(small, 1)  # 200000 + 100000 slots do not fit
        results = {}
        for _ in range(100):
            drain(E, results, 2)
            if 0 in results:
                break
        assert 0 in results
        assert E.admit(small, 1)  # the big request's slots were freed
        for _ in range(100):
            drain(E, results, 2)
            if 1 in results:
                break
        assert [int(v) for v in results[0]] == expect_hull(big)
        assert [int(v) for v in results[1]] == expect_hull(small)
        with pytest.raises(sqh.SqhError):
            E.admit(workloads.square((1 << 18) + 1, 7), 2)  # can never fit
    finally:
        E.close()


def test_engine_bad_and_empty_requests(H):
    say("engine: non-finite and empty requests")
    E = H.engine(1 << 20, 64)
    try:
        good = requests(9, 6, 10, 50_000)
        bad = workloads.disk(5000, 3)
        bad[1234, 0] = np.inf
        results = {}
        for i, xy in enumerate(good[:3]):
            assert E.admit(xy, i)
        assert E.admit(bad, 100)
        assert E.admit(np.zeros((0, 2), np.float32), 200)
        for i, xy in enumerate(good[3:], start=3):
            assert E.admit(xy, i)
        for _ in range(300):
            drain(E, results, 3)
            if len(results) == len(good) + 2:
                break
        assert results[100] is None
        assert len(results[200]) == 0
        for i, xy in enumerate(good):
            assert [int(v) for v in results[i]] == expect_hull(xy), i
    finally:
        E.close()


def test_engine_device_input_and_fp64(H):
    import torch
    say("engine: device input, fp64-only mode")
    reqs = requests(11, 10, 100, 300_000)
    H2 = sqh.Hull(0, precision=sqh.SQH_FP64_ONLY)
    E = H2.engine(1 << 22, 64)
    try:
        results = {}
        for i, xy in enumerate(reqs):
            assert E.admit(torch.from_numpy(xy).cuda(), i)
        for _ in range(300):
            drain(E, results, 4)
            if len(results) == len(reqs):
                break
        for i, xy in enumerate(reqs):
            assert [int(v) for v in results[i]] == expect_hull(xy), i
    finally:
        E.close()
        H2.close()


def test_engine_admit_while_step_in_flight(H):
    import torch
    say("engine: admissions on a copy stream overlap launched steps")
    reqs = requests(13, 40, 50, 400_000)
    pinned = [torch.from_numpy(xy).pin_memory() for xy in reqs]
    copy = torch.cuda.Stream()
    E = H.engine(1 << 22, 128, 1 << 20)
    try:
        results = {}
        nxt = 0
        inflight = False
        rounds = 0
        while len(results) < len(reqs):
            # admit two per round: these copies run while the launched step computes
            for _ in range(2):
                if nxt < len(reqs) and E.admit(pinned[nxt], nxt, stream=copy):
                    nxt += 1
            if inflight:
                E.finish()
                while True:
                    r = E.poll()
                    if r is None:
                        break
                    results[r[0]] = r[1]
            inflight = E.launch(2)
            rounds += 1
            assert rounds < 2000
        with pytest.raises(sqh.SqhError):
            # a second launch while one is in flight is refused
            assert E.admit(pinned[0], 999, stream=copy)
            E.launch(2)
            E.launch(2)
        E.finish()
        for i, xy in enumerate(reqs):
            assert [int(v) for v in results[i]] == expect_hull(xy), i
    finally:
        E.close()


def serving_requests(seed, count, lo=1_000_000, hi=4_000_000):
    """Requests from the upper part of the serving size range (log-uniform),
    kinds square/disk/circle as the serving workload draws them."""
    rng = np.random.default_rng(seed)
    kinds = ["square", "disk", "circle"]
    out = []
    for i in range(count):
        n = int(np.floor(np.exp(rng.uniform(np.log(lo), np.log(hi)))))
        out.append(workloads.make(kinds[int(rng.integers(0, 3))], n, seed * 1000 + i))
    return out


def test_engine_large_requests_alone_and_mixed(H):
    # 1M .. 4M-point requests: each alone, then all of them in flight at once
    # with admissions staggered over the steps; every result is the oracle's
    reqs = serving_requests(21, 5)
    say("engine: large requests " + ", ".join(str(len(r)) for r in reqs))
    want = [[int(v) for v in oracle.c_hull(xy)] for xy in reqs]
    E = H.engine(1 << 24, 64, 1 << 23)
    try:
        for i, xy in enumerate(reqs):
            results = {}
            assert E.admit(xy, i)
            for _ in range(400):
                drain(E, results, 4)
                if i in results:
                    break
            assert [int(v) for v in results[i]] == want[i], ("alone", i, len(xy))
        results = {}
        pending = list(range(len(reqs)))
        steps = 0
        while len(results) < len(reqs):
            if pending and E.admit(reqs[pending[0]], 100 + pending[0]):
                pending.pop(0)
            drain(E, results, 2)
            steps += 1
            assert steps < 4000
        for i in range(len(reqs)):
            assert [int(v) for v in results[100 + i]] == want[i], ("mixed", i, len(reqs[i]))
        assert E.status()["free_slots"] == E.slots
    finally:
        E.close()
