"""CPU: the C oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

The oracle is the parity reference, so its own memory safety matters: the
harness `tests/oracle_sanitize.c` is linked with `oracle/monotone_chain.c`,
both built with `-fsanitize=address,undefined`, and run on random,
duplicate-heavy, collinear and degenerate inputs (also with an output
capacity one short of the hull); every run must be clean and print the
hull the normal build returns.
"""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from paper_1501_04706_amd import workloads

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def harness():
    gcc = shutil.which("gcc")
    if not gcc:
        pytest.skip("gcc not found")
    d = tempfile.mkdtemp(prefix="oracle_san_")
    exe = os.path.join(d, "oracle_san")
    cmd = [gcc, "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-ffp-contract=off", "-std=c11",
           "-o", exe, os.path.join(HERE, "oracle_sanitize.c"), oracle.SRC_PATH, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("sanitizer build unavailable: " + r.stderr[-300:])
    yield exe, d
    shutil.rmtree(d, ignore_errors=True)


def cases():
    rng = np.random.default_rng(41)
    yield "empty", np.zeros((0, 2), np.float32)
    yield "one", np.array([[1.5, -2.0]], np.float32)
    yield "two equal", np.array([[1, 1], [1, 1]], np.float32)
    yield "collinear", np.stack([np.arange(500), 3 * np.arange(500)], 1).astype(np.float32)[::-1].copy()
    yield "all equal", np.full((3000, 2), 0.25, np.float32)
    yield "signed zeros", np.array([[-0.0, 0.0], [0.0, -0.0], [1, 0], [0, 1]], np.float32)
    yield "small grids", (rng.integers(-3, 4, size=(400, 2)) * 0.5).astype(np.float32)
    for kind in ("square", "disk", "circle", "grid"):
        yield kind, workloads.make(kind, 20_000, 7)


@pytest.mark.parametrize("name,xy", list(cases()))
def test_oracle_clean_under_sanitizers(harness, name, xy):
    exe, d = harness
    path = os.path.join(d, "in.bin")
    with open(path, "wb") as f:
        f.write(np.int64(len(xy)).tobytes())
        f.write(np.ascontiguousarray(xy, dtype=np.float32).tobytes())
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe, path], capture_output=True, text=True, env=env)
    assert r.returncode == 0, (name, r.returncode, r.stderr[-2000:])
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-2000:]
    got = [int(v) for v in r.stdout.split()]
    assert got == [int(v) for v in oracle.c_hull(xy)], name
