"""CPU oracle for the planar convex hull -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s
``cpu_baseline`` leg may import, call, link or execute anything here. The
library in ``paper_1501_04706_amd`` never does and shares no code with it.

* ``hull_exact``      -- Andrew's monotone chain on exact integers, an O(n^3)
                          brute-force hull and the invariant checker (Python).
* ``monotone_chain.c`` -- the same monotone chain in C with exact expansion
                          orientation; the timed CPU baseline (``c_hull``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle_hull.so")
SRC_PATH = os.path.join(HERE, "monotone_chain.c")

_lib = None


def build(force: bool = True, path: str | None = None, native: bool = False) -> str:
    """Compile the C oracle with gcc (no fast-math, no FMA contraction).

    The in-tree copy is built for a portable x86-64 level (it is built on one
    machine and may run on another); ``native=True`` builds a copy for the
    machine it runs on (the timed CPU baseline)."""
    path = path or LIB_PATH
    if force or not os.path.exists(path):
        tmp = path + ".tmp"
        subprocess.check_call([
            "gcc", "-O3", "-march=native" if native else "-march=x86-64-v2", "-ffp-contract=off",
            "-fno-fast-math", "-fPIC", "-shared", "-std=c11", "-o", tmp, SRC_PATH, "-lm",
        ])
        os.replace(tmp, path)
    return path


def load_lib(path: str) -> ctypes.CDLL:
    lib = ctypes.CDLL(path)
    lib.oracle_hull.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
    lib.oracle_hull.restype = ctypes.c_int
    lib.oracle_orient_sign.argtypes = [ctypes.c_float] * 6
    lib.oracle_orient_sign.restype = ctypes.c_int
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = load_lib(LIB_PATH)
    return _lib


class OracleError(RuntimeError):
    pass


def c_hull(xy: np.ndarray, lib: ctypes.CDLL | None = None) -> np.ndarray:
    """Hull indices (int32) from the C oracle (``lib``: another build of it)."""
    a = np.ascontiguousarray(np.asarray(xy, dtype=np.float32).reshape(-1, 2))
    n = a.shape[0]
    out = np.empty(max(n, 1), dtype=np.int32)
    h = ctypes.c_int64(0)
    rc = (lib or _load()).oracle_hull(a.ctypes.data, n, out.ctypes.data, out.shape[0], ctypes.byref(h))
    if rc != 0:
        raise OracleError(f"oracle_hull returned {rc}")
    return out[:h.value].copy()


def c_hull_sharded(xy: np.ndarray, threads: int, lib: ctypes.CDLL | None = None) -> np.ndarray:
    """The same hull on ``threads`` host threads: the C oracle on contiguous
    index ranges at once (ctypes releases the GIL during the call), then once
    more on the union of the range hulls, whose hull is the hull of all
    points. Ranges are in index order and each range hull names the lowest
    index at its positions, so the first copy of a position in the union is
    its lowest input index, as the oracle's tie rule requires."""
    from concurrent.futures import ThreadPoolExecutor
    a = np.ascontiguousarray(np.asarray(xy, dtype=np.float32).reshape(-1, 2))
    n = a.shape[0]
    threads = max(1, min(int(threads), max(n, 1)))
    cuts = [n * k // threads for k in range(threads + 1)]
    with ThreadPoolExecutor(max_workers=threads) as ex:
        parts = list(ex.map(lambda k: c_hull(a[cuts[k]:cuts[k + 1]], lib) + cuts[k], range(threads)))
    ids = np.concatenate(parts).astype(np.int64) if parts else np.zeros(0, np.int64)
    local = c_hull(a[ids], lib)
    return ids[local].astype(np.int32)


def c_orient_sign(a, b, c) -> int:
    return int(_load().oracle_orient_sign(float(a[0]), float(a[1]), float(b[0]), float(b[1]),
                                          float(c[0]), float(c[1])))
