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


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call([
            "gcc", "-O3", "-march=x86-64-v2", "-ffp-contract=off", "-fno-fast-math",
            "-fPIC", "-shared", "-std=c11", "-o", tmp, SRC_PATH, "-lm",
        ])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        lib = ctypes.CDLL(LIB_PATH)
        lib.oracle_hull.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                    ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
        lib.oracle_hull.restype = ctypes.c_int
        lib.oracle_orient_sign.argtypes = [ctypes.c_float] * 6
        lib.oracle_orient_sign.restype = ctypes.c_int
        _lib = lib
    return _lib


class OracleError(RuntimeError):
    pass


def c_hull(xy: np.ndarray) -> np.ndarray:
    """Hull indices (int32) from the C oracle."""
    a = np.ascontiguousarray(np.asarray(xy, dtype=np.float32).reshape(-1, 2))
    n = a.shape[0]
    out = np.empty(max(n, 1), dtype=np.int32)
    h = ctypes.c_int64(0)
    rc = _load().oracle_hull(a.ctypes.data, n, out.ctypes.data, out.shape[0], ctypes.byref(h))
    if rc != 0:
        raise OracleError(f"oracle_hull returned {rc}")
    return out[:h.value].copy()


def c_orient_sign(a, b, c) -> int:
    return int(_load().oracle_orient_sign(float(a[0]), float(a[1]), float(b[0]), float(b[1]),
                                          float(c[0]), float(c[1])))
