"""Seeded synthetic point sets for the planar convex-hull workloads.

This module only draws numbers: it holds none of the hull method's arithmetic,
so both the CPU oracle (``oracle/``) and the HIP path read their inputs from
here. Every generator returns a C-contiguous ``float32`` array of shape
``(n, 2)`` holding ``(x, y)`` pairs (array-of-structures, 8 bytes per point).

The paper evaluates points drawn uniformly in the unit square (section 5,
Table 2, n = 100K ... 20M). The other recipes widen that to the unit disk, a
jittered circle (most points on or near the hull) and an integer grid with
duplicates and collinear runs on the bounding box, which exercise the exact
predicates; their recipes are stated next to each function.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

KINDS = ("square", "disk", "circle", "grid")


def square(n: int, seed: int = 0) -> np.ndarray:
    """Uniform in [0, 1)^2: ``default_rng(seed).random((n, 2), float32)``.

    numpy draws float32 uniforms as k * 2**-24, so every coordinate lies on a
    2**-24 grid in [0, 1)."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.random((n, 2), dtype=np.float32))


def disk(n: int, seed: int = 0) -> np.ndarray:
    """Uniform in the unit disk: r = sqrt(U1), theta = 2 pi U2, evaluated in
    float64 and rounded to float32."""
    rng = np.random.default_rng(seed)
    u1 = rng.random(n)
    u2 = rng.random(n)
    r = np.sqrt(u1)
    th = 2.0 * math.pi * u2
    out = np.empty((n, 2), dtype=np.float32)
    out[:, 0] = r * np.cos(th)
    out[:, 1] = r * np.sin(th)
    return out


def circle(n: int, seed: int = 0, jitter: float = 1e-6) -> np.ndarray:
    """Unit circle with radial jitter: theta = 2 pi U1, r = 1 + jitter*(2 U2 - 1),
    in float64, rounded to float32. The jitter is only ~8-17 float32 ulps at
    radius 1, so most points are on or within a few ulps of the hull."""
    rng = np.random.default_rng(seed)
    u1 = rng.random(n)
    u2 = rng.random(n)
    th = 2.0 * math.pi * u1
    r = 1.0 + jitter * (2.0 * u2 - 1.0)
    out = np.empty((n, 2), dtype=np.float32)
    out[:, 0] = r * np.cos(th)
    out[:, 1] = r * np.sin(th)
    return out


def grid(n: int, seed: int = 0, side: int = 4096, dup_frac: float = 0.3,
         edge_frac: float = 0.02) -> np.ndarray:
    """Integer grid [0, side)^2 cast to float32 (exact).

    0.7n base points are drawn i.i.d. on the grid; ``edge_frac`` of them are
    snapped onto a random bounding-box edge (x or y set to 0 or side-1), which
    creates long collinear runs on the hull; the remaining 0.3n points are
    copies of random base points (duplicates). The result is shuffled."""
    rng = np.random.default_rng(seed)
    nb = n - int(round(dup_frac * n))
    if n > 0 and nb == 0:
        nb = 1
    base = rng.integers(0, side, size=(nb, 2), dtype=np.int64)
    ns = int(edge_frac * nb)
    if ns > 0:
        who = rng.choice(nb, size=ns, replace=False)
        edge = rng.integers(0, 4, size=ns)
        base[who[edge == 0], 0] = 0
        base[who[edge == 1], 0] = side - 1
        base[who[edge == 2], 1] = 0
        base[who[edge == 3], 1] = side - 1
    nd = n - nb
    dups = base[rng.integers(0, nb, size=nd)] if nd > 0 else np.empty((0, 2), np.int64)
    pts = np.concatenate([base, dups], axis=0)
    pts = pts[rng.permutation(len(pts))]
    return np.ascontiguousarray(pts.astype(np.float32))


def make(kind: str, n: int, seed: int = 0) -> np.ndarray:
    if kind == "square":
        return square(n, seed)
    if kind == "disk":
        return disk(n, seed)
    if kind == "circle":
        return circle(n, seed)
    if kind == "grid":
        return grid(n, seed)
    raise ValueError(f"unknown workload kind {kind!r}")


@dataclass
class Batch:
    """Many independent point sets stored back to back.

    ``xy`` is (N, 2) float32; set s owns rows ``offsets[s]:offsets[s+1]``."""
    xy: np.ndarray
    offsets: np.ndarray  # int64, nsets + 1
    kinds: list

    @property
    def nsets(self) -> int:
        return len(self.offsets) - 1

    def set(self, s: int) -> np.ndarray:
        return self.xy[self.offsets[s]:self.offsets[s + 1]]


def log_uniform_sizes(rng: np.random.Generator, count: int, lo: float, hi: float) -> np.ndarray:
    """floor(exp(U(ln lo, ln hi))) for ``count`` draws."""
    u = rng.random(count)
    return np.floor(np.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))).astype(np.int64)


def batch(nsets: int = 4096, seed: int = 4, lo: int = 64, hi: int = 1 << 20,
          kinds=("square", "disk", "circle"), total: int | None = None) -> Batch:
    """``nsets`` independent sets with log-uniform sizes in [lo, hi]; each set's
    distribution is drawn uniformly from ``kinds`` and its points from its own
    child seed. With ``total`` the sizes are rescaled so they sum to about
    ``total`` (each at least ``lo``)."""
    rng = np.random.default_rng(seed)
    sizes = log_uniform_sizes(rng, nsets, lo, hi)
    if total is not None and sizes.sum() > 0:
        sizes = np.maximum(lo, np.floor(sizes * (total / sizes.sum()))).astype(np.int64)
    which = rng.integers(0, len(kinds), size=nsets)
    offsets = np.zeros(nsets + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    xy = np.empty((int(offsets[-1]), 2), dtype=np.float32)
    child = np.random.SeedSequence(seed).spawn(nsets)
    names = []
    for s in range(nsets):
        kind = kinds[which[s]]
        names.append(kind)
        sub_seed = int(child[s].generate_state(1)[0])
        xy[offsets[s]:offsets[s + 1]] = make(kind, int(sizes[s]), sub_seed)
    return Batch(xy=xy, offsets=offsets, kinds=names)


@dataclass
class Request:
    arrival_s: float
    xy: np.ndarray
    kind: str
    tag: int


def request_stream(count: int, qps: float, seed: int = 5, lo: int = 1000,
                   hi: int = 4_000_000, kinds=("square", "disk", "circle")):
    """Poisson arrivals at rate ``qps``; sizes log-uniform in [lo, hi]; mixed
    distributions. Returns a list of ``Request`` sorted by arrival time."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / qps, size=count) if qps > 0 else np.zeros(count)
    t = np.cumsum(gaps)
    sizes = log_uniform_sizes(rng, count, lo, hi)
    which = rng.integers(0, len(kinds), size=count)
    child = np.random.SeedSequence(seed).spawn(count)
    out = []
    for i in range(count):
        kind = kinds[which[i]]
        out.append(Request(float(t[i]), make(kind, int(sizes[i]), int(child[i].generate_state(1)[0])),
                           kind, i))
    return out


def request_windows(count: int, seed: int = 5, lo: int = 1000, hi: int = 4_000_000, nkinds: int = 3):
    """Request recipes for the serving workload without materialising every
    set: request i takes ``sizes[i]`` consecutive points, from ``starts[i]``,
    of the ``kinds[i]``-th pool of ``hi`` points (one pool per distribution,
    drawn once by ``make(kind, hi, seed)``). Sizes are log-uniform in
    [lo, hi], kinds uniform, starts uniform over the pool; returns three
    int64 arrays (kinds, starts, sizes)."""
    rng = np.random.default_rng(seed)
    sizes = log_uniform_sizes(rng, count, lo, hi).astype(np.int64)
    kinds = rng.integers(0, nkinds, size=count).astype(np.int64)
    starts = np.floor(rng.random(count) * (hi - sizes + 1)).astype(np.int64)
    return kinds, starts, sizes
