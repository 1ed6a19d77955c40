#!/usr/bin/env python3
"""Benchmark of the segmented QuickHull library on one MI355X.

Default workload: one convex hull of n = 20,000,000 float32 points drawn
uniformly in the unit square (seed 0) -- the largest size of the paper's
Table 2 workload. A step is one full sqh_hull call (seed, first split, first
compaction, every segmented pass, table rebuilds, ordered emission) with the
input already resident in device memory; the call returns the hull size to
the host, so each step ends synchronised.

Prints one JSON line:
  value      whole-job throughput in Mpoints/s (n / step time), warm caches
  roofline   the dominant kernel (largest device time per step): its
             algorithmic HBM bytes per launch divided by its average launch
             time, from HIP events the library records on the launch stream
             before and after every kernel during the timed steps, against
             the 8 TB/s HBM3E peak; `traffic` is the measured HBM bytes per
             launch from the committed rocprofv3 counter runs
  kernels    the same figures for every kernel of the call
  cold       the same call after writing 1 GiB of scratch before each
             repetition (the 256 MB last-level cache no longer holds the
             160 MB input)
  config3    the adversarial 20M-point workloads (jittered circle, integer
             grid): time, predicate fallback rates, passes
  filters    the static line filter against the semi-static filter alone:
             time and fallback rate per workload
  cpu_baseline  the C oracle (monotone chain, exact predicates) timed on
             this host on the same input, on one core and on all cores
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "traffic.json")
# launch names reported by the library -> the kernel's name in rocprofv3
PROFILER_NAME = {"k_sfirst<line>": "k_sfirst<true>", "k_sfirst<semistatic>": "k_sfirst<false>"}


def call_bytes(st: dict, n: int) -> int:
    """Algorithmic HBM bytes of one whole sqh_hull call.

    seed   reads the (x, y) input once: 8 B/pt
    split  reads it again: 8 B/pt
    first  reads it a third time and writes each survivor (x, y, index): 12 B
    pass   reads each point entering the pass (12 B) and writes each point
           kept for the next pass (12 B)
    Segment tables, counters and the output are O(h + segments) and left out.
    """
    pts = list(st["pass_points"])[: int(st["passes"])]
    pass_bytes = 0
    for k, v in enumerate(pts):
        nxt = pts[k + 1] if k + 1 < len(pts) else 0
        pass_bytes += 12 * v + 12 * nxt
    return 8 * n + 8 * n + 8 * n + 12 * int(st["first_survivors"]) + pass_bytes


def launch_sequence(st: dict, n_spass: int) -> list:
    """The launches of a plain sqh_hull call, as (name, 0.0) pairs: the
    streaming path (with n_spass k_spass launches; the passes kernel when the
    call needed it) or the general path's one hull kernel."""
    if int(st.get("stream_path", 0)) == 0:
        names = ["k_reset", "k_hull<plain>"]
    else:
        names = ["k_reset", "k_sseed", "k_ssplit", "k_sfirst<line>", "k_sfirst<semistatic>"] + \
                ["k_spass"] * n_spass + ["k_stail"] + (["k_hull<passes>"] if int(st["stream_path"]) == 2 else [])
    return [(x, 0.0) for x in names]


def launch_bytes(launches: list, st: dict, n: int) -> list:
    """Algorithmic HBM bytes of each launch of one call on the streaming path
    (k_sseed, k_ssplit: one read of the input, 8 B/pt; the first compaction:
    one read plus 12 B per survivor written -- its second read of each tile
    is meant to hit the cache and is not counted; the k-th k_spass launch:
    pass k's reads and writes, 12 B per point each way, when it ran that
    pass; the passes kernel when it ran, else the tail: the rest)."""
    pts = list(st["pass_points"])[: int(st["passes"])]

    def pass_b(k):
        nxt = pts[k + 1] if k + 1 < len(pts) else 0
        return 12 * pts[k] + 12 * nxt

    line = int(st.get("line_filter", 0))
    fallback = any(name == "k_hull<passes>" for name, _ in launches)
    out, k_spass, spass_ran = [], 0, 0
    for name, _ in launches:
        b = 0
        if name == "k_hull<plain>":
            b = call_bytes(st, n)
        elif name in ("k_sseed", "k_ssplit"):
            b = 8 * n
        elif name == "k_sfirst<line>":
            b = (8 * n + 12 * int(st["first_survivors"])) if line else 0
        elif name == "k_sfirst<semistatic>":
            b = 0 if line else 8 * n + 12 * int(st["first_survivors"])
        elif name == "k_spass":
            # a streaming pass runs while the table qualifies: more than 6144
            # points (fewer: the LDS passes) in at most 256 segments
            if k_spass < len(pts) and k_spass == spass_ran and pts[k_spass] > 6144 and \
                    int(st["pass_segments"][k_spass]) <= 256:
                b = pass_b(k_spass)
                spass_ran += 1
            k_spass += 1
        elif name == "k_hull<passes>" or (name == "k_stail" and not fallback):
            b = sum(pass_b(k) for k in range(spass_ran, len(pts)))
        out.append(b)
    return out


def load_traffic(kernel: str):
    """Measured HBM bytes per launch of `kernel` (its rocprofv3 name) from the
    committed counter summary, if it was taken for the current build."""
    try:
        with open(PROFILE_TRAFFIC) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    rec = d.get(kernel)
    if not rec or rec.get("build") != library_fingerprint():
        return None
    return rec.get("bytes_per_launch")


def _counter_per_dispatch(run_dir: str, counter: str, name_part: str) -> tuple:
    """Average over dispatches of `counter` (summed over its instances) for
    the kernels whose name contains name_part, from a rocprofv3 --pmc
    directory (its *counter_collection.csv)."""
    import csv
    import glob
    files = glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {run_dir}")
    per = {}
    for path in files:
        with open(path, newline="") as f:
            for row in csv.DictReader(f):
                if row.get("Counter_Name") != counter or name_part not in row.get("Kernel_Name", ""):
                    continue
                key = (path, row.get("Dispatch_Id") or row.get("Correlation_Id"))
                per[key] = per.get(key, 0.0) + float(row["Counter_Value"])
    if not per:
        raise SystemExit(f"no {counter} rows for kernels matching {name_part!r} in {run_dir}")
    return sum(per.values()) / len(per), len(per)


def write_traffic(kname: str, fetch_dir: str, write_dir: str, copy_fetch_dir: str, copy_write_dir: str,
                  copy_bytes: int = 160_000_000) -> dict:
    """HBM bytes per launch of kernel `kname` (a part of its rocprofv3 name)
    from two counter runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch), each
    scaled by what the same counter reads for a device-to-device copy of
    copy_bytes in each direction; merged into profiles/traffic.json with the
    build's fingerprint."""
    f_k, nk = _counter_per_dispatch(fetch_dir, "FETCH_SIZE", kname)
    w_k, _ = _counter_per_dispatch(write_dir, "WRITE_SIZE", kname)
    f_c, nc = _counter_per_dispatch(copy_fetch_dir, "FETCH_SIZE", "copy")
    w_c, _ = _counter_per_dispatch(copy_write_dir, "WRITE_SIZE", "copy")
    ff = copy_bytes / (f_c * 1024.0)
    fw = copy_bytes / (w_c * 1024.0)
    rec = {
        "build": library_fingerprint(),
        "bytes_per_launch": int(f_k * 1024.0 * ff + w_k * 1024.0 * fw),
        "fetch_kib": round(f_k, 1), "write_kib": round(w_k, 1), "dispatches": nk,
        "copy_fetch_kib": round(f_c, 1), "copy_write_kib": round(w_c, 1), "copy_dispatches": nc,
        "fetch_scale": round(ff, 4), "write_scale": round(fw, 4),
    }
    try:
        with open(PROFILE_TRAFFIC) as f:
            allrec = json.load(f)
    except (OSError, ValueError):
        allrec = {}
    allrec[kname] = rec
    with open(PROFILE_TRAFFIC, "w") as f:
        json.dump(allrec, f, indent=1)
        f.write("\n")
    return rec


def library_fingerprint() -> str:
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1501_04706_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def host_threads() -> int:
    """Threads the CPU baseline may use: every core the process may run on,
    at most the job's thread allowance (OMP_NUM_THREADS where it is set)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    cap = os.environ.get("OMP_NUM_THREADS")
    if cap and cap.isdigit() and int(cap) > 0:
        n = min(n, int(cap))
    return max(1, n)


def cpu_baseline(xy, budget_s: float = 25.0) -> dict:
    """The C oracle on this host: built for this machine (-march=native, else
    the portable in-tree build), timed on one core and on all the cores the
    job may use (contiguous index ranges at once, then the hull of their
    hulls; the result is checked against the one-core result)."""
    import tempfile
    import numpy as np
    import oracle
    n = len(xy)
    lib, build = None, "portable in-tree build (-march=x86-64-v2)"
    try:
        d = tempfile.mkdtemp(prefix="sqh_oracle_")
        lib = oracle.load_lib(oracle.build(force=True, path=os.path.join(d, "liboracle_native.so"), native=True))
        build = "gcc -O3 -march=native"
    except Exception as e:  # compiler missing or the flag refused: time the portable build
        build += f" (native build failed: {type(e).__name__})"
    threads = host_threads()

    def timed(fn, cap):
        times, res = [], None
        t_start = time.perf_counter()
        while True:
            t0 = time.perf_counter()
            res = fn()
            times.append(time.perf_counter() - t0)
            if time.perf_counter() - t_start + times[-1] > budget_s / 2 or len(times) >= cap:
                break
        return statistics.median(times), len(times), res

    t1, r1, h1 = timed(lambda: oracle.c_hull(xy, lib), 3)
    tN, rN, hN = timed(lambda: oracle.c_hull_sharded(xy, threads, lib), 5)
    same = bool(np.array_equal(h1, hN))
    return {
        "value": round(n / tN / 1e6, 3),
        "unit": "Mpoints/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"C monotone chain (exact predicates), {build}, on the same {n}-point input: "
                  f"{threads} threads on contiguous index ranges plus the hull of their hulls, "
                  f"median of {rN} run(s) {tN:.2f} s; one core: median of {r1} run(s) {t1:.2f} s",
        "single_core_value": round(n / t1 / 1e6, 3),
        "nproc": os.cpu_count(),
        "threads_identical_to_one_core": same,
    }


def bench_batched(H, sqh, torch, workloads, total, steps: int, warmup: int, seed: int = 4) -> dict:
    """4096 independent sets (log-uniform sizes in [64, 2^20], kinds drawn from
    square/disk/circle) as one batched call, against one sqh_hull call per set
    on the same GPU, the same build and the same device-resident sets."""
    import numpy as np
    b = workloads.batch(4096, seed=seed, total=total)
    dev = torch.device("cuda", 0)
    xy_d = torch.from_numpy(b.xy).to(dev)
    off_d = torch.from_numpy(b.offsets).to(dev)
    n_total = int(b.offsets[-1])
    out = torch.empty(max(n_total, 1), dtype=torch.int32, device=dev)
    for _ in range(warmup):
        H.hull_batched(xy_d, off_d, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kern = 0.0
    for _ in range(steps):
        hv, _ = H.hull_batched(xy_d, off_d, out=out)
        kern += H.stats()["ms_kernel"]
    torch.cuda.synchronize()
    ms_batched = (time.perf_counter() - t0) * 1000.0 / steps
    st = H.stats()

    # one hull per launch: each set through sqh_hull, synchronising per hull
    sizes = np.diff(b.offsets)
    H.workspace(int(sizes.max()), 1)
    out1 = torch.empty(int(sizes.max()), dtype=torch.int32, device=dev)
    views = [xy_d[int(b.offsets[s]):int(b.offsets[s + 1])] for s in range(b.nsets)]
    for v in views[:64]:
        H.hull(v, out=out1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for v in views:
        H.hull(v, out=out1)
    torch.cuda.synchronize()
    ms_loop = (time.perf_counter() - t0) * 1000.0
    hps_b = b.nsets / (ms_batched / 1000.0)
    hps_l = b.nsets / (ms_loop / 1000.0)
    del xy_d, off_d, out, out1
    return {
        "workload": f"4096 sets, log-uniform sizes in [64, 2^20]"
                    + (f" rescaled to about {total} points" if total else "")
                    + f", square/disk/circle, seed {seed}",
        "points": n_total,
        "hulls_per_s": round(hps_b, 1),
        "ms_per_batch": round(ms_batched, 3),
        "kernel_ms_per_batch": round(kern / steps, 3),
        "Mpoints_per_s": round(n_total / (ms_batched / 1000.0) / 1e6, 1),
        "hull_vertices": int(hv.numel()),
        "passes": int(st["passes"]),
        "per_hull_loop_hulls_per_s": round(hps_l, 1),
        "per_hull_loop_ms": round(ms_loop, 2),
        "speedup_vs_per_hull_loop": round(hps_b / hps_l, 2),
    }


def bench_breakdown(H, sqh, torch, workloads, steps: int = 5, warmup: int = 2) -> list:
    """Per-phase device time of single hulls at the paper's sizes (1M .. 20M
    points, square and disk), plain, with each pre-filter and in the sorted-
    chain layout: the phase times come from the kernels' own clock stamps,
    the total from HIP events. sort_bytes: the radix sort's algorithmic
    traffic (4 passes x (4 B key read + 12 B read + 12 B write) per point)."""
    modes = (("plain", sqh.SQH_PREFILTER_NONE, sqh.SQH_VARIANT_PARTITION),
             ("quad", sqh.SQH_PREFILTER_QUAD, sqh.SQH_VARIANT_PARTITION),
             ("octagon", sqh.SQH_PREFILTER_OCTAGON, sqh.SQH_VARIANT_PARTITION),
             ("sorted", sqh.SQH_PREFILTER_NONE, sqh.SQH_VARIANT_SORTED))
    dev = torch.device("cuda", 0)
    rows = []
    for kind in ("square", "disk"):
        for n in (1_000_000, 5_000_000, 10_000_000, 20_000_000):
            xy_d = torch.from_numpy(workloads.make(kind, n, 0)).to(dev)
            out = torch.empty(n, dtype=torch.int32, device=dev)
            H.workspace(n, 1)
            for name, mode, variant in modes:
                H.set_prefilter(mode)
                H.set_variant(variant)
                for _ in range(warmup):
                    H.hull(xy_d, out=out)
                acc = {}
                for _ in range(steps):
                    H.hull(xy_d, out=out)
                    st = H.stats()
                    for k in ("ms_kernel", "ms_prefilter", "ms_seed", "ms_split", "ms_first", "ms_sort", "ms_pass",
                              "ms_emit"):
                        acc[k] = acc.get(k, 0.0) + st[k] / steps
                row = {"kind": kind, "n": n, "mode": name,
                       "Mpoints_per_s": round(n / (acc["ms_kernel"] / 1000.0) / 1e6, 1),
                       "subset": int(st["prefilter_points"]), "passes": int(st["passes"]),
                       "survivors_total": int(st["survivors_total"]),
                       **{k[3:]: round(v, 4) for k, v in acc.items()}}
                if variant == sqh.SQH_VARIANT_SORTED:
                    row["sorted_points"] = int(st["sorted_points"])
                    row["sort_violations"] = int(st["sort_violations"])
                    row["sort_bytes"] = 112 * max(int(st["sorted_points"]), 0)
                rows.append(row)
            H.set_prefilter(sqh.SQH_PREFILTER_NONE)
            H.set_variant(sqh.SQH_VARIANT_PARTITION)
            del xy_d, out
    return rows


def modes_at(rows: list, kind: str, n: int) -> dict:
    """Kernel throughput of each method variant (plain, pre-filters, sorted
    layout) on the benchmarked workload, taken from the breakdown rows."""
    return {r["mode"]: {"Mpoints_per_s": r["Mpoints_per_s"], "ms_kernel": r["kernel"]}
            for r in rows if r["kind"] == kind and r["n"] == n}


def _percentiles(lat_ms):
    import numpy as np
    v = np.asarray(lat_ms, dtype=np.float64)
    return {"p50_ms": round(float(np.percentile(v, 50)), 3), "p99_ms": round(float(np.percentile(v, 99)), 3),
            "mean_ms": round(float(v.mean()), 3)}


def bench_serving(H, sqh, torch, workloads, count: int = 2000, warm: int = 200, max_passes: int = 32,
                  seed: int = 5) -> dict:
    """Poisson stream of hull requests (sizes log-uniform in [1e3, 4e6], kinds
    square/disk/circle): `warm` requests, then `count` fresh ones, each a
    distinct window of points from pinned host memory. The engine
    (continuous batching) against one sqh_hull per request in arrival order
    (the plain path), both timed from arrival to the hull indices in host
    memory; saturated (everything arrives at once), then Poisson arrivals at
    0.5 and 0.8 of the engine's saturated rate."""
    import numpy as np
    kinds_ = ("square", "disk", "circle")
    hi = 4_000_000
    # one pinned pool per distribution; a request is a window into one
    pools = [torch.from_numpy(workloads.make(k, hi, seed + 1 + i)).pin_memory() for i, k in enumerate(kinds_)]
    kk, ss, nn = workloads.request_windows(warm + count, seed=seed, lo=1000, hi=hi)
    sets = [pools[int(kk[i])][int(ss[i]):int(ss[i]) + int(nn[i])] for i in range(warm + count)]
    dev = torch.device("cuda", 0)
    dev_ms = [0.0]  # device time of the engine's steps

    def run_engine(H_, reqs, arrivals):
        # admissions copy on their own stream while the previous step computes
        E = H_.engine(1 << 25, 1024, 1 << 24)
        copy = torch.cuda.Stream()
        dev_ms[0] = 0.0
        m = len(reqs)
        try:
            res = {}
            done_t = {}
            t0 = time.perf_counter()
            nxt = 0
            inflight = False
            while len(done_t) < m:
                now = time.perf_counter() - t0
                while nxt < m and arrivals[nxt] <= now and E.admit(sets[reqs[nxt]], nxt, stream=copy):
                    nxt += 1
                if inflight:
                    E.finish()
                    dev_ms[0] += H_.stats()["ms_total"]
                    inflight = False
                    while True:
                        r = E.poll()
                        if r is None:
                            break
                        done_t[r[0]] = time.perf_counter() - t0
                        res[r[0]] = r[1]
                inflight = E.launch(max_passes)
                if not inflight and nxt < m:
                    time.sleep(max(0.0, arrivals[nxt] - (time.perf_counter() - t0)))
            wall = max(done_t.values())
            lat = [(done_t[i] - arrivals[i]) * 1000.0 for i in range(m)]
            return wall, lat, res
        finally:
            E.close()

    out1 = torch.empty(hi, dtype=torch.int32, device=dev)
    H.workspace(hi, 1)

    def run_plain(reqs, arrivals):
        t0 = time.perf_counter()
        lat = []
        res = {}
        for i, q in enumerate(reqs):
            now = time.perf_counter() - t0
            if arrivals[i] > now:
                time.sleep(arrivals[i] - now)
            xy = sets[q].to(dev, non_blocking=True)
            hv = H.hull(xy, out=out1).cpu().numpy()
            t = time.perf_counter() - t0
            lat.append((t - arrivals[i]) * 1000.0)
            res[i] = hv
        return time.perf_counter() - t0, lat, res

    warm_reqs = list(range(warm))
    reqs = list(range(warm, warm + count))
    zero = np.zeros(count)
    run_engine(H, warm_reqs, np.zeros(warm))  # warm-up requests
    run_plain(warm_reqs, np.zeros(warm))
    wall_e, _, res_e = run_engine(H, reqs, zero)
    dev_e = dev_ms[0]
    T = count / wall_e
    wall_p, _, res_p = run_plain(reqs, zero)
    Tp = count / wall_p
    same = all(np.array_equal(res_e[i], res_p[i]) for i in range(count))
    H64 = sqh.Hull(0, precision=sqh.SQH_FP64_ONLY)
    try:
        wall_64, _, res_64 = run_engine(H64, reqs, zero)
    finally:
        H64.close()
    same64 = all(np.array_equal(res_e[i], res_64[i]) for i in range(count))
    pts = int(sum(int(nn[q]) for q in reqs))
    out = {
        "workload": f"{warm} warm-up then {count} requests, each a distinct window of a 4M-point pool per "
                    f"distribution (square/disk/circle), sizes log-uniform in [1e3, 4e6], seed {seed}, "
                    f"pinned host input, {max_passes} passes per engine step",
        "points": pts,
        "saturated_hulls_per_s": round(T, 1),
        "plain_saturated_hulls_per_s": round(Tp, 1),
        "speedup_vs_plain": round(T / Tp, 2),
        "engine_device_ms": round(dev_e, 1),
        "engine_wall_ms": round(wall_e * 1000.0, 1),
        "plain_wall_ms": round(wall_p * 1000.0, 1),
        "fp64_only_saturated_hulls_per_s": round(count / wall_64, 1),
        "fp32_filter_vs_fp64_only": round(T / (count / wall_64), 3),
        "identical_to_plain": bool(same),
        "fp64_identical": bool(same64),
    }
    for frac in (0.5, 0.8):
        lam = frac * T
        gaps = np.random.default_rng(seed + 1).exponential(1.0 / lam, size=count)
        arr = np.cumsum(gaps)
        _, lat_e, _ = run_engine(H, reqs, arr)
        _, lat_p, _ = run_plain(reqs, arr)
        out[f"qps_{frac}T"] = round(lam, 1)
        out[f"engine_{frac}T"] = _percentiles(lat_e)
        out[f"plain_{frac}T"] = _percentiles(lat_p)
    del out1
    return out


def timed_calls(H, xy_d, out, n: int, steps: int, warmup: int, scratch=None, only=None) -> dict:
    """`steps` sqh_hull calls (after `warmup` untimed ones) with per-launch
    events on. Each call returns synchronised; wall_ms is the mean time
    inside the calls, loop_ms the mean including the reading of the stats
    and launch times between calls. With `scratch`, 1 GiB of it is
    rewritten before each call (outside the call's time). With `only`,
    events bracket only that kernel's launches."""
    import torch
    H.set_launch_timing(True, only)
    for _ in range(warmup):
        H.hull(xy_d, out=out)
    torch.cuda.synchronize()
    keys = ("ms_total", "ms_kernel", "ms_seed", "ms_split", "ms_first", "ms_pass", "ms_emit")
    agg = {k: 0.0 for k in keys}
    per = {}  # kernel -> [ms, launches, bytes]
    exact = evals = cmpx = 0
    totals = []
    last = None
    wall = 0.0
    torch.cuda.synchronize()
    l0 = time.perf_counter()
    for r in range(steps):
        if scratch is not None:
            scratch.fill_(float(r))
            torch.cuda.synchronize()
        t0 = time.perf_counter()
        H.hull(xy_d, out=out)
        wall += time.perf_counter() - t0
        st = H.stats()
        lt = H.launch_times()
        if only:
            # the byte model follows the call's whole launch sequence
            seq = launch_sequence(st, len(lt) if only == "k_spass" else 0)
            bl = [b for (x, _), b in zip(seq, launch_bytes(seq, st, n)) if x == only]
        else:
            bl = launch_bytes(lt, st, n)
        for name, b, (_, ms) in zip((x for x, _ in lt), bl, lt):
            e = per.setdefault(name, [0.0, 0, 0])
            e[0] += ms
            e[1] += 1
            e[2] += b
        for k in agg:
            agg[k] += st[k]
        totals.append(st["ms_total"])
        evals += st["orient_evals"]
        exact += st["orient_exact"]
        cmpx += st["cmp_exact"]
        last = st
    torch.cuda.synchronize()
    loop = time.perf_counter() - l0
    H.set_launch_timing(False)
    return {"wall_ms": wall * 1000.0 / steps, "loop_ms": loop * 1000.0 / steps, "agg": {k: v / steps for k, v in agg.items()}, "per": per,
            "totals": totals, "evals": evals, "exact": exact, "cmpx": cmpx, "last": last, "steps": steps}


def kernel_table(m: dict) -> dict:
    """Per-kernel device time per call, average launch time, algorithmic
    bytes per launch and the bandwidth they imply."""
    steps = m["steps"]
    rows = {}
    for name, (ms, nl, b) in m["per"].items():
        avg = ms / nl
        bpl = b / nl
        rows[name] = {"ms_per_call": round(ms / steps, 4), "launches_per_call": round(nl / steps, 2),
                      "avg_launch_ms": round(avg, 5), "alg_bytes_per_launch": int(bpl),
                      "GB_s": round(bpl / (avg / 1000.0) / 1e9, 1) if avg > 0 else 0.0}
    return rows


def filter_modes(H, sqh, torch, workloads, n: int, steps: int = 3, warmup: int = 1) -> dict:
    """The adversarial workloads and the square under both float32 filter
    modes: time per call and the predicates' exact-path rates."""
    dev = torch.device("cuda", 0)
    res = {}
    for kind in ("square", "circle", "grid"):
        xy_d = torch.from_numpy(workloads.make(kind, n, 0)).to(dev)
        out = torch.empty(n, dtype=torch.int32, device=dev)
        H.workspace(n, 1)
        row = {}
        for name, mode in (("fp32_filter", sqh.SQH_FP32_FILTER), ("fp32_semistatic", sqh.SQH_FP32_SEMISTATIC)):
            H.set_precision(mode)
            m = timed_calls(H, xy_d, out, n, steps, warmup, only="-")  # (no kernel has that name: no events)
            st = m["last"]
            row[name] = {
                "ms_per_call": round(m["wall_ms"], 4),
                "device_ms_per_call": round(m["agg"]["ms_total"], 4),
                "Mpoints_per_s": round(n / (m["wall_ms"] / 1000.0) / 1e6, 1),
                "orient_fallback_rate": m["exact"] / m["evals"] if m["evals"] else 0.0,
                "orient_exact_per_call": m["exact"] // steps,
                "cmp_exact_per_call": m["cmpx"] // steps,
                "line_filter": int(st["line_filter"]),
                "stream_path": int(st["stream_path"]),
                "passes": int(st["passes"]),
                "max_segments": int(st["max_segments"]),
                "hull_size": int(st["hull_size"]),
            }
        H.set_precision(sqh.SQH_FP32_FILTER)
        f, s_ = row["fp32_filter"]["ms_per_call"], row["fp32_semistatic"]["ms_per_call"]
        row["faster"] = "fp32_filter" if f <= s_ else "fp32_semistatic"
        res[kind] = row
        del xy_d, out
    return res


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=20_000_000)
    ap.add_argument("--kind", default="square", choices=["square", "disk", "circle", "grid"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp32-semistatic", "fp64"],
                    help="fp32: float32 filters with exact fallback (the static line filter where it "
                         "applies); fp32-semistatic: without the line filter; fp64: every predicate exact")
    ap.add_argument("--no-streaming", action="store_true",
                    help="run the general path (the persistent cooperative kernel) instead of the streaming "
                         "kernels of a large single hull")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve", type=int, default=2000, help="serving requests after 200 warm-up (0: skip)")
    ap.add_argument("--no-breakdown", action="store_true",
                    help="skip the per-phase breakdown over sizes and pre-filter modes")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the cold-cache leg, the adversarial workloads and the filter comparison")
    ap.add_argument("--batch", default="64M", choices=["64M", "full", "none"],
                    help="batched comparison: 4096 sets rescaled to ~64M points, the literal "
                         "log-uniform sizes (~4.4e8 points), or skip it")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device-to-device copy of the 20M-point input "
                         "(160 MB read + 160 MB written per launch), to scale HBM counters")
    ap.add_argument("--write-traffic", nargs=5, metavar=("KERNEL", "FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR",
                                                          "COPY_WRITE_DIR"),
                    help="no GPU work: turn four rocprofv3 --pmc result directories (FETCH_SIZE and "
                         "WRITE_SIZE of this bench, then of --copy-calibration) into KERNEL's entry "
                         "of profiles/traffic.json")
    args = ap.parse_args()

    if args.write_traffic:
        print(json.dumps(write_traffic(*args.write_traffic)), flush=True)
        return 0

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the hull of one point set runs on one device "
              "(see DESIGN.md for how it would shard); run with --gpus 1", file=sys.stderr)
        return 2

    import torch
    from paper_1501_04706_amd import sqh, workloads

    dev = torch.device("cuda", 0)
    if args.copy_calibration:
        src = torch.empty((args.n, 2), dtype=torch.float32, device=dev).uniform_()
        dst = torch.empty_like(src)
        for _ in range(args.warmup + args.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4,
                          "launches": args.warmup + args.steps}), flush=True)
        return 0
    xy = workloads.make(args.kind, args.n, args.seed)
    xy_d = torch.from_numpy(xy).to(dev)
    H = sqh.Hull(0)
    H.set_precision({"fp32": sqh.SQH_FP32_FILTER, "fp32-semistatic": sqh.SQH_FP32_SEMISTATIC,
                     "fp64": sqh.SQH_FP64_ONLY}[args.precision])
    if args.no_streaming:
        H.set_streaming(False)
    out = torch.empty(max(args.n, 1), dtype=torch.int32, device=dev)
    H.workspace(args.n, 1)

    # every kernel's time from an event pair around each launch (these
    # events cost device time, so these steps are not the timed region)
    mk = timed_calls(H, xy_d, out, args.n, args.steps, args.warmup)
    kernels = kernel_table(mk)
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_call"])
    # the timed region: K calls, HIP events on the launch stream around the
    # dominant kernel's launches only
    m = timed_calls(H, xy_d, out, args.n, args.steps, 2, only=dom)
    ms_step = m["wall_ms"]
    value = args.n / (ms_step / 1000.0) / 1e6
    last = m["last"]
    dk = kernel_table(m)[dom]
    achieved = dk["GB_s"]
    traffic = load_traffic(PROFILER_NAME.get(dom, dom))

    line = {
        "metric": "Mpoints/s + HBM GB/s (20M-pt hull); batched hulls/s & p99 latency vs plain",
        "value": round(value, 2),
        "unit": "Mpoints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"single hull, {args.kind}, n={args.n}, float32, seed {args.seed}",
                   "n": args.n, "kind": args.kind, "seed": args.seed,
                   "precision": args.precision, "streaming": not args.no_streaming},
        "roofline": {
            "bound": "hbm",
            "kernel": dom,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "alg_bytes_per_launch": dk["alg_bytes_per_launch"],
            "avg_launch_ms": dk["avg_launch_ms"],
            "launches": int(m["per"][dom][1]),
        },
        "kernels": {"note": "separate steps with an event pair around every launch", **kernels},
        "detail": {
            "hull_size": int(last["hull_size"]),
            "passes": int(last["passes"]),
            "stream_path": int(last["stream_path"]),
            "line_filter": int(last["line_filter"]),
            "device_ms_per_call": {k[3:]: round(v, 4) for k, v in m["agg"].items()},
            "ms_per_step_with_bookkeeping": round(m["loop_ms"], 4),
            "device_ms_median": round(statistics.median(m["totals"]), 4),
            "device_ms_min": round(min(m["totals"]), 4),
            "call_alg_bytes": call_bytes(last, args.n),
            "call_GB_s": round(call_bytes(last, args.n) / (statistics.median(m["totals"]) / 1000.0) / 1e9, 1),
            "one_read_floor_frac": round(8 * args.n / (ms_step / 1000) / 1e9 / HBM_PEAK_GBS, 4),
            "orient_fallback_rate": (m["exact"] / m["evals"]) if m["evals"] else 0.0,
            "orient_evals_per_call": m["evals"] / args.steps,
            "cmp_exact_per_call": m["cmpx"] / args.steps,
            "pass_points": list(last["pass_points"])[: int(last["passes"])],
            "pass_segments": list(last["pass_segments"])[: int(last["passes"])],
            "pass_ms": [round(v, 4) for v in list(last["pass_ms"])[: int(last["passes"])]],
        },
    }
    if not args.no_extra:
        # cold: 1 GiB of scratch rewritten before each call
        scratch = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        mc = timed_calls(H, xy_d, out, args.n, 10, 2, scratch=scratch, only=dom)
        del scratch
        kc = kernel_table(mc)
        med = statistics.median(mc["totals"])
        line["cold"] = {
            "repetitions": 10,
            "scratch_bytes": 1 << 30,
            "device_ms_median": round(med, 4),
            "device_ms_min": round(min(mc["totals"]), 4),
            "Mpoints_per_s": round(args.n / (med / 1000.0) / 1e6, 1),
            "call_GB_s": round(call_bytes(mc["last"], args.n) / (med / 1000.0) / 1e9, 1),
            "dominant_kernel": {"kernel": dom, **kc.get(dom, {}),
                                "frac": round(kc.get(dom, {}).get("GB_s", 0.0) / HBM_PEAK_GBS, 4)},
        }
        filt = filter_modes(H, sqh, torch, workloads, args.n)
        line["filters"] = filt
        line["config3"] = {k: {"workload": f"{k}, n={args.n}, seed 0", **filt[k]["fp32_filter"]}
                           for k in ("circle", "grid")}
    if args.batch != "none":
        line["batched"] = bench_batched(H, sqh, torch, workloads,
                                        64_000_000 if args.batch == "64M" else None,
                                        steps=3, warmup=1)
    if args.serve > 0:
        line["serving"] = bench_serving(H, sqh, torch, workloads, count=args.serve)
    if not args.no_breakdown:
        line["breakdown"] = bench_breakdown(H, sqh, torch, workloads)
        line["modes"] = modes_at(line["breakdown"], args.kind, args.n)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(xy)
    else:
        line["cpu_baseline"] = None
    H.close()
    del xy_d, out
    torch.cuda.synchronize()
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    rc = main()
    if rc:
        sys.exit(rc)
