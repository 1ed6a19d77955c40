#!/usr/bin/env python3
"""Benchmark of the segmented QuickHull library on one MI355X.

Default workload: one convex hull of n = 20,000,000 float32 points drawn
uniformly in the unit square (seed 0) -- the largest size of the paper's
Table 2 workload. A step is one full sqh_hull call (seed, first split, first
compaction, every segmented pass, table rebuilds, ordered emission) with the
input already resident in device memory; the call returns the hull size to
the host, so each step ends synchronised.

Prints one JSON line:
  value      whole-job throughput in Mpoints/s (n / step time)
  roofline   the dominant kernel's algorithmic HBM bytes per launch divided
             by its average launch time (HIP events recorded by the library
             on the launch stream around every launch, over the timed steps)
             against the 8 TB/s HBM3E peak
  cpu_baseline  the C oracle (monotone chain, exact predicates) timed on
             this host on the same input, single thread
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
KERNEL = "k_hull"      # the persistent kernel that runs the whole hull
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "traffic.json")


def kernel_bytes(st: dict, n: int) -> int:
    """Algorithmic HBM bytes of one hull-kernel launch (one sqh_hull call).

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


def load_traffic(kernel: str):
    """Measured HBM bytes per launch from the committed rocprofv3 counter
    summary, if it was taken for the current kernel build."""
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


def write_traffic(fetch_dir: str, write_dir: str, copy_fetch_dir: str, copy_write_dir: str,
                  copy_bytes: int = 160_000_000) -> dict:
    """HBM bytes per launch of the hull kernel from two counter runs
    (FETCH_SIZE, WRITE_SIZE; KiB per dispatch), each scaled by what the same
    counter reads for a device-to-device copy of copy_bytes in each
    direction; written to profiles/traffic.json with the build's fingerprint."""
    kname = "k_hull"
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
    with open(PROFILE_TRAFFIC, "w") as f:
        json.dump({KERNEL: rec}, f, indent=1)
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


def bench_serving(H, sqh, torch, workloads, count: int = 600, pool: int = 48, max_passes: int = 32,
                  seed: int = 5) -> dict:
    """Poisson stream of hull requests (sizes log-uniform in [1e3, 4e6], kinds
    square/disk/circle) from host memory. The engine (continuous batching)
    against one sqh_hull per request in arrival order (the plain path), both
    timed from arrival to the hull indices in host memory."""
    import numpy as np
    rng = np.random.default_rng(seed)
    sizes = workloads.log_uniform_sizes(rng, pool, 1000, 4_000_000)
    kinds = ("square", "disk", "circle")
    which = rng.integers(0, 3, size=pool)
    child = np.random.SeedSequence(seed).spawn(pool)
    # request payloads live in pinned host memory, as network receive buffers would
    sets = [torch.from_numpy(workloads.make(kinds[which[i]], int(sizes[i]),
                                            int(child[i].generate_state(1)[0]))).pin_memory()
            for i in range(pool)]
    pick = rng.integers(0, pool, size=count)
    dev = torch.device("cuda", 0)

    dev_ms = [0.0]  # device time of the engine's steps

    def run_engine(H_, arrivals):
        # admissions copy on their own stream while the previous step computes
        E = H_.engine(1 << 25, 1024, 1 << 24)
        copy = torch.cuda.Stream()
        dev_ms[0] = 0.0
        try:
            res = {}
            done_t = {}
            t0 = time.perf_counter()
            nxt = 0
            inflight = False
            while len(done_t) < count:
                now = time.perf_counter() - t0
                while nxt < count and arrivals[nxt] <= now and E.admit(sets[pick[nxt]], nxt, stream=copy):
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
                if not inflight and nxt < count:
                    time.sleep(max(0.0, arrivals[nxt] - (time.perf_counter() - t0)))
            wall = max(done_t.values())
            lat = [(done_t[i] - arrivals[i]) * 1000.0 for i in range(count)]
            return wall, lat, res
        finally:
            E.close()

    def run_plain(arrivals):
        out = torch.empty(4_000_000, dtype=torch.int32, device=dev)
        H.workspace(4_000_000, 1)
        t0 = time.perf_counter()
        lat = []
        res = {}
        for i in range(count):
            now = time.perf_counter() - t0
            if arrivals[i] > now:
                time.sleep(arrivals[i] - now)
            xy = sets[pick[i]].to(dev, non_blocking=True)
            hv = H.hull(xy, out=out).cpu().numpy()
            t = time.perf_counter() - t0
            lat.append((t - arrivals[i]) * 1000.0)
            res[i] = hv
        return time.perf_counter() - t0, lat, res

    zero = np.zeros(count)
    run_engine(H, zero)  # warm-up
    runs = []
    for _ in range(3):  # saturated throughput: median of three runs of each path
        wall_e, _, res_e = run_engine(H, zero)
        runs.append((wall_e, dev_ms[0]))
    wall_e, dev_e = sorted(runs)[1]
    T = count / wall_e
    walls_p = []
    for _ in range(3):
        wall_p, _, res_p = run_plain(zero)
        walls_p.append(wall_p)
    wall_p = sorted(walls_p)[1]
    Tp = count / wall_p
    same = all(np.array_equal(res_e[i], res_p[i]) for i in range(count))
    H64 = sqh.Hull(0, precision=sqh.SQH_FP64_ONLY)
    try:
        wall_64, _, res_64 = run_engine(H64, zero)
    finally:
        H64.close()
    same64 = all(np.array_equal(res_e[i], res_64[i]) for i in range(count))
    out = {
        "workload": f"{count} requests drawn from {pool} point sets, sizes log-uniform in [1e3, 4e6], "
                    f"square/disk/circle, seed {seed}, pinned host input, {max_passes} passes per engine step",
        "saturated_hulls_per_s": round(T, 1),
        "saturated_runs": 3,
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
        _, lat_e, _ = run_engine(H, arr)
        _, lat_p, _ = run_plain(arr)
        out[f"qps_{frac}T"] = round(lam, 1)
        out[f"engine_{frac}T"] = _percentiles(lat_e)
        out[f"plain_{frac}T"] = _percentiles(lat_p)
    return out


def release_device(torch) -> None:
    """Reset the HIP device (end of process)."""
    import ctypes
    torch.cuda.synchronize()
    ctypes.CDLL("libamdhip64.so").hipDeviceReset()


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=20_000_000)
    ap.add_argument("--kind", default="square", choices=["square", "disk", "circle", "grid"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"],
                    help="fp32: float32 filter with exact fallback; fp64: every predicate exact")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve", type=int, default=600, help="serving requests (0: skip)")
    ap.add_argument("--no-breakdown", action="store_true",
                    help="skip the per-phase breakdown over sizes and pre-filter modes")
    ap.add_argument("--batch", default="64M", choices=["64M", "full", "none"],
                    help="batched comparison: 4096 sets rescaled to ~64M points, the literal "
                         "log-uniform sizes (~4.4e8 points), or skip it")
    ap.add_argument("--release-device", action="store_true",
                    help="reset the HIP device before exiting (lets a profiler that wraps this "
                         "process write its results before it tears down)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device-to-device copy of the 20M-point input "
                         "(160 MB read + 160 MB written per launch), to scale HBM counters")
    ap.add_argument("--write-traffic", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR",
                                                          "COPY_WRITE_DIR"),
                    help="no GPU work: turn four rocprofv3 --pmc result directories (FETCH_SIZE and "
                         "WRITE_SIZE of this bench, then of --copy-calibration) into "
                         "profiles/traffic.json")
    args = ap.parse_args()

    if args.write_traffic:
        print(json.dumps(write_traffic(*args.write_traffic)), flush=True)
        return 0

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the hull of one point set runs on one device "
              "(see DESIGN.md for how it would shard); run with --gpus 1", file=sys.stderr)
        return 2

    import numpy as np
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
        del src, dst
        if args.release_device:
            release_device(torch)
        return 0
    xy = workloads.make(args.kind, args.n, args.seed)
    xy_d = torch.from_numpy(xy).to(dev)
    H = sqh.Hull(0)
    if args.precision == "fp64":
        H.set_precision(sqh.SQH_FP64_ONLY)
    out = torch.empty(max(args.n, 1), dtype=torch.int32, device=dev)
    H.workspace(args.n, 1)
    for _ in range(args.warmup):
        H.hull(xy_d, out=out)
    torch.cuda.synchronize()

    keys = ("ms_total", "ms_kernel", "ms_seed", "ms_split", "ms_first", "ms_pass", "ms_emit")
    agg = {k: 0.0 for k in keys}
    exact = evals = cmpx = 0
    last = None
    t0 = time.perf_counter()
    for _ in range(args.steps):
        h = H.hull(xy_d, out=out)
        st = H.stats()
        for k in agg:
            agg[k] += st[k]
        evals += st["orient_evals"]
        exact += st["orient_exact"]
        cmpx += st["cmp_exact"]
        last = st
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1000.0 / args.steps
    value = args.n / (ms_step / 1000.0) / 1e6

    nbytes = kernel_bytes(last, args.n)
    avg_launch_ms = agg["ms_kernel"] / args.steps
    achieved = nbytes / (avg_launch_ms / 1000.0) / 1e9
    traffic = load_traffic(KERNEL)

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
                   "precision": args.precision},
        "roofline": {
            "bound": "hbm",
            "kernel": KERNEL,
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "alg_bytes_per_launch": int(nbytes),
            "avg_launch_ms": round(avg_launch_ms, 5),
        },
        "detail": {
            "hull_size": int(last["hull_size"]),
            "passes": int(last["passes"]),
            "ms_per_call": {k[3:]: round(v / args.steps, 4) for k, v in agg.items()},
            "one_read_floor_frac": round(8 * args.n / (ms_step / 1000) / 1e9 / HBM_PEAK_GBS, 4),
            "orient_fallback_rate": (exact / evals) if evals else 0.0,
            "orient_evals_per_call": evals / args.steps,
            "cmp_exact_per_call": cmpx / args.steps,
            "pass_points": list(last["pass_points"])[: int(last["passes"])],
        },
    }
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
    print(json.dumps(line), flush=True)
    if args.release_device:
        release_device(torch)
    return 0


if __name__ == "__main__":
    rc = main()
    if rc:
        sys.exit(rc)
