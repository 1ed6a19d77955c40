"""Build libsqh.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1501_04706_amd.build

The library is one translation unit (csrc/sqh_host.hip includes the kernels).
Flags: -ffp-contract=off keeps every floating-point operation separately
rounded, which the predicate error bounds assume; packed fp32 instructions
are disabled for all device code.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsqh.so")
ARCH = os.environ.get("SQH_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def flags(extra=()):
    return [
        f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
        "-ffp-contract=off", "-fno-fast-math",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-but-set-variable",
        f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}",
        *extra,
    ]


def build(verbose: bool = False, extra=()) -> str:
    src = os.path.join(CSRC, "sqh_host.hip")
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *flags(extra), "-o", tmp, src]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    out = (res.stdout or "") + (res.stderr or "")
    # the host pass does not know the gfx target feature; that note is expected
    lines = [l for l in out.splitlines() if "packed-fp32-ops" not in l and l.strip()]
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + "\n".join(lines))
    if verbose and lines:
        print("\n".join(lines))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
    print(LIB)
