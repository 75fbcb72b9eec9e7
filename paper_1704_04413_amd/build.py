"""Builds librrlbm.so (the HIP C-ABI library) in-tree for gfx950 with hipcc.

The kernels are split over translation units that compile in parallel: the
2D step once per (lattice, storage) pair, the 3D step six times per lattice
(pull, in-place, and in-place with non-temporal stores, for two storages), the
moment representation once per lattice, the batch kernel once per storage,
the closure, and the host-side C-ABI.  Objects go to _build/ next to this
file and are linked into one shared library.
"""
from __future__ import annotations

import os
import re
import subprocess
import sys
import time
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "librrlbm.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]

# (object name, source, defines); the heaviest units first so that the
# parallel build ends soonest
UNITS = (
    [(f"step2d_{lat}_{st}", "step2d.hip", {"RR_LAT": lat, "RR_STORE": st}) for lat in (2, 1, 0) for st in (0, 1, 2, 3)]
    + [(f"step3d_{lat}{('', '_aa', '_aant')[aa]}{'_f32' if st else ''}", "step3d.hip",
        {"RR_LAT3": lat, "RR_AA3": aa, "RR_STORE3": st})
       for lat in (6, 5, 4, 3) for aa in (0, 1, 2) for st in (0, 3)]
    + [("closure", "closure.hip", {})]
    + [(f"batch_{st}", "batch.hip", {"RR_STORE": st}) for st in (0, 1, 2, 3)]
    + [(f"mom_{lat}", "mom.hip", {"RR_LAT": lat}) for lat in (2, 1, 0)]
    + [("api", "api.hip", {})]
)


def _jobs() -> int:
    n = os.environ.get("MAX_JOBS") or os.cpu_count() or 4
    return max(1, min(16, int(n)))


def _deps(src: str) -> set[str]:
    """The source and every project header it includes, transitively."""
    seen, todo = set(), [os.path.join(CSRC, src)]
    while todo:
        path = todo.pop()
        if path in seen or not os.path.exists(path):
            continue
        seen.add(path)
        for line in open(path):
            m = re.match(r'\s*#\s*include\s*"([^"]+)"', line)
            if m:
                todo += [os.path.join(d, m.group(1)) for d in (CSRC, INCLUDE)]
    return seen


def _compile(unit, extra, verbose, incremental):
    name, src, defs = unit
    obj = os.path.join(OBJDIR, name + ".o")
    newest = max(os.path.getmtime(f) for f in _deps(src))
    if incremental and os.path.exists(obj) and os.path.getmtime(obj) >= newest:
        return name, 0.0, False
    cmd = [HIPCC, *FLAGS, *extra, *[f"-D{k}={v}" for k, v in defs.items()], "-I", INCLUDE, "-I", CSRC,
           "-c", "-o", obj + ".tmp", os.path.join(CSRC, src)]
    if verbose:
        print(" ".join(cmd), flush=True)
    t0 = time.time()
    subprocess.run(cmd, check=True)
    os.replace(obj + ".tmp", obj)
    return name, time.time() - t0, True


def build(verbose: bool = False, extra: list[str] | None = None, out: str | None = None,
          incremental: bool = False) -> str:
    """Compile every unit (all of them unless `incremental`, which skips
    objects newer than their source and the headers it includes) and link
    librrlbm.so."""
    os.makedirs(OBJDIR, exist_ok=True)
    extra = list(extra or [])
    t0 = time.time()
    with ThreadPoolExecutor(max_workers=_jobs()) as ex:
        futs = [ex.submit(_compile, u, extra, verbose, incremental) for u in UNITS]
        done = [f.result() for f in futs]
    if verbose:
        for name, dt, built in done:
            if built:
                print(f"  {name}: {dt:.0f} s", flush=True)
    target = out or LIB
    objs = [os.path.join(OBJDIR, u[0] + ".o") for u in UNITS]
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", target + ".tmp", *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(target + ".tmp", target)
    if verbose:
        print(f"built {target} in {time.time() - t0:.0f} s", flush=True)
    return target


if __name__ == "__main__":
    args = sys.argv[1:]
    inc = "--incremental" in args
    build(verbose=True, extra=[a for a in args if a != "--incremental"], incremental=inc)
