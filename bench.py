"""Throughput benchmark of the recursive-regularized LBM step on one MI355X.

Default workload: D2V37, isothermal recursive regularization at the lattice's
full order (N = 4), doubly periodic shear layer on 1024 x 1024 nodes, FP64
populations (the plain form), Re = 1e5, Mach 0.1.  A step is one fused
stream-and-collide launch over the whole grid.

Prints ONE JSON line: MLUPS over the timed steps, the HBM roofline of the
step kernel (algorithmic bytes 2 Q sizeof(f) per node over the kernel's
average duration, from HIP events recorded around every launch on the
library's stream), the CPU oracle timed on a bounded sample of the same
workload, and a per-lattice / per-precision sweep.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 vector
METRIC = "MLUPS and % of HBM roofline per lattice; closure/low-precision vs plain at stated error"
STORAGE_FLAGS = {"fp64": 0, "fp32": 0x2, "bf16": 0x4, "moments": 0x8, "fp32d": 0x2 | 0x400}
STORAGE_BYTES = {"fp64": 8, "fp32": 4, "bf16": 2, "fp32d": 4}


def bytes_per_node(q: int, storage: str, thermal: bool = False) -> int:
    """Algorithmic HBM bytes of one node update: every stored value read once
    and written once (Q populations, or the six FP64 moments; eleven for the
    thermal moment state)."""
    if storage == "moments":
        return 2 * (11 if thermal else 6) * 8
    return 2 * q * STORAGE_BYTES[storage]


def _code_only(text: str) -> str:
    """C/C++ source without comments and with whitespace collapsed (string
    literals are kept as they are; none of the sources holds a comment
    marker inside one)."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash(unit: str = "step2d.hip") -> str:
    """Hash of the code of one kernel unit and the headers it includes (a
    counter summary is valid only while it is unchanged; comments and
    layout do not count)."""
    from paper_1704_04413_amd import build

    h = hashlib.sha256()
    for p in sorted(build._deps(unit)):
        with open(p) as f:
            h.update(os.path.basename(p).encode())
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]


def kernel_unit(storage: str = "fp64", closure: bool = False) -> str:
    """The source unit of the kernel a profile of this storage covers."""
    return "closure.hip" if closure else "mom.hip" if storage == "moments" else "step2d.hip"


def read_profile(name: str, unit: str):
    """The key: value lines of profiles/<name>, or None if the file is missing
    or the kernel's code has changed since it was written."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    return kv if kv.get("kernel_source_hash") == kernel_source_hash(unit) else None


def moment_step_roofline(row):
    """The moment-form step is bound by vector ALU issue, not HBM: its FP64
    rate against the 78.6 TFLOP/s FP64 vector peak, with the VALU busy
    fraction and instruction counts of its rocprofv3 profile (per node, so
    they hold at any grid size)."""
    kv = read_profile("d2v37_moments_2048_valu.txt", "mom.hip")
    if kv is None or row is None:
        return None
    flops = float(kv["fp64_flops_per_node"])
    achieved = row["MLUPS"] * 1e6 * flops / 1e12
    return {"bound": "alu", "lattice": row["lattice"], "n": row["n"], "MLUPS": row["MLUPS"],
            "fp64_flops_per_node": flops, "valu_insts_per_node": float(kv["valu_insts_per_node"]),
            "achieved": round(achieved, 2), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
            "valu_busy_percent_2048": float(kv["valu_busy_percent"]),
            "profile": "profiles/d2v37_moments_2048_valu.txt"}


def read_traffic(name: str):
    """HBM bytes per launch measured by rocprofv3 counters (profiles/<name>),
    valid only if the kernel sources have not changed since."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_hash") != kernel_source_hash("mom.hip" if "_moments_" in name else "step2d.hip"):
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


# ------------------------------------------------------------------ profiles
# Turning rocprofv3 output into the summaries under profiles/ (runs on any
# host, after the profiled runs on the GPU).

PROFILE_RUN = "python3 bench.py --steps 20 --warmup 2 --only-headline"


def _pmc_per_kernel(csv_dir: str, counter: str):
    """{kernel name: [values per dispatch]} of one rocprofv3 --pmc run (csv)."""
    import csv

    out = {}
    for path in glob.glob(os.path.join(csv_dir, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as f:
            for row in csv.DictReader(f):
                if row["Counter_Name"] == counter:
                    out.setdefault(row["Kernel_Name"], []).append(float(row["Counter_Value"]))
    return out


def _busiest(d):
    name = max(d, key=lambda k: len(d[k]))
    return name, float(np.mean(d[name]))


def _step_kernel(d, scheme):
    """(name, mean per dispatch, dispatches) of the step kernel: the busiest
    kernel, or for the single-buffer scheme its two kernels (one per
    placement of the state, alternating) taken together."""
    if scheme == "aa":
        names = sorted(k for k in d if "k_stream_collide_aa" in k)
        vals = [v for k in names for v in d[k]]
        return " + ".join(names), float(np.mean(vals)), len(vals)
    name, mean = _busiest(d)
    return name, mean, len(d[name])


def _scheme_tag(scheme):
    return "_aa" if scheme == "aa" else ""


def _run_flags(args):
    """The bench.py options that select the profiled workload's storage and
    scheme (the moment representation has one scheme)."""
    flag = "" if args.storage == "fp64" else f" --storage {args.storage}"
    return flag if args.storage == "moments" else flag + f" --scheme {args.scheme}"


def summarize_pmc(args) -> str:
    """Writes profiles/<lattice>_<storage>_<n>_traffic.txt from the four PMC runs
    (step FETCH_SIZE, step WRITE_SIZE, copy FETCH_SIZE, copy WRITE_SIZE)."""
    fetch_dir, write_dir, cfetch_dir, cwrite_dir = args.summarize_pmc
    kname, fetch, ndisp = _step_kernel(_pmc_per_kernel(fetch_dir, "FETCH_SIZE"), args.scheme)
    kname2, write, _ = _step_kernel(_pmc_per_kernel(write_dir, "WRITE_SIZE"), args.scheme)
    assert kname == kname2, (kname, kname2)
    cname, cfetch = _busiest(_pmc_per_kernel(cfetch_dir, "FETCH_SIZE"))
    _, cwrite = _busiest(_pmc_per_kernel(cwrite_dir, "WRITE_SIZE"))
    copy_kib = float(1 << 20)  # 1 GiB read and written by the calibration copy
    fs, ws = copy_kib / cfetch, copy_kib / cwrite
    q = {"D2Q9": 9, "D2V17": 17, "D2V37": 37}[args.lattice]
    alg = bytes_per_node(q, args.storage) * args.n * args.n
    alg_formula = ("2*6*8" if args.storage == "moments" else f"2*{q}*{STORAGE_BYTES[args.storage]}") + f"*{args.n}^2"
    rd, wr = fetch * fs * 1024, write * ws * 1024
    name = f"{args.lattice.lower()}_{args.storage}_{args.n}{_scheme_tag(args.scheme)}_traffic.txt"
    flag = _run_flags(args)
    what = "single-buffer in-place (AA)" if args.scheme == "aa" else "pull"
    lines = [
        f"# HBM traffic of the {args.lattice} {args.storage.upper()} {args.n}x{args.n} {what} stream-collide step (rocprofv3 PMC)",
        "#",
        "# Commands (repo root on an MI355X; one counter per run):",
        f"#   rocprofv3 --pmc FETCH_SIZE --output-format csv -d {fetch_dir} -o run -- {PROFILE_RUN} --lattice {args.lattice} --n {args.n}{flag}",
        f"#   rocprofv3 --pmc WRITE_SIZE --output-format csv -d {write_dir} -o run -- {PROFILE_RUN} --lattice {args.lattice} --n {args.n}{flag}",
        f"# Calibration with a device copy of 1 GiB (torch copy_, kernel {cname}):",
        f"#   rocprofv3 --pmc FETCH_SIZE --output-format csv -d {cfetch_dir} -o run -- python3 bench.py --copy-only",
        f"#   rocprofv3 --pmc WRITE_SIZE --output-format csv -d {cwrite_dir} -o run -- python3 bench.py --copy-only",
        f"# Summary: python3 bench.py --lattice {args.lattice} --n {args.n}{flag} --summarize-pmc {fetch_dir} {write_dir} {cfetch_dir} {cwrite_dir}",
        "#",
        f"# copy: FETCH_SIZE {cfetch:.1f} KiB, WRITE_SIZE {cwrite:.1f} KiB per dispatch for {copy_kib:.0f} KiB read and written",
        f"#   -> scale factors fetch {fs:.4f}, write {ws:.4f}",
        f"# step kernel ({ndisp} dispatches): FETCH_SIZE {fetch:.1f} KiB, WRITE_SIZE {write:.1f} KiB per dispatch",
        f"#   -> read {rd / 1e6:.1f} MB, written {wr / 1e6:.1f} MB per launch; algorithmic {alg_formula} = {alg / 1e6:.1f} MB",
        f"#   -> measured / algorithmic = {(rd + wr) / alg:.4f}",
        f"kernel: {kname}",
        f"kernel_source_hash: {kernel_source_hash(kernel_unit(args.storage))}",
        f"fetch_scale: {fs:.6f}",
        f"write_scale: {ws:.6f}",
        f"read_bytes_per_launch: {rd:.0f}",
        f"write_bytes_per_launch: {wr:.0f}",
        f"hbm_bytes_per_launch: {rd + wr:.0f}",
    ]
    path = os.path.join(ROOT, "profiles", name)
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    return path


def summarize_trace(args) -> str:
    """Writes profiles/<lattice>_<storage>_<n>_kernel_trace.md from the rocpd
    database of a --kernel-trace --stats run, plus the live HIP-event timing
    of the bench JSON line printed by the same run."""
    import sqlite3

    db, bench_json = args.summarize_trace
    rows = sqlite3.connect(db).execute(
        "select name, total_calls, total_duration, average, percentage from top_kernels").fetchall()
    line = [ln for ln in open(bench_json) if ln.startswith("{")][-1]
    live = json.loads(line)
    roof = live["roofline"]
    flag = "" if args.only_closure else _run_flags(args)
    mode = "--only-closure" if args.only_closure else "--only-headline"
    what = ("fused closure step" if args.only_closure else
            "single-buffer in-place (AA) stream-collide" if args.scheme == "aa" else "pull stream-collide")
    name = (f"{args.lattice.lower()}_{'closure' if args.only_closure else args.storage}_{args.n}"
            f"{_scheme_tag(args.scheme)}_kernel_trace.md")
    out = [f"# rocprofv3 kernel trace: {args.lattice} {args.storage.upper()} {args.n}x{args.n} shear layer ({what})",
           "", "Command (repo root on an MI355X):", "",
           f"    rocprofv3 --kernel-trace --stats -d gpurun_out/prof -o run -- python3 bench.py --steps {args.steps} "
           f"--warmup {args.warmup} {mode} --lattice {args.lattice} --n {args.n}{flag}",
           "", f"Summary: `python3 bench.py --steps {args.steps} --warmup {args.warmup} --lattice {args.lattice} "
               f"--n {args.n}{flag}{' --only-closure' if args.only_closure else ''} "
               f"--summarize-trace <run_results.db> <bench output>`",
           "", "From the `top_kernels` view of the run's database (durations in microseconds):", "",
           "| kernel | calls | total us | average us | % |", "|---|---|---|---|---|"]
    for n, c, tot, avg, pct in rows:
        out.append(f"| `{n}` | {c} | {tot:.1f} | {avg:.2f} | {pct:.1f} |")
    if args.scheme == "aa":
        aa = [(c, tot) for n, c, tot, avg, pct in rows if "k_stream_collide_aa" in n]
        calls, tot = sum(c for c, _ in aa), sum(t for _, t in aa)
        out += ["", f"The two AA kernels (one per placement of the state, alternating) together: {calls} calls, "
                    f"average {tot / calls:.2f} us per launch (the initial state's collision is one of them)."]
    out += ["", f"Live HIP-event timing of the step kernel inside the same run ({live['steps']} timed steps): "
                f"average {roof['kernel_ms_avg'] * 1e3:.2f} us per launch (events at both ends of the region).",
            "", f"Algorithmic bytes per launch: {roof['bytes_per_launch']} B -> {roof['achieved']:.1f} GB/s = "
                f"{roof['frac'] * 100:.1f}% of the 8 TB/s HBM3E peak.",
            f"kernel_source_hash: {kernel_source_hash(kernel_unit(args.storage, args.only_closure))}"]
    path = os.path.join(ROOT, "profiles", name)
    with open(path, "w") as f:
        f.write("\n".join(out) + "\n")
    return path


def _pmc_sums(csv_dir: str, kernel_hint: str, scheme: str = "pull"):
    """{counter: mean value per dispatch} for the busiest kernel whose name
    contains kernel_hint (for the single-buffer scheme: its two step kernels
    together), from one rocprofv3 --pmc csv run."""
    import csv

    per = {}
    for path in glob.glob(os.path.join(csv_dir, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as f:
            for row in csv.DictReader(f):
                if kernel_hint in row["Kernel_Name"]:
                    per.setdefault((row["Kernel_Name"], row["Counter_Name"]), []).append(float(row["Counter_Value"]))
    if not per:
        raise SystemExit(f"no dispatch of a kernel matching {kernel_hint!r} in {csv_dir}")
    if scheme == "aa":
        names = sorted({k for k, _ in per if "k_stream_collide_aa" in k})
        merged = {}
        for (k, c), v in per.items():
            if k in names:
                merged.setdefault(c, []).extend(v)
        return " + ".join(names), {c: float(np.mean(v)) for c, v in merged.items()}
    kname = max({k for k, _ in per}, key=lambda k: sum(len(v) for (kk, _), v in per.items() if kk == k))
    return kname, {c: float(np.mean(v)) for (k, c), v in per.items() if k == kname}


def summarize_pmc3d(args) -> str:
    """HBM traffic of the 3D step kernels of one lattice at 128^3 under the
    default policy and under RRLBM_CACHE_POLICY=1 (ordinary stores for the
    single-buffer step), from FETCH_SIZE / WRITE_SIZE runs of `bench.py
    --only-3d <lattice>:RR` scaled by the same counters of a 1 GiB device copy
    (profiles/<lattice>_128_traffic.txt)."""
    lat = args.lattice3d
    fd, wd, fd1, wd1, fc, wc = args.summarize_pmc3d
    q = {"D3Q19": 19, "D3Q27": 27, "D3V39": 39, "D3Q103": 103}[lat]
    n = 128
    _, cf = _busiest(_pmc_per_kernel(fc, "FETCH_SIZE"))
    _, cw = _busiest(_pmc_per_kernel(wc, "WRITE_SIZE"))
    copy_kib = float(1 << 20)  # 1 GiB read and written by the calibration copy
    fs, ws = copy_kib / cf, copy_kib / cw
    run = f"python3 bench.py --only-3d {lat}:RR --steps 30 --warmup 3 --n3 {n}"
    out = [f"# HBM traffic of the {lat} 3D step kernels at {n}^3 (rocprofv3 PMC), default policy and policy 1",
           "#", "# Commands (repo root on an MI355X; one counter per run):"]
    for tag, pre in (("", ""), ("1", "RRLBM_CACHE_POLICY=1 ")):
        for c, d in (("FETCH_SIZE", "f"), ("WRITE_SIZE", "w")):
            out.append(f"#   {pre}rocprofv3 --pmc {c} --output-format csv -d gpurun_out/prof/{d}3_{lat}{tag} -o run -- {run}")
    out += ["# Calibration with a device copy of 1 GiB (torch copy_):",
            "#   rocprofv3 --pmc FETCH_SIZE --output-format csv -d gpurun_out/prof/fcopy -o run -- python3 bench.py --copy-only",
            "#   rocprofv3 --pmc WRITE_SIZE --output-format csv -d gpurun_out/prof/wcopy -o run -- python3 bench.py --copy-only",
            f"# Summary: python3 bench.py --lattice3d {lat} --summarize-pmc3d <the six csv dirs in that order>",
            f"# scale factors: fetch {fs:.4f}, write {ws:.4f}",
            "# algorithmic bytes per launch: 2 Q E n^3 (E = 8 for FP64, 4 for FP32 storage)", "#",
            "policy  kernel  dispatches  read_MB  written_MB  measured/algorithmic"]
    for tag, (fdir, wdir) in (("default", (fd, wd)), ("1", (fd1, wd1))):
        f, w = _pmc_per_kernel(fdir, "FETCH_SIZE"), _pmc_per_kernel(wdir, "WRITE_SIZE")
        for k in sorted(k for k in f if "k_stream_collide3" in k and k in w):
            e = 4 if "StoreF32D" in k else 8
            alg = 2 * q * e * n ** 3
            rd, wr = float(np.mean(f[k])) * 1024 * fs, float(np.mean(w[k])) * 1024 * ws
            short = k.split("(")[0].replace("void rr::", "").replace("rr::", "")
            out.append(f"{tag}  {short}  {len(f[k])}  {rd / 1e6:.1f}  {wr / 1e6:.1f}  {(rd + wr) / alg:.4f}")
    out.append(f"kernel_source_hash: {kernel_source_hash('step3d.hip')}")
    path = os.path.join(ROOT, "profiles", f"{lat.lower()}_128_traffic.txt")
    with open(path, "w") as fh:
        fh.write("\n".join(out) + "\n")
    return path


def summarize_requests(args) -> str:
    """Cross-check of the FETCH_SIZE / WRITE_SIZE calibration with request
    counters: bytes = 128 R128 + 64 R64 + 32 R32 for reads and 64 W64 +
    32 (W - W64) for writes, for the step kernel and for a 1 GiB device copy
    (profiles/<lattice>_<storage>_<n>_requests.txt)."""
    rd_dir, wr_dir, crd_dir, cwr_dir = args.summarize_requests
    kname, rd = _pmc_sums(rd_dir, "k_stream_collide", args.scheme)
    _, wr = _pmc_sums(wr_dir, "k_stream_collide", args.scheme)
    cname, crd = _pmc_sums(crd_dir, "")
    _, cwr = _pmc_sums(cwr_dir, "")

    def rbytes(d):
        return 128 * d["TCC_EA0_RDREQ_128B_sum"] + 64 * d["TCC_EA0_RDREQ_64B_sum"] + 32 * d["TCC_EA0_RDREQ_32B_sum"]

    def wbytes(d):
        return 64 * d["TCC_EA0_WRREQ_64B_sum"] + 32 * (d["TCC_EA0_WRREQ_sum"] - d["TCC_EA0_WRREQ_64B_sum"])

    q = {"D2Q9": 9, "D2V17": 17, "D2V37": 37}[args.lattice]
    alg = bytes_per_node(q, args.storage) * args.n * args.n
    gib = float(1 << 30)
    flag = _run_flags(args)
    rdc = "TCC_EA0_RDREQ_sum TCC_EA0_RDREQ_128B_sum TCC_EA0_RDREQ_64B_sum TCC_EA0_RDREQ_32B_sum"
    wrc = "TCC_EA0_WRREQ_sum TCC_EA0_WRREQ_64B_sum"
    lines = [
        f"# Request-counter cross-check of HBM traffic: {args.lattice} {args.storage.upper()} {args.n}x{args.n} step",
        "#",
        "# Commands (repo root on an MI355X):",
        f"#   rocprofv3 --pmc {rdc} --output-format csv -d {rd_dir} -o run -- {PROFILE_RUN} --lattice {args.lattice} --n {args.n}{flag}",
        f"#   rocprofv3 --pmc {wrc} --output-format csv -d {wr_dir} -o run -- {PROFILE_RUN} --lattice {args.lattice} --n {args.n}{flag}",
        f"#   the same two with -- python3 bench.py --copy-only (dirs {crd_dir}, {cwr_dir})",
        f"# Summary: python3 bench.py --lattice {args.lattice} --n {args.n}{flag} --summarize-requests {rd_dir} {wr_dir} {crd_dir} {cwr_dir}",
        "#",
        f"# copy kernel {cname[:60]}: reads 128B/64B/32B = {crd['TCC_EA0_RDREQ_128B_sum']:.0f}/{crd['TCC_EA0_RDREQ_64B_sum']:.0f}/"
        f"{crd['TCC_EA0_RDREQ_32B_sum']:.0f} of {crd['TCC_EA0_RDREQ_sum']:.0f} requests -> {rbytes(crd) / gib:.4f} GiB read (1 GiB copied)",
        f"#   writes 64B {cwr['TCC_EA0_WRREQ_64B_sum']:.0f} of {cwr['TCC_EA0_WRREQ_sum']:.0f} -> {wbytes(cwr) / gib:.4f} GiB written",
        f"# step kernel: reads 128B/64B/32B = {rd['TCC_EA0_RDREQ_128B_sum']:.0f}/{rd['TCC_EA0_RDREQ_64B_sum']:.0f}/"
        f"{rd['TCC_EA0_RDREQ_32B_sum']:.0f} of {rd['TCC_EA0_RDREQ_sum']:.0f} requests -> {rbytes(rd) / 1e6:.1f} MB read",
        f"#   writes 64B {wr['TCC_EA0_WRREQ_64B_sum']:.0f} of {wr['TCC_EA0_WRREQ_sum']:.0f} -> {wbytes(wr) / 1e6:.1f} MB written",
        f"#   -> measured / algorithmic ({alg / 1e6:.1f} MB) = {(rbytes(rd) + wbytes(wr)) / alg:.4f}",
        f"kernel: {kname}",
        f"kernel_source_hash: {kernel_source_hash()}",
        f"copy_read_over_true: {rbytes(crd) / gib:.6f}",
        f"copy_write_over_true: {wbytes(cwr) / gib:.6f}",
        f"read_bytes_per_launch: {rbytes(rd):.0f}",
        f"write_bytes_per_launch: {wbytes(wr):.0f}",
        f"hbm_bytes_per_launch: {rbytes(rd) + wbytes(wr):.0f}",
    ]
    path = os.path.join(ROOT, "profiles",
                        f"{args.lattice.lower()}_{args.storage}_{args.n}{_scheme_tag(args.scheme)}_requests.txt")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    return path


CLOSURE_COUNTERS = ("SQ_INSTS_VALU SQ_ACTIVE_INST_VALU SQ_INSTS_VALU_TRANS_F32 SQ_INSTS_MFMA SQ_VALU_MFMA_BUSY_CYCLES "
                    "SQ_WAVE_CYCLES SQ_WAIT_INST_ANY SQ_BUSY_CYCLES GRBM_GUI_ACTIVE")


def summarize_closure_pmc(args) -> str:
    """Instruction mix of the fused closure step against the plain step of
    the same grid from two rocprofv3 --pmc runs with the same counters
    (profiles/d2v37_closure_<n>_counters.txt)."""
    cdir, pdir = args.summarize_closure_pmc
    nodes = args.n * args.n
    cus, xccs = 256, 8
    rows = []
    for label, d_, hint in (("closure", cdir, "k_stream_collide_closure"), ("plain", pdir, "k_stream_collide<")):
        kname, d = _pmc_sums(d_, hint)
        cyc = d["GRBM_GUI_ACTIVE"] / xccs
        rows.append((label, kname, {
            "valu_insts_per_node": d["SQ_INSTS_VALU"] * 64 / nodes,
            "transcendental_insts_per_node": d["SQ_INSTS_VALU_TRANS_F32"] * 64 / nodes,
            "mfma_insts_per_wave_of_64_nodes": d["SQ_INSTS_MFMA"] * 64 / nodes,
            "valu_busy_percent": 100.0 * d["SQ_ACTIVE_INST_VALU"] / cus / cyc,
            "mfma_busy_percent": 100.0 * d["SQ_VALU_MFMA_BUSY_CYCLES"] / cus / cyc / 4,
            "wait_inst_any_percent_of_wave_cycles": 100.0 * d["SQ_WAIT_INST_ANY"] / d["SQ_WAVE_CYCLES"],
            "gpu_cycles_per_xcc": cyc,
        }))
    lines = [f"# Fused closure step against the plain step: D2V37 FP64 {args.n}x{args.n} (rocprofv3 PMC)", "#",
             "# Commands (repo root on an MI355X):",
             f"#   rocprofv3 --pmc {CLOSURE_COUNTERS} --output-format csv -d {cdir} -o run -- python3 bench.py "
             f"--steps 20 --warmup 2 --only-closure --lattice D2V37 --n {args.n}",
             f"#   rocprofv3 --pmc {CLOSURE_COUNTERS} --output-format csv -d {pdir} -o run -- {PROFILE_RUN} "
             f"--lattice D2V37 --n {args.n} --scheme pull",
             f"# Summary: python3 bench.py --n {args.n} --summarize-closure-pmc {cdir} {pdir}",
             "# Per node in the lane view (one lane per node); busy fractions over the kernel's GPU cycles.",
             "# MFMA busy: SQ_VALU_MFMA_BUSY_CYCLES / 256 CUs / 4 SIMDs per kernel cycle."]
    for label, kname, v in rows:
        lines.append(f"{label}.kernel: {kname}")
        lines += [f"{label}.{k}: {x:.1f}" for k, x in v.items()]
    lines.append(f"kernel_source_hash: {kernel_source_hash('closure.hip')}")
    path = os.path.join(ROOT, "profiles", f"d2v37_closure_{args.n}_counters.txt")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    return path


def summarize_valu(args) -> str:
    """VALU instruction mix and busy fraction of the step kernel from one
    rocprofv3 --pmc run (profiles/<lattice>_<storage>_<n>_valu.txt)."""
    (vdir,) = args.summarize_valu
    kname, d = _pmc_sums(vdir, "k_mom_step" if args.storage == "moments" else "k_stream_collide", args.scheme)
    nodes = args.n * args.n
    f64 = d["SQ_INSTS_VALU_FMA_F64"] + d["SQ_INSTS_VALU_MUL_F64"] + d["SQ_INSTS_VALU_ADD_F64"]
    flops = 64 * (2 * d["SQ_INSTS_VALU_FMA_F64"] + d["SQ_INSTS_VALU_MUL_F64"] + d["SQ_INSTS_VALU_ADD_F64"])
    cus, xccs = 256, 8
    # SQ_ACTIVE_INST_VALU counts quad-cycles summed over every SIMD; GRBM_GUI_ACTIVE
    # comes summed over the 8 XCCs: per XCC (the kernel's duration in cycles) is 1/8
    busy = 100.0 * d["SQ_ACTIVE_INST_VALU"] / cus / (d["GRBM_GUI_ACTIVE"] / xccs)
    counters = "SQ_INSTS_VALU SQ_INSTS_VALU_FMA_F64 SQ_INSTS_VALU_MUL_F64 SQ_INSTS_VALU_ADD_F64 SQ_ACTIVE_INST_VALU GRBM_GUI_ACTIVE"
    flag = _run_flags(args)
    lines = [
        f"# VALU profile: {args.lattice} {args.storage} {args.n}x{args.n} step (rocprofv3 PMC)",
        "#",
        f"#   rocprofv3 --pmc {counters} --output-format csv -d {vdir} -o run -- {PROFILE_RUN} --lattice {args.lattice} --n {args.n}{flag}",
        f"# Summary: python3 bench.py --lattice {args.lattice} --n {args.n}{flag} --summarize-valu {vdir}",
        "#",
        f"# per node: {d['SQ_INSTS_VALU'] * 64 / nodes:.0f} VALU instructions (lane view), of which FP64 "
        f"{f64 * 64 / nodes:.0f} (FMA {d['SQ_INSTS_VALU_FMA_F64'] * 64 / nodes:.0f}); {flops / nodes:.0f} FP64 flops",
        f"# VALUBusy = 100 SQ_ACTIVE_INST_VALU / {cus} CUs / (GRBM_GUI_ACTIVE / {xccs} XCCs) = {busy:.1f}%",
        f"kernel: {kname}",
        f"kernel_source_hash: {kernel_source_hash(kernel_unit(args.storage))}",
        f"valu_insts_per_node: {d['SQ_INSTS_VALU'] * 64 / nodes:.1f}",
        f"fp64_flops_per_node: {flops / nodes:.1f}",
        f"valu_busy_percent: {busy:.2f}",
    ]
    path = os.path.join(ROOT, "profiles",
                        f"{args.lattice.lower()}_{args.storage}_{args.n}{_scheme_tag(args.scheme)}_valu.txt")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    return path


def summarize_trace3d(args) -> str:
    """Writes profiles/lattices3d_<n>_kernel_trace.md from the rocpd database of
    a --kernel-trace --stats run of `bench.py --only-3d all` and that run's
    JSON line (live HIP-event timing of each case)."""
    import sqlite3

    db, bench_json = args.summarize_trace3d
    rows = sqlite3.connect(db).execute(
        "select name, total_calls, total_duration, average, percentage from top_kernels").fetchall()
    line = [ln for ln in open(bench_json) if ln.startswith("{")][-1]
    cases = json.loads(line)["lattices_3d"]
    n = cases[0]["n"]
    cmd = (f"rocprofv3 --kernel-trace --stats -d gpurun_out/prof3d -o run -- python3 bench.py --only-3d all "
           f"--steps {args.steps} --warmup {args.warmup} --n3 {n}")
    out = [f"# rocprofv3 kernel trace: 3D lattices (Table II), {n}^3 extruded shear layer, FP64", "",
           "Command (repo root on an MI355X):", "", f"    {cmd}", "",
           f"Summary: `python3 bench.py --summarize-trace3d <run_results.db> <bench output>`", "",
           "From the `top_kernels` view (durations in microseconds; the pull step of each lattice and "
           "collision is one template instance, `k_stream_collide3<L, MODE, POL>` with MODE 0 RR, 2 BGK; the "
           "single-buffer step two, `k_stream_collide3_aa<L, MODE, SHIFTED, NT>`, alternating):", "",
           "| kernel | calls | total us | average us | % |", "|---|---|---|---|---|"]
    for name, c, tot, avg, pct in rows:
        out.append(f"| `{name[:110]}` | {c} | {tot:.1f} | {avg:.2f} | {pct:.1f} |")
    out += ["", "Live HIP-event timing inside the same run (average step-kernel duration, algorithmic "
                "bytes 2 Q 8 per node, fraction of the 8 TB/s HBM3E peak), pull step and single-buffer step:", "",
            "| lattice | collision | pull us per step | GB/s | % of peak | AA us per step | GB/s | % of peak |",
            "|---|---|---|---|---|---|---|---|"]
    for r in cases:
        out.append(f"| {r['lattice']} | {r['collision']} | {r['kernel_ms_avg'] * 1e3:.1f} | {r['kernel_GBs']:.0f} | "
                   f"{r['frac_hbm'] * 100:.1f} | {r['aa_kernel_ms_avg'] * 1e3:.1f} | {r['aa_kernel_GBs']:.0f} | "
                   f"{r['aa_frac_hbm'] * 100:.1f} |")
    f32 = [r for r in cases if "fp32_kernel_ms_avg" in r]
    if f32:
        out += ["", "FP32 storage with FP64 arithmetic (algorithmic bytes 2 Q 4 per node), same run:", "",
                "| lattice | collision | pull us per step | GB/s | % of peak | AA us per step | GB/s | % of peak |",
                "|---|---|---|---|---|---|---|---|"]
        for r in f32:
            out.append(f"| {r['lattice']} | {r['collision']} | {r['fp32_kernel_ms_avg'] * 1e3:.1f} | "
                       f"{r['fp32_kernel_GBs']:.0f} | {r['fp32_frac_hbm'] * 100:.1f} | "
                       f"{r['fp32_aa_kernel_ms_avg'] * 1e3:.1f} | {r['fp32_aa_kernel_GBs']:.0f} | "
                       f"{r['fp32_aa_frac_hbm'] * 100:.1f} |")
    out += ["", f"kernel_source_hash: {kernel_source_hash('step3d.hip')}"]
    path = os.path.join(ROOT, "profiles", f"lattices3d_{n}_kernel_trace.md")
    with open(path, "w") as f:
        f.write("\n".join(out) + "\n")
    return path


def summarize_trace_batch(args) -> str:
    """Writes profiles/batch64_<storage>_kernel_trace.md from the rocpd
    database of a --kernel-trace --stats run of `bench.py --only-batch` and
    that run's JSON line.  The timed steps are the last `steps` dispatches of each persistent
    batch kernel of the chosen tile shape (the autotuner's trials come before
    them)."""
    import sqlite3

    db, bench_json = args.summarize_trace_batch
    con = sqlite3.connect(db)
    rows = con.execute("select name, total_calls, total_duration, average, percentage from top_kernels").fetchall()
    line = [ln for ln in open(bench_json) if ln.startswith("{")][-1]
    live = json.loads(line)["batched"]
    k = live["steps"]
    disp = con.execute("select name, duration, grid_x, workgroup_x, workgroup_y, vgpr_count, accum_vgpr_count, "
                       "sgpr_count, scratch_size from kernels where name like '%k_batch<%' order by start").fetchall()
    # the timed launches use the chosen tile's kernels: one-row (WIDE) ones for tiles of 256 and more
    wide = live["tile_x"] >= 256
    names = sorted({d[0] for d in disp if (", true>" in d[0]) == wide})
    st = live["storage"]
    cmd = (f"rocprofv3 --kernel-trace --stats -d gpurun_out/profb{'' if st == 'fp32' else '_' + st} -o run -- "
           f"python3 bench.py --only-batch{'' if st == 'fp32' else ' --batch-storage ' + st} --steps {k}")
    out = [f"# rocprofv3 kernel trace: batch of {live['workload']}", "",
           "Command (repo root on an MI355X):", "", f"    {cmd}", "",
           "Summary: `python3 bench.py --summarize-trace-batch <run_results.db> <bench output>`", "",
           "From the `top_kernels` view (durations in microseconds; the run also times one launch per instance "
           "per step, and the autotuner's trials):", "",
           "| kernel | calls | total us | average us | % |", "|---|---|---|---|---|"]
    for name, c, tot, avg, pct in rows[:12]:
        out.append(f"| `{name[:110]}` | {c} | {tot:.1f} | {avg:.2f} | {pct:.1f} |")
    out += ["", f"Timed region: the last {k} dispatches of each batch kernel (tile_x {live['tile_x']}, "
                f"{live['blocks_per_cu']} blocks per CU after autotuning):", "",
            "| kernel | grid | block | VGPR | AGPR | SGPR | scratch | average us |", "|---|---|---|---|---|---|---|---|"]
    total_us = 0.0
    for nm in names:
        last = [d for d in disp if d[0] == nm][-k:]
        avg = float(np.mean([d[1] for d in last])) / 1e3
        total_us += avg
        d = last[-1]
        out.append(f"| `{nm[:80]}` | {d[2]} | {d[3]}x{d[4]} | {d[5]} | {d[6]} | {d[7]} | {d[8]} | {avg:.2f} |")
    nbytes = live["bytes_per_step"]
    out += ["", f"Algorithmic bytes per step (every member: 2 Q bytes-per-value per node): {nbytes} B.",
            f"Kernel time per step {total_us:.2f} us -> {nbytes / (total_us * 1e-6) / 1e9:.1f} GB/s = "
            f"{nbytes / (total_us * 1e-6) / 1e9 / HBM_PEAK_GBS * 100:.1f}% of the 8 TB/s HBM3E peak.",
            f"Live HIP-event timing of the replayed graph in the same run: {live['batched_ms_per_step'] * 1e3:.2f} us "
            f"per step ({live['batched_MLUPS']} MLUPS, {live['batched_frac_hbm'] * 100:.1f}% of peak).",
            f"kernel_source_hash: {kernel_source_hash('batch.hip')}"]
    path = os.path.join(ROOT, "profiles", f"batch64_{st}_kernel_trace.md")
    with open(path, "w") as f:
        f.write("\n".join(out) + "\n")
    return path


def make_sim(b, wl, lattice, n, storage, re=1e5, thermal=False, seed=0, noise=True, coll=0, scheme="pull"):
    """The shear-layer workload (noise=False skips the 1e-8 w_i noise, which
    changes nothing in the timing of a large grid); scheme "aa": one buffer,
    in-place steps."""
    q, reach, n_eq, cs2 = b.lbm_lattice_info(lattice)
    u0, tau = wl.shear_layer_params(cs2, n, re)
    rho, ux, uy = wl.shear_layer_fields(n, n, u0)
    flags = STORAGE_FLAGS[storage] | (b.LBM_THERMAL if thermal else 0) | coll
    flags |= b.LBM_SCHEME_AA if scheme == "aa" else 0
    theta = np.ones_like(rho) if thermal else None
    nz = wl.uniform_noise(seed, q, n, n) if noise else None
    sim = b.Simulation(lattice, n, n, tau, rho, ux, uy, theta=theta, noise=nz, noise_amp=1e-8 if noise else 0.0,
                       flags=flags)
    return sim, dict(q=q, tau=tau, u0=u0, rho=rho, ux=ux, uy=uy, noise=nz)


def make_sim3(b, wl, lattice, n, re=1e5, flags=0, seed=0):
    """The shear layer extruded along z (with a z perturbation) on an n^3
    periodic box, FP64 populations."""
    q, reach, n_eq, cs2 = b.lbm_lattice_info(lattice)
    u0, tau = wl.shear_layer_params(cs2, n, re)
    rho, ux, uy, uz = wl.shear_layer_fields_3d(n, n, n, u0)
    sim = b.Simulation3D(lattice, n, n, n, tau, rho, ux, uy, uz, flags=flags)
    return sim, dict(q=q, tau=tau, u0=u0)


LATTICES_3D = [("D3Q19", "RR"), ("D3Q19", "BGK"), ("D3Q27", "RR"), ("D3V39", "RR"), ("D3Q103", "RR")]


def suite_3d(torch, b, wl, n=128, steps=30, warmup=3, only=None):
    rows = []
    for lat, coll in LATTICES_3D:
        if only is not None and (lat, coll) != only:
            continue
        flags = b.LBM_COLL_BGK if coll == "BGK" else 0
        nodes = n ** 3
        row = {"lattice": lat, "collision": coll, "n": n,
               "order": b.lbm_lattice_info(lat)[2] if coll == "RR" else None}
        # the pull step, then the single-buffer step on the same workload, in
        # FP64 and (RR) in FP32 storage with FP64 arithmetic
        f32 = b.LBM_STORE_FP32 | b.LBM_MATH_FP64
        runs = [("", flags, "fp64"), ("aa_", flags | b.LBM_SCHEME_AA, "fp64")]
        if coll == "RR":
            runs += [("fp32_", f32, "fp32d"), ("fp32_aa_", f32 | b.LBM_SCHEME_AA, "fp32d")]
        for tag, fl, st in runs:
            sim, meta = make_sim3(b, wl, lat, n, flags=fl)
            wall, kms = time_steps(torch, sim, steps, warmup)
            bad = int(sim.moments()["sums"][7])
            sim.close()
            gbs = bytes_per_node(meta["q"], st) * nodes / (kms * 1e-3) / 1e9
            row.update({f"{tag}MLUPS": round(nodes * steps / wall / 1e6, 1), f"{tag}kernel_ms_avg": round(kms, 4),
                        f"{tag}kernel_GBs": round(gbs, 1), f"{tag}frac_hbm": round(gbs / HBM_PEAK_GBS, 4),
                        f"{tag}nonfinite": bad})
        row["aa_over_pull"] = round(row["aa_MLUPS"] / row["MLUPS"], 3)
        rows.append(row)
    return rows


def time_steps(torch, sim, steps, warmup):
    """Wall time of the timed region (bracketed by synchronizations) and the
    average launch duration: HIP events recorded on the library's stream at
    both ends of the region, divided by the number of launches (one launch
    per step; events between launches would add their own gaps)."""
    sim.step(warmup)
    torch.cuda.synchronize()
    stream = sim.stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return t1 - t0, e0.elapsed_time(e1) / steps


def time_regions(torch, sim, steps, regions=5):
    """Average launch duration (ms) of each of `regions` timed regions of
    `steps` launches (HIP events at both ends of each region, on the
    library's stream); the state keeps evolving between regions."""
    stream = sim.stream
    out = []
    for _ in range(regions):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        sim.step(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        out.append(e0.elapsed_time(e1) / steps)
    return out


def roofline_point(torch, b, wl, lattice, n, storage, steps=100, regions=5, thermal=False, coll=0, scheme="pull"):
    """Median-of-regions step time of one workload and its fraction of the
    8 TB/s HBM peak (algorithmic bytes 2 Q sizeof per node)."""
    sim, meta = make_sim(b, wl, lattice, n, storage, thermal=thermal, noise=False, coll=coll, scheme=scheme)
    sim.step(5)
    ms = time_regions(torch, sim, steps, regions)
    bad = int(sim.moments(vorticity=False)["sums"][8])
    sim.close()
    med = float(np.median(ms))
    bpl = bytes_per_node(meta["q"], storage, thermal) * n * n
    gbs = bpl / (med * 1e-3) / 1e9
    buf = bpl // 2
    return {"lattice": lattice, "storage": storage, "thermal": thermal,
            "collision": {0: "RR", 0x10: "PR", 0x20: "BGK"}[coll], "scheme": scheme, "n": n,
            "buffer_MiB": round(buf / 2 ** 20, 1), "MLUPS": round(n * n / (med * 1e-3) / 1e6, 1),
            "kernel_ms_median": round(med, 5), "kernel_ms_regions": [round(x, 5) for x in ms],
            "kernel_GBs": round(gbs, 1), "frac_hbm": round(gbs / HBM_PEAK_GBS, 4), "nonfinite": bad}


# Sizes where one state buffer fits the 256 MiB memory-side cache but two do
# not (the band the single-buffer scheme is for), and two above it.
AA_CASES = [("D2V37", 768, "fp64"), ("D2V17", 1024, "fp64"), ("D2V37", 1024, "fp32"), ("D2Q9", 2048, "fp64"),
            ("D2V37", 1024, "fp64"), ("D2V37", 2048, "fp64")]


def aa_suite(torch, b, wl, steps=50):
    """The pull step against the single-buffer (AA) step on the same workload
    (an even number of steps per timed region, so both AA kernels count
    alike); frac_hbm is algorithmic bytes per second over the HBM peak."""
    rows = []
    for lat, n, st in AA_CASES:
        pull = roofline_point(torch, b, wl, lat, n, st, steps=steps)
        aa = roofline_point(torch, b, wl, lat, n, st, steps=steps, scheme="aa")
        rows.append({"lattice": lat, "n": n, "storage": st, "buffer_MiB": aa["buffer_MiB"],
                     "pull_MLUPS": pull["MLUPS"], "aa_MLUPS": aa["MLUPS"], "pull_frac_hbm": pull["frac_hbm"],
                     "aa_frac_hbm": aa["frac_hbm"], "aa_over_pull": round(aa["MLUPS"] / pull["MLUPS"], 3),
                     "nonfinite": pull["nonfinite"] + aa["nonfinite"]})
    return rows


def copy_bandwidth(torch, nbytes=1 << 30, reps=20):
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        b.copy_(a)
    e.record()
    torch.cuda.synchronize()
    return 2.0 * nbytes * reps / (s.elapsed_time(e) * 1e-3) / 1e9


def batched_suite(torch, b, wl, storage="fp32", steps=40):
    """All instances advanced by one autotuned, graph-replayed persistent
    launch per step, against one launch per instance per step."""
    inst = wl.batch_instances()
    sims, nodes, nbytes = [], 0, 0
    for lat, n, re in inst:
        q, _, _, cs2 = b.lbm_lattice_info(lat)
        u0, tau = wl.shear_layer_params(cs2, n, re)
        rho, ux, uy = wl.shear_layer_fields(n, n, u0)
        sims.append(b.Simulation(lat, n, n, tau, rho, ux, uy, flags=STORAGE_FLAGS[storage]))
        nodes += n * n
        nbytes += 2 * q * STORAGE_BYTES[storage] * n * n
    torch.cuda.synchronize()
    stream = sims[0].stream

    def timed(fn, k):
        fn(2)
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record(stream)
        fn(k)
        e.record(stream)
        torch.cuda.synchronize()
        return s.elapsed_time(e) * 1e-3

    def per_instance(k):
        for _ in range(k):
            for sim in sims:
                sim.step(1)

    t_sep = timed(per_instance, steps)
    batch = b.lbm_batch_create([s.ctx for s in sims], 64, 4)
    tune = b.lbm_batch_autotune(batch, 6)
    t_bat = timed(lambda k: b.lbm_batch_step(batch, k), steps)
    cfg = b.lbm_batch_config(batch)
    b.lbm_batch_destroy(batch)
    bad = 0
    for sim in sims:
        bad += int(sim.moments(vorticity=False)["sums"][8])
        sim.close()
    mix = {l: sum(1 for x in inst if x[0] == l) for l in ("D2Q9", "D2V17", "D2V37")}
    return {
        "workload": f"{len(inst)} shear-layer instances, sides 128..1024, lattices {mix}, Re 1e4..1e6, "
                    f"{storage} shifted storage" + (" (FP64 arithmetic)" if storage == "fp32d" else ""),
        "storage": storage, "nodes": nodes, "bytes_per_step": nbytes, "steps": steps,
        "batched_MLUPS": round(nodes * steps / t_bat / 1e6, 1),
        "batched_ms_per_step": round(t_bat / steps * 1e3, 5),
        "batched_GBs": round(nbytes * steps / t_bat / 1e9, 1),
        "batched_frac_hbm": round(nbytes * steps / t_bat / 1e9 / HBM_PEAK_GBS, 4),
        "per_instance_MLUPS": round(nodes * steps / t_sep / 1e6, 1),
        "per_instance_GBs": round(nbytes * steps / t_sep / 1e9, 1),
        "tile_x": cfg[0], "blocks_per_cu": cfg[1],
        "autotune": [list(r) for r in tune],
        "nonfinite_nodes": bad,
    }


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(wl, lattice_name, n, steps, seed=0):
    import oracle as orc

    lat = orc.lattice(lattice_name)
    u0, tau = wl.shear_layer_params(lat.cs2, n, 1e5)
    rho, ux, uy = wl.shear_layer_fields(n, n, u0)
    noise = wl.uniform_noise(seed, lat.Q, n, n)
    f = orc.init_populations(lat, rho, ux, uy, None, noise, 1e-8)
    t0 = time.perf_counter()
    orc.step(lat, f, tau, steps)
    dt = time.perf_counter() - t0
    return n * n * steps / dt / 1e6, dt, orc.threads()


def cpu_baseline(wl, lattice_name, n, steps, steps_1t=2, seed=0):
    """The oracle as it stands, timed on the host cores on `steps` steps of
    the full grid (MLUPS), and on one thread (a child process with
    OMP_NUM_THREADS=1) on `steps_1t` steps."""
    import subprocess

    mlups, dt, threads = _oracle_rate(wl, lattice_name, n, steps, seed)
    code = (f"import sys; sys.path.insert(0, {ROOT!r}); import bench; from paper_1704_04413_amd import workloads as wl; "
            f"r = bench._oracle_rate(wl, {lattice_name!r}, {n}, {steps_1t}); print(r[0], r[1], r[2])")
    env = dict(os.environ, OMP_NUM_THREADS="1")
    one = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, check=True)
    m1, dt1, th1 = one.stdout.split()[-3:]
    return dict(value=round(mlups, 4), unit="MLUPS", cores=threads, kind="oracle",
                sample=f"{steps} steps of the {lattice_name} {n}x{n} FP64 RR shear layer ({dt:.1f} s)",
                cpu_model=cpu_model(), host_cpus=os.cpu_count(),
                one_thread={"value": round(float(m1), 4), "unit": "MLUPS", "threads": int(th1),
                            "sample": f"{steps_1t} steps of the same grid ({float(dt1):.1f} s)"})


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--lattice", default="D2V37")
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--storage", default="fp64", choices=list(STORAGE_FLAGS))
    ap.add_argument("--thermal", action="store_true", help="thermal form of the --only-headline workload (D2V37)")
    ap.add_argument("--scheme", choices=["pull", "aa"],
                    help="single-buffer in-place (AA) step or two-buffer pull step for the headline workload "
                         "(the same states bit for bit; default: AA, the faster at the headline size, for "
                         "population storage; the moment representation has the pull step only)")
    ap.add_argument("--no-aa", action="store_true", help="skip the pull-against-AA lines")
    ap.add_argument("--only-aa", action="store_true", help="time the pull-against-AA lines alone")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=25)
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-storage", default="fp32", choices=["fp64", "fp32", "fp32d", "bf16"],
                    help="member storage of --only-batch")
    ap.add_argument("--no-3d", action="store_true", help="skip the 3D lattice lines (128^3)")
    ap.add_argument("--only-3d", metavar="LATTICE:COLL",
                    help="time one 3D case (e.g. D3Q19:RR, or 'all') for --steps and print its line alone")
    ap.add_argument("--n3", type=int, default=128, help="edge of the 3D box")
    ap.add_argument("--summarize-pmc3d", nargs=6, metavar="DIR",
                    help="3D traffic summary: FETCH and WRITE csv dirs (default policy), the same with "
                         "RRLBM_CACHE_POLICY=1, then the copy's FETCH and WRITE dirs")
    ap.add_argument("--lattice3d", default="D3V39", help="lattice of --summarize-pmc3d")
    ap.add_argument("--summarize-trace3d", nargs=2, metavar=("DB", "BENCH_OUT"),
                    help="write the 3D kernel-trace summary under profiles/ and exit")
    ap.add_argument("--no-studies", action="store_true", help="skip the precision, Sod and stability studies")
    ap.add_argument("--closure", choices=["full", "small", "none"], default="full",
                    help="learned-closure study: D2V37 256^2 coarse / 1024^2 fine (full) or 64^2 / 256^2")
    ap.add_argument("--only-closure", action="store_true",
                    help="time the fused closure step (D2V37, random network) at --n only")
    ap.add_argument("--summarize-requests", nargs=4, metavar="DIR",
                    help="request-counter cross-check from --pmc csv dirs: step reads, step writes, copy reads, copy writes")
    ap.add_argument("--summarize-valu", nargs=1, metavar="DIR", help="VALU summary from one --pmc csv dir")
    ap.add_argument("--summarize-closure-pmc", nargs=2, metavar="DIR",
                    help="closure-step counters against the plain step: closure csv dir, plain csv dir")
    ap.add_argument("--only-batch", action="store_true",
                    help="time the 64-instance batch (autotuned; storage from --batch-storage) alone and print its line")
    ap.add_argument("--summarize-trace-batch", nargs=2, metavar=("DB", "BENCH_OUT"),
                    help="write the batch kernel-trace summary from a rocprofv3 database and that run's output")
    ap.add_argument("--only-headline", action="store_true",
                    help="time the headline workload only (no sweeps, studies, closure or CPU baseline)")
    ap.add_argument("--no-hbm-points", action="store_true",
                    help="skip the out-of-cache roofline points (buffers of 0.5-1.2 GB)")
    ap.add_argument("--regions", type=int, default=5, help="timed regions for the median step time")
    ap.add_argument("--region-steps", type=int, default=200, help="steps per region of the median step time")
    ap.add_argument("--copy-only", action="store_true", help="only run 1 GiB device copies (counter calibration)")
    ap.add_argument("--summarize-pmc", nargs=4, metavar="DIR",
                    help="write the traffic summary from rocprofv3 --pmc csv dirs: step FETCH_SIZE, step WRITE_SIZE, "
                         "copy FETCH_SIZE, copy WRITE_SIZE (no GPU needed)")
    ap.add_argument("--summarize-trace", nargs=2, metavar=("DB", "BENCH_OUT"),
                    help="write the kernel-trace summary from a rocprofv3 database and that run's output")
    args = ap.parse_args()
    if args.scheme is None:
        # the moment representation and the closure have the pull step only
        args.scheme = "pull" if args.storage == "moments" or args.only_closure else "aa"
    if args.scheme == "aa" and (args.storage == "moments" or args.only_closure):
        ap.error("the moment representation and the closure have the pull step only")

    if args.summarize_pmc:
        print(summarize_pmc(args))
        return
    if args.summarize_trace:
        print(summarize_trace(args))
        return
    if args.summarize_requests:
        print(summarize_requests(args))
        return
    if args.summarize_valu:
        print(summarize_valu(args))
        return
    if args.summarize_closure_pmc:
        print(summarize_closure_pmc(args))
        return
    if args.summarize_trace3d:
        print(summarize_trace3d(args))
        return
    if args.summarize_pmc3d:
        print(summarize_pmc3d(args))
        return
    if args.summarize_trace_batch:
        print(summarize_trace_batch(args))
        return

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(this benchmark times one GPU's share of the work)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1704_04413_amd import binding as b
    from paper_1704_04413_amd import workloads as wl

    if not os.path.exists(b.LIB_PATH):
        from paper_1704_04413_amd import build as hipbuild

        hipbuild.build()
    b.lib()
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    if args.copy_only:
        print(json.dumps({"copy_GBs": round(copy_bandwidth(torch), 1)}), flush=True)
        return

    if args.only_3d:
        only = None if args.only_3d == "all" else tuple(args.only_3d.split(":"))
        print(json.dumps({"lattices_3d": suite_3d(torch, b, wl, n=args.n3, steps=args.steps, warmup=args.warmup,
                                                  only=only)}), flush=True)
        return

    if args.only_batch:
        print(json.dumps({"batched": batched_suite(torch, b, wl, storage=args.batch_storage, steps=args.steps)}),
              flush=True)
        return

    if args.only_aa:
        print(json.dumps({"scheme_aa": aa_suite(torch, b, wl)}), flush=True)
        return

    if args.only_closure:
        # the fused closure step with a random network (every node inside a wide
        # normalisation range): its cost does not depend on the weights
        from paper_1704_04413_amd import closure as cl

        theta = torch.as_tensor(cl.init_theta(3)).cuda()
        nv = np.zeros(b.LBM_MLP_NNORM)
        nv[8:16] = 1.0
        nv[16:24], nv[24:32] = -1e30, 1e30
        nv[48:64] = 1e-6
        nv[64:80], nv[80:96] = -1e30, 1e30
        norm = torch.as_tensor(nv, dtype=torch.float32).cuda()
        sim, meta = make_sim(b, wl, "D2V37", args.n, args.storage, re=3e4, noise=False)
        b.lbm_closure_set(sim.ctx, theta, norm)
        wall, kms = time_steps(torch, sim, args.steps, args.warmup)
        sim.close()
        bpl = bytes_per_node(meta["q"], args.storage) * args.n * args.n
        print(json.dumps({"closure_step": True, "value": round(args.n * args.n * args.steps / wall / 1e6, 2),
                          "unit": "MLUPS", "steps": args.steps,
                          "roofline": {"bytes_per_launch": bpl, "kernel_ms_avg": round(kms, 5),
                                       "achieved": round(bpl / (kms * 1e-3) / 1e9, 1),
                                       "frac": round(bpl / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}}), flush=True)
        return

    if args.only_headline:
        args.no_sweep = args.no_batch = args.no_3d = args.no_studies = args.no_cpu_baseline = args.no_aa = True
        args.no_hbm_points = True
        args.closure = "none"
        args.regions = 0

    sim, meta = make_sim(b, wl, args.lattice, args.n, args.storage, thermal=args.thermal, scheme=args.scheme)
    wall, kms = time_steps(torch, sim, args.steps, args.warmup)
    med = time_regions(torch, sim, args.region_steps, args.regions) if args.regions > 0 else []
    mom = sim.moments()
    buffer_mib = b.lbm_buffer_elems(args.lattice, args.n, args.n,
                                    STORAGE_FLAGS[args.storage] | (b.LBM_THERMAL if args.thermal else 0)) * \
        (8 if args.storage in ("fp64", "moments") else STORAGE_BYTES[args.storage]) / 2 ** 20
    sim.close()
    nodes = args.n * args.n
    mlups = nodes * args.steps / wall / 1e6
    bytes_per_launch = bytes_per_node(meta["q"], args.storage, args.thermal) * nodes
    kavg = kms * 1e-3
    achieved = bytes_per_launch / kavg / 1e9
    traffic = read_traffic(f"{args.lattice.lower()}_{args.storage}_{args.n}{_scheme_tag(args.scheme)}_traffic.txt")
    out = {
        "metric": METRIC,
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.storage in ("fp32", "bf16") else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{args.lattice} {'thermal' if args.thermal else 'isothermal'} recursive-regularized "
                        f"shear layer {args.n}x{args.n}, "
                        f"{args.storage} populations, order {b.lbm_lattice_info(args.lattice)[2]}, "
                        "Re 1e5, Mach 0.1",
            "lattice": args.lattice, "nx": args.n, "ny": args.n, "storage": args.storage, "scheme": args.scheme,
            "tau": meta["tau"],
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "bytes_per_launch": bytes_per_launch,
            "kernel_ms_avg": round(kms, 5),
            "buffer_MiB": round(buffer_mib, 1),
            "memory": (("cache-assisted: the one state buffer of the in-place steps is a little larger than "
                        "the 256 MiB memory-side cache, which still serves part of each step's traffic (the "
                        "out-of-cache point is roofline_out_of_cache)") if args.scheme == "aa" else
                       ("cache-assisted: the state buffer is within the 256-320 MiB band where the step keeps "
                        "what it writes in the 256 MiB memory-side cache (the out-of-cache point is "
                        "roofline_out_of_cache)")) if 256 < buffer_mib <= 320 else
                      ("cache-resident" if buffer_mib <= 256 else "out of cache"),
        },
        "nonfinite_nodes": int(mom["sums"][8]),
    }
    if med:
        mk = float(np.median(med))
        out["median_of_regions"] = {
            "regions": len(med), "steps_per_region": args.region_steps,
            "kernel_ms_regions": [round(x, 5) for x in med], "kernel_ms_median": round(mk, 5),
            "MLUPS": round(nodes / (mk * 1e-3) / 1e6, 1),
            "frac_hbm": round(bytes_per_launch / (mk * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    if not args.no_hbm_points:
        # the same step with state buffers of 0.5-1.2 GB, far above the 256 MiB
        # memory-side cache: these fractions are HBM bandwidth
        pt = roofline_point(torch, b, wl, "D2V37", 2048, "fp64")
        pt["traffic"] = read_traffic("d2v37_fp64_2048_traffic.txt")
        out["roofline_out_of_cache"] = pt
        cases = [("D2Q9", 4096, "fp64", False, 0), ("D2V17", 2048, "fp64", False, 0),
                 ("D2V37", 2048, "fp64", True, 0), ("D2V37", 2048, "fp64", False, 0x20),
                 ("D2V37", 2048, "fp64", False, 0x10), ("D2Q9", 4096, "fp32", False, 0),
                 ("D2V17", 3072, "fp32", False, 0), ("D2V37", 2048, "fp32", False, 0),
                 ("D2V37", 2048, "fp32d", False, 0),
                 ("D2V37", 4096, "bf16", False, 0), ("D2Q9", 4096, "moments", False, 0),
                 ("D2V17", 4096, "moments", False, 0), ("D2V37", 4096, "moments", False, 0),
                 ("D2V37", 2048, "moments", True, 0)]
        out["per_lattice_hbm"] = [roofline_point(torch, b, wl, lat, n, st, steps=50, thermal=th, coll=co)
                                  for lat, n, st, th, co in cases]
        mom = [r for r in out["per_lattice_hbm"]
               if r["storage"] == "moments" and r["lattice"] == "D2V37" and not r["thermal"]]
        out["roofline_moment_step"] = moment_step_roofline(mom[0] if mom else None)
    if not args.no_sweep:
        # 1024^2: buffers of 37-310 MB, inside or about the size of the 256 MiB
        # memory-side cache, so these are MLUPS only (no HBM fraction); the
        # BGK and PR lines give the cost of the regularization on the GPU
        sweep = []
        cases = [("D2Q9", "fp64", False, 0), ("D2V17", "fp64", False, 0), ("D2V37", "fp64", False, 0),
                 ("D2Q9", "fp64", False, 0x20), ("D2V17", "fp64", False, 0x20), ("D2V37", "fp64", False, 0x20),
                 ("D2Q9", "fp64", False, 0x10), ("D2V17", "fp64", False, 0x10), ("D2V37", "fp64", False, 0x10),
                 ("D2V37", "fp64", True, 0), ("D2Q9", "fp32", False, 0), ("D2V17", "fp32", False, 0),
                 ("D2V37", "fp32", False, 0), ("D2V37", "fp32d", False, 0), ("D2V37", "bf16", False, 0),
                 ("D2Q9", "moments", False, 0),
                 ("D2V17", "moments", False, 0), ("D2V37", "moments", False, 0), ("D2V37", "moments", True, 0)]
        for lat, st, th, co in cases:
            s2, m2 = make_sim(b, wl, lat, args.n, st, thermal=th, coll=co, noise=False)
            s2.step(5)
            k2 = float(np.median(time_regions(torch, s2, 50, 3)))
            s2.close()
            sweep.append({"lattice": lat, "storage": st, "thermal": th,
                          "collision": {0: "RR", 0x10: "PR", 0x20: "BGK"}[co],
                          "MLUPS": round(nodes / (k2 * 1e-3) / 1e6, 1), "memory": "cache-resident or cache-assisted"})
        rr = {(r["lattice"]): r["MLUPS"] for r in sweep if r["storage"] == "fp64" and r["collision"] == "RR"
              and not r["thermal"]}
        ratios = {}
        for r in sweep:
            if r["storage"] == "fp64" and not r["thermal"] and r["collision"] != "RR":
                ratios[f"{r['lattice']} t_RR/t_{r['collision']}"] = round(r["MLUPS"] / rr[r["lattice"]], 3)
        out["per_lattice"] = sweep
        out["cost_ratios_1024"] = ratios
        out["copy_GBs"] = round(copy_bandwidth(torch), 1)
    if not args.no_aa:
        out["scheme_aa"] = aa_suite(torch, b, wl)
    if not args.no_3d:
        out["lattices_3d"] = suite_3d(torch, b, wl, n=args.n3)
    if not args.no_batch:
        out["batched"] = batched_suite(torch, b, wl)
        out["batched_fp32d"] = batched_suite(torch, b, wl, storage="fp32d")
    if not args.no_studies:
        from paper_1704_04413_amd import studies

        out["precision"] = studies.precision_study(torch)
        out["sod"] = studies.sod_study(torch)
        out["stability"] = studies.stability_range(torch)
        out["re3e4_study"] = studies.comparison_study(torch)
        machs = [round(0.40 + 0.01 * k, 2) for k in range(36)]
        out["stability_scan_d2v37"] = [
            studies.stability_scan(torch, "D2V37", [("RR", 2), ("RR", 3), ("RR", 4), ("PR", 4)], re, machs)
            for re in (3e5, 1e6)]
    if args.closure != "none":
        from paper_1704_04413_amd import closure as cl

        if args.closure == "full":
            # the paper's D2V37 Mach (Fig. 4), where ranks 3-4 carry weight, and the workload's Mach 0.1
            out["closure"] = cl.experiment(torch, snaps=tuple(range(100, 1001, 100)), mach=0.57)
            out["closure_mach01"] = cl.experiment(torch)
        else:
            out["closure"] = cl.experiment(torch, range(6), range(6, 8), 64, 4, 3e4, tuple(range(50, 401, 50)),
                                           1500, 8192)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.lattice, args.n, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
