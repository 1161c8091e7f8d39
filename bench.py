#!/usr/bin/env python3
"""Throughput of the coupled LBM / hard-sphere step on one MI355X.

A step is one pass of the whole method over the bed: deposition, modified
collision + streaming, drag + integration, binning, contact detection and
collisions.  Default workload: the riser-shaped bed with the precision
pattern (512 x 4096 D2Q9 lattice, 2 000 000 spheres of d = 0.5, y periodic,
x walls, body-force-driven gas; FP32, with FP16 and BF16 deviation storage as
variants), inputs resident in HBM before timing.

Prints ONE JSON line:
  value             coupled MLUPS (lattice cells updated per second / 1e6)
  particle_updates  particles advanced per second
  roofline          the dominant kernel: the bytes the whole-step model gives
                    its phase (model_kernel_bytes) per launch over its mean
                    launch time (events its dispatch stamps, on the library's
                    stream, timed region), against the 8 TB/s HBM3E peak; the
                    bytes the kernel itself must move as built are beside it
                    (impl_*)
  cpu_baseline      the FP64 oracle timed on the host on a bounded sample, on
                    all cores (per-cell loops over OpenMP threads) and on one
  variants          the same workload with FP16 / BF16 population storage

--workload beds: the batching pattern, 64 independent beds of uneven size
(64x256 to 256x1024, 2 000 to 200 000 spheres) with FP16 population storage,
advanced by one launch per phase for all beds and replayed from a captured
hipGraph; compared with the same beds stepped one after another through the
plain single-bed FP32 path.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "coupled MLUPS + particle-updates/s, % HBM peak; FP16-store vs FP32 at stated err"
WORKLOADS = {
    "bubble": lambda: __import__("synth").bubble(),
    "bubble_small": lambda: __import__("synth").bubble_small(),
    "riser": lambda: __import__("synth").riser(),
    "riser_random_ids": lambda: __import__("synth").riser(sort_ids=False),
    "riser_crop": lambda: __import__("synth").riser_crop(),
    "riser_large": lambda: __import__("synth").riser_large(),
    "beds": lambda: __import__("synth").beds(64),
    "paper_bubble": lambda: __import__("synth").paper_bubble(),
    "paper_riser": lambda: __import__("synth").paper_riser(),
    "riser3d": None,  # the 3-D coupled step: run_riser3d
    "d3q19_gas": None,  # the 3-D gas lattice alone: run_d3q19
    "d3q19_psm": None,  # the 3-D lattice with solids given per cell: run_d3q19
}
SIZES = {"fp64": (8, 8), "fp32": (4, 4), "fp16": (2, 4), "bf16": (2, 4)}  # (population, scalar) bytes


def model_kernel_bytes(kernel: str, prec: str, C: int, N: int, pairs: int) -> float:
    """The whole-step byte model (model_bytes_per_step) split over the phases
    that the kernels carry.  Per cell: populations in and out (18 s_f), the
    deposited solid velocity written and read (4 s_c), the six node fields
    u_gas, beta, p, F_pg written by the collision and read by the drag
    (12 s_c), the count n written once and read twice, the cell start written
    and read.  Per particle: the state read and written by the integration
    (8 s_p), the position read by the binning and by the contact search, the
    velocity read by the deposition (2 s_p each), key and permutation (16 B).
    Per contact pair: its two indices written and read (16 B), the two
    positions and velocities read by the collision (8 s_p)."""
    sf, st = SIZES[prec]
    if kernel == "collide":   # deposition + collision + streaming
        return C * (18 * sf + 10 * st + 4) + N * 2 * st
    if kernel == "drag":      # interpolation, drag, integration
        return C * (6 * st + 4) + N * 8 * st
    if kernel == "scan":      # counts in, cell starts out
        return C * 8
    if kernel == "scatter":   # binning read of the position, key and permutation
        return N * (2 * st + 16)
    if kernel == "contacts":  # cell starts, positions, pairs written
        return C * 4 + N * 2 * st + pairs * 8
    if kernel == "resolve":   # pairs read, both particles' positions and velocities
        return pairs * (8 + 8 * st)
    raise KeyError(kernel)


def algorithmic_bytes(kernel: str, prec: str, C: int, N: int, pairs: int) -> float:
    """Bytes a launch of `kernel` must move at minimum as built (each operand
    it reads or writes once, including its own keys, degrees and counters)."""
    sf, st = SIZES[prec]
    if kernel == "collide":   # f read + write, cell starts, 6 node fields written, particle velocities read
        return C * (18 * sf + 4 + 6 * st) + N * 2 * st
    if kernel == "drag":      # cell starts, F_pg, 4 interpolated fields; particle record read + write, rank, count
        return C * (4 + 2 * st + 4 * st + 4) + N * (2 * (4 + 4 * st) + 4)
    if kernel == "resolve":   # slot, degree; positions and velocities; updated velocities; contact rows
        return N * (4 + 4 + 4 + 4 * st + 2 * st) + pairs * 2 * (8 + 4)
    if kernel == "contacts":  # record read, cell starts, degree and counter written, contact rows written
        return N * (4 + 4 + 2 * st + 4 + 4) + C * 4 + pairs * 2 * 8
    if kernel == "scatter":   # record read and written, rank and cell start read, slot map written
        return N * (2 * (8 + 4 * st) + 4 + 4 + 4)
    if kernel == "scan":      # counts read (and cleared), cell starts written
        return C * 12
    raise KeyError(kernel)


# Error bounds of the storage precisions against the FP64 oracle (norm-wise
# relative error of populations and gas fields after 10 steps from one state
# on the 64 x 512 riser crop), asserted by tests/test_precision_study.py; the
# measured errors are in profiles/precision_riser-crop-64x512.md.
STATED_ERR = {p: {"bound": b, "fields": "f, rho, u_gas, F_pg, beta", "after_steps": 10,
                  "source": "profiles/precision_riser-crop-64x512.md"}
              for p, b in (("fp16", 1e-2), ("bf16", 1.5e-2))}
STATED_ERR["fp32"] = {"bound": {"f": 1e-8, "rho": 1e-8, "beta": 1e-6, "u_gas": 1e-4, "F_pg": 3e-4},
                      "fields": "f, rho, u_gas, F_pg, beta", "after_steps": 10,
                      "source": "profiles/precision_riser-crop-64x512.md"}


def workload_name(name: str, prec: str) -> str:
    """A workload's name with the storage precision actually run in place of
    the one the recipe names."""
    head, _, tail = name.rpartition("-")
    return f"{head}-{prec}" if tail in SIZES else name


def model_bytes_per_step(prec: str, C: int, N: int, pairs: int) -> float:
    """Whole-step byte model: 18 s_f + 16 s_c + 20 per cell, 14 s_p + 16 per
    particle, 16 + 8 s_p per contact pair."""
    sf, st = SIZES[prec]
    return C * (18 * sf + 16 * st + 20) + N * (14 * st + 16) + pairs * (16 + 8 * st)


def run_gpu(cfg, prec, steps, warmup, torch, L, dominant=None, tuning=None):
    sim = L.Sim(cfg, precision=prec)
    stream = sim.stream
    sim.step(warmup)
    if tuning is None:
        tuning = sim.autotune(4)  # launch shapes (results do not depend on them)
    else:
        sim.set_tuning(**tuning)
    torch.cuda.synchronize()
    # per-kernel breakdown (separate pass): find the dominant kernel
    sim.time_kernels(L.KERNELS)
    nb = max(5, min(steps, 20))
    sim.step(nb)
    bd = sim.kernel_times()
    sim.time_kernels([])
    breakdown = {k: ms / max(n, 1) * 1e3 for k, (ms, n) in bd.items()}  # us per launch
    if dominant is None:
        dominant = max(breakdown, key=lambda k: breakdown[k])
    # timed region: whole steps, with only the dominant kernel's launches carrying timing events
    torch.cuda.synchronize()
    sim.time_kernels([dominant])
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    e1.synchronize()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    kt = sim.kernel_times()[dominant]
    sim.time_kernels([])
    counters = sim.counters()
    sums, dstep = sim.diag_last()  # the periodic FP64 check (raises if it found a non-finite value)
    hist = sim.count_histogram(8)
    out = dict(ms=ms, breakdown_us=breakdown, dominant=dominant, dom_ms=kt[0], dom_launches=kt[1],
               pairs=counters["pairs"], tuning=sim.tuning(), diag=(sums, dstep), hist=hist)
    sim.close()
    return out


CSRC = os.path.join(ROOT, "paper_1303_2653_amd", "csrc")
KERNEL_SOURCES = ("kernels.hpp", "device.hpp", "lattice3d.hpp", "spheres_tile.hpp")
# the 3-D coupled step's kernels also live in coupled3d.hpp
KERNEL_SOURCES_3D = KERNEL_SOURCES + ("coupled3d.hpp",)
# the kernels of each phase (either form of a kernel, and every launch of the
# phase: the collision stage's tile kernel with the contact kernel on what it
# left, the cluster kernel with the ordered sweep)
KERNEL_KEYS = {"collide": ("k_collide",), "drag": ("k_drag", "k_drag_flat"), "scan": ("k_scan_cells",),
               "scatter": ("k_scatter",), "contacts": ("k_spheres_tile", "k_contacts", "k_contacts_small"),
               "resolve": ("k_resolve_clusters", "k_resolve"), "k3_bgk": ("k3_bgk", "k3_bgk_pairs"), "k3_psm": ("k3_psm", "k3_psm_pairs")}
# the whole 3-D coupled step: every kernel it launches once per step
STEP3D_KEYS = {"step3d": ("k3c_collide", "k3c_gradp", "k3c_drag", "k_scan_reduce", "k_scan_top", "k_scan_apply",
                          "k3c_scatter", "k3c_contacts", "k3c_clusters", "k3c_resolve")}


def kernel_source_hash(sources=KERNEL_SOURCES) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, kernel: str):
    """HBM-side bytes per launch of `kernel` from the committed counter summary,
    or None if there is none or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_source_hash") != kernel_source_hash(tuple(t.get("kernel_sources", KERNEL_SOURCES))):
        return None
    v = t.get("bytes_per_launch", {}).get(kernel)
    return None if v is None else int(v)


def summarize(args):
    """Turn rocprofv3 CSV output into the short summaries kept under profiles/:
    <label>.md (per-kernel duration statistics and counter bytes) and
    traffic_<workload>.json (HBM-side bytes per launch, scaled by the copy probe)."""
    import csv
    import glob

    def rows(d, pattern):
        out = []
        for f in glob.glob(os.path.join(d, "**", pattern), recursive=True):
            with open(f) as fh:
                out += list(csv.DictReader(fh))
        return out

    def short(name):
        n = name.split("(")[0].split("<")[0].split("::")[-1]
        return n

    stats = rows(args.stats, "*kernel_stats.csv")
    lines = [f"# rocprofv3 summary: {args.label}", "", "Command (run from /tmp, repository at $R):", "",
             "```", args.command, "```", "", "| kernel | calls | mean us | min us | max us | share % |",
             "|---|---:|---:|---:|---:|---:|"]
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"])):
        lines.append(f"| {r['Name'].split('(')[0][:70]} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.1f} |")
    traffic = {}
    if args.fetch and args.write and args.copy_fetch and args.copy_write:
        def per_kernel(d):
            acc = {}
            for r in rows(d, "*counter_collection.csv"):
                acc.setdefault(short(r["Kernel_Name"]), []).append(float(r["Counter_Value"]) * 1024.0)
            return {k: sum(v) / len(v) for k, v in acc.items()}
        fetch, write = per_kernel(args.fetch), per_kernel(args.write)
        cf, cw = per_kernel(args.copy_fetch), per_kernel(args.copy_write)
        copy_name = max(cf, key=lambda k: cf[k])  # the copy: the only probe kernel that reads
        f_scale = args.copy_bytes / cf[copy_name]
        w_scale = args.copy_bytes / cw[copy_name]
        lines += ["", f"HBM-side bytes per launch: FETCH_SIZE x {f_scale:.3f} + WRITE_SIZE x {w_scale:.3f}; the factors "
                  f"make a plain {args.copy_bytes} byte copy ({copy_name}) read and write exactly its size.", "",
                  "| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | bytes per launch |", "|---|---:|---:|---:|"]
        keys = STEP3D_KEYS if args.workload == "riser3d" else KERNEL_KEYS
        for key, knames in keys.items():
            names = [n for n in knames if n in fetch and n in write]
            if names:
                b = 0.0
                for kname in names:
                    bk = fetch[kname] * f_scale + write[kname] * w_scale
                    b += bk
                    lines.append(f"| {kname} | {fetch[kname] / 1024:.1f} | {write[kname] / 1024:.1f} | {int(bk)} |")
                traffic[key] = int(b)
        lines += ["", "Counter commands: the same program under `rocprofv3 --pmc FETCH_SIZE` and "
                  "`rocprofv3 --pmc WRITE_SIZE` (one counter per run), and `bench.py --copy-probe "
                  f"{args.copy_bytes}` under each for the scale factors."]
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", f"{args.label}.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    if traffic:
        with open(os.path.join(ROOT, "profiles", f"traffic_{args.workload}.json"), "w") as fh:
            srcs = KERNEL_SOURCES_3D if args.workload == "riser3d" else KERNEL_SOURCES
            json.dump({"workload": args.workload, "kernel_sources": list(srcs),
                       "kernel_source_hash": kernel_source_hash(srcs),
                       "bytes_per_launch": traffic, "fetch_scale": f_scale, "write_scale": w_scale}, fh, indent=1)
    print("\n".join(lines))


def cpu_baseline(cfg, seconds):
    """The FP64 oracle stepping the bed from its initial state for about
    `seconds` each: first the OpenMP build (per-cell loops on every host core,
    bit-identical results), then the single-thread build."""
    import oracle
    C, N = cfg["nx"] * cfg["ny"], len(cfg["pos"])

    def leg(omp):
        sim = oracle.Sim(cfg, omp=omp)
        t0 = time.perf_counter()
        steps = 0
        while True:
            sim.step()
            steps += 1
            if time.perf_counter() - t0 >= seconds:
                break
        return steps, time.perf_counter() - t0

    threads = oracle.threads(omp=True)
    s_all, t_all = leg(True)
    s_one, t_one = leg(False)
    nproc = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return dict(value=round(C * s_all / t_all / 1e6, 4), unit="MLUPS", cores=threads, kind="oracle",
                sample=f"{cfg['name']}: first {s_all} coupled steps from the initial state, FP64, per-cell loops "
                       f"on {threads} OpenMP threads ({t_all:.1f} s; host nproc {nproc}); particle updates/s "
                       f"{N * s_all / t_all:.3e}",
                single_thread=dict(value=round(C * s_one / t_one / 1e6, 4), unit="MLUPS", cores=1,
                                   sample=f"first {s_one} coupled steps, FP64, one thread ({t_one:.1f} s); "
                                          f"particle updates/s {N * s_one / t_one:.3e}"))


def copy_bandwidth(torch, nbytes: int, reps: int = 5) -> dict:
    """A plain device-to-device copy of nbytes: read + write bytes over the mean
    time of reps copies (the measured HBM ceiling beside the published peak)."""
    n = nbytes // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"copy_probe_bytes": n * 4, "launches": reps + 1, "ms_per_copy": round(ms, 4),
            "GBs": round(2 * n * 4 / (ms * 1e-3) / 1e9, 1)}


def time_region(torch, stream, fn):
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    fn()
    e1.record(stream)
    e1.synchronize()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def run_d3q19(args, torch, L):
    """The 3-D gas lattice alone (D3Q19 BGK collide-stream, periodic box) on the
    3-D riser's lattice, 256 x 256 x 1024 cells, in FP16 deviation storage by
    default: MLUPS, and the kernel against the HBM roofline (each step reads
    and writes 19 populations per cell)."""
    prec = args.precision if args.precision_given else "fp16"
    nx, ny, nz = 256, 256, 1024
    C = nx * ny * nz
    code = {"fp64": L.LBDPS_FP64, "fp32": L.LBDPS_FP32, "fp16": L.LBDPS_FP32_STORE_FP16,
            "bf16": L.LBDPS_FP32_STORE_BF16}[prec]
    dt = {"fp64": torch.float64, "fp32": torch.float32, "fp16": torch.float16, "bf16": torch.bfloat16}[prec]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        a = torch.zeros(19 * C, dtype=dt, device="cuda")  # deviations 0: gas at rest (FP64: filled below)
        if prec == "fp64":
            for i, w in enumerate([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12):
                a[i * C:(i + 1) * C] = w
        b = torch.empty_like(a)
    stream.synchronize()

    psm = args.workload == "d3q19_psm"
    sT = SIZES[prec][1]
    if psm:
        # the 3-D riser's solids: 10 M spheres of d = 0.5 over the 67.1 M cells,
        # Poisson counts per cell (mean 0.149), velocities up to 0.01
        with torch.cuda.stream(stream):
            g = torch.Generator(device="cuda").manual_seed(7)
            n_cell = torch.poisson(torch.full((C,), 1.0e7 / C, device="cuda"), generator=g).to(torch.int32)
            vdt = torch.float64 if prec == "fp64" else torch.float32
            vs = ((torch.rand(3 * C, device="cuda", generator=g) - 0.5) * 0.02).to(vdt)
            force = torch.empty_like(vs)
        stream.synchronize()

    def step(n):
        nonlocal a, b
        for _ in range(n):
            if psm:
                L.check(L.lbdps3_psm_step(a.data_ptr(), b.data_ptr(), n_cell.data_ptr(), vs.data_ptr(),
                                          force.data_ptr(), nx, ny, nz, 0.6, 0.5, code, stream.cuda_stream),
                        "lbdps3_psm_step")
            else:
                L.check(L.lbdps3_bgk_step(a.data_ptr(), b.data_ptr(), nx, ny, nz, 0.6, code, stream.cuda_stream),
                        "lbdps3_bgk_step")
            a, b = b, a

    step(args.warmup)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stream.synchronize()
    e0.record(stream)
    step(args.steps)
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1)
    us = ms / args.steps * 1e3
    # populations in and out; with solids also the count, v_s in and F out
    nbytes = (2 * 19 * SIZES[prec][0] + (4 + 6 * sT if psm else 0)) * C
    kern = "k3_psm" if psm else "k3_bgk"
    achieved = nbytes / (us * 1e-6) / 1e9
    cb = copy_bandwidth(torch, 1 << 30)
    return {"metric": METRIC, "value": round(C * args.steps / (ms / 1e3) / 1e6, 2), "unit": "MLUPS", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms / args.steps, 5),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": {"fp64": "f64", "fp32": "f32", "fp16": "f32 (f16 storage)", "bf16": "f32 (bf16 storage)"}[prec],
            "data": "synthetic (gas at rest, periodic box" + (", seeded Poisson solids per cell)" if psm else ")"),
            "config": {"workload": f"d3q19-{'psm' if psm else 'gas'}-{nx}x{ny}x{nz}-{prec}", "nx": nx, "ny": ny,
                       "nz": nz, "precision": prec, "tau": 0.6, "particles": int(1e7) if psm else 0,
                       # the sphere count is kept, so the mean solid fraction is
                       # 1e7 (pi d^3 / 6) / C, not the 0.1 a denser riser would have
                       **({"d_p": 0.5, "solid_fraction_3d": round(1e7 * math.pi * 0.5 ** 3 / 6 / C, 5)}
                          if psm else {})},
            "roofline": {"bound": "hbm", "kernel": kern, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                         "traffic": measured_traffic(args.workload, kern) if prec == "fp16" else None,
                         "bytes_per_launch": int(nbytes), "us_per_launch": round(us, 3), "copy_GBs": cb["GBs"],
                         "frac_of_copy": round(achieved / cb["GBs"], 4)}}


def model_bytes_per_step_3d(prec: str, C: int, N: int, pairs: int) -> float:
    """The whole-step byte model in 3-D: per cell 38 s_f (19 populations in
    and out) + 22 s_c (the deposited solid velocity written and read, 3 + 3;
    u_gas, beta, p, F_pg written by the collision and read by the drag, 8 + 8)
    + 20 (the count written and read twice, the cell start written and read);
    per particle 21 s_p + 16 (state read and written, 12; position read by the
    binning and the contact search and velocity read by the deposition, 3
    each; key and permutation); per pair 16 + 12 s_p."""
    sf, st = SIZES[prec]
    return C * (38 * sf + 22 * st + 20) + N * (21 * st + 16) + pairs * (16 + 12 * st)


def run_riser3d(args, torch, L):
    """The 3-D coupled step (config: D3Q19 256 x 256 x 1024, 10 000 000 spheres
    of d = 0.5, periodic, gravity-driven riser, FP16 deviation storage with
    FP32 arithmetic by default): MLUPS, particle updates/s and the whole-step
    model bandwidth."""
    import synth
    prec = args.precision if args.precision_given else "fp16"
    cfg = synth.riser3d()
    C, N = cfg["nx"] * cfg["ny"] * cfg["nz"], len(cfg["pos"])
    sim = L.Sim3(cfg, precision=prec)
    st = sim.stream
    sim.step(args.warmup)
    ms = time_region(torch, st, lambda: sim.step(args.steps))
    pairs = sim.counters()["pairs"]
    cons = sim.conservation()  # FP64 sums after the timed steps (raises on a non-finite value)
    sim.close()
    del sim
    s = ms / 1e3
    model = model_bytes_per_step_3d(prec, C, N, pairs)
    bw = model * args.steps / s / 1e9
    line = {"metric": METRIC, "value": round(C * args.steps / s / 1e6, 2), "unit": "MLUPS", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms / args.steps, 5),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": {"fp64": "f64", "fp32": "f32", "fp16": "f32 (f16 storage)", "bf16": "f32 (bf16 storage)"}[prec],
            "data": "synthetic (seeded splitmix64 spheres, gas at rest)",
            "config": {"workload": f"riser3d-{cfg['nx']}x{cfg['ny']}x{cfg['nz']}-{N}-{prec}", "nx": cfg["nx"],
                       "ny": cfg["ny"], "nz": cfg["nz"], "particles": N, "precision": prec, "d_p": cfg["d"],
                       "tau": cfg["tau"], "solid_fraction_3d": round(N * math.pi * cfg["d"] ** 3 / 6 / C, 5)},
            "particle_updates_per_s": float(f"{N * args.steps / s:.4e}"),
            "model_bytes_per_step": int(model), "model_bw_frac": round(bw / HBM_PEAK_GBS, 4),
            "contact_pairs": int(pairs),
            "roofline": {"bound": "hbm", "kernel": "step", "achieved": round(bw, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(bw / HBM_PEAK_GBS, 4),
                         "traffic": measured_traffic("riser3d", "step3d") if prec == "fp16" else None,
                         "bytes_per_launch": int(model), "us_per_launch": round(ms / args.steps * 1e3, 3)}}
    if not args.no_cpu_baseline:
        import oracle
        sub = synth.riser3d(64, 64, 64, int(round(N * 64 ** 3 / C)), seed=5)
        o = oracle.Sim3(sub, omp=True)
        t0, k = time.perf_counter(), 0
        while time.perf_counter() - t0 < args.cpu_seconds:
            o.step()
            k += 1
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = dict(value=round(64 ** 3 * k / dt / 1e6, 4), unit="MLUPS",
                                    cores=oracle.threads(omp=True), kind="oracle",
                                    sample=f"a 64 x 64 x 64 box at the same density ({len(sub['pos'])} spheres), "
                                           f"{k} coupled steps from rest, FP64, per-cell loops on OpenMP threads "
                                           f"({dt:.1f} s)")
    line["conservation"] = {"mass": float(cons[0]), "gas_momentum": [float(v) for v in cons[1:4]],
                            "particle_momentum": [float(v) for v in cons[4:7]], "nonfinite": int(cons[7])}
    return line


def run_beds(args, torch, L):
    """The batching workload: one JSON line (see the module docstring)."""
    cfgs = WORKLOADS["beds"]()
    prec = args.precision if args.precision_given else "fp16"
    Cs = [c["nx"] * c["ny"] for c in cfgs]
    Ns = [len(c["pos"]) for c in cfgs]
    K = args.steps + (args.steps & 1)  # graphs hold an even number of steps
    batch = L.Batch(cfgs, precision=prec)
    st = batch.stream
    batch.step(args.warmup)
    # launch shapes per bed size class; two rounds of 2 steps per candidate and
    # class keep the tuning run within the beds' stable span (they are reset below)
    tunings = batch.autotune(steps=2)
    # every measured region starts again from the initial beds, after the warmup
    batch.reset()
    batch.step(args.warmup)
    batch.time_kernels(L.KERNELS)
    batch.step(max(4, min(K, 20)))
    bd = batch.kernel_times()
    batch.sync()
    breakdown = {k: ms / max(n, 1) * 1e3 for k, (ms, n) in bd.items()}
    dom = max(breakdown, key=lambda k: breakdown[k])
    batch.reset()
    batch.step(args.warmup)
    batch.time_kernels([dom])
    ms_eager = time_region(torch, st, lambda: batch.step(K))
    kt = batch.kernel_times()[dom]
    batch.time_kernels([])
    batch.sync()
    batch.reset()
    batch.step(args.warmup)
    batch.capture(K)
    ms_first = time_region(torch, st, batch.launch)  # the first replay also uploads the graph
    batch.sync()
    batch.reset()
    batch.step(args.warmup)
    batch.capture(K)
    batch.sync()
    ms_graph = time_region(torch, st, batch.launch)
    batch.sync()
    pairs = [b.counters()["pairs"] for b in batch.beds]
    batch.close()
    del batch
    def sequential_ms(p):
        """The same beds stepped one after another through the single-bed path
        in storage precision p (each bed autotuned as the batch was)."""
        sims = [L.Sim(c, precision=p) for c in cfgs]
        for sm in sims:
            sm.step(args.warmup)
            sm.autotune(2)
            sm.set_state(None, sm.cfg["pos"], sm.cfg["vel"])
            sm.step(args.warmup)

        def sequential():
            for sm in sims:
                sm.step(K)

        ms = time_region(torch, torch.cuda.current_stream(), sequential)
        for sm in sims:
            sm.close()
        return ms

    ms_seq = sequential_ms("fp32")
    ms_seq_same = sequential_ms(prec)
    s = ms_graph / 1e3
    dom_us = kt[0] / max(kt[1], 1) * 1e3
    dom_bytes = sum(model_kernel_bytes(dom, prec, C, N, pr) for C, N, pr in zip(Cs, Ns, pairs))
    impl_bytes = sum(algorithmic_bytes(dom, prec, C, N, pr) for C, N, pr in zip(Cs, Ns, pairs))
    achieved = dom_bytes / (dom_us * 1e-6) / 1e9
    impl_achieved = impl_bytes / (dom_us * 1e-6) / 1e9
    model = sum(model_bytes_per_step(prec, C, N, pr) for C, N, pr in zip(Cs, Ns, pairs))
    line = {
        "metric": METRIC, "value": round(sum(Cs) * K / s / 1e6, 2), "unit": "MLUPS", "n_gpus": 1, "steps": K,
        "warmup": args.warmup, "ms_per_step": round(ms_graph / K, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp16": "f32 (f16 storage)", "bf16": "f32 (bf16 storage)"}[prec],
        "data": "synthetic (seeded splitmix64 beds)",
        "config": {"workload": f"beds-64-uneven-{prec}", "beds": len(cfgs), "cells": sum(Cs), "particles": sum(Ns),
                   "precision": prec, "launch": "hipGraph of batched phases"},
        "particle_updates_per_s": float(f"{sum(Ns) * K / s:.4e}"),
        "model_bytes_per_step": int(model),
        "model_bw_frac": round(model * K / s / 1e9 / HBM_PEAK_GBS, 4),
        "contact_pairs": int(sum(pairs)),
        "kernel_us": {k: round(v, 2) for k, v in breakdown.items()},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "bytes_per_launch": int(dom_bytes), "us_per_launch": round(dom_us, 3),
                     "bytes_model": "model_kernel_bytes",
                     "impl_bytes_per_launch": int(impl_bytes), "impl_achieved": round(impl_achieved, 1),
                     "impl_frac": round(impl_achieved / HBM_PEAK_GBS, 4)},
        "autotune": sorted({(t["cluster_lists"], t["cluster_groups_max"]) for t in tunings}),
        "batched_eager_ms_per_step": round(ms_eager / K, 5),
        "graph_first_replay_ms_per_step": round(ms_first / K, 5),
        "sequential_fp32_ms_per_step": round(ms_seq / K, 5),
        "speedup_vs_sequential_fp32": round(ms_seq / ms_graph, 3),
        f"sequential_{prec}_ms_per_step": round(ms_seq_same / K, 5),
        f"speedup_vs_sequential_{prec}": round(ms_seq_same / ms_graph, 3),
        "drag_tile": sorted({t["drag_tile"] for t in tunings}),
    }
    if not args.no_cpu_baseline:
        import oracle
        t0, cells, n = time.perf_counter(), 0, 0
        sims_o = []
        while time.perf_counter() - t0 < args.cpu_seconds:
            if n < len(cfgs):
                sims_o.append(oracle.Sim(cfgs[n]))
            o = sims_o[n % len(cfgs)]
            o.step()
            cells += o.p.nx * o.p.ny
            n += 1
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = dict(value=round(cells / dt / 1e6, 4), unit="MLUPS", cores=1, kind="oracle",
                                    sample=f"first coupled step of beds 0..{min(n, len(cfgs)) - 1} in turn, FP64, "
                                           f"single thread ({n} bed-steps, {dt:.1f} s)")
    return line


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="riser", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default=None, choices=sorted(SIZES))
    ap.add_argument("--n-sub", type=int, default=1, help="particle sub-steps per lattice step")
    ap.add_argument("--cs-smag", type=float, default=None, help="Smagorinsky constant (sub-grid model on)")
    ap.add_argument("--diag-every", type=int, default=100,
                    help="steps between the FP64 conservation checks inside lbdps_step (0: off)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="seconds of each oracle leg")
    ap.add_argument("--tuning", default=None, metavar="LISTS,GROUPS[,DRAG[,SPHERE]]",
                    help="fixed launch shapes instead of the autotuner (profiling runs): cluster lists and "
                         "groups, drag tile, collision-stage tile")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (HBM counter calibration)")
    ap.add_argument("--summarize", action="store_true", help="write profiles/ summaries from rocprofv3 output")
    ap.add_argument("--stats", help="directory of a rocprofv3 --kernel-trace --stats run")
    ap.add_argument("--fetch", help="directory of the --pmc FETCH_SIZE run")
    ap.add_argument("--write", help="directory of the --pmc WRITE_SIZE run")
    ap.add_argument("--copy-fetch", help="directory of the copy probe under --pmc FETCH_SIZE")
    ap.add_argument("--copy-write", help="directory of the copy probe under --pmc WRITE_SIZE")
    ap.add_argument("--copy-bytes", type=int, default=1 << 30)
    ap.add_argument("--label", default="profile")
    ap.add_argument("--command", default="")
    args = ap.parse_args()
    args.precision_given = args.precision is not None
    if args.precision is None:
        args.precision = "fp32"
    if args.summarize:
        summarize(args)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    torch.cuda.set_device(0)
    if args.copy_probe:
        print(json.dumps(copy_bandwidth(torch, args.copy_probe)), flush=True)
        return
    from paper_1303_2653_amd import lbdps as L

    if args.workload == "riser3d":
        print(json.dumps(run_riser3d(args, torch, L)), flush=True)
        return
    if args.workload in ("d3q19_gas", "d3q19_psm"):
        print(json.dumps(run_d3q19(args, torch, L)), flush=True)
        return
    if args.workload == "beds":
        print(json.dumps(run_beds(args, torch, L)), flush=True)
        return
    cfg = WORKLOADS[args.workload]()
    if args.n_sub > 1:
        cfg["n_sub"] = args.n_sub
    if args.cs_smag is not None:
        cfg["cs_smag"] = args.cs_smag
    cfg["diag_every"] = args.diag_every  # the FP64 conservation check inside the timed steps
    C, N = cfg["nx"] * cfg["ny"], len(cfg["pos"])
    fixed = None
    if args.tuning:
        vals = [int(v) for v in args.tuning.split(",")]
        fixed = dict(zip(("cluster_lists", "cluster_groups_max", "drag_tile", "sphere_tile"), vals))
    r = run_gpu(cfg, args.precision, args.steps, args.warmup, torch, L, tuning=fixed)
    s = r["ms"] / 1e3
    mlups = C * args.steps / s / 1e6
    pups = N * args.steps / s
    dom = r["dominant"]
    # the kernel's own duration per launch, from events its dispatch stamps
    dom_us = r["dom_ms"] / max(r["dom_launches"], 1) * 1e3
    dom_bytes = model_kernel_bytes(dom, args.precision, C, N, r["pairs"])
    impl_bytes = algorithmic_bytes(dom, args.precision, C, N, r["pairs"])
    if args.n_sub > 1:  # the phase's time per step covers every sub-step's launch
        sf, st = SIZES[args.precision]
        if dom == "drag":
            dom_bytes += (args.n_sub - 1) * N * 8 * st
            impl_bytes += (args.n_sub - 1) * N * (2 * (4 + 4 * st) + 4 + 2 * st + 8)
        elif dom != "collide":
            dom_bytes *= args.n_sub
            impl_bytes *= args.n_sub
    achieved = dom_bytes / (dom_us * 1e-6) / 1e9
    impl_achieved = impl_bytes / (dom_us * 1e-6) / 1e9
    model = model_bytes_per_step(args.precision, C, N, r["pairs"])
    traffic = None if args.n_sub > 1 or args.cs_smag is not None else measured_traffic(
        args.workload if args.precision == "fp32" else f"{args.workload}-{args.precision}", dom)
    line = {
        "metric": METRIC,
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms"] / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp16": "f32 (f16 storage)", "bf16": "f32 (bf16 storage)"}[args.precision],
        "data": "synthetic (seeded splitmix64 bed)",
        "config": {"workload": workload_name(cfg["name"], args.precision)
                   + (f"-nsub{args.n_sub}" if args.n_sub > 1 else "")
                   + (f"-les{args.cs_smag:g}" if args.cs_smag is not None else ""), "nx": cfg["nx"], "ny": cfg["ny"],
                   "particles": N,
                   "precision": args.precision, "d_p": cfg["d"], "tau": cfg["tau"],
                   "n_sub": cfg.get("n_sub", 1), "cs_smag": cfg.get("cs_smag", 0.0),
                   "diag_every": args.diag_every},
        "particle_updates_per_s": float(f"{pups:.4e}"),
        "model_bytes_per_step": int(model),
        "model_bw_frac": round(model * args.steps / s / 1e9 / HBM_PEAK_GBS, 4),
        "contact_pairs": r["pairs"],
        "conservation": {"last_check_step": r["diag"][1], "mass": float(r["diag"][0][0]),
                         "gas_momentum": [float(v) for v in r["diag"][0][1:3]],
                         "particle_momentum": [float(v) for v in r["diag"][0][3:5]],
                         "nonfinite": int(r["diag"][0][5])},
        "cells_by_particle_count": [int(v) for v in r["hist"]],  # 0, 1, ... 6, 7 or more
        "autotune": [r["tuning"][f] for f in ("cluster_lists", "cluster_groups_max", "drag_tile", "sphere_tile")],
        "kernel_us": {k: round(v, 2) for k, v in r["breakdown_us"].items()},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "bytes_per_launch": int(dom_bytes), "us_per_launch": round(dom_us, 3),
                     "bytes_model": "model_kernel_bytes",
                     "impl_bytes_per_launch": int(impl_bytes), "impl_achieved": round(impl_achieved, 1),
                     "impl_frac": round(impl_achieved / HBM_PEAK_GBS, 4)},
    }
    if fixed is not None:
        line["tuning_fixed"] = True
    cb = copy_bandwidth(torch, 1 << 30)
    line["roofline"]["copy_GBs"] = cb["GBs"]
    line["roofline"]["frac_of_copy"] = round(achieved / cb["GBs"], 4)
    if not args.no_variants and args.precision == "fp32":
        var = {}
        for p in ("fp16", "bf16"):
            rv = run_gpu(cfg, p, args.steps, args.warmup, torch, L, dominant=dom, tuning=fixed)
            sv = rv["ms"] / 1e3
            var[p] = {"MLUPS": round(C * args.steps / sv / 1e6, 2), "ms_per_step": round(rv["ms"] / args.steps, 5),
                      "speedup_vs_fp32": round(r["ms"] / rv["ms"], 3),
                      "stated_err_vs_fp64_oracle": STATED_ERR[p]}
        line["variants"] = var
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(cfg, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
