#!/usr/bin/env python3
"""Throughput of the coupled LBM / hard-sphere step on one MI355X.

A step is one pass of the whole method over the bed: deposition, modified
collision + streaming, drag + integration, binning, contact detection and
collisions.  Default workload: the bubble-injection-shaped bed (256 x 1024
D2Q9 lattice, 200 000 spheres, FP32), inputs resident in HBM before timing.

Prints ONE JSON line:
  value             coupled MLUPS (lattice cells updated per second / 1e6)
  particle_updates  particles advanced per second
  roofline          the dominant kernel: algorithmic bytes per launch over its
                    mean launch time (hipEvents on the library's stream, timed
                    region), against the 8 TB/s HBM3E peak
  cpu_baseline      the FP64 oracle timed on the host on a bounded sample
  variants          the same workload with FP16 / BF16 population storage
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
    "riser_crop": lambda: __import__("synth").riser_crop(),
    "riser_large": lambda: __import__("synth").riser_large(),
}
SIZES = {"fp64": (8, 8), "fp32": (4, 4), "fp16": (2, 4), "bf16": (2, 4)}  # (population, scalar) bytes


def algorithmic_bytes(kernel: str, prec: str, C: int, N: int, pairs: int) -> float:
    """Bytes a launch of `kernel` must move at minimum (each operand once)."""
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


def model_bytes_per_step(prec: str, C: int, N: int, pairs: int) -> float:
    """Whole-step byte model: 18 s_f + 16 s_c + 20 per cell, 14 s_p + 16 per
    particle, 16 + 8 s_p per contact pair."""
    sf, st = SIZES[prec]
    return C * (18 * sf + 16 * st + 20) + N * (14 * st + 16) + pairs * (16 + 8 * st)


def run_gpu(cfg, prec, steps, warmup, torch, L, dominant=None):
    sim = L.Sim(cfg, precision=prec)
    stream = sim.stream
    sim.step(warmup)
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
    # timed region: whole steps, with only the dominant kernel bracketed by events
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
    out = dict(ms=ms, breakdown_us=breakdown, dominant=dominant, dom_ms=kt[0], dom_launches=kt[1],
               pairs=counters["pairs"])
    sim.close()
    return out


def cpu_baseline(cfg, seconds):
    import oracle
    sim = oracle.Sim(cfg)
    t0 = time.perf_counter()
    steps = 0
    while True:
        sim.step()
        steps += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    C = cfg["nx"] * cfg["ny"]
    return dict(value=round(C * steps / dt / 1e6, 4), unit="MLUPS", cores=1, kind="oracle",
                sample=f"{cfg['name']}: first {steps} coupled steps from the initial state, FP64, single thread "
                       f"({dt:.1f} s); particle updates/s {len(cfg['pos']) * steps / dt:.3e}")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="bubble", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp32", choices=sorted(SIZES))
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1303_2653_amd import lbdps as L

    torch.cuda.set_device(0)
    cfg = WORKLOADS[args.workload]()
    C, N = cfg["nx"] * cfg["ny"], len(cfg["pos"])
    r = run_gpu(cfg, args.precision, args.steps, args.warmup, torch, L)
    s = r["ms"] / 1e3
    mlups = C * args.steps / s / 1e6
    pups = N * args.steps / s
    dom = r["dominant"]
    dom_us = r["dom_ms"] / max(r["dom_launches"], 1) * 1e3
    dom_bytes = algorithmic_bytes(dom, args.precision, C, N, r["pairs"])
    achieved = dom_bytes / (dom_us * 1e-6) / 1e9
    model = model_bytes_per_step(args.precision, C, N, r["pairs"])
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
        "data": "synthetic (seeded splitmix64 bed, recipe in DESIGN.md)",
        "config": {"workload": cfg["name"], "nx": cfg["nx"], "ny": cfg["ny"], "particles": N,
                   "precision": args.precision, "d_p": cfg["d"], "tau": cfg["tau"]},
        "particle_updates_per_s": float(f"{pups:.4e}"),
        "model_bytes_per_step": int(model),
        "model_bw_frac": round(model * args.steps / s / 1e9 / HBM_PEAK_GBS, 4),
        "contact_pairs": r["pairs"],
        "kernel_us": {k: round(v, 2) for k, v in r["breakdown_us"].items()},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "bytes_per_launch": int(dom_bytes), "us_per_launch": round(dom_us, 3)},
    }
    if not args.no_variants and args.precision == "fp32":
        var = {}
        for p in ("fp16", "bf16"):
            rv = run_gpu(cfg, p, args.steps, args.warmup, torch, L, dominant=dom)
            sv = rv["ms"] / 1e3
            var[p] = {"MLUPS": round(C * args.steps / sv / 1e6, 2), "ms_per_step": round(rv["ms"] / args.steps, 5),
                      "speedup_vs_fp32": round(r["ms"] / rv["ms"], 3)}
        line["variants"] = var
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(cfg, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
