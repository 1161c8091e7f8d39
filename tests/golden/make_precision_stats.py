"""Writes tests/golden/precision_riser_crop_stats.json: time-averaged
statistics of the FP64 oracle on the 64x512 riser crop (31 250 spheres), steps
1000-5000 sampled every 10 steps, started from the state the library holds in
its FP32-position modes (equilibrium gas at rest, positions as cell + float32
offset, zero velocities).  Calls the oracle only.

Statistics: column solid area fraction phi(x) (particles with floor(P_x) = x,
times pi d^2 / 4, over ny), mean gas velocity u_y over the cells, mean particle
velocity v_y, and their difference (mean slip).

The particle system is chaotic, so the same statistics are also taken from two
more oracle runs whose initial x positions are moved by +-2^-40 cells
(alternating in sign by particle).  Their largest relative difference from the
reference run is the spread that divergence alone produces ("noise").

    python tests/golden/make_precision_stats.py      (about 2-3 minutes)
"""
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import storage_repr  # noqa: E402
import synth  # noqa: E402

STEPS, START, EVERY = 5000, 1000, 10


def sample(cfg, pos, vel, ugas):
    nx, ny = cfg["nx"], cfg["ny"]
    col = np.bincount(np.floor(pos[:, 0]).astype(np.int64), minlength=nx)[:nx]
    phi = col * (math.pi * cfg["d"] ** 2 / 4) / ny
    uy = float(np.mean(ugas[:, 1]))
    vy = float(np.mean(vel[:, 1]))
    return phi, uy, vy


def run(cfg, f0, pos0, vel0):
    sim = oracle.Sim(cfg, f=f0, pos=pos0, vel=vel0)
    acc_phi, acc_uy, acc_vy, ns = np.zeros(cfg["nx"]), 0.0, 0.0, 0
    t0 = time.time()
    for k in range(1, STEPS + 1):
        rec = k >= START and k % EVERY == 0
        out = sim.step(record=rec)
        if rec:
            phi, uy, vy = sample(cfg, sim.pos, sim.vel, out.ugas)
            acc_phi += phi
            acc_uy += uy
            acc_vy += vy
            ns += 1
        if k % 500 == 0:
            print(f"step {k}  {time.time() - t0:.0f} s", flush=True)
    return dict(samples=ns, phi_x=acc_phi / ns, mean_uy=acc_uy / ns, mean_vy=acc_vy / ns,
                mean_slip=(acc_uy - acc_vy) / ns)


def rel_diff(a, b):
    return dict(phi_x=float(np.abs(a["phi_x"] - b["phi_x"]).max() / b["phi_x"].max()),
                **{k: abs(a[k] - b[k]) / abs(b[k]) for k in ("mean_uy", "mean_vy", "mean_slip")})


def main():
    cfg = synth.riser_crop()
    f0, pos0, vel0 = storage_repr.state(cfg, oracle.equilibrium_state(cfg["nx"], cfg["ny"]), cfg["pos"],
                                        cfg["vel"], "fp32")
    ref = run(cfg, f0, pos0, vel0)
    noise = {k: 0.0 for k in ("phi_x", "mean_uy", "mean_vy", "mean_slip")}
    sign = np.where(np.arange(len(pos0)) % 2 == 0, 1.0, -1.0)
    for j in (1, 2):
        pj = pos0.copy()
        pj[:, 0] += (-1) ** j * sign * 2.0 ** -40
        d = rel_diff(run(cfg, f0, pj, vel0), ref)
        print("perturbed run", j, d, flush=True)
        noise = {k: max(noise[k], d[k]) for k in noise}
    res = dict(workload=cfg["name"], steps=STEPS, start=START, every=EVERY, samples=ref["samples"],
               phi_x=ref["phi_x"].tolist(), mean_uy=ref["mean_uy"], mean_vy=ref["mean_vy"],
               mean_slip=ref["mean_slip"], noise=noise,
               note="FP64 oracle; initial positions as cell + float32 offset; noise = largest relative "
                    "difference of two runs with x moved by +-2^-40")
    with open(os.path.join(HERE, "precision_riser_crop_stats.json"), "w") as fh:
        json.dump(res, fh, indent=1)
    print({k: v for k, v in res.items() if k != "phi_x"})


if __name__ == "__main__":
    main()
