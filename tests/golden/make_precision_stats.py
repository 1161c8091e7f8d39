"""Writes tests/golden/precision_riser_crop_stats.json: time-averaged
statistics of the FP64 oracle on the 64x512 riser crop (31 250 spheres), steps
1000-5000 sampled every 10 steps, started from the state the library holds in
its FP32-position modes (equilibrium gas at rest, positions as cell + float32
offset, zero velocities).  Calls the oracle only.

Statistics: column solid area fraction phi(x) (particles with floor(P_x) = x,
times pi d^2 / 4, over ny), mean gas velocity u_y over the cells, mean particle
velocity v_y, and their difference (mean slip).

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


def main():
    cfg = synth.riser_crop()
    f0, pos0, vel0 = storage_repr.state(cfg, oracle.equilibrium_state(cfg["nx"], cfg["ny"]), cfg["pos"],
                                        cfg["vel"], "fp32")
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
    res = dict(workload=cfg["name"], steps=STEPS, start=START, every=EVERY, samples=ns,
               phi_x=(acc_phi / ns).tolist(), mean_uy=acc_uy / ns, mean_vy=acc_vy / ns,
               mean_slip=(acc_uy - acc_vy) / ns,
               note="FP64 oracle; initial positions as cell + float32 offset")
    with open(os.path.join(HERE, "precision_riser_crop_stats.json"), "w") as fh:
        json.dump(res, fh, indent=1)
    print({k: v for k, v in res.items() if k != "phi_x"})


if __name__ == "__main__":
    main()
