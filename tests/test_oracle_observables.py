"""Pins of the oracle's voidage statistics (the observables of Sec. 3) and of
the paper-faithful workloads' parameters against Tables 1 and 2 (no GPU)."""
import json
import math
import os

import numpy as np
import pytest

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _tables():
    with open(os.path.join(GOLDEN, "paper_tables.json")) as fh:
        return json.load(fh)


def _cfg(**kw):
    c = dict(synth.DEFAULTS)
    c.update(nx=12, ny=10, bc=["wall", "wall", "periodic", "periodic"], pos=np.zeros((0, 2)), vel=np.zeros((0, 2)))
    c.update(kw)
    return c


def _fill(counts):
    """Particle centres realising a [ny][nx] array of per-cell counts."""
    pos = []
    ny, nx = counts.shape
    for j in range(ny):
        for i in range(nx):
            for q in range(counts[j, i]):
                pos.append((i + (q + 0.5) / (counts[j, i] + 1), j + 0.5))
    return np.array(pos, np.float64).reshape(-1, 2)


def test_voidage_rows_columns_and_count(orc):
    """Sec. 3 (R42): each cell's voidage is the Eq. 11 voidage of its count, so a
    lattice whose row j holds j mod 4 particles per cell has row sums
    nx eps_g(j mod 4), column sums over a row window of the window's eps_g, and
    counts the cells above a threshold by their count alone."""
    nx, ny = 12, 10
    counts = np.repeat((np.arange(ny) % 4)[:, None], nx, axis=1)
    p = orc.make_params(_cfg(nx=nx, ny=ny))
    eg = [orc.cell_props(p, k)["eps_g"] for k in range(4)]
    assert eg[0] == 1.0 and eg[1] > eg[2] > eg[3]  # more particles, less gas
    rows, cols, count = orc.voidage(p, _fill(counts), 2, 7, threshold=eg[2])
    assert np.allclose(rows, [nx * eg[j % 4] for j in range(ny)], rtol=1e-15)
    assert np.allclose(cols, sum(eg[j % 4] for j in range(2, 7)), rtol=1e-15)
    # rows 2..6 hold counts 2, 3, 0, 1, 2: eps_g > eps_g(2) for counts 0 and 1
    assert count == 2 * nx
    rows0, cols0, count0 = orc.voidage(p, np.zeros((0, 2)), 0, ny)
    assert (rows0 == nx).all() and (cols0 == ny).all() and count0 == nx * ny


def test_bubble_area_of_a_hole(orc):
    """Sec. 3.1: the equivalent bubble diameter is that of the circle with the
    area of the cells whose voidage exceeds 0.85.  A bed of 16 particles per
    cell (d = 0.2: 2-D solid fraction 0.503, eps_g = 0.784) with an empty disc of
    cells has exactly the disc's cells above 0.85."""
    nx, ny, R = 24, 30, 5.0
    y, x = np.mgrid[0:ny, 0:nx] + 0.5
    hole = (x - 12) ** 2 + (y - 14) ** 2 < R * R
    counts = np.where(hole, 0, 16)
    p = orc.make_params(_cfg(nx=nx, ny=ny, d=0.2))
    assert orc.cell_props(p, 16)["eps_g"] == pytest.approx(0.784, abs=1e-3)
    _, _, count = orc.voidage(p, _fill(counts), 0, ny, threshold=0.85)
    assert count == int(hole.sum())
    assert abs(math.sqrt(4 * count / math.pi) - 2 * R) < 1.0


def test_paper_bubble_at_incipient_fluidization(orc):
    """The Table 1 bed is packed where the drag of Eqs. 19-22 (Eq. 26 per
    sphere) at v_mf carries the spheres' weight: at the bed's mean count per
    cell the ratio of drag to weight lies between 0.8 and 1.25."""
    c = synth.paper_bubble()
    p = orc.make_params(c)
    pos = c["pos"]
    cell = (np.floor(pos[:, 1]) * c["nx"] + np.floor(pos[:, 0])).astype(int)
    counts = np.bincount(cell, minlength=c["nx"] * c["ny"])
    n = int(round(counts[: 23 * c["nx"]].mean()))  # the full rows of the bed
    pr = orc.cell_props(p, n)
    u = min(c["inlet_uy"]) / pr["eps_2"]  # actual gas velocity at the superficial v_mf (R6)
    vp = math.pi * c["d"] ** 3 / 6
    drag = n * vp * orc.beta(p, pr["eps_g"], pr["omega"], u) / (1 - pr["eps_g"]) * u
    weight = n * c["rho_s"] * vp * (1 - 1 / c["rho_s"]) * -c["g"][1]
    assert 0.8 < drag / weight < 1.25, (n, drag / weight)


def test_paper_bubble_parameters():
    """Table 1 in lattice units: the lattice, orifice, particle size and number
    are the dimensionless column; v_mf, the jet, tau and gravity follow from
    the dimensional column with h = 2.7e-4 m and dt = 1.35e-6 s.  The printed
    dimensionless jet (0.04) is ten times its conversion (R31)."""
    t = _tables()["table1"]
    c = synth.paper_bubble()
    h, dt = t["h_m"], t["dt_s"]
    assert (c["nx"], c["ny"]) == (round(t["W_m"] / h), round(t["H_m"] / h)) == (t["W_lu"], t["H_lu"])
    assert len(c["pos"]) == t["N"] and c["d"] == pytest.approx(t["d_p_m"] / h) == t["d_lu"]
    assert c["rho_s"] == t["rho_s_lu"] and abs(t["rho_s"] / t["rho_g"] / t["rho_s_lu"] - 1) < 1e-4
    inlet = np.asarray(c["inlet_uy"])
    jet = inlet > inlet.min()
    assert jet.sum() == round(t["r_inj_m"] / h) == t["r_inj_lu"]
    assert np.flatnonzero(jet).mean() == pytest.approx((c["nx"] - 1) / 2)  # centred
    assert inlet.min() == pytest.approx(t["v_mf_lu"]) == pytest.approx(t["v_mf_ms"] * dt / h)
    assert inlet.max() == pytest.approx(t["v_inj_ms"] * dt / h)
    assert t["v_inj_lu_printed"] == pytest.approx(10 * inlet.max())
    assert np.all(np.asarray(c["inlet_after"]) == inlet.min())
    assert c["pulse_steps"] == int(t["injection_s"] / dt)
    mu_lu = t["mu_g"] * dt / (t["rho_g"] * h * h)
    assert mu_lu == pytest.approx(t["mu_lu"], rel=2e-3)
    assert c["tau"] == pytest.approx(3 * mu_lu + 0.5, rel=1e-15)
    assert c["g"][1] == pytest.approx(-9.81 * dt * dt / h)
    assert c["e_pp"] == t["e"] and c["bc"] == ["wall", "wall", "inlet", "outlet"]
    # no two spheres touch at t = 0
    from scipy.spatial import cKDTree
    dist, _ = cKDTree(c["pos"]).query(c["pos"], 2)
    assert dist[:, 1].min() > c["d"]
    assert c["pos"][:, 0].min() >= c["d"] / 2 and c["pos"][:, 0].max() <= c["nx"] - c["d"] / 2


def test_paper_riser_parameters():
    """Table 2 in lattice units: 60 x 720, 123 921 spheres of d = 0.2 whose 2-D
    solid fraction reproduces the printed 0.09007; tau from the converted
    viscosity (the printed 1.32e-4 is a tenth of it, R31); gas in through the
    bottom at the converted inlet velocity, out through the top; the spheres
    circulate through the y faces (R43, R44)."""
    t = _tables()["table2"]
    c = synth.paper_riser()
    h, dt = t["h_m"], t["dt_s"]
    assert (c["nx"], c["ny"]) == (t["W_lu"], t["H_lu"])
    assert round(t["W_m"] / h) == t["W_lu"] and abs(t["H_m"] / h / t["H_lu"] - 1) < 3e-3  # 0.194 m printed rounded
    n = len(c["pos"])
    assert n == t["N"] and c["d"] == t["d_lu"]
    theta = n * math.pi * c["d"] ** 2 / 4 / (c["nx"] * c["ny"])
    assert theta == pytest.approx(t["theta_s"], rel=1e-3)
    mu_lu = t["mu_g"] * dt / (t["rho_g"] * h * h)
    assert mu_lu == pytest.approx(10 * t["mu_lu_printed"], rel=3e-3)
    assert c["tau"] == pytest.approx(3 * mu_lu + 0.5, rel=1e-15)
    assert c["u0"][1] == pytest.approx(t["v_inlet_ms"] * dt / h) == pytest.approx(t["v_inlet_lu"], rel=1e-3)
    g = 9.81 * dt * dt / h
    assert c["g"][1] == pytest.approx(-g)
    assert c["bc"] == ["wall", "wall", "inlet", "outlet"] and c["particles_periodic_y"] == 1
    assert np.allclose(c["inlet_uy"], c["u0"][1])
    x = c["pos"][:, 0]
    assert x.min() >= c["d"] / 2 and x.max() <= c["nx"] - c["d"] / 2
