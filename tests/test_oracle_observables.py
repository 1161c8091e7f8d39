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


# ---------------------------------------------------------------- outlet solids flux (Sec. 3.2)
def _loop_cfg(**kw):
    """A tiny circulating bed: gas inlet at the bottom, outlet at the top,
    walls at x, particles periodic in y (R44)."""
    return _cfg(nx=12, ny=16, bc=["wall", "wall", "inlet", "outlet"], particles_periodic_y=1,
                inlet_uy=np.full(12, 0.01), g=(0.0, 0.0), **kw)


def test_outlet_crossings_of_a_constructed_bed(orc):
    """R47: the step counts the particles that cross the outlet plane y = ny
    upward, less those that cross it downward (leaving through the bottom of
    a circulating bed).  Five spheres 0.1 below the top moving up at 0.3, two
    0.1 above the bottom moving down at 0.3, and three in mid-bed: net 3, and
    the flux is m 3 / nx per step.  With walls in y the spheres reflect and
    nothing crosses."""
    pos = np.array([[1.5 + 2 * k, 15.9] for k in range(5)] + [[2.5, 0.1], [6.5, 0.1]] +
                   [[3.5, 8.0], [7.5, 8.0], [10.5, 8.0]])
    vel = np.array([[0.0, 0.3]] * 5 + [[0.0, -0.3]] * 2 + [[0.01, 0.0]] * 3)
    cfg = _loop_cfg(pos=pos, vel=vel)
    sim = orc.Sim(cfg)
    o = sim.step(record=True)
    assert o.ncross == 3
    assert (sim.pos[:5, 1] < 1.0).all() and (sim.pos[5:7, 1] > 15.0).all()
    m = cfg["rho_s"] * math.pi * cfg["d"] ** 3 / 6
    assert abs(orc.solids_flux(sim.p, o.ncross, 1) - m * 3 / 12) <= 1e-15 * m
    walls = dict(cfg, particles_periodic_y=0, bc=["wall", "wall", "wall", "wall"])
    sim_w = orc.Sim(walls)
    assert sim_w.step(record=True).ncross == 0 and (sim_w.pos[:, 1] < 16).all() and (sim_w.pos[:, 1] > 0).all()


def test_outlet_crossings_close_the_displacement_balance(orc):
    """R47 against the move itself: over one step of a circulating bed with
    fast random motion, the particles' summed displacement, unwrapped by ny
    for each counted crossing, equals the summed velocity they moved with
    (the previous velocity plus the acceleration of Eq. 16, h = 1)."""
    rng = np.random.default_rng(3)
    n = 300
    pos = np.stack([0.3 + 11.4 * rng.random(n), 16 * rng.random(n)], 1)
    vel = (rng.random((n, 2)) - 0.5) * np.array([0.1, 1.6])
    cfg = _loop_cfg(pos=pos, vel=vel)
    sim = orc.Sim(cfg)
    y0, v0 = sim.pos[:, 1].copy(), sim.vel.copy()
    o = sim.step(record=True)
    moved = (v0[:, 1] + o.acc[:, 1]).sum()
    disp = (sim.pos[:, 1] - y0).sum() + 16 * o.ncross
    assert abs(o.ncross) > 0 and np.abs(sim.pos[:, 1] - y0).max() > 8  # wraps happened
    assert abs(disp - moved) < 1e-12 * n
