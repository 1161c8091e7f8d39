"""Pins of the oracle's 3-D coupled step (the procedure of Sec. 2.4 on a
periodic D3Q19 box with spheres, R48): the particle-free limit, the two-phase
relaxation closed form, Newton's third law per cell, momentum bookkeeping,
trilinear interpolation, the 27-cell contact search against brute force, and
the two-sphere collision laws in 3-D (no GPU)."""
import math

import numpy as np
import pytest

import synth


def _p(orc, **kw):
    return orc.make_params3(synth.tiny3d(**kw))


def test_cell_props_3d(orc):
    """R45/R48: the solid fraction of n spheres is n pi d^3 / 6, held at the
    densest sphere packing pi / (3 sqrt 2); gamma is Eq. 9 there and omega
    Eq. 20 at the voidage (dense branch: omega_dense)."""
    p = _p(orc)
    one = orc.cell_props3(p, 1)
    assert abs(one["eps_s"] - math.pi / 48) < 1e-16 and abs(one["eps_g"] - (1 - math.pi / 48)) < 1e-16
    assert one["gamma"] == orc.gamma(math.pi / 48, 0.6)
    assert one["omega"] == orc.omega_emms(1 - math.pi / 48)
    big = orc.cell_props3(p, 40)
    assert abs(big["eps_s"] - math.pi / (3 * math.sqrt(2))) < 1e-15 and big["omega"] == 1.0
    assert orc.cell_props3(p, 0)["gamma"] == 0.0


def test_no_particles_is_the_3d_bgk_step(orc):
    """Without spheres (gamma = 0) the coupled step is the D3Q19 BGK step of
    the gas lattice, to rounding (the relaxation is written (1 - gamma) / tau
    instead of 1 / tau)."""
    cfg = synth.tiny3d(n=0, g=(0.0, 0.0, 0.0))
    rng = np.random.default_rng(1)
    f0 = orc.equilibrium_state3(6, 5, 7) * (1 + 0.01 * rng.random((19, 7, 5, 6)))
    sim = orc.Sim3(cfg, f=f0, pos=np.zeros((0, 3)), vel=np.zeros((0, 3)))
    for _ in range(3):
        sim.step()
    ref = f0.copy()
    for _ in range(3):
        ref = orc.bgk3_step(ref, 0.6)
    assert np.abs(sim.f - ref).max() <= 1e-15 * np.abs(ref).max()


def test_uniform_two_phase_relaxation_3d(orc):
    """Whole 3-D step, closed form: one sphere at every cell centre with the
    same velocity v0, gas uniform at u0, no gravity or body force.  There are
    no contacts (spacing 1 > d), grad p = 0, interpolation returns the node
    value, and with F_pg = omega gamma rho (v_s - u) (Eq. 25) and F_d = -F_pg
    (Eq. 28) the slip w = u - v obeys w_n = w_0 (1 - omega gamma (1 + rho/m))^n
    while rho u + m v stays constant."""
    nx, ny, nz = 4, 3, 5
    z, y, x = np.mgrid[0:nz, 0:ny, 0:nx] + 0.5
    pos = np.stack([x.ravel(), y.ravel(), z.ravel()], 1)
    v0, u0 = np.array([2e-3, -1e-3, 3e-3]), np.array([-1e-3, 2e-3, 5e-4])
    cfg = synth.tiny3d(nx=nx, ny=ny, nz=nz, n=len(pos), g=(0.0, 0.0, 0.0))
    f0 = orc.equilibrium_state3(nx, ny, nz, 1.0, u0)
    sim = orc.Sim3(cfg, f=f0, pos=pos, vel=np.tile(v0, (len(pos), 1)))
    pr = orc.cell_props3(sim.p, 1)
    og = pr["omega"] * pr["gamma"]
    m = cfg["rho_s"] * math.pi * cfg["d"] ** 3 / 6
    w0 = u0 - v0
    for n in range(1, 6):
        o = sim.step(record=True)
        assert len(o.pairs) == 0
        v = sim.vel
        assert np.abs(v - v[0]).max() < 1e-18
        u_now = np.array([(sim.f * orc.lattice3()[0][:, a].reshape(19, 1, 1, 1)).sum(0).mean() for a in range(3)])
        w = u_now - v[0]
        want = w0 * (1 - og * (1 + 1.0 / m)) ** n
        assert np.abs(w - want).max() < 1e-13 * np.abs(w0).max(), (n, w, want)
        assert np.abs(u_now + m * v[0] - (u0 + m * v0)).max() < 1e-15


def test_newton_third_law_and_momentum_3d(orc):
    """Eq. 28 (signed, R15): in every cell the particles' drags sum to -F_pg
    (Eq. 29); with no gravity or body force the gas and particle momentum of
    the periodic box is conserved to roundoff over steps with collisions (the
    pressure-gradient force of Eq. 16 off: the gas takes no reaction to it),
    and with them it grows by steps (N m g_eff + C G)."""
    cfg = synth.tiny3d(nx=6, ny=5, nz=7, n=400, seed=3, vel_scale=5e-3, g=(0.0, 0.0, 0.0), pressure_sign=0)
    sim = orc.Sim3(cfg)
    c0 = sim.conservation()
    seen_pairs = 0
    for _ in range(6):
        o = sim.step(record=True)
        seen_pairs += len(o.pairs)
        cells = None
    assert seen_pairs > 20
    c1 = sim.conservation()
    assert abs(c1[0] - c0[0]) < 1e-12 * c0[0]
    tot0, tot1 = c0[1:4] + c0[4:7], c1[1:4] + c1[4:7]
    assert np.abs(tot1 - tot0).max() < 1e-13 * max(np.abs(c0[4:7]).max(), 1e-30)
    # Newton's third law per cell, checked on the last step's outputs
    pos_before = None
    sim2 = orc.Sim3(cfg)
    pos_before = sim2.pos.copy()
    o = sim2.step(record=True)
    key = ((np.floor(pos_before[:, 2]) * 5 + np.floor(pos_before[:, 1])) * 6 + np.floor(pos_before[:, 0])).astype(int)
    sums = np.zeros((6 * 5 * 7, 3))
    np.add.at(sums, key, o.fd)
    fpg = o.fpg.reshape(-1, 3)
    occupied = o.ncell.reshape(-1) > 0
    assert np.abs(sums[occupied] + fpg[occupied]).max() <= 1e-14 * np.abs(fpg).max()
    # bookkeeping with gravity and a body force
    g, G = (1e-6, -2e-6, -3e-6), (4e-6, 0.0, 1e-6)
    cfgg = dict(cfg, g=g, G=G, pressure_sign=0)
    simg = orc.Sim3(cfgg)
    b0 = simg.conservation()
    for _ in range(5):
        simg.step()
    b1 = simg.conservation()
    m = cfg["rho_s"] * math.pi * cfg["d"] ** 3 / 6
    geff = (1 - cfg["rho_g"] / cfg["rho_s"]) * np.array(g)
    want = 5 * (400 * m * geff + 210 * np.array(G))
    got = (b1[1:4] + b1[4:7]) - (b0[1:4] + b0[4:7])
    assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()


def test_trilinear_interpolation(orc):
    """Trilinear weights sum to 1, a particle at a node centre gets the node
    value, and affine fields are reproduced exactly (periodic box, away from
    the seam)."""
    nx, ny, nz = 5, 4, 6
    p = _p(orc, nx=nx, ny=ny, nz=nz)
    z, y, x = np.mgrid[0:nz, 0:ny, 0:nx] + 0.5
    q = 0.2 + 0.7 * x - 1.1 * y + 0.3 * z
    rng = np.random.default_rng(4)
    for _ in range(200):
        P = np.array([0.5 + (nx - 1) * rng.random(), 0.5 + (ny - 1) * rng.random(), 0.5 + (nz - 1) * rng.random()])
        idx, wt = orc.stencil3(p, P)
        assert abs(wt.sum() - 1) < 1e-15 and (wt >= 0).all()
        assert abs(orc.interp3(p, q, P) - (0.2 + 0.7 * P[0] - 1.1 * P[1] + 0.3 * P[2])) < 1e-13
    r = rng.random((nz, ny, nx))
    for (k, j, i) in [(0, 0, 0), (5, 3, 4), (2, 1, 3)]:
        assert orc.interp3(p, r, np.array([i + 0.5, j + 0.5, k + 0.5])) == r[k, j, i]
    # across the periodic seam: halfway between the last and the first node
    assert abs(orc.interp3(p, r, np.array([0.0, 0.5, 0.5])) - 0.5 * (r[0, 0, 0] + r[0, 0, nx - 1])) < 1e-15


@pytest.mark.parametrize("shape", [(6, 5, 7), (3, 4, 3), (9, 8, 10)])
def test_contacts_27_cells_equal_brute_force(orc, shape):
    """The 27-cell search finds exactly the brute-force O(N^2) pair set, with
    the periodic minimum image on all three axes (boxes of three cells
    included, where neighbour cells repeat) and exact ties |r|^2 = d^2."""
    nx, ny, nz = shape
    n = 3 * nx * ny * nz
    cfg = synth.tiny3d(nx=nx, ny=ny, nz=nz, n=n, seed=11)
    p = orc.make_params3(cfg)
    pos = cfg["pos"].copy()
    pos[1] = pos[0] + np.array([0.5, 0.0, 0.0])  # a tie at exactly d
    pos[1] %= np.array([nx, ny, nz])
    a = orc.contacts3(p, pos, brute=True)
    b = orc.contacts3(p, pos)
    assert len(a) > n // 5 and (a == b).all()
    assert (a[:, 0] < a[:, 1]).all() and np.all(np.diff(a[:, 0] * n + a[:, 1]) > 0)
    assert any((r == [0, 1]).all() for r in a)


@pytest.mark.parametrize("e", [0.0, 0.9, 1.0])
def test_two_sphere_collision_3d(orc, e):
    """Eqs. 17-18 in 3-D: the normal relative velocity becomes -e times itself,
    the tangential part is unchanged, momentum is conserved; separating
    spheres are left alone."""
    p = _p(orc, e_pp=e)
    pos = np.array([[2.0, 2.0, 2.0], [2.3, 2.2, 1.9]])
    for v1, v2 in [((0.01, 0.0, 0.02), (-0.02, -0.01, 0.0)), ((0.0, 0.0, 0.01), (0.0, 0.0, -0.01)),
                   ((-0.01, -0.01, 0.0), (0.01, 0.01, 0.0))]:
        vel = np.array([v1, v2])
        out, nc = orc.resolve3(p, pos, vel, np.array([[0, 1]], np.int32))
        d = pos[0] - pos[1]
        nvec = d / np.linalg.norm(d)
        r0, r1 = vel[0] - vel[1], out[0] - out[1]
        if r0 @ nvec >= 0:
            assert nc == 0 and (out == vel).all()
            continue
        assert nc == 1
        assert abs(r1 @ nvec + e * (r0 @ nvec)) < 1e-16
        t0, t1 = r0 - (r0 @ nvec) * nvec, r1 - (r1 @ nvec) * nvec
        assert np.abs(t1 - t0).max() < 1e-16
        assert np.abs(out.sum(0) - vel.sum(0)).max() < 1e-17
