"""Pins of the oracle's particle side: interpolation, integration, contacts,
collisions, walls, drag correction and the whole coupled step (no GPU)."""
import math

import numpy as np
import pytest

import synth


def _cfg(**kw):
    c = dict(synth.DEFAULTS)
    c.update(nx=8, ny=8, bc=["periodic"] * 4, pos=np.zeros((0, 2)), vel=np.zeros((0, 2)))
    c.update(kw)
    return c


# ---------------------------------------------------------------- interpolation
def test_bilinear_interpolation(orc):
    """Sec. 2.3 after Eq. 26 (R11): bilinear weights sum to 1, a particle at a
    node centre returns the node value, and affine fields are reproduced exactly
    away from clamped walls."""
    nx, ny = 9, 7
    p = orc.make_params(_cfg(nx=nx, ny=ny, bc=["wall", "wall", "inlet", "outlet"]))
    y, x = np.mgrid[0:ny, 0:nx] + 0.5
    q = 0.3 + 0.7 * x - 1.1 * y
    rng = np.random.default_rng(2)
    for _ in range(200):
        px, py = 0.5 + (nx - 1) * rng.random(), 0.5 + (ny - 1) * rng.random()
        idx, wt = orc.stencil(p, px, py)
        assert abs(wt.sum() - 1) < 1e-15 and (wt >= 0).all()
        assert abs(orc.interp(p, q, px, py) - (0.3 + 0.7 * px - 1.1 * py)) < 1e-13
    r = rng.random((ny, nx))
    for j in range(ny):
        for i in range(nx):
            assert orc.interp(p, r, i + 0.5, j + 0.5) == r[j, i]
    # own cell's node always in the stencil with weight >= 1/4 (R11)
    for _ in range(200):
        px, py = nx * rng.random(), ny * rng.random()
        idx, wt = orc.stencil(p, px, py)
        own = int(py) * nx + int(px)
        assert wt[idx == own].sum() >= 0.25 - 1e-15


def test_pressure_gradient_stencil(orc):
    """R17: central differences of p reproduce a linear field's gradient in the
    interior; at a non-periodic face the ghost equals the boundary value, so the
    boundary node gets (p1 - p0)/2."""
    nx, ny = 6, 5
    p = orc.make_params(_cfg(nx=nx, ny=ny, bc=["wall", "wall", "wall", "wall"]))
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    pres = 2.0 + 0.25 * x - 0.5 * y
    g = orc.grad_p(p, pres).reshape(ny, nx, 2)
    assert np.allclose(g[1:-1, 1:-1, 0], 0.25) and np.allclose(g[1:-1, 1:-1, 1], -0.5)
    assert np.allclose(g[:, 0, 0], 0.125) and np.allclose(g[:, -1, 0], 0.125)
    assert np.allclose(g[0, :, 1], -0.25) and np.allclose(g[-1, :, 1], -0.25)
    pp = orc.make_params(_cfg(nx=nx, ny=ny))
    gper = orc.grad_p(pp, np.sin(2 * np.pi * x / nx)).reshape(ny, nx, 2)
    want = (np.sin(2 * np.pi * (x + 1) / nx) - np.sin(2 * np.pi * (x - 1) / nx)) / 2
    assert np.allclose(gper[..., 0], want, atol=1e-15)


# ---------------------------------------------------------------- integrator
def test_free_particle_integration(orc):
    """Eq. 16 with no drag and no pressure force, symplectic Euler with unit
    step (R18): v_n = v0 + n a, P_n = P0 + n v0 + a n(n+1)/2, with the effective
    gravity (1 - rho_g/rho_s) g of Sec. 3."""
    nx, ny = 400, 400
    p = orc.make_params(_cfg(nx=nx, ny=ny, bc=["periodic"] * 4, g=(2e-4, -3e-4)))
    a = (1 - p.rho_g / p.rho_s) * np.array([2e-4, -3e-4])
    pos0 = np.array([[100.25, 300.5]])
    vel0 = np.array([[0.01, 0.02]])
    pos, vel = pos0.copy(), vel0.copy()
    z = np.zeros((1, 2))
    for _ in range(50):
        pos, vel = orc.integrate(p, pos, vel, z, z)
    n = 50
    assert np.allclose(vel, vel0 + n * a, rtol=0, atol=1e-15)
    assert np.allclose(pos, pos0 + n * vel0 + a * n * (n + 1) / 2, rtol=0, atol=1e-12)


def test_wrap_and_mirror(orc):
    """Periodic wrap (R26) and mirror at a wall plane (R23)."""
    p = orc.make_params(_cfg(nx=10, ny=10, bc=["wall", "wall", "periodic", "periodic"], g=(0, 0)))
    z = np.zeros((2, 2))
    pos = np.array([[0.2, 9.9], [9.7, 0.1]])
    vel = np.array([[-0.5, 0.3], [0.6, -0.3]])
    pos1, vel1 = orc.integrate(p, pos, vel, z, z)
    assert np.allclose(pos1[0], [0.3, 0.2], atol=1e-14)   # x mirrored, y wrapped
    assert np.allclose(pos1[1], [9.7, 9.8], atol=1e-14)
    assert (vel1 == vel).all()  # mirroring moves the centre only; the wall collision flips v


# ---------------------------------------------------------------- contacts
def _brute_numpy(pos, d, nx, ny, per_x, per_y):
    out = []
    for i in range(len(pos)):
        for j in range(i + 1, len(pos)):
            dx, dy = pos[i] - pos[j]
            if per_x:
                dx -= nx * round(dx / nx) if abs(dx) > nx / 2 else 0
            if per_y:
                dy -= ny * round(dy / ny) if abs(dy) > ny / 2 else 0
            if dx * dx + dy * dy <= d * d:
                out.append((i, j))
    return np.array(out, np.int32).reshape(-1, 2)


@pytest.mark.parametrize("bc,ppy", [(("periodic",) * 4, 0), (("wall", "wall", "periodic", "periodic"), 0),
                                    (("periodic", "periodic", "inlet", "outlet"), 0), (("wall",) * 4, 0),
                                    (("wall", "wall", "inlet", "outlet"), 1)])
def test_contacts_cells_equal_brute(orc, bc, ppy):
    """Sec. 2.2 contact set: the 3x3-cell search returns exactly the O(N^2) set,
    with periodic minimum images and exact ties (distance == d) included (R25);
    with particles periodic in y over an inlet and an outlet (R44) the image
    across the y faces counts too."""
    cfg = synth.tiny(nx=7, ny=6, n=90, seed=11, bc=bc, particles_periodic_y=ppy)
    pos = cfg["pos"].copy()
    # plant exact ties and a wrap-around pair
    pos[0] = (1.0, 1.0)
    pos[1] = (1.5, 1.0)
    pos[2] = (3.0, 2.5)
    pos[3] = (3.0, 3.0)
    pos[4] = (0.1, 4.0)
    pos[5] = (6.8, 4.1)
    p = orc.make_params(cfg)
    a = orc.contacts(p, pos, brute=True)
    b = orc.contacts(p, pos, brute=False)
    c = _brute_numpy(pos, p.d, p.nx, p.ny, bc[0] == "periodic", bc[2] == "periodic" or ppy == 1)
    assert a.shape == c.shape and (a == c).all()
    assert (a == b).all()
    assert {(0, 1), (2, 3)} <= set(map(tuple, a.tolist()))
    assert ((4, 5) in set(map(tuple, a.tolist()))) == (bc[0] == "periodic")
    # a pair touching only through the y faces
    pos[6], pos[7] = (5.0, 0.1), (5.2, 5.9)
    pairs = set(map(tuple, orc.contacts(p, pos).tolist()))
    assert ((6, 7) in pairs) == (bc[2] == "periodic" or ppy == 1)


@pytest.mark.slow
def test_contacts_full_bubble_small(orc):
    """The whole 2000-particle initial bed: cell search == brute force."""
    cfg = synth.bubble_small()
    p = orc.make_params(cfg)
    a = orc.contacts(p, cfg["pos"], brute=True)
    b = orc.contacts(p, cfg["pos"], brute=False)
    assert len(a) > 1000 and (a == b).all()


def test_contacts_f32(orc):
    """Single-precision predicate on a cell + offset state (R25, R27): cell search
    == brute force, and it agrees with the FP64 set on the same positions except
    for pairs whose distance is within float rounding of d."""
    rng = np.random.default_rng(4)
    nx, ny, n = 9, 8, 150
    cell = np.stack([rng.integers(0, nx, n), rng.integers(0, ny, n)], 1).astype(np.int32)
    off = rng.random((n, 2)).astype(np.float32)
    a = orc.contacts_f32(nx, ny, 1, 0, 0.5, cell, off, brute=True)
    b = orc.contacts_f32(nx, ny, 1, 0, 0.5, cell, off, brute=False)
    assert (a == b).all() and len(a) > 10
    pos = cell.astype(np.float64) + off.astype(np.float64)
    p = orc.make_params(_cfg(nx=nx, ny=ny, bc=["periodic", "periodic", "wall", "wall"]))
    c = orc.contacts(p, pos, brute=True)
    sa, sc = set(map(tuple, a.tolist())), set(map(tuple, c.tolist()))
    for i, j in sa ^ sc:
        dx, dy = pos[i] - pos[j]
        dx -= nx * round(dx / nx)
        assert abs(math.hypot(dx, dy) - 0.5) < 1e-6


# ---------------------------------------------------------------- collisions
def _two(orc, e, v1, v2, P1=(2.0, 2.0), P2=(2.4, 2.3)):
    p = orc.make_params(_cfg(nx=8, ny=8, e_pp=e))
    pos = np.array([P1, P2])
    vel = np.array([v1, v2], float)
    out, nc = orc.resolve(p, pos, vel, np.array([[0, 1]], np.int32))
    return p, pos, vel, out, nc


@pytest.mark.parametrize("e", [0.0, 0.5, 0.9, 1.0])
def test_two_sphere_collision(orc, e):
    """Eqs. 17-18: momentum is conserved, the normal relative velocity becomes
    -e times itself, the tangential part is unchanged, and the kinetic energy
    drops by mu_red (1 - e^2) v_n^2 / 2."""
    for v1, v2 in [((0.3, 0.1), (-0.2, -0.05)), ((0.01, 0.0), (0.0, 0.0)), ((0.0, 0.2), (0.1, -0.4))]:
        p, pos, vel, out, nc = _two(orc, e, v1, v2)
        nvec = (pos[0] - pos[1]) / np.linalg.norm(pos[0] - pos[1])
        t = np.array([-nvec[1], nvec[0]])
        rel0, rel1 = vel[0] - vel[1], out[0] - out[1]
        if rel0 @ nvec >= 0:
            assert nc == 0 and (out == vel).all()
            continue
        assert nc == 1
        assert np.allclose(out.sum(0), vel.sum(0), atol=1e-16)
        assert abs(rel1 @ nvec + e * (rel0 @ nvec)) < 1e-15
        assert abs(rel1 @ t - rel0 @ t) < 1e-15
        m = 1.0
        ke0 = 0.5 * m * (vel ** 2).sum()
        ke1 = 0.5 * m * (out ** 2).sum()
        assert abs((ke0 - ke1) - 0.5 * (m / 2) * (1 - e * e) * (rel0 @ nvec) ** 2) < 1e-15


def test_head_on_restitution(orc):
    """Head-on equal spheres: velocities (u, 0) and (-u, 0) leave as (-e u, 0)
    and (e u, 0) (Eqs. 17-18, the restitution coefficient as the speed ratio)."""
    p, pos, vel, out, nc = _two(orc, 0.9, (0.02, 0.0), (-0.02, 0.0), P1=(2.0, 2.0), P2=(2.45, 2.0))
    assert np.allclose(out, [[-0.018, 0.0], [0.018, 0.0]], atol=1e-17)


def test_separating_overlap_untouched(orc):
    """Sec. 2.2: overlapping particles that move apart do not collide."""
    p, pos, vel, out, nc = _two(orc, 0.9, (-0.02, 0.0), (0.02, 0.0), P1=(2.0, 2.0), P2=(2.45, 2.0))
    assert nc == 0 and (out == vel).all()


def test_wall_collision(orc):
    """Sec. 2.2 (walls as infinitely heavy particles) and R23: within r of a wall
    and moving into it, v_n -> -e_w v_n; tangential unchanged; moving away untouched."""
    p = orc.make_params(_cfg(nx=10, ny=10, bc=["wall"] * 4, e_pw=0.7))
    pos = np.array([[0.2, 5.0], [9.9, 5.0], [5.0, 0.25], [5.0, 9.8], [0.2, 5.0], [5.0, 5.0]])
    vel = np.array([[-0.1, 0.3], [0.2, 0.1], [0.05, -0.4], [0.0, 0.3], [0.1, 0.0], [-1.0, -1.0]])
    out, nw = orc.walls(p, pos, vel)
    want = vel.copy()
    want[0, 0] *= -0.7
    want[1, 0] *= -0.7
    want[2, 1] *= -0.7
    want[3, 1] *= -0.7
    assert nw == 4 and np.allclose(out, want, atol=0)


def _levels_schedule(orc, p, pos, vel, pairs, reverse_within_level=True):
    """Resolve the pairs by dependency level: a pair's predecessors are the
    previous pair (in list order) of each of its two particles.  Pairs of one
    level touch disjoint particles, so any order inside a level is valid."""
    last = {}
    level = np.zeros(len(pairs), int)
    for q, (i, j) in enumerate(pairs):
        level[q] = 1 + max(last.get(i, -1), last.get(j, -1))
        last[i] = last[j] = level[q]
    v = vel.copy()
    for L in range(level.max() + 1 if len(pairs) else 0):
        qs = np.nonzero(level == L)[0]
        if reverse_within_level:
            qs = qs[::-1]
        for q in qs:
            v, _ = orc.resolve(p, pos, v, pairs[q:q + 1])
    return v, level.max() + 1 if len(pairs) else 0


def test_collision_order_schedules_agree(orc):
    """R24 fixes the order as sequential over the lexicographic pair list.  Any
    schedule that keeps each particle's own pairs in that order gives the same
    result bit for bit, because a pair only reads and writes its two particles.
    Here: dependency levels, each level in reverse, against the sequential sweep."""
    cfg = synth.bubble_small()
    p = orc.make_params(cfg)
    pos = cfg["pos"]
    rng = np.random.default_rng(8)
    vel = (rng.random(pos.shape) - 0.5) * 1e-3
    pairs = orc.contacts(p, pos)
    seq, nc = orc.resolve(p, pos, vel, pairs)
    lev, depth = _levels_schedule(orc, p, pos, vel, pairs)
    assert nc > 100 and depth > 1
    assert (seq == lev).all()


# ---------------------------------------------------------------- coupled step
def test_uniform_two_phase_relaxation(orc):
    """Whole step, closed form (A1-A5 together).  Periodic lattice, one particle
    at every cell centre with the same velocity v0, gas uniform at u0, no
    gravity or body force: no contacts (spacing 1 > d), grad p = 0, and per cell
    F_p->g = omega gamma rho (v - u) (Eq. 25), F_d = -F_p->g (Eq. 28 with one
    particle).  Hence the slip w = u - v obeys w_n = w0 (1 - omega gamma (1 + rho/m))^n
    and rho u + m v stays constant."""
    nx = ny = 6
    y, x = np.mgrid[0:ny, 0:nx] + 0.5
    pos = np.stack([x.ravel(), y.ravel()], 1)
    v0, u0 = np.array([1e-3, -2e-3]), np.array([-1e-3, 5e-4])
    cfg = _cfg(nx=nx, ny=ny, pos=pos, vel=np.tile(v0, (len(pos), 1)), g=(0.0, 0.0))
    f = orc.equilibrium_state(nx, ny, 1.0, *u0)
    sim = orc.Sim(cfg, f=f)
    pr = orc.cell_props(sim.p, 1)
    og = pr["omega"] * pr["gamma"]
    m = sim.p.rho_s * math.pi * sim.p.d ** 3 / 6
    r = 1 - og * (1 + 1.0 / m)
    c, _, _ = orc.lattice()
    for n in range(1, 41):
        sim.step()
        j = np.einsum("ia,iyx->yxa", c.astype(float), sim.f)
        rho = sim.f.sum(0)
        u = j / rho[..., None]
        w = u.reshape(-1, 2) - sim.vel
        assert np.allclose(w, (u0 - v0) * r ** n, rtol=1e-11, atol=1e-18)
        mom = rho[..., None].reshape(-1, 1) * u.reshape(-1, 2) + m * sim.vel
        assert np.allclose(mom, u0 + m * v0, rtol=1e-13)


def test_drag_correction_newton3(orc):
    """Eqs. 27-29 (SIGNED reading R15): in every cell the corrected drags sum to
    -F_p->g, and inside a cell F_d,k is proportional to F^pre_k."""
    cfg = synth.tiny(nx=10, ny=12, n=160, seed=21, vel_scale=2e-3, band=8.0)
    sim = orc.Sim(cfg)
    sim.step()  # develop a flow first
    pos0, vel0 = sim.pos.copy(), sim.vel.copy()
    o = sim.step(record=True)
    cell = (np.floor(pos0[:, 1]) * cfg["nx"] + np.floor(pos0[:, 0])).astype(int)
    tot = np.zeros((cfg["nx"] * cfg["ny"], 2))
    np.add.at(tot, cell, o.fd)
    fpg = o.fpg.reshape(-1, 2)
    occupied = np.bincount(cell, minlength=len(tot)) > 0
    scale = np.abs(fpg).max()
    assert np.abs(tot[occupied] + fpg[occupied]).max() < 1e-12 * scale
    assert np.abs(fpg[~occupied]).max() == 0.0


def test_momentum_bookkeeping(orc):
    """Periodic bed, SIGNED Eq. 28, pressure force off: gas + particle momentum is
    conserved to roundoff; with gravity g and gas body force G it grows by
    steps * (N m g_eff + C G) exactly (contacts and walls conserve it), with
    one or three particle sub-steps per lattice step (R41)."""
    for g, G, nsub in (((0.0, 0.0), (0.0, 0.0), 1), ((0.0, -1e-5), (2e-6, 3e-6), 1),
                       ((0.0, -1e-5), (2e-6, 3e-6), 3)):
        cfg = synth.tiny(nx=12, ny=12, n=120, seed=5, bc=("periodic",) * 4, vel_scale=2e-3,
                         pressure_sign=0, g=g, G=G, n_sub=nsub)
        sim = orc.Sim(cfg)
        c0 = sim.conservation()
        steps = 25
        sim.run(steps)
        c1 = sim.conservation()
        m = sim.p.rho_s * math.pi * sim.p.d ** 3 / 6
        geff = (1 - sim.p.rho_g / sim.p.rho_s) * np.array(g)
        want = steps * (len(sim.pos) * m * geff + 144 * np.array(G))
        got = (c1[1:3] + c1[3:5]) - (c0[1:3] + c0[3:5])
        assert np.allclose(got, want, rtol=1e-9, atol=1e-13)


def test_deposition_counts_and_means(orc):
    """Step 2 of Sec. 2.4 (Eq. 8): n_tot per cell equals a histogram of the
    particle cells and v_s the mean of their velocities, summed in index order."""
    cfg = synth.tiny(nx=9, ny=9, n=200, seed=3, vel_scale=1e-2)
    sim = orc.Sim(cfg)
    pos, vel = sim.pos.copy(), sim.vel.copy()
    o = sim.step(record=True)
    cell = (np.floor(pos[:, 1]) * 9 + np.floor(pos[:, 0])).astype(int)
    assert (o.ncell.ravel() == np.bincount(cell, minlength=81)).all()
    want = np.zeros((81, 2))
    for k in range(len(pos)):
        want[cell[k]] += vel[k]
    cnt = np.bincount(cell, minlength=81)
    want[cnt > 0] /= cnt[cnt > 0, None]
    assert (o.vs.reshape(-1, 2) == want).all()


# ---------------------------------------------------------------- sub-steps (R41)
@pytest.mark.parametrize("nsub", [2, 3, 8])
def test_substep_free_flight(orc, nsub):
    """R41: the accelerations of Eq. 16 are held over the lattice step, so n
    symplectic Euler sub-steps of h = 1/n leave the velocity at v0 + a (as one
    step does) and move the particle by v0 + a (n + 1) / (2 n).  The same state
    stepped once with n = 1 gives a = v1 - v0; dilute periodic bed, no walls or
    contacts (the largest speed keeps every pair apart)."""
    rng = np.random.default_rng(8)
    y, x = np.mgrid[0:6, 0:6] * 2.0 + 1.0
    pos = np.stack([x.ravel(), y.ravel()], 1) + (rng.random((36, 2)) - 0.5) * 0.4
    vel = (rng.random((36, 2)) - 0.5) * 4e-3
    cfg = _cfg(nx=12, ny=12, pos=pos, vel=vel, g=(0.0, -1e-5), G=(1e-6, 2e-6))
    one = orc.Sim(cfg)
    one.run(3)  # develop a flow
    f, pos0, vel0 = one.f.copy(), one.pos.copy(), one.vel.copy()
    o1 = one.step(record=True)
    assert len(o1.pairs) == 0
    a = one.vel - vel0
    sub = orc.Sim(dict(cfg, n_sub=nsub), f=f, pos=pos0, vel=vel0)
    on = sub.step(record=True)
    assert len(on.pairs) == 0 and on.nwall == 0
    assert np.array_equal(on.fd, o1.fd)  # forces from the state at the start of the step
    assert np.allclose(sub.vel, one.vel, rtol=0, atol=1e-15)
    want = pos0 + vel0 + a * (nsub + 1) / (2 * nsub)
    dx = (sub.pos - want + 6.0) % 12.0 - 6.0
    assert np.abs(dx).max() < 1e-13
    assert np.abs(a).max() > 1e-7  # the test has an acceleration to integrate
    # n = 1 is the plain step, bit for bit
    same = orc.Sim(dict(cfg, n_sub=1), f=f, pos=pos0, vel=vel0)
    same.step()
    assert np.array_equal(same.pos, one.pos) and np.array_equal(same.vel, one.vel)


@pytest.mark.parametrize("nsub", [1, 2, 4, 7, 8])
def test_substep_collision_time(orc, nsub):
    """R41 with Eqs. 17-18: two equal spheres approach head-on at 0.3 each, one
    cell apart (d = 0.5, e = 1).  Contacts are tested after every sub-step, so
    the collision happens at the first sub-step k whose separation
    1 - 0.6 k h is at most d, the velocities swap there and the spheres recede
    for the remaining sub-steps.  A huge solid density makes the gas forces on
    the spheres negligible (below 1e-12 per step)."""
    h = 1.0 / nsub
    k = next(j for j in range(1, nsub + 1) if 1.0 - 0.6 * j * h <= 0.5)
    xa = 4.0 + 0.3 * k * h - 0.3 * (nsub - k) * h
    xb = 5.0 - 0.3 * k * h + 0.3 * (nsub - k) * h
    pos = np.array([[4.0, 8.2], [5.0, 8.2]])
    vel = np.array([[0.3, 0.0], [-0.3, 0.0]])
    cfg = _cfg(nx=16, ny=16, pos=pos, vel=vel, d=0.5, e_pp=1.0, rho_s=1e12, g=(0.0, 0.0), n_sub=nsub)
    sim = orc.Sim(cfg)
    o = sim.step(record=True)
    assert np.allclose(sim.pos[:, 0], [xa, xb], rtol=0, atol=1e-11)
    assert np.allclose(sim.pos[:, 1], 8.2, rtol=0, atol=1e-11)
    assert np.allclose(sim.vel, [[-0.3, 0.0], [0.3, 0.0]], rtol=0, atol=1e-11)
    # the counters describe the last sub-step: the collision is counted only if it fell there
    assert o.ncollisions == (1 if k == nsub else 0)



def test_circulating_loop_wraps_particles_not_gas(orc):
    """R44: with the particles periodic in y over an inlet and an outlet, a
    sphere rising through the top re-enters at the bottom without a wall
    collision, while the gas keeps its inlet and outlet (the step with the
    flag off mirrors the sphere at the top and reverses it)."""
    pos = np.array([[3.5, 5.95]])
    vel = np.array([[0.0, 0.2]])
    base = dict(nx=7, ny=6, bc=["wall", "wall", "inlet", "outlet"], pos=pos, vel=vel, g=(0.0, 0.0),
                inlet_uy=np.full(7, 0.01))
    on = orc.Sim(_cfg(**base, particles_periodic_y=1))
    o = on.step(record=True)
    assert 0.0 <= on.pos[0, 1] < 0.2 and on.vel[0, 1] > 0.19 and o.nwall == 0
    off = orc.Sim(_cfg(**base))
    o2 = off.step(record=True)
    assert 5.8 < off.pos[0, 1] < 6.0 and off.vel[0, 1] < 0 and o2.nwall == 1
    # the gas is the same in both runs: the flag does not touch the lattice
    assert np.abs(on.f - off.f).max() < 1e-6


# ---------------------------------------------------------------- the hard-sphere stage in single precision
def _split(pos):
    cell = np.floor(pos)
    return cell.astype(np.int32), (pos - cell).astype(np.float32)


@pytest.mark.parametrize("e", [0.0, 0.9, 1.0])
def test_f32_two_sphere_collision(orc, e):
    """orc_collide_f32, Eqs. 17-18 in float: for two spheres in contact the
    normal relative velocity becomes -e times itself and the tangential part
    and the momentum are kept, each to float rounding; spheres moving apart or
    not touching are left alone; the pair list is the float predicate's."""
    p = orc.make_params(_cfg(nx=8, ny=8, e_pp=e))
    cases = [((2.25, 3.5), (2.625, 3.5), (0.01, 0.0), (-0.01, 0.0)),    # head-on along x, one cell
             ((2.75, 3.75), (3.125, 4.0), (0.02, 0.01), (-0.01, -0.03)),  # oblique, across cells
             ((7.875, 0.125), (0.25, 7.875), (0.01, -0.01), (-0.01, 0.02)),  # across the periodic corner
             ((2.25, 3.5), (2.625, 3.5), (-0.01, 0.0), (0.01, 0.0)),     # separating overlap
             ((2.0, 2.0), (2.75, 2.0), (0.05, 0.0), (-0.05, 0.0))]       # 0.75 apart: no contact
    for P1, P2, v1, v2 in cases:
        pos = np.array([P1, P2], float)
        cell, off = _split(pos)
        vel = np.array([v1, v2], np.float32)
        pairs, out, nc, nw = orc.collide_f32(p, cell, off, vel)
        d = pos[0] - pos[1]
        d -= 8 * np.round(d / 8)
        touching = np.hypot(*d) <= 0.5
        assert len(pairs) == int(touching) and nw == 0
        n = d / np.linalg.norm(d)
        t = np.array([-n[1], n[0]])
        r0 = vel[0].astype(float) - vel[1]
        if not touching or r0 @ n >= 0:
            assert nc == 0 and (out == vel).all()
            continue
        assert nc == 1
        r1 = out[0].astype(float) - out[1]
        eps = 4 * np.finfo(np.float32).eps * np.abs(vel).max()
        assert abs(r1 @ n + e * (r0 @ n)) < eps
        assert abs(r1 @ t - r0 @ t) < eps
        assert np.abs(out.astype(float).sum(0) - vel.astype(float).sum(0)).max() < eps


def test_f32_wall_collision(orc):
    """Walls in float (R23): in the first or last cell within r of the wall
    plane and moving into it, v_n -> -e_w v_n exactly (one float product);
    tangential and outward motion untouched; periodic axes have no walls."""
    p = orc.make_params(_cfg(nx=10, ny=10, bc=["wall", "wall", "periodic", "periodic"], e_pw=0.7))
    pos = np.array([[0.2, 5.5], [9.875, 5.5], [5.5, 0.125], [0.2, 5.5], [3.5, 5.5]])
    vel = np.array([[-0.1, 0.3], [0.2, 0.1], [0.05, -0.4], [0.1, 0.0], [-1.0, -1.0]], np.float32)
    # spread them out so none touch: one per row
    pos[:, 1] = [1.5, 3.5, 5.5, 7.5, 9.5]
    pos[2] = (5.5, 5.5)
    cell, off = _split(pos)
    pairs, out, nc, nw = orc.collide_f32(p, cell, off, vel)
    want = vel.copy()
    want[0, 0] = np.float32(-0.7) * vel[0, 0]
    want[1, 0] = np.float32(-0.7) * vel[1, 0]
    assert len(pairs) == 0 and nc == 0 and nw == 2 and (out == want).all()
    pw = orc.make_params(_cfg(nx=10, ny=10, bc=["wall"] * 4, e_pw=0.5))
    pos = np.array([[5.5, 0.125], [5.5, 9.9], [2.5, 0.3]])
    vel = np.array([[0.05, -0.4], [0.0, 0.3], [0.0, -0.2]], np.float32)
    cell, off = _split(pos)
    _, out, _, nw = orc.collide_f32(pw, cell, off, vel)
    assert nw == 2 and out[0, 1] == np.float32(0.2) and out[1, 1] == np.float32(-0.5) * np.float32(0.3)
    assert out[2, 1] == vel[2, 1]


def test_f32_stage_follows_the_fp64_sweep(orc):
    """On a whole bed (the 64 x 512 riser crop, 31 250 spheres, random
    velocities) the float stage takes the same decisions as the FP64 oracle's
    sequential sweep and walls on the same float-held state, and its
    velocities agree to float rounding; pair lists are identical."""
    cfg = synth.riser_crop()
    p = orc.make_params(cfg)
    pos = cfg["pos"].copy()
    rng = np.random.default_rng(5)
    near = rng.choice(len(pos), 400, replace=False)  # some spheres within r of the x walls
    pos[near[:200], 0] = 0.05 + 0.2 * rng.random(200)
    pos[near[200:], 0] = 63.95 - 0.2 * rng.random(200)
    cell, off = _split(pos)
    pos32 = cell + off.astype(np.float64)
    vel = ((rng.random(pos.shape) - 0.5) * 2e-2).astype(np.float32)
    pairs, out, nc, nw = orc.collide_f32(p, cell, off, vel)
    ref_pairs = orc.contacts(p, pos32)
    assert (pairs == ref_pairs).all()
    v64, nc64 = orc.resolve(p, pos32, vel.astype(np.float64), ref_pairs)
    v64, nw64 = orc.walls(p, pos32, v64)
    assert nc == nc64 and nw == nw64 and nc > 1000 and nw > 10
    assert np.abs(out - v64).max() <= 1e-5 * np.abs(v64).max()


def _cancelling_bed(mode):
    """A crowded periodic bed with fast random velocities (the regime where a
    cell's pre-drags can nearly cancel), after one step to develop a flow."""
    return synth.tiny(nx=8, ny=8, n=400, seed=31, bc=("periodic",) * 4, vel_scale=2e-2, g=(0.0, 0.0),
                      drag_ratio_mode=mode)


def test_regularised_drag_splits_cancelling_cells(orc):
    """R49 (drag_ratio_mode 2): in a cell whose pre-drags cancel, sum |F_pre|
    above 100 |sum F_pre| (sums in index order), every particle takes
    -F_p->g / n, the split of an exactly zero sum (R16); in every other cell
    the signed ratio of Eq. 28, -F_p->g F_pre,k / sum F_pre.  Both classes
    occur on this bed, and the drags still sum to -F_p->g per cell."""
    cfg = _cancelling_bed(2)
    sim = orc.Sim(cfg)
    sim.step()
    pos0 = sim.pos.copy()
    o = sim.step(record=True)
    nx = cfg["nx"]
    cell = (np.floor(pos0[:, 1]) * nx + np.floor(pos0[:, 0])).astype(int)
    C = nx * cfg["ny"]
    S = np.zeros((C, 2))
    A = np.zeros((C, 2))
    np.add.at(S, cell, o.fpre)
    np.add.at(A, cell, np.abs(o.fpre))
    n = np.bincount(cell, minlength=C)
    fpg = o.fpg.reshape(-1, 2)
    split = A > 100.0 * np.abs(S)
    nsplit = 0
    for k in range(len(pos0)):
        c = cell[k]
        for a in range(2):
            if split[c, a]:
                want = -fpg[c, a] / n[c]
                nsplit += 1
            else:
                want = -fpg[c, a] * o.fpre[k, a] / S[c, a]
            assert o.fd[k, a] == want, (k, a, split[c, a])
    assert nsplit > 0 and nsplit < 2 * len(pos0)
    tot = np.zeros((C, 2))
    np.add.at(tot, cell, o.fd)
    occ = n > 0
    assert np.abs(tot[occ] + fpg[occ]).max() < 1e-12 * np.abs(fpg).max()


def test_regularised_drag_equals_signed_without_cancellation(orc):
    """R49: on a dilute bed where no cell's pre-drags cancel, drag_ratio_mode 2
    steps exactly as the signed Eq. 28 (mode 0)."""
    runs = []
    for mode in (0, 2):
        cfg = synth.tiny(nx=16, ny=24, n=60, seed=7, vel_scale=1e-3, drag_ratio_mode=mode)
        sim = orc.Sim(cfg)
        for _ in range(10):
            o = sim.step(record=True)
        runs.append((sim.f.copy(), sim.pos.copy(), sim.vel.copy(), o))
    assert (runs[1][3].ncell > 1).any()  # cells where the ratio of Eq. 28 applies
    for a, b in zip(runs[0][:3], runs[1][:3]):
        assert np.array_equal(a, b)
