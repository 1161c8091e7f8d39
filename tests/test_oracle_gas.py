"""Pins of the oracle's collision and streaming against identities, closed-form
flows and an independent textbook BGK implementation (no GPU)."""
import math

import numpy as np
import pytest

import synth


def _cfg(**kw):
    c = dict(synth.DEFAULTS)
    c.update(nx=8, ny=8, bc=["periodic"] * 4, pos=np.zeros((0, 2)), vel=np.zeros((0, 2)))
    c.update(kw)
    return c


def _rand_f(rng, rho=1.0):
    u = (rng.random(2) - 0.5) * 0.1
    import oracle
    fe = np.array([oracle.feq(i, rho, u[0], u[1]) for i in range(9)])
    return fe * (1 + 0.05 * (rng.random(9) - 0.5))


def test_collide_identities(orc):
    """Eqs. 7, 23-25 with the plain moment velocity (R5):
    sum Om^s = 0, sum c Om^s = rho (v_s - u)  =>  F_pg = omega gamma rho (v_s - u);
    the collision keeps mass and adds exactly F_pg + G of momentum; and
    u_sup = (1 - omega gamma / 2) u + (omega gamma / 2) v_s + G / (2 rho)."""
    c, w, _ = orc.lattice()
    rng = np.random.default_rng(3)
    for n in (0, 1, 2, 3, 7):
        for G in ((0.0, 0.0), (1e-5, -3e-6)):
            p = orc.make_params(_cfg(G=G, u_gas_porosity=2))
            f = _rand_f(rng)
            vs = (rng.random(2) - 0.5) * 0.05 if n else np.zeros(2)
            fs, o = orc.collide_node(p, f, n, vs)
            pr = orc.cell_props(p, n)
            og = pr["omega"] * pr["gamma"]
            rho = f.sum()
            j = (c * f[:, None]).sum(0)
            u = j / rho
            assert abs(o["rho"] - rho) < 1e-15
            assert np.allclose(o["fpg"], og * rho * (vs - u), atol=1e-16, rtol=1e-12)
            assert abs(fs.sum() - rho) < 2e-15
            assert np.allclose((c * fs[:, None]).sum(0), j + o["fpg"] + np.array(G), atol=1e-16, rtol=1e-12)
            usup = (1 - og / 2) * u + og / 2 * vs + np.array(G) / (2 * rho)
            assert np.allclose(o["usup"], usup, atol=1e-16, rtol=1e-12)


def test_zero_particle_limit_is_bgk(orc):
    """With no particles gamma = 0 and Eq. 23 reduces to the BGK collision of
    Eqs. 2-3.  Compare the oracle's step against an independent textbook D2Q9 BGK
    written here with numpy (np.roll streaming, vectorised equilibrium)."""
    nx, ny, tau = 12, 10, 0.7
    cfg = _cfg(nx=nx, ny=ny, tau=tau)
    rng = np.random.default_rng(5)
    c = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]])
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    rho0 = 1 + 0.01 * rng.random((ny, nx))
    u0 = 0.02 * (rng.random((2, ny, nx)) - 0.5)

    def eq(rho, ux, uy):
        cu = c[:, 0, None, None] * ux + c[:, 1, None, None] * uy
        return w[:, None, None] * rho * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * (ux ** 2 + uy ** 2))

    f = eq(rho0, u0[0], u0[1]) * (1 + 0.01 * (rng.random((9, ny, nx)) - 0.5))
    sim = orc.Sim(cfg, f=f)
    g = f.copy()
    for _ in range(25):
        sim.step()
        rho = g.sum(0)
        ux = (c[:, 0, None, None] * g).sum(0) / rho
        uy = (c[:, 1, None, None] * g).sum(0) / rho
        g = g - (g - eq(rho, ux, uy)) / tau
        g = np.stack([np.roll(np.roll(g[i], c[i, 0], axis=1), c[i, 1], axis=0) for i in range(9)])
    assert np.abs(sim.f - g).max() < 1e-13


def _tg_amplitude(ux, kx, ky, X, Y):
    mode = -np.cos(kx * X) * np.sin(ky * Y)
    return (ux * mode).sum() / (mode * mode).sum()


def _taylor_green_rate(orc, L, tau=0.6, t1=40, t2=240):
    nu = (tau - 0.5) / 3
    k = 2 * math.pi / L
    y, x = np.mgrid[0:L, 0:L] + 0.5
    u0 = 1e-3
    ux = -u0 * np.cos(k * x) * np.sin(k * y)
    uy = u0 * np.sin(k * x) * np.cos(k * y)
    f = np.stack([np.vectorize(lambda a, b, i=i: orc.feq(i, 1.0, a, b))(ux, uy) for i in range(9)])
    sim = orc.Sim(_cfg(nx=L, ny=L, tau=tau), f=f)
    amps = {}
    for t in range(1, t2 + 1):
        o = sim.step(record=(t in (t1, t2)))
        if o is not None:
            amps[t] = _tg_amplitude(o.ugas[..., 0], k, k, x, y)
    rate = -math.log(amps[t2] / amps[t1]) / (t2 - t1)
    return rate, 2 * nu * k * k


def test_taylor_green_decay(orc):
    """Periodic Taylor-Green vortex: the BGK gas (Eqs. 2-4, tau = 3 nu + 1/2)
    decays as exp(-2 nu k^2 t); the rate error falls at second order in 1/L."""
    errs = []
    for L in (16, 32):
        rate, want = _taylor_green_rate(orc, L)
        errs.append(abs(rate - want) / want)
    assert errs[1] < 1e-3
    assert errs[0] / errs[1] > 3.0


def _poiseuille(orc, nx, tau=0.8, G=1e-6, steps=None):
    nu = (tau - 0.5) / 3
    steps = steps or int(8 * nx * nx / nu)
    sim = orc.Sim(_cfg(nx=nx, ny=4, tau=tau, bc=["wall", "wall", "periodic", "periodic"], G=(0.0, G)))
    sim.run(steps - 1)
    o = sim.step(record=True)
    uy = o.ugas[:, :, 1].mean(0)
    x = np.arange(nx) + 0.5
    want = G / (2 * nu) * x * (nx - x)
    return np.abs(uy - want).max() / want.max()


@pytest.mark.slow
def test_poiseuille_channel(orc):
    """Walls at x = 0 and x = nx (halfway bounce-back, R20), periodic in y, gas
    body force G (R29): the steady profile is G/(2 nu) x (nx - x); the error
    falls at second order in the channel width."""
    e16 = _poiseuille(orc, 16)
    e32 = _poiseuille(orc, 32)
    assert e32 < 1e-3
    assert e16 / e32 > 3.0


def test_uniform_inflow_is_steady(orc):
    """Equilibrium inlet (R21) and zero-gradient outlet (R22): the uniform state
    f^eq(1, (0, u_in)) is a fixed point of collision + streaming."""
    nx, ny, uin = 6, 9, 0.02
    cfg = _cfg(nx=nx, ny=ny, bc=["periodic", "periodic", "inlet", "outlet"], inlet_uy=np.full(nx, uin))
    f = orc.equilibrium_state(nx, ny, 1.0, 0.0, uin)
    sim = orc.Sim(cfg, f=f)
    sim.run(5)
    assert np.abs(sim.f - f).max() < 1e-14


def test_walls_and_inlet_sources(orc):
    """Streaming rules: on a closed box (walls on all faces) streaming only moves
    and reflects populations, so every value of f* reappears once; the inlet
    writes f^eq(1, u_in(x)) into the upward populations of row 0 except where an
    x wall takes precedence (R20, R21)."""
    nx, ny = 5, 4
    rng = np.random.default_rng(9)
    fstar = rng.random((9, ny, nx))
    p = orc.make_params(_cfg(nx=nx, ny=ny, bc=["wall"] * 4))
    out = orc.stream(p, fstar)
    assert np.allclose(np.sort(out.ravel()), np.sort(fstar.ravel()), atol=0, rtol=0)
    uin = np.linspace(0.01, 0.05, nx)
    p2 = orc.make_params(_cfg(nx=nx, ny=ny, bc=["wall", "wall", "inlet", "outlet"]))
    out2 = orc.stream(p2, fstar, inlet_uy=uin)
    for x in range(nx):
        for i in (2, 5, 6):  # c_y = +1
            cx = (0, 1, 0, -1, 0, 1, -1, -1, 1)[i]
            if 0 <= x - cx < nx:
                assert out2[i, 0, x] == orc.feq(i, 1.0, 0.0, uin[x])
            else:
                opp = (0, 3, 4, 1, 2, 7, 8, 5, 6)[i]
                assert out2[i, 0, x] == fstar[opp, 0, x]
    # outlet: downward populations of the top row come from the top row itself
    for x in range(nx):
        for i in (4, 7, 8):  # c_y = -1
            cx = (0, 1, 0, -1, 0, 1, -1, -1, 1)[i]
            if 0 <= x - cx < nx:
                assert out2[i, ny - 1, x] == fstar[i, ny - 1, x - cx]


def test_mass_conservation_periodic(orc):
    """Periodic bed with particles, no forcing: sum f is conserved to roundoff."""
    cfg = synth.tiny(nx=16, ny=16, n=80, bc=("periodic",) * 4, vel_scale=1e-3, g=(0.0, 0.0))
    sim = orc.Sim(cfg)
    m0 = sim.conservation()[0]
    sim.run(30)
    assert abs(sim.conservation()[0] - m0) < 1e-12 * m0


def _poiseuille_les(orc, nx, tau=0.8, G=2e-5, cs=4.0):
    """Steady channel flow with the Smagorinsky model on: returns the oracle's
    profile, the closed form and the laminar profile at the nodes."""
    nu = (tau - 0.5) / 3
    steps = int(8 * nx * nx / nu)
    sim = orc.Sim(_cfg(nx=nx, ny=4, tau=tau, bc=["wall", "wall", "periodic", "periodic"], G=(0.0, G),
                       cs_smag=cs))
    sim.run(steps - 1)
    o = sim.step(record=True)
    uy = o.ugas[:, :, 1].mean(0)
    x = np.arange(nx) + 0.5
    # Steady momentum balance with nu_t = nu + C_s^2 |u'| (Eq. 12, |S| = |u'| in
    # simple shear, dx = 1): (nu + a |u'|) |u'| = G |s| at s = x - nx/2, a = C_s^2;
    # |u'| = (sqrt(nu^2 + 4 a G |s|) - nu) / (2 a), integrated from the wall.
    a = cs * cs

    def W(s):
        return ((nu * nu + 4 * a * G * s) ** 1.5 / (6 * a * G) - nu * s) / (2 * a)

    h = nx / 2
    want = W(h) - W(np.abs(x - h))
    lam = G / (2 * nu) * x * (nx - x)
    return uy, want, lam


@pytest.mark.slow
def test_poiseuille_channel_smagorinsky(orc):
    """Eqs. 12-15: the sub-grid viscosity nu_e = C_s^2 |S| added to nu turns the
    parabola of the channel flow into the closed-form profile of
    (nu + C_s^2 |u'|) u' = -G (x - nx/2); the error falls at second order in the
    channel width, and the profile stands 20 % below the laminar one."""
    errs = []
    for nx in (16, 32):
        uy, want, lam = _poiseuille_les(orc, nx)
        errs.append(np.abs(uy - want).max() / want.max())
    assert errs[1] < 2e-3, errs
    assert errs[0] / errs[1] > 3.0, errs
    assert (lam.max() - want.max()) / lam.max() > 0.15


def test_smagorinsky_off_at_equilibrium(orc):
    """Q = 0 gives tau_t = tau (Eq. 15, text after it): a lattice at equilibrium
    steps identically with and without the sub-grid model."""
    import oracle
    rng = np.random.default_rng(3)
    u = (rng.random(2) - 0.5) * 0.05
    f = np.array([oracle.feq(i, 1.0, u[0], u[1]) for i in range(9)])
    f0 = np.broadcast_to(f[:, None, None], (9, 8, 8)).copy()
    a = orc.Sim(_cfg(), f=f0)
    b = orc.Sim(_cfg(cs_smag=0.3), f=f0)
    for _ in range(5):
        a.step()
        b.step()
    assert np.array_equal(a.f, b.f)
