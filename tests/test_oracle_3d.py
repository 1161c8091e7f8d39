"""Pins of the oracle's 3-D gas lattice (D3Q19), the first piece of the 3-D
extension: lattice isotropy, equilibrium moments, conservation and the
viscous decay of a shear wave (no GPU)."""
import itertools
import math

import numpy as np
import pytest


def test_d3q19_isotropy(orc):
    """Weights 1/3, 1/18, 1/36 with c_s^2 = 1/3: every velocity has its
    opposite, and the weighted moments are isotropic through fourth order,
    sum w c_a c_b c_c c_d = (d_ab d_cd + d_ac d_bd + d_ad d_bc) / 9."""
    c, w = orc.lattice3()
    assert len({tuple(v) for v in c}) == 19 and abs(w.sum() - 1.0) < 1e-15
    assert all(any((c[j] == -c[i]).all() for j in range(19)) for i in range(19))
    d = np.eye(3)
    assert np.abs(w @ c).max() < 1e-16
    assert np.allclose(np.einsum("i,ia,ib->ab", w, c, c), d / 3.0, atol=1e-16)
    assert np.abs(np.einsum("i,ia,ib,ic->abc", w, c, c, c)).max() < 1e-16
    m4 = np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)
    for a, b, e, f in itertools.product(range(3), repeat=4):
        want = (d[a, b] * d[e, f] + d[a, e] * d[b, f] + d[a, f] * d[b, e]) / 9.0
        assert abs(m4[a, b, e, f] - want) < 1e-15


def test_d3q19_equilibrium_moments(orc):
    """sum f^eq = rho, sum c f^eq = rho u, sum c c f^eq = rho (I/3 + u u)."""
    c, _ = orc.lattice3()
    rng = np.random.default_rng(3)
    for _ in range(20):
        rho = 0.8 + 0.4 * rng.random()
        u = (rng.random(3) - 0.5) * 0.1
        fe = np.array([orc.feq3(i, rho, *u) for i in range(19)])
        assert abs(fe.sum() - rho) < 1e-14
        assert np.allclose(c.T @ fe, rho * u, atol=1e-15)
        assert np.allclose(np.einsum("i,ia,ib->ab", fe, c, c), rho * (np.eye(3) / 3 + np.outer(u, u)), atol=1e-15)


def test_d3q19_conservation_and_uniform_flow(orc):
    """A periodic box conserves mass and momentum to roundoff; a uniform flow
    at equilibrium is a fixed point of the step."""
    c, _ = orc.lattice3()
    rng = np.random.default_rng(5)
    nx, ny, nz = 5, 4, 6
    f = np.empty((19, nz, ny, nx))
    for i in range(19):
        f[i] = orc.feq3(i, 1.0, 0.01, -0.02, 0.005)
    f += (rng.random(f.shape) - 0.5) * 1e-3
    m0, j0 = f.sum(), np.einsum("ia,izyx->a", c.astype(float), f)
    g = f
    for _ in range(10):
        g = orc.bgk3_step(g, 0.7)
    assert abs(g.sum() - m0) < 1e-11
    assert np.allclose(np.einsum("ia,izyx->a", c.astype(float), g), j0, atol=1e-12)
    u = np.array([0.02, 0.01, -0.03])
    fe = np.empty((19, nz, ny, nx))
    for i in range(19):
        fe[i] = orc.feq3(i, 1.0, *u)
    assert np.abs(orc.bgk3_step(fe, 0.8) - fe).max() < 1e-16


@pytest.mark.slow
def test_d3q19_shear_wave_decay(orc):
    """A shear wave u_x = U sin(2 pi z / L) decays as exp(-nu k^2 t) with
    nu = (tau - 1/2) / 3 (Eq. 3 in three dimensions); the error of the decay
    falls at second order as L doubles."""
    tau, U = 0.8, 1e-3
    nu = (tau - 0.5) / 3.0
    errs = []
    for L in (16, 32):
        k = 2 * math.pi / L
        z = np.arange(L)
        f = np.empty((19, L, 2, 2))
        for i in range(19):
            for zz in z:
                f[i, zz] = orc.feq3(i, 1.0, U * math.sin(k * zz), 0.0, 0.0)
        steps = int(round(0.5 / (nu * k * k)))  # decay to about exp(-0.5)
        for _ in range(steps):
            f = orc.bgk3_step(f, tau)
        c, _ = orc.lattice3()
        rho = f.sum(0)
        ux = np.einsum("i,izyx->zyx", c[:, 0].astype(float), f) / rho
        amp = 2.0 / L * float((ux[:, 0, 0] * np.sin(k * z)).sum())
        errs.append(abs(amp / (U * math.exp(-nu * k * k * steps)) - 1.0))
    assert errs[1] < 5e-3, errs
    assert errs[0] / errs[1] > 3.0, errs


def _eq_state(orc, rho, u):
    """f = f^eq(rho, u) cell by cell; rho [nz][ny][nx], u [3][nz][ny][nx]."""
    f = np.empty((19,) + rho.shape)
    for i in range(19):
        f[i] = np.vectorize(lambda r, a, b, c: orc.feq3(i, r, a, b, c))(rho, u[0], u[1], u[2])
    return f


def _solids(shape, seed):
    rng = np.random.default_rng(seed)
    n = rng.integers(0, 4, shape).astype(np.int32)
    vs = (rng.random((3,) + shape) - 0.5) * 0.06
    return n, vs


def test_psm3_without_solids_is_bgk(orc):
    """No spheres anywhere: gamma = 0, so the step is the plain BGK step (to
    rounding: the relaxation is written (1 - gamma) / tau times the
    non-equilibrium part there) and the force is zero."""
    shape = (4, 5, 6)
    rng = np.random.default_rng(1)
    f = np.array([w for w in orc.lattice3()[1]])[:, None, None, None] + (rng.random((19,) + shape) - 0.5) * 1e-2
    n = np.zeros(shape, np.int32)
    _, vs = _solids(shape, 2)
    got, force = orc.psm3_step(f, 0.8, 0.7, n, vs)
    assert np.abs(got - orc.bgk3_step(f, 0.8)).max() < 1e-16
    assert not force.any()


@pytest.mark.parametrize("tau", [0.55, 1.0])
def test_psm3_force_on_equilibrium_is_drag_of_gamma(orc, tau):
    """For a cell at equilibrium the non-equilibrium bounce-back of Eq. 7
    sums to c-moments that give F = gamma rho (v_s - u) exactly (the
    momentum of f^eq is rho u, that of its reflection -rho u); the dense
    cells are held at the densest sphere packing pi / (3 sqrt 2)."""
    shape = (3, 4, 5)
    rng = np.random.default_rng(3)
    rho = 1.0 + (rng.random(shape) - 0.5) * 0.1
    u = (rng.random((3,) + shape) - 0.5) * 0.08
    n, vs = _solids(shape, 4)
    n[0, 0, 0] = 40  # far beyond the densest packing
    d = 0.9
    _, force = orc.psm3_step(_eq_state(orc, rho, u), tau, d, n, vs)
    es = np.minimum(n * math.pi * d ** 3 / 6.0, math.pi / (3.0 * math.sqrt(2.0)))
    gam = np.vectorize(lambda e: orc.gamma(e, tau))(es)
    assert abs(es[0, 0, 0] - 0.7404804896930609) < 1e-15
    want = gam * rho * (vs - u)
    assert np.abs(force - want).max() < 1e-15


def test_psm3_conserves_mass_and_balances_momentum(orc):
    """Eq. 7's term carries no mass, and the gas gains exactly the force of
    Eq. 25: total mass is unchanged and total momentum moves by the summed
    force (streaming on the periodic box moves populations, not momentum)."""
    shape = (5, 4, 6)
    rng = np.random.default_rng(5)
    c, w = orc.lattice3()
    f = w[:, None, None, None] * (1.0 + (rng.random((19,) + shape) - 0.5) * 0.2)
    n, vs = _solids(shape, 6)
    got, force = orc.psm3_step(f, 0.7, 0.8, n, vs)
    assert abs(got.sum() - f.sum()) < 1e-12
    mom = lambda g: np.array([(c[:, a][:, None, None, None] * g).sum() for a in range(3)])
    assert np.abs(mom(got) - mom(f) - force.reshape(3, -1).sum(axis=1)).max() < 1e-13


def test_psm3_solids_moving_with_the_gas_leave_it_steady(orc):
    """Uniform gas at equilibrium with every sphere moving at the gas
    velocity: Eq. 7's term vanishes, the force is zero and the state does
    not change (to rounding)."""
    shape = (3, 4, 5)
    u0 = np.array([0.03, -0.02, 0.01])
    u = np.broadcast_to(u0[:, None, None, None], (3,) + shape).copy()
    f = _eq_state(orc, np.ones(shape), u)
    n, _ = _solids(shape, 7)
    got, force = orc.psm3_step(f, 0.6, 1.0, n, u)
    assert np.abs(force).max() < 1e-16
    assert np.abs(got - f).max() < 5e-16


def test_psm3_opposite_directions(orc):
    """A dropped or mismatched opposite would break Eq. 7: a single cell whose
    only non-equilibrium part sits in one direction i reflects it into
    opp(i), whatever i is."""
    c, w = orc.lattice3()
    shape = (3, 3, 3)
    for i in range(1, 19):
        f = np.broadcast_to(w[:, None, None, None], (19,) + shape).copy()
        f[i, 1, 1, 1] += 1e-3
        n = np.zeros(shape, np.int32)
        n[1, 1, 1] = 1
        vs = np.zeros((3,) + shape)
        _, force = orc.psm3_step(f, 1.0, 1.0, n, vs)
        # moments: rho = 1 + 1e-3, j = 1e-3 c_i; F = gamma (sum c Om) and
        # sum c_k (f_opp(k) - f_k) = -2 j, sum c feq(v_s = 0) = 0,
        # sum c_k feq_opp(k)(u) = -j
        gam = orc.gamma(math.pi / 6.0, 1.0)
        want = gam * (-2e-3 * c[i] + 1e-3 * c[i])
        assert np.abs(force[:, 1, 1, 1] - want).max() < 1e-17, i
