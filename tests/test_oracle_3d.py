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
