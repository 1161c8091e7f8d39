"""Pins of the oracle's gas-phase pieces against closed forms, invariants and
the paper's printed numbers (no GPU).  Each test names the passage it pins."""
import json
import math
import os

import numpy as np
import pytest

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)


def _params(orc, **kw):
    cfg = dict(synth.DEFAULTS)
    cfg.update(nx=8, ny=8, bc=["periodic"] * 4)
    cfg.update(kw)
    return orc.make_params(cfg)


# ---------------------------------------------------------------- D2Q9 lattice
def test_d2q9_isotropy(orc):
    """Sec. 2.1 after Eq. 4: weights 4/9, 1/9, 1/36 and c_s^2 = 1/3.  A D2Q9
    lattice with those weights must satisfy sum w = 1, sum w c = 0,
    sum w c c = I/3 and the 4th-order isotropy sum w c_a^2 c_b^2 = 1/9
    (a != b), 1/3 (a = b); a garbled diagonal (the printed sqrt(2) form) fails."""
    c, w, opp = orc.lattice()
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.abs((w[:, None] * c).sum(0)).max() == 0.0
    m2 = np.einsum("i,ia,ib->ab", w, c, c)
    assert np.allclose(m2, np.eye(2) / 3.0, atol=1e-15)
    m4 = np.einsum("i,ia,ib->ab", w, c.astype(float) ** 2, c.astype(float) ** 2)
    assert np.allclose(m4, [[1 / 3, 1 / 9], [1 / 9, 1 / 3]], atol=1e-15)
    assert (c[opp] == -c).all()
    assert set(map(tuple, c.tolist())) == {(x, y) for x in (-1, 0, 1) for y in (-1, 0, 1)}


def test_feq_moments(orc):
    """Eq. 4/5: sum f^eq = rho, sum c f^eq = rho u, sum c c f^eq = rho (I/3 + u u)."""
    c, w, _ = orc.lattice()
    rng = np.random.default_rng(1)
    for _ in range(20):
        rho = 0.5 + rng.random()
        u = (rng.random(2) - 0.5) * 0.2
        fe = np.array([orc.feq(i, rho, u[0], u[1]) for i in range(9)])
        assert abs(fe.sum() - rho) < 1e-14
        assert np.allclose((c * fe[:, None]).sum(0), rho * u, atol=1e-15)
        m2 = np.einsum("i,ia,ib->ab", fe, c, c)
        assert np.allclose(m2, rho * (np.eye(2) / 3 + np.outer(u, u)), atol=1e-14)


# ---------------------------------------------------------------- porosity, gamma, omega
def test_gamma_limits(orc):
    """Sec. 2.1 after Eq. 9: gamma = 0 is pure fluid, gamma = 1 pure solid."""
    for tau in (0.51, 0.6, 1.0, 2.0):
        assert orc.gamma(0.0, tau) == 0.0
        assert orc.gamma(1.0, tau) == 1.0
        g = [orc.gamma(e, tau) for e in np.linspace(0, 1, 21)]
        assert all(b > a for a, b in zip(g, g[1:]))


def test_eps3_at_packing_clamp(orc):
    """Eq. 11 at the densest disc packing pi/(2 sqrt 3) (the clamp of R7) gives
    the 3-D fraction pi/6 exactly (derived: coeff * (pi/(2 sqrt3))^1.5 = pi/6)."""
    p = _params(orc)
    pr = orc.cell_props(p, 50)
    assert abs(pr["eps_s2"] - math.pi / (2 * math.sqrt(3))) < 1e-15
    assert abs(pr["eps_s3"] - math.pi / 6) < 1e-14
    # n = 0: pure fluid
    pr0 = orc.cell_props(p, 0)
    assert pr0["eps_s2"] == 0.0 and pr0["eps_g"] == 1.0 and pr0["gamma"] == 0.0


def test_table2_solids_fraction(orc):
    """Table 2: 123 921 particles of d = 0.2 in a 60 x 720 riser give the printed
    initial solids fraction 0.09007 when each particle counts its Eq. 10 disc area."""
    g = _golden("table2_riser.json")
    p = _params(orc, d=g["d"])
    per_particle = orc.cell_props(p, 1)["eps_s2"]  # one particle in a unit cell
    theta = g["n_particles"] * per_particle / (g["width"] * g["height"])
    assert abs(theta - g["theta_s_printed"]) / g["theta_s_printed"] < g["rel_tol"]


def test_omega_printed_range(orc):
    """Sec. 2.3 after Eq. 22: omega of Eq. 20 lies between 0.0152 and 4.2876."""
    g = _golden("omega_range.json")
    eg = np.linspace(0.7400001, 1.0, 200001)
    om = np.array([orc.omega_emms(e) for e in eg])
    assert round(om.max(), g["digits"]) == g["omega_max_printed"]
    assert abs(eg[om.argmax()] - 0.7463) < 2e-6
    assert round(orc.omega_emms(0.97), g["digits"]) == g["omega_min_printed"]
    # the branch-3 limit just above 0.97 is within 1.1e-4 of it (printed tie-break, R32)
    assert abs(orc.omega_emms(0.9700001) - orc.omega_emms(0.97)) < 1.1e-4
    assert abs(orc.omega_emms(1.0) - 1.0) < 1e-12


def test_omega_by_count_table(orc):
    """Appendix numbers of the build plan for d = 0.5, tau = 0.6: gamma and omega
    per particle count (n = 1, 2 in the dilute branches; n >= 3 dense -> 1)."""
    p = _params(orc)
    want = {1: (0.02173, 0.02228), 2: (0.05552, 0.14386), 3: (0.11528, 1.0)}
    for n, (gam, om) in want.items():
        pr = orc.cell_props(p, n)
        assert abs(pr["gamma"] - gam) < 6e-6
        assert abs(pr["omega"] - om) < 6e-6


# ---------------------------------------------------------------- drag laws
def test_cd0_near_continuous(orc):
    """Eq. 21: 24/Re (1 + 0.15 Re^0.687) reaches 0.438 at Re -> 1000, next to 0.44."""
    assert abs(orc.cd0(999.999999) - 0.44) < 0.002
    assert orc.cd0(1000.0) == 0.44


def test_beta_dilute_rewrite_matches_literal(orc):
    """Eqs. 19, 21, 22: the Re-cancelled dilute branch used by the oracle (R12)
    equals the literal 3/4 (1-eg) eg rho |u-v| / d * C_d0(Re) * omega for Re > 0."""
    p = _params(orc, tau=0.55, d=0.2)
    mu = p.rho_g * (p.tau - 0.5) / 3.0
    for eg in (0.75, 0.8, 0.9, 0.99):
        om = orc.omega_emms(eg)
        for slip in (1e-6, 1e-3, 0.05, 0.5):
            re = eg * p.rho_g * slip * p.d / mu
            lit = 0.75 * (1 - eg) * eg * p.rho_g * slip / p.d * orc.cd0(re) * om
            got = orc.beta(p, eg, om, slip)
            assert abs(got - lit) <= 1e-12 * abs(lit)


def test_beta_limits_and_units(orc):
    """Eq. 19: beta = 0 in a particle-free cell (eps_g = 1); Stokes limit
    18 (1-eg) omega mu / d^2 as slip -> 0, with mu from tau = 3 nu + 1/2 (Eq. 3)
    at the Table 1 viscosity converted to lattice units (h = dt = 1, R2)."""
    t1 = _golden("table1_bubble.json")
    nu_lu = t1["mu_g"] / t1["rho_g"] * t1["dt"] / t1["h"] ** 2
    assert abs(nu_lu - t1["mu_lu"]) / t1["mu_lu"] < t1["rel_tol"]
    assert abs(t1["v_mf"] * t1["dt"] / t1["h"] - t1["v_mf_lu"]) / t1["v_mf_lu"] < t1["rel_tol"]
    assert abs(t1["d_p"] / t1["h"] - t1["d_lu"]) < 1e-12
    p = _params(orc, tau=3 * nu_lu + 0.5, d=t1["d_lu"])
    assert orc.beta(p, 1.0, 1.0, 0.3) == 0.0
    eg, om = 0.9, orc.omega_emms(0.9)
    stokes = 18 * (1 - eg) * om * nu_lu / p.d ** 2
    assert abs(orc.beta(p, eg, om, 0.0) - stokes) <= 1e-12 * stokes
    # dense branch: Ergun viscous term alone at zero slip
    eg = 0.6
    erg = 150 * (1 - eg) ** 2 * nu_lu / (eg * p.d ** 2)
    assert abs(orc.beta(p, eg, 1.0, 0.0) - erg) <= 1e-12 * erg
