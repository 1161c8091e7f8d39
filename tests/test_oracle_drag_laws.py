"""Pins of the oracle's drag coefficient beta (Eqs. 19, 21, 22) against the
textbook drag laws it is built from (no GPU).

Eq. 19's dense branch is the Ergun equation, its dilute branch the Wen & Yu
law with the voidage function replaced by the EMMS factor omega, and Eq. 21 is
the Schiller & Naumann drag of a single sphere.  Each test below states the
textbook law in its own form (pressure drop per length of a packed bed; force
on one sphere at the superficial velocity; the standard drag curve) and checks
the oracle's beta against it, so a wrong prefactor, voidage factor, power of
d_p or branch constant in the oracle fails one of them.
"""
import math

import numpy as np

import synth


def _params(orc, tau=0.6, d=0.5, rho_g=1.0):
    c = dict(synth.DEFAULTS)
    c.update(nx=8, ny=8, bc=["periodic"] * 4, pos=np.zeros((0, 2)), vel=np.zeros((0, 2)), tau=tau, d=d,
             rho_g=rho_g)
    return orc.make_params(c)


def _mu(p):
    """Dynamic viscosity from tau = 3 nu + 1/2 (Eq. 3, h = dt = 1)."""
    return p.rho_g * (p.tau - 0.5) / 3.0


def _force_per_sphere(p, beta, eg, slip):
    """beta is a force per unit bed volume per unit slip; the spheres of that
    volume take the fraction 1 - eg, so one sphere of volume pi d^3/6 takes
    beta slip (pi d^3 / 6) / (1 - eg)."""
    return beta * slip * (math.pi * p.d ** 3 / 6.0) / (1.0 - eg)


def _schiller_naumann(re):
    """Single-sphere drag coefficient of Schiller & Naumann (1935): Stokes'
    24/Re with the 0.15 Re^0.687 inertial correction, constant 0.44 in the
    Newton regime from Re = 1000."""
    return 24.0 / re * (1.0 + 0.15 * re ** 0.687) if re < 1000.0 else 0.44


def test_cd0_follows_the_standard_drag_curve(orc):
    """Eq. 21 against the standard drag curve of a sphere (measured C_D at
    Re = 0.1, 1, 10, 100, 1000: about 244, 27, 4.2, 1.09, 0.47), which the
    Schiller-Naumann fit follows within about 7 %; and Stokes' law
    C_D -> 24/Re as Re -> 0."""
    curve = {0.1: 244.0, 1.0: 27.0, 10.0: 4.2, 100.0: 1.09, 1000.0: 0.47}
    for re, cd in curve.items():
        assert abs(orc.cd0(re) - cd) / cd < 0.07, (re, orc.cd0(re), cd)
    for re in (1e-6, 1e-4):
        assert abs(orc.cd0(re) * re / 24.0 - 1.0) < 2e-3
    for re in (1000.0, 5e3, 1e5):
        assert orc.cd0(re) == 0.44


def test_dense_beta_is_the_ergun_pressure_drop(orc):
    """Eq. 19, eps_g <= 0.74: Ergun's packed-bed pressure drop per length at
    superficial velocity U = eps_g |u - v|,
        dP/L = 150 mu (1-eps)^2 U / (eps^3 d^2) + 1.75 rho (1-eps) U^2 / (eps^3 d),
    is balanced by the drag on the bed: beta |u - v| = eps_g dP/L.  Checked
    over voidages and slips where either the viscous or the inertial term
    dominates; the correction omega does not enter this branch (R9)."""
    seen_inertial = seen_viscous = False
    for tau, d, rho in ((0.6, 0.5, 1.0), (0.5009, 0.2, 1.0), (0.9, 0.35, 1.3)):
        p = _params(orc, tau=tau, d=d, rho_g=rho)
        mu = _mu(p)
        for eg in (0.36, 0.45, 0.55, 0.65, 0.74):
            for slip in (1e-5, 1e-3, 0.02, 0.3, 3.0):
                U = eg * slip
                visc = 150.0 * mu * (1 - eg) ** 2 * U / (eg ** 3 * d ** 2)
                inert = 1.75 * rho * (1 - eg) * U * U / (eg ** 3 * d)
                want = eg * (visc + inert) / slip
                for om in (1.0, 0.3):
                    got = orc.beta(p, eg, om, slip)
                    assert abs(got - want) <= 1e-13 * want, (tau, d, rho, eg, slip, om, got, want)
                seen_inertial |= inert > 10 * visc
                seen_viscous |= visc > 10 * inert
    assert seen_inertial and seen_viscous


def test_dilute_beta_is_the_wen_yu_force(orc):
    """Eq. 19, eps_g > 0.74, with omega = eps_g^-2.65 is the Wen & Yu drag: the
    force on one sphere is its single-sphere drag at the superficial velocity
    U = eps_g |u - v| times the voidage function eps_g^-3.65,
        F = C_D(Re) (1/2) rho U^2 (pi d^2 / 4) eps_g^-3.65,
    with Re = rho U d / mu (Eq. 22) and C_D of Schiller & Naumann.  Covers
    both branches of Eq. 21 (Re from 1e-4 to above 1e4)."""
    seen_newton = seen_sn = False
    for tau, d, rho in ((0.6, 0.5, 1.0), (0.5001, 0.2, 1.0), (0.50002, 0.5, 1.2)):
        p = _params(orc, tau=tau, d=d, rho_g=rho)
        mu = _mu(p)
        for eg in (0.7401, 0.78, 0.85, 0.93, 0.98, 0.999):
            om = eg ** -2.65
            for slip in (1e-5, 1e-3, 0.01, 0.05, 0.2, 1.0):
                U = eg * slip
                re = rho * U * d / mu
                want = _schiller_naumann(re) * 0.5 * rho * U * U * (math.pi * d * d / 4.0) * eg ** -3.65
                got = _force_per_sphere(p, orc.beta(p, eg, om, slip), eg, slip)
                assert abs(got - want) <= 1e-12 * want, (tau, d, eg, slip, re, got, want)
                seen_newton |= re >= 1000.0
                seen_sn |= re < 1000.0
    assert seen_newton and seen_sn


def test_isolated_sphere_limit(orc):
    """eps_g -> 1 with omega = 1 (Eq. 20 gives omega(1) = 1): one sphere alone
    in the gas takes the Schiller-Naumann drag 3 pi mu d |u - v| (1 + 0.15
    Re^0.687) below Re = 1000 (Stokes' 3 pi mu d |u - v| at small Re), and the
    Newton drag 0.44 (1/2) rho |u - v|^2 (pi d^2 / 4) above."""
    eg = 1.0 - 1e-9
    for tau, d in ((0.6, 0.5), (0.50001, 0.2)):
        p = _params(orc, tau=tau, d=d)
        mu = _mu(p)
        for slip in (1e-6, 1e-3, 0.1, 2.0):
            re = p.rho_g * slip * d / mu
            got = _force_per_sphere(p, orc.beta(p, eg, orc.omega_emms(1.0), slip), eg, slip)
            if re < 1000.0:
                want = 3.0 * math.pi * mu * d * slip * (1.0 + 0.15 * re ** 0.687)
            else:
                want = 0.44 * 0.5 * p.rho_g * slip * slip * math.pi * d * d / 4.0
            assert abs(got - want) <= 1e-7 * want, (tau, d, slip, re, got, want)
        # Stokes: the drag of a slow sphere grows linearly with its slip
        f1 = _force_per_sphere(p, orc.beta(p, eg, 1.0, 1e-9), eg, 1e-9)
        assert abs(f1 - 3.0 * math.pi * mu * d * 1e-9) <= 1e-3 * f1


def test_branch_switch_at_re_1000_uses_the_voidage(orc):
    """Eq. 22 puts eps_g in Re: at eps_g = 0.9 the Newton constant 0.44 takes
    over where eps_g rho |u - v| d / mu reaches 1000, not rho |u - v| d / mu;
    across the switch beta jumps by 0.44 / C_D(1000-) = 1.0039."""
    p = _params(orc, tau=0.5001, d=0.5)
    mu, eg, om = _mu(p), 0.9, 1.0
    s_switch = 1000.0 * mu / (eg * p.rho_g * p.d)
    below = orc.beta(p, eg, om, s_switch * (1 - 1e-12))
    above = orc.beta(p, eg, om, s_switch)
    cd_below = 24.0 / 1000.0 * (1.0 + 0.15 * 1000.0 ** 0.687)
    assert abs(above / below - 0.44 / cd_below) < 1e-9
    # at rho |u-v| d / mu = 1050 the Reynolds number of Eq. 22 is 945: still Schiller-Naumann
    s = 1050.0 * mu / (p.rho_g * p.d)
    re = eg * p.rho_g * s * p.d / mu
    want = 0.75 * eg * (1 - eg) * p.rho_g * s / p.d * (24.0 / re * (1.0 + 0.15 * re ** 0.687)) * om
    assert abs(orc.beta(p, eg, om, s) - want) <= 1e-12 * want


def test_openmp_oracle_is_bit_identical(orc):
    """The all-cores build (per-cell loops over OpenMP threads) steps a bed to
    the same bits as the single-thread build."""
    import oracle
    cfg = synth.bubble_small()
    a, b = oracle.Sim(cfg), oracle.Sim(cfg, omp=True)
    for _ in range(3):
        oa, ob = a.step(record=True), b.step(record=True)
    assert np.array_equal(a.f, b.f) and np.array_equal(a.pos, b.pos) and np.array_equal(a.vel, b.vel)
    assert np.array_equal(oa.ugas, ob.ugas) and np.array_equal(oa.beta, ob.beta) and np.array_equal(oa.fd, ob.fd)
