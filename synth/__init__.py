"""Seeded synthetic inputs for the LBM discrete-particle workloads.

This module holds random-number generation and workload recipes only (lattice
sizes, boundary faces, parameters and initial particle positions).  It carries
none of the simulation method's arithmetic.  Both the FP64 oracle runs and the
GPU runs take their inputs from here, so they start from the same state.

Random numbers: splitmix64 (Steele, Lea & Flood, OOPSLA 2014), output k of a
stream with seed s is mix(s + (k+1) * 0x9E3779B97F4A7C15); a uniform double is
(x >> 11) * 2^-53.  Draws are consumed in particle-index order, x then y.

The workloads borrow the shapes of the paper's two experiments (bubble
injection, Table 1; riser, Table 2) at the sizes of the benchmark plan;
paper_bubble and paper_riser take the tables' own sizes and parameters.  No
dataset is involved.
"""
from __future__ import annotations

import math

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """Outputs offset .. offset+count-1 of the splitmix64 stream for ``seed``."""
    k = np.arange(offset + 1, offset + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + k * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """Uniform doubles in [0, 1) from splitmix64."""
    return (splitmix64(seed, count, offset) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


# Physical defaults shared by every workload (lattice units): tau = 0.6,
# gas density 1, solid density 788.5 (Tables 1-2, dimensionless column),
# restitution 0.9 (Tables 1-2), particle diameter 0.5 cells.
DEFAULTS = dict(tau=0.6, rho_g=1.0, rho_s=788.5, d=0.5, e_pp=0.9, e_pw=0.9,
                drag_ratio_mode=0, u_gas_porosity=0, omega_mode=0, pressure_sign=-1,
                omega_dense=1.0, cs_smag=0.0, G=(0.0, 0.0))

DISC = math.pi * 0.25 / 4.0  # area of a d = 0.5 disc, used only to size seeding bands


def _cfg(name, nx, ny, bc, pos, steps, **kw):
    c = dict(DEFAULTS)
    c.update(kw)
    c.update(name=name, nx=nx, ny=ny, bc=list(bc), steps=steps,
             pos=np.ascontiguousarray(pos, np.float64),
             vel=np.ascontiguousarray(kw.get("vel", np.zeros_like(pos)), np.float64))
    return c


def cell_order(pos: np.ndarray, nx: int) -> np.ndarray:
    """Permutation that numbers particles in row-major cell order of their
    position (ties by draw order): the numbering a spatially sorted injector
    would give."""
    key = np.floor(pos[:, 1]).astype(np.int64) * nx + np.floor(pos[:, 0]).astype(np.int64)
    return np.argsort(key, kind="stable")


def bubble_small(seed: int = 1) -> dict:
    """64x256 bed, x periodic, inflow u = 0.01 at the bottom, zero-gradient
    outlet at the top, 2000 spheres (d = 0.5) seeded uniformly in a bottom band
    whose 2-D solid area fraction is 0.35 (band height N pi d^2/(4 0.35 nx) =
    17.53 rows), zero velocity, gravity 1e-5, 100 steps.  FP64."""
    nx, ny, n, phi, r = 64, 256, 2000, 0.35, 0.25
    band = n * DISC / (phi * nx)
    u = uniform(seed, 2 * n).reshape(n, 2)
    pos = np.empty((n, 2))
    pos[:, 0] = nx * u[:, 0]
    pos[:, 1] = r + (band - 2 * r) * u[:, 1]
    return _cfg("bubble-64x256-2k-fp64", nx, ny, ["periodic", "periodic", "inlet", "outlet"], pos, 100,
                inlet_uy=np.full(nx, 0.01), g=(0.0, -1e-5), precision="fp64")


def bubble(seed: int = 2, v_mf: float = 0.005) -> dict:
    """Bubble-injection shape: 256x1024 bed, 200 000 spheres on a jittered
    square lattice (365 columns, 548 rows, the last row holding 345) filling a
    bottom band of 2-D solid fraction 0.4 (383.5 rows), jitter uniform +-0.09
    per axis so no two spheres touch at t = 0.  Inflow v_mf = 0.005 everywhere
    except 3 v_mf on the 8 central columns x in [124, 132).  Gravity 4.35e-7,
    which balances the bed's weight against the drag at v_mf (cell force balance
    at solid fraction 0.4).  2000 steps, FP32."""
    nx, ny, n, phi = 256, 1024, 200_000, 0.4
    band = n * DISC / (phi * nx)
    ncol = 365
    nrow = -(-n // ncol)
    dx, dy = nx / ncol, band / nrow
    k = np.arange(n)
    col, row = k % ncol, k // ncol
    jit = (uniform(seed, 2 * n).reshape(n, 2) * 2.0 - 1.0) * 0.09
    pos = np.empty((n, 2))
    pos[:, 0] = (col + 0.5) * dx + jit[:, 0]
    pos[:, 1] = (row + 0.5) * dy + jit[:, 1]
    inlet = np.full(nx, v_mf)
    inlet[124:132] = 3.0 * v_mf
    return _cfg("bubble-256x1024-200k-fp32", nx, ny, ["periodic", "periodic", "inlet", "outlet"], pos, 2000,
                inlet_uy=inlet, g=(0.0, -4.35e-7), precision="fp32")


# Riser shape: a body force on the gas balances the particles' weight.  With
# m = 788.5 pi 0.5^3/6 = 51.607, g_eff = (1 - 1/788.5) 2.82e-7 and 0.95367
# particles per cell, N m g_eff / C = 1.38614e-5 per cell.
RISER_G = (0.0, -2.82e-7)
RISER_BODY = (0.0, 1.38614e-5)


def riser(nx: int = 512, ny: int = 4096, n: int = 2_000_000, seed: int = 3, sort_ids: bool = True,
          precision: str = "fp32") -> dict:
    """Riser shape: y periodic, x walls, n spheres uniform in
    x in [r, nx - r), y in [0, ny), zero velocity, gas driven upward by a body
    force, particle gravity 2.82e-7.  Default 512x4096 with 2 000 000 spheres
    (0.954 per cell).  sort_ids numbers particles in cell order."""
    r = 0.25
    u = uniform(seed, 2 * n).reshape(n, 2)
    pos = np.empty((n, 2))
    pos[:, 0] = r + (nx - 2 * r) * u[:, 0]
    pos[:, 1] = ny * u[:, 1]
    if sort_ids:
        pos = pos[cell_order(pos, nx)]
    ids = "" if sort_ids else "-random-ids"
    return _cfg(f"riser-{nx}x{ny}-{n}{ids}-{precision}", nx, ny, ["wall", "wall", "periodic", "periodic"], pos,
                5000, inlet_uy=None, g=RISER_G, G=RISER_BODY, precision=precision)


def riser_crop(seed: int = 3, precision: str = "fp32") -> dict:
    """64x512 bed at the riser's density: 31 250 spheres."""
    return riser(64, 512, 31_250, seed, True, precision)


def riser_large(seed: int = 3) -> dict:
    """2048x8192 bed (16.8 M cells) at the riser's density: 16 000 000 spheres."""
    return riser(2048, 8192, 16_000_000, seed, True, "fp32")


# The paper's own experiments in lattice units (Tables 1 and 2; h = 2.7e-4 m).
# Velocities convert by dt / h, gravity 9.81 m/s^2 to 9.81 dt^2 / h, and the gas
# viscosity to mu_lu = mu_g dt / (rho_g h^2), which gives tau = 3 mu_lu + 1/2
# (Eq. 3, rho_g = 1 in lattice units).  Where a printed dimensionless value
# disagrees with its dimensional one (the bubble's jet velocity, the riser's
# viscosity), the converted value is taken.  tau lies so close to 1/2 that the
# Smagorinsky model (Eqs. 12-15) is on, with C_s = PAPER_CS (the paper gives no
# value).
PAPER_H = 2.7e-4
PAPER_CS = 0.3


def paper_gravity(dt: float) -> float:
    """9.81 m/s^2 in lattice units for time step dt (s) and cell size PAPER_H."""
    return 9.81 * dt * dt / PAPER_H


def paper_tau(dt: float, mu_g: float = 1.8872e-5, rho_g: float = 1.1795) -> float:
    """tau = 3 mu_lu + 1/2 with mu_lu = mu_g dt / (rho_g h^2)."""
    return 3.0 * mu_g * dt / (rho_g * PAPER_H * PAPER_H) + 0.5


def paper_bubble(seed: int = 11) -> dict:
    """Table 1: a 25 x 100 bed (walls at x, gas inlet at the bottom, outlet at
    the top) holding 15 000 spheres of d = 0.2 at incipient fluidization; gas
    enters at v_mf = 0.0025 m/s = 1.25e-5 except through the 3-cell central
    orifice x in [11, 14), where a jet of 0.8 m/s = 0.004 lasts 0.006 s = 4 444
    steps of 1.35e-6 s (cfg["pulse_steps"]; cfg["inlet_after"] is the profile
    afterwards).  tau = 3 (2.963e-4) + 1/2.  Incipient fluidization: the drag
    of Eqs. 19-22 at v_mf carries the weight of a cell of about 25.3 spheres
    (2-D solid fraction 0.795, 3-D voidage 0.57), so the spheres sit on a
    hexagonal lattice of that fraction (spacing 0.2137; rows of 117 and 116
    alternately, 23.9 rows in all, the outer centres 0.104 from the walls),
    with a jitter of +-0.004 per axis so no two touch at t = 0 and none
    reaches a wall."""
    nx, ny, n, d = 25, 100, 15_000, 0.2
    a = (nx - d - 0.008) / 116.0       # spacing: 117 centres from x = 0.104 to 24.896
    dy = a * math.sqrt(3.0) / 2.0
    pos = np.empty((n, 2))
    k, row = 0, 0
    while k < n:
        cols = 117 if row % 2 == 0 else 116
        m = min(cols, n - k)
        x0 = 0.5 * d + 0.004 + (0.0 if row % 2 == 0 else 0.5 * a)
        pos[k:k + m, 0] = x0 + a * np.arange(m)
        pos[k:k + m, 1] = 0.5 * d + 0.004 + dy * row
        k += m
        row += 1
    pos += (uniform(seed, 2 * n).reshape(n, 2) * 2.0 - 1.0) * 0.004
    v_mf, v_inj = 0.0025 * 1.35e-6 / PAPER_H, 0.8 * 1.35e-6 / PAPER_H
    after = np.full(nx, v_mf)
    inlet = after.copy()
    inlet[11:14] = v_inj
    return _cfg("paper-bubble-25x100-15k-fp64", nx, ny, ["wall", "wall", "inlet", "outlet"], pos, 26_000,
                d=d, tau=paper_tau(1.35e-6), cs_smag=PAPER_CS, inlet_uy=inlet, inlet_after=after,
                pulse_steps=int(0.006 / 1.35e-6), g=(0.0, -paper_gravity(1.35e-6)), precision="fp64")


def paper_riser(seed: int = 12) -> dict:
    """Table 2: a 60 x 720 riser holding 123 921 spheres of d = 0.2 (2-D solid
    fraction 0.09012, uniform), time step 6e-6 s, tau = 3 (1.317e-3) + 1/2.
    Gas enters at the bottom at the table's 1.52 m/s = 0.0338 and leaves at
    the top; the spheres circulate: one leaving through the top re-enters at
    the bottom (cfg["particles_periodic_y"]), as the riser's solids return
    through the loop of a circulating bed.  The gas starts uniform at the
    inlet velocity (cfg["u0"]) (R43)."""
    nx, ny, n, d = 60, 720, 123_921, 0.2
    r = 0.5 * d
    u = uniform(seed, 2 * n).reshape(n, 2)
    pos = np.empty((n, 2))
    pos[:, 0] = r + (nx - 2 * r) * u[:, 0]
    pos[:, 1] = ny * u[:, 1]
    pos = pos[cell_order(pos, nx)]
    v_in = 1.52 * 6.0e-6 / PAPER_H
    return _cfg("paper-riser-60x720-124k-fp64", nx, ny, ["wall", "wall", "inlet", "outlet"], pos, 100_000,
                d=d, tau=paper_tau(6.0e-6), cs_smag=PAPER_CS, inlet_uy=np.full(nx, v_in), u0=(0.0, v_in),
                particles_periodic_y=1, g=(0.0, -paper_gravity(6.0e-6)), precision="fp64")


# Gravity of the batched beds: the bubble bed's balance of bed weight against
# drag at minimum fluidization (4.35e-7 at v_mf = 0.005), scaled to their
# inlet velocity 0.01.  With 1e-5, beds this tall (bands up to 512 rows) are
# unstable under the method itself: in cells whose particles' pre-drags nearly
# cancel, the per-cell ratio of Eq. 28 (condition numbers 1e3 - 3e4) gives
# kicks of 0.1 - 0.5 and the FP64 oracle reaches speeds above 0.05 cells/step
# within 120 - 140 steps.
BEDS_G = (0.0, -8.7e-7)


def beds(count: int = 64, seed0: int = 1000) -> list:
    """Batch of uneven beds: bed b draws s, phi from seed seed0 + b; nx =
    round(64 4^s), ny = 4 nx, 2-D solid fraction phi = 0.05 + 0.35 u, particle
    count clip(round(phi nx ny / 2 / (pi d^2/4)), 2000, 200000) seeded
    uniformly in a bottom band of that fraction; faces and inflow as
    bubble_small, gravity BEDS_G."""
    out = []
    for b in range(count):
        s, uphi = uniform(seed0 + b, 2)
        nx = int(round(64 * 4.0 ** s))
        ny = 4 * nx
        phi = 0.05 + 0.35 * uphi
        n = int(np.clip(round(phi * nx * ny / 2 / DISC), 2000, 200_000))
        band = min(n * DISC / (phi * nx), ny - 1.0)
        u = uniform(seed0 + b, 2 * n, offset=2).reshape(n, 2)
        pos = np.empty((n, 2))
        pos[:, 0] = nx * u[:, 0]
        pos[:, 1] = 0.25 + (band - 0.5) * u[:, 1]
        pos = pos[cell_order(pos, nx)]
        out.append(_cfg(f"bed{b}-{nx}x{ny}-{n}", nx, ny, ["periodic", "periodic", "inlet", "outlet"], pos, 200,
                        inlet_uy=np.full(nx, 0.01), g=BEDS_G, precision="fp16"))
    return out


def tiny(nx: int = 16, ny: int = 24, n: int = 60, seed: int = 7, bc=("periodic", "periodic", "inlet", "outlet"),
         band: float | None = None, vel_scale: float = 0.0, **kw) -> dict:
    """Small random bed for unit and parity tests: n spheres uniform in
    [0, nx) x [r, band - r) (band defaults to ny), velocities uniform in
    +-vel_scale."""
    r = 0.5 * kw.get("d", DEFAULTS["d"])
    band = ny if band is None else band
    u = uniform(seed, 4 * n).reshape(n, 4)
    pos = np.empty((n, 2))
    xlo = 0.0 if bc[0] == "periodic" else r
    xhi = nx if bc[0] == "periodic" else nx - r
    pos[:, 0] = xlo + (xhi - xlo) * u[:, 0]
    ylo = 0.0 if bc[2] == "periodic" else r
    yhi = band if bc[2] == "periodic" else band - r
    pos[:, 1] = ylo + (yhi - ylo) * u[:, 1]
    vel = (u[:, 2:4] * 2.0 - 1.0) * vel_scale
    inlet = kw.pop("inlet_uy", np.full(nx, 0.01) if "inlet" in bc else None)
    kw.setdefault("g", (0.0, -1e-5))
    return _cfg(f"tiny-{nx}x{ny}-{n}", nx, ny, list(bc), pos, 10, vel=vel, inlet_uy=inlet, **kw)


# ---------------------------------------------------------------- 3-D beds
# 3-D riser: gravity along -z (the long axis), a body force on the gas balances
# the particles' weight, every face periodic.
RISER3_G = 2.82e-7


def riser3d(nx: int = 256, ny: int = 256, nz: int = 1024, n: int = 10_000_000, seed: int = 5,
            sort_ids: bool = True) -> dict:
    """3-D riser shape: a fully periodic D3Q19 box, n spheres of d = 0.5
    uniform in it at rest (default 256 x 256 x 1024 with 10 000 000: 0.149 per
    cell, 3-D solid fraction 0.0098), particle gravity 2.82e-7 along -z, and
    the gas driven along +z by the body force n m g_eff / C that balances the
    particles' weight.  sort_ids numbers particles in cell order (z, y, x)."""
    u = uniform(seed, 3 * n).reshape(n, 3)
    pos = u * np.array([nx, ny, nz], np.float64)
    if sort_ids:
        key = (np.floor(pos[:, 2]).astype(np.int64) * ny + np.floor(pos[:, 1]).astype(np.int64)) * nx \
            + np.floor(pos[:, 0]).astype(np.int64)
        pos = pos[np.argsort(key, kind="stable")]
    c = dict(DEFAULTS)
    m = c["rho_s"] * math.pi * c["d"] ** 3 / 6
    geff = (1 - c["rho_g"] / c["rho_s"]) * RISER3_G
    c.update(name=f"riser3d-{nx}x{ny}x{nz}-{n}", nx=nx, ny=ny, nz=nz, pos=np.ascontiguousarray(pos),
             vel=np.zeros_like(pos), g=(0.0, 0.0, -RISER3_G), G=(0.0, 0.0, n * m * geff / (nx * ny * nz)),
             steps=500)
    return c


def tiny3d(nx: int = 6, ny: int = 5, nz: int = 7, n: int = 60, seed: int = 7, vel_scale: float = 0.0,
           **kw) -> dict:
    """Small periodic 3-D bed for unit and parity tests: n spheres uniform in
    the box, velocities uniform in +-vel_scale."""
    u = uniform(seed, 6 * n).reshape(n, 6)
    pos = u[:, :3] * np.array([nx, ny, nz], np.float64)
    vel = (u[:, 3:] * 2.0 - 1.0) * vel_scale
    c = dict(DEFAULTS)
    c.update(name=f"tiny3d-{nx}x{ny}x{nz}-{n}", nx=nx, ny=ny, nz=nz, pos=pos, vel=vel, g=(0.0, 0.0, -1e-5),
             G=(0.0, 0.0, 0.0), steps=10)
    c.update(kw)
    return c
