"""FP64 CPU oracle of the LBM-based discrete particle step (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``.  The product library under
``paper_1303_2653_amd/`` never imports, links or calls anything here, and the
two share no code.

The arithmetic lives in ``lbdps_oracle.c`` (plain C99, FP64, contraction off);
this module only builds it, loads it and marshals numpy arrays.  Section,
equation and reading references are in the C source next to each function.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbdps_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
# The same source built with -fopenmp: the per-cell loops run over all host
# cores, bit-identical results (the all-cores CPU baseline of the benchmark).
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")

PERIODIC, WALL, INLET, OUTLET = 0, 1, 2, 3
BC_NAMES = {"periodic": PERIODIC, "wall": WALL, "inlet": INLET, "outlet": OUTLET}


def build(force: bool = True) -> str:
    """Compile liboracle.so (single thread) and liboracle_omp.so (per-cell
    loops over OpenMP threads) with gcc (FP64, -ffp-contract=off)."""
    for out, extra in ((LIB, []), (LIB_OMP, ["-fopenmp"])):
        if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(SRC):
            cmd = ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fPIC", "-shared", *extra,
                   "-o", out + ".tmp", SRC, "-lm"]
            subprocess.run(cmd, check=True)
            os.replace(out + ".tmp", out)
    return LIB


class OrcParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("bc", ctypes.c_int32 * 4),
        ("tau", ctypes.c_double),
        ("rho_g", ctypes.c_double), ("rho_s", ctypes.c_double), ("d", ctypes.c_double),
        ("e_pp", ctypes.c_double), ("e_pw", ctypes.c_double),
        ("g", ctypes.c_double * 2), ("G", ctypes.c_double * 2),
        ("drag_ratio_mode", ctypes.c_int32), ("u_gas_porosity", ctypes.c_int32),
        ("omega_mode", ctypes.c_int32), ("pressure_sign", ctypes.c_int32),
        ("omega_dense", ctypes.c_double),
        ("cs_smag", ctypes.c_double),
        ("n_sub", ctypes.c_int32),
        ("particles_periodic_y", ctypes.c_int32),
    ]


class OrcOut(ctypes.Structure):
    _fields_ = [
        ("ncell", ctypes.c_void_p), ("vs", ctypes.c_void_p), ("rho", ctypes.c_void_p),
        ("ugas", ctypes.c_void_p), ("fpg", ctypes.c_void_p), ("beta", ctypes.c_void_p),
        ("fd", ctypes.c_void_p), ("fpre", ctypes.c_void_p), ("upart", ctypes.c_void_p),
        ("acc", ctypes.c_void_p),
        ("pairs", ctypes.c_void_p),
        ("pair_cap", ctypes.c_int64), ("npairs", ctypes.c_int64),
        ("ncollisions", ctypes.c_int64), ("nwall", ctypes.c_int64),
        ("nzero_den", ctypes.c_int64), ("ncross", ctypes.c_int64),
    ]


class Orc3Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("tau", ctypes.c_double), ("rho_g", ctypes.c_double), ("rho_s", ctypes.c_double),
                ("d", ctypes.c_double), ("e_pp", ctypes.c_double), ("g", ctypes.c_double * 3),
                ("G", ctypes.c_double * 3), ("omega_dense", ctypes.c_double), ("pressure_sign", ctypes.c_int32)]


class Orc3Out(ctypes.Structure):
    _fields_ = [("ncell", ctypes.c_void_p), ("vs", ctypes.c_void_p), ("rho", ctypes.c_void_p),
                ("ugas", ctypes.c_void_p), ("fpg", ctypes.c_void_p), ("beta", ctypes.c_void_p),
                ("fd", ctypes.c_void_p), ("acc", ctypes.c_void_p), ("pairs", ctypes.c_void_p),
                ("pair_cap", ctypes.c_int64), ("npairs", ctypes.c_int64), ("ncollisions", ctypes.c_int64)]


_libs = {}


def lib(omp: bool = False):
    """The loaded oracle library; omp=True: the OpenMP build."""
    path = LIB_OMP if omp else LIB
    if path not in _libs:
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(SRC):
            build(force=False)
        L = ctypes.CDLL(path)
        P = ctypes.POINTER(OrcParams)
        vp = ctypes.c_void_p
        i64 = ctypes.c_int64
        L.orc_threads.restype = ctypes.c_int32
        L.orc_feq.restype = ctypes.c_double
        L.orc_feq.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.orc_gamma.restype = ctypes.c_double
        L.orc_gamma.argtypes = [ctypes.c_double, ctypes.c_double]
        L.orc_omega_emms.restype = ctypes.c_double
        L.orc_omega_emms.argtypes = [ctypes.c_double]
        L.orc_cd0.restype = ctypes.c_double
        L.orc_cd0.argtypes = [ctypes.c_double]
        L.orc_beta.restype = ctypes.c_double
        L.orc_beta.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.orc_cell_props.argtypes = [P, i64, vp]
        L.orc_collide_node.argtypes = [P, vp, i64, vp, vp, vp]
        L.orc_stream.argtypes = [P, vp, vp, vp]
        L.orc_stencil.argtypes = [P, ctypes.c_double, ctypes.c_double, vp, vp]
        L.orc_interp.restype = ctypes.c_double
        L.orc_interp.argtypes = [P, vp, ctypes.c_double, ctypes.c_double]
        L.orc_grad_p.argtypes = [P, vp, vp]
        L.orc_integrate.argtypes = [P, i64, vp, vp, vp, vp]
        L.orc_contacts_brute.restype = ctypes.c_int
        L.orc_contacts_brute.argtypes = [P, i64, vp, vp, i64, ctypes.POINTER(i64)]
        L.orc_contacts_cells.restype = ctypes.c_int
        L.orc_contacts_cells.argtypes = [P, i64, vp, vp, i64, ctypes.POINTER(i64)]
        L.orc_contacts_f32.restype = ctypes.c_int
        L.orc_contacts_f32.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_float, i64, vp, vp, ctypes.c_int32, vp, i64,
                                       ctypes.POINTER(i64)]
        L.orc_solids_flux.restype = ctypes.c_double
        L.orc_solids_flux.argtypes = [P, i64, i64]
        L.orc_collide_f32.restype = ctypes.c_int
        L.orc_collide_f32.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, i64,
                                      vp, vp, vp, vp, i64, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                      ctypes.POINTER(i64)]
        L.orc_resolve.argtypes = [P, i64, vp, vp, vp, i64, ctypes.POINTER(i64)]
        L.orc_walls.argtypes = [P, i64, vp, vp, ctypes.POINTER(i64)]
        L.orc_step.restype = ctypes.c_int
        L.orc_step.argtypes = [P, vp, vp, i64, vp, vp, ctypes.POINTER(OrcOut)]
        L.orc_conservation.argtypes = [P, vp, i64, vp, vp]
        L.orc_lattice.argtypes = [vp, vp, vp]
        L.orc3_lattice.argtypes = [vp, vp]
        P3 = ctypes.POINTER(Orc3Params)
        L.orc3_cell_props.argtypes = [P3, i64, vp]
        L.orc3_stencil.argtypes = [P3, vp, vp, vp]
        L.orc3_interp.restype = ctypes.c_double
        L.orc3_interp.argtypes = [P3, vp, vp]
        L.orc3_contacts_brute.restype = ctypes.c_int
        L.orc3_contacts_brute.argtypes = [P3, i64, vp, vp, i64, ctypes.POINTER(i64)]
        L.orc3_contacts_cells.restype = ctypes.c_int
        L.orc3_contacts_cells.argtypes = [P3, i64, vp, vp, i64, ctypes.POINTER(i64)]
        L.orc3_resolve.argtypes = [P3, vp, vp, vp, i64, ctypes.POINTER(i64)]
        L.orc3_step.restype = ctypes.c_int
        L.orc3_step.argtypes = [P3, vp, i64, vp, vp, ctypes.POINTER(Orc3Out)]
        L.orc3_conservation.argtypes = [P3, vp, i64, vp, vp]
        L.orc3_feq.restype = ctypes.c_double
        L.orc3_feq.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.orc3_bgk_step.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, vp]
        L.orc3_psm_step.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                    vp, vp, vp, vp]
        _libs[path] = L
    return _libs[path]


def threads(omp: bool = False) -> int:
    """Threads the oracle's per-cell loops use (1 for the plain build)."""
    return int(lib(omp).orc_threads())


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _bc_code(v):
    return BC_NAMES[v] if isinstance(v, str) else int(v)


def make_params(cfg: dict) -> OrcParams:
    """Build the oracle's parameter struct from a workload dict (see ``synth``)."""
    p = OrcParams()
    p.nx, p.ny = int(cfg["nx"]), int(cfg["ny"])
    for k, v in enumerate(cfg["bc"]):
        p.bc[k] = _bc_code(v)
    p.tau = float(cfg.get("tau", 0.6))
    p.rho_g = float(cfg.get("rho_g", 1.0))
    p.rho_s = float(cfg.get("rho_s", 788.5))
    p.d = float(cfg.get("d", 0.5))
    p.e_pp = float(cfg.get("e_pp", 0.9))
    p.e_pw = float(cfg.get("e_pw", cfg.get("e_pp", 0.9)))
    g = cfg.get("g", (0.0, 0.0))
    G = cfg.get("G", (0.0, 0.0))
    p.g[0], p.g[1] = float(g[0]), float(g[1])
    p.G[0], p.G[1] = float(G[0]), float(G[1])
    p.drag_ratio_mode = int(cfg.get("drag_ratio_mode", 0))
    p.u_gas_porosity = int(cfg.get("u_gas_porosity", 0))
    p.omega_mode = int(cfg.get("omega_mode", 0))
    p.pressure_sign = int(cfg.get("pressure_sign", -1))
    p.omega_dense = float(cfg.get("omega_dense", 1.0))
    p.cs_smag = float(cfg.get("cs_smag", 0.0))
    p.n_sub = int(cfg.get("n_sub", 1))
    p.particles_periodic_y = int(cfg.get("particles_periodic_y", 0))
    return p


# ---------------------------------------------------------------- small pieces
def lattice():
    c = np.zeros((9, 2), np.int32)
    w = np.zeros(9)
    opp = np.zeros(9, np.int32)
    lib().orc_lattice(_ptr(c), _ptr(w), _ptr(opp))
    return c, w, opp


def feq(i, rho, ux, uy):
    return lib().orc_feq(int(i), float(rho), float(ux), float(uy))


def gamma(eps_s, tau):
    return lib().orc_gamma(float(eps_s), float(tau))


def omega_emms(eps_g):
    return lib().orc_omega_emms(float(eps_g))


def cd0(re):
    return lib().orc_cd0(float(re))


def beta(p: OrcParams, eps_g, om, slip):
    return lib().orc_beta(ctypes.byref(p), float(eps_g), float(om), float(slip))


def cell_props(p: OrcParams, n: int):
    out = np.zeros(6)
    lib().orc_cell_props(ctypes.byref(p), int(n), _ptr(out))
    return dict(eps_s2=out[0], eps_2=out[1], eps_s3=out[2], eps_g=out[3], gamma=out[4], omega=out[5])


def collide_node(p: OrcParams, f, n, vs):
    f = np.ascontiguousarray(f, np.float64)
    vs = np.ascontiguousarray(vs, np.float64)
    fs = np.zeros(9)
    o = np.zeros(8)
    lib().orc_collide_node(ctypes.byref(p), _ptr(f), int(n), _ptr(vs), _ptr(fs), _ptr(o))
    return fs, dict(rho=o[0], ugas=o[1:3].copy(), fpg=o[3:5].copy(), beta=o[5], usup=o[6:8].copy())


def stream(p: OrcParams, fstar, inlet_uy=None):
    fstar = np.ascontiguousarray(fstar, np.float64)
    out = np.zeros_like(fstar)
    iu = None if inlet_uy is None else np.ascontiguousarray(inlet_uy, np.float64)
    lib().orc_stream(ctypes.byref(p), _ptr(iu), _ptr(fstar), _ptr(out))
    return out


def stencil(p: OrcParams, px, py):
    idx = np.zeros(4, np.int64)
    wt = np.zeros(4)
    lib().orc_stencil(ctypes.byref(p), float(px), float(py), _ptr(idx), _ptr(wt))
    return idx, wt


def interp(p: OrcParams, q, px, py):
    q = np.ascontiguousarray(q, np.float64).reshape(-1)
    return lib().orc_interp(ctypes.byref(p), _ptr(q), float(px), float(py))


def grad_p(p: OrcParams, pres):
    pres = np.ascontiguousarray(pres, np.float64).reshape(-1)
    g = np.zeros((pres.size, 2))
    lib().orc_grad_p(ctypes.byref(p), _ptr(pres), _ptr(g))
    return g


def integrate(p: OrcParams, pos, vel, fd, gpk):
    pos = np.ascontiguousarray(pos, np.float64).copy()
    vel = np.ascontiguousarray(vel, np.float64).copy()
    fd = np.ascontiguousarray(fd, np.float64)
    gpk = np.ascontiguousarray(gpk, np.float64)
    lib().orc_integrate(ctypes.byref(p), len(pos), _ptr(pos), _ptr(vel), _ptr(fd), _ptr(gpk))
    return pos, vel


def contacts(p: OrcParams, pos, brute=False, cap=None):
    pos = np.ascontiguousarray(pos, np.float64)
    n = len(pos)
    cap = cap if cap is not None else max(16, 32 * n)
    pairs = np.zeros((cap, 2), np.int32)
    m = ctypes.c_int64(0)
    fn = lib().orc_contacts_brute if brute else lib().orc_contacts_cells
    rc = fn(ctypes.byref(p), n, _ptr(pos), _ptr(pairs), cap, ctypes.byref(m))
    if rc != 0:
        raise RuntimeError(f"oracle contacts failed rc={rc}")
    return pairs[: m.value].copy()


def contacts_f32(nx, ny, per_x, per_y, d, cell, off, brute=False, cap=None):
    cell = np.ascontiguousarray(cell, np.int32)
    off = np.ascontiguousarray(off, np.float32)
    n = len(cell)
    cap = cap if cap is not None else max(16, 32 * n)
    pairs = np.zeros((cap, 2), np.int32)
    m = ctypes.c_int64(0)
    rc = lib().orc_contacts_f32(int(nx), int(ny), int(per_x), int(per_y), float(np.float32(d)), n,
                                _ptr(cell), _ptr(off), int(bool(brute)), _ptr(pairs), cap,
                                ctypes.byref(m))
    if rc != 0:
        raise RuntimeError(f"oracle contacts_f32 failed rc={rc}")
    return pairs[: m.value].copy()


def collide_f32(p: OrcParams, cell, off, vel, cap=None):
    """The hard-sphere stage in single precision (orc_collide_f32): contacts,
    binary collisions in lexicographic order, then walls, on the cell
    [N][2] int32 + offset [N][2] float32 state with float32 velocities.
    Returns (pairs, new velocities float32 [N][2], collisions, wall hits)."""
    cell = np.ascontiguousarray(cell, np.int32)
    off = np.ascontiguousarray(off, np.float32)
    v = np.array(vel, np.float32, copy=True).reshape(-1, 2)
    n = len(cell)
    cap = cap if cap is not None else max(16, 32 * n)
    pairs = np.zeros((cap, 2), np.int32)
    m, nc, nw = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
    per_x = int(p.bc[0] == PERIODIC)
    per_y = int(p.bc[2] == PERIODIC or p.particles_periodic_y)
    rc = lib().orc_collide_f32(p.nx, p.ny, per_x, per_y, p.d, p.rho_s, p.e_pp, p.e_pw, n, _ptr(cell), _ptr(off),
                               _ptr(v), _ptr(pairs), cap, ctypes.byref(m), ctypes.byref(nc), ctypes.byref(nw))
    if rc != 0:
        raise RuntimeError(f"oracle collide_f32 failed rc={rc}")
    return pairs[: m.value].copy(), v, nc.value, nw.value


def resolve(p: OrcParams, pos, vel, pairs):
    pos = np.ascontiguousarray(pos, np.float64)
    vel = np.ascontiguousarray(vel, np.float64).copy()
    pairs = np.ascontiguousarray(pairs, np.int32)
    nc = ctypes.c_int64(0)
    lib().orc_resolve(ctypes.byref(p), len(pos), _ptr(pos), _ptr(vel), _ptr(pairs), len(pairs),
                      ctypes.byref(nc))
    return vel, nc.value


def walls(p: OrcParams, pos, vel):
    pos = np.ascontiguousarray(pos, np.float64)
    vel = np.ascontiguousarray(vel, np.float64).copy()
    nw = ctypes.c_int64(0)
    lib().orc_walls(ctypes.byref(p), len(pos), _ptr(pos), _ptr(vel), ctypes.byref(nw))
    return vel, nw.value


def conservation(p: OrcParams, f, vel):
    f = np.ascontiguousarray(f, np.float64)
    vel = np.ascontiguousarray(vel, np.float64)
    out = np.zeros(5)
    lib().orc_conservation(ctypes.byref(p), _ptr(f), len(vel), _ptr(vel), _ptr(out))
    return out


def voidage(p: OrcParams, pos, y0=0, y1=None, threshold=0.85):
    """Voidage statistics of Sec. 3 at particle positions pos [N][2]: the gas
    voidage of each cell is the 3-D one of Eq. 11 for the cell's count (the
    voidage of the drag laws, R42).  Returns (row_sum [ny]: sum over x of
    eps_g per row; col_sum [nx]: sum over rows y0..y1-1 per column; count:
    cells of rows y0..y1-1 with eps_g > threshold).  The equivalent bubble
    diameter of Sec. 3.1 is then sqrt(4 count / pi) cells."""
    nx, ny = p.nx, p.ny
    y1 = ny if y1 is None else y1
    pos = np.asarray(pos, np.float64).reshape(-1, 2)
    cell = (np.floor(pos[:, 1]).astype(np.int64) * nx + np.floor(pos[:, 0]).astype(np.int64))
    n = np.bincount(cell, minlength=nx * ny).reshape(ny, nx)
    eg = {k: cell_props(p, k)["eps_g"] for k in np.unique(n)}
    e = np.vectorize(eg.get, otypes=[np.float64])(n)
    rows = e.sum(axis=1)
    cols = e[y0:y1].sum(axis=0)
    count = int((e[y0:y1] > threshold).sum())
    return rows, cols, count


def solids_flux(p: OrcParams, net: int, steps: int) -> float:
    """Outlet solids mass flux (Sec. 3.2) of `net` particles across the outlet
    plane over `steps` steps: m net / (nx steps) in lattice units (R47)."""
    return lib().orc_solids_flux(ctypes.byref(p), int(net), int(steps))


# ---------------------------------------------------------------- 3-D gas lattice
def lattice3():
    c = np.zeros((19, 3), np.int32)
    w = np.zeros(19)
    lib().orc3_lattice(_ptr(c), _ptr(w))
    return c, w


def feq3(i, rho, ux, uy, uz):
    return lib().orc3_feq(int(i), float(rho), float(ux), float(uy), float(uz))


def bgk3_step(f, tau):
    """One periodic D3Q19 BGK step of f [19][nz][ny][nx] (returns a new array)."""
    f = np.array(f, np.float64, copy=True)
    _, nz, ny, nx = f.shape
    lib().orc3_bgk_step(nx, ny, nz, float(tau), _ptr(f))
    return f


def psm3_step(f, tau, d, n, vs):
    """One periodic D3Q19 step with the solids' partial saturation (Eqs. 6-7,
    9, 25 on the 3-D lattice): n [nz][ny][nx] spheres of diameter d per cell
    moving with vs [3][nz][ny][nx].  Returns (new f, force [3][nz][ny][nx])."""
    f = np.array(f, np.float64, copy=True)
    _, nz, ny, nx = f.shape
    n = np.ascontiguousarray(n, np.int32)
    vs = np.ascontiguousarray(vs, np.float64)
    assert n.shape == (nz, ny, nx) and vs.shape == (3, nz, ny, nx)
    force = np.zeros((3, nz, ny, nx))
    lib().orc3_psm_step(nx, ny, nz, float(tau), float(d), _ptr(n), _ptr(vs), _ptr(f), _ptr(force))
    return f, force


def equilibrium_state(nx, ny, rho=1.0, ux=0.0, uy=0.0):
    """f = f^eq(rho, u) on every node, [9][ny][nx] (R33 initial state)."""
    f = np.empty((9, ny, nx))
    for i in range(9):
        f[i] = feq(i, rho, ux, uy)
    return f


# ---------------------------------------------------------------- the step
@dataclass
class StepOut:
    ncell: np.ndarray
    vs: np.ndarray
    rho: np.ndarray
    ugas: np.ndarray
    fpg: np.ndarray
    beta: np.ndarray
    fd: np.ndarray
    fpre: np.ndarray
    upart: np.ndarray
    acc: np.ndarray
    pairs: np.ndarray
    ncollisions: int
    nwall: int
    nzero_den: int
    ncross: int


class Sim:
    """Holds an oracle state (f, pos, vel) and advances it with orc_step."""

    def __init__(self, cfg: dict, f=None, pos=None, vel=None, omp: bool = False):
        self.cfg = cfg
        self.omp = omp
        self.p = make_params(cfg)
        nx, ny = self.p.nx, self.p.ny
        self.inlet_uy = None
        if cfg.get("inlet_uy") is not None:
            self.inlet_uy = np.ascontiguousarray(cfg["inlet_uy"], np.float64)
        self.f = equilibrium_state(nx, ny) if f is None else np.array(f, np.float64, copy=True)
        pos = cfg["pos"] if pos is None else pos
        vel = cfg["vel"] if vel is None else vel
        self.pos = np.array(pos, np.float64, copy=True).reshape(-1, 2)
        self.vel = np.array(vel, np.float64, copy=True).reshape(-1, 2)
        self.nstep = 0

    def step(self, record=False, pair_cap=None):
        nx, ny = self.p.nx, self.p.ny
        C = nx * ny
        n = len(self.pos)
        o = OrcOut()
        bufs = {}
        if record:
            bufs = dict(ncell=np.zeros(C, np.int32), vs=np.zeros((C, 2)), rho=np.zeros(C),
                        ugas=np.zeros((C, 2)), fpg=np.zeros((C, 2)), beta=np.zeros(C),
                        fd=np.zeros((max(n, 1), 2)), fpre=np.zeros((max(n, 1), 2)),
                        upart=np.zeros((max(n, 1), 2)), acc=np.zeros((max(n, 1), 2)))
            cap = pair_cap if pair_cap is not None else max(16, 32 * n)
            bufs["pairs"] = np.zeros((cap, 2), np.int32)
            for k, v in bufs.items():
                setattr(o, k, v.ctypes.data)
            o.pair_cap = cap
        rc = lib(self.omp).orc_step(ctypes.byref(self.p), _ptr(self.inlet_uy), _ptr(self.f), n,
                            _ptr(self.pos), _ptr(self.vel), ctypes.byref(o))
        if rc != 0:
            raise RuntimeError(f"oracle step failed rc={rc}")
        self.nstep += 1
        if not record:
            return None
        return StepOut(ncell=bufs["ncell"].reshape(ny, nx), vs=bufs["vs"].reshape(ny, nx, 2),
                       rho=bufs["rho"].reshape(ny, nx), ugas=bufs["ugas"].reshape(ny, nx, 2),
                       fpg=bufs["fpg"].reshape(ny, nx, 2), beta=bufs["beta"].reshape(ny, nx),
                       fd=bufs["fd"][:n].copy(), fpre=bufs["fpre"][:n].copy(),
                       upart=bufs["upart"][:n].copy(), acc=bufs["acc"][:n].copy(), pairs=bufs["pairs"][: o.npairs].copy(),
                       ncollisions=o.ncollisions, nwall=o.nwall, nzero_den=o.nzero_den,
                       ncross=o.ncross)

    def run(self, nsteps):
        for _ in range(nsteps):
            self.step()

    def conservation(self):
        return conservation(self.p, self.f, self.vel)


# ---------------------------------------------------------------- the 3-D coupled step
def make_params3(cfg: dict) -> Orc3Params:
    """3-D parameters from a workload dict (nx, ny, nz, tau, rho_g, rho_s, d,
    e_pp, g[3], G[3], omega_dense)."""
    p = Orc3Params()
    p.nx, p.ny, p.nz = int(cfg["nx"]), int(cfg["ny"]), int(cfg["nz"])
    for k in ("tau", "rho_g", "rho_s", "d", "e_pp", "omega_dense"):
        setattr(p, k, float(cfg[k]))
    p.pressure_sign = int(cfg.get("pressure_sign", -1))
    for a in range(3):
        p.g[a] = float(cfg["g"][a])
        p.G[a] = float(cfg["G"][a])
    return p


def cell_props3(p: Orc3Params, n: int) -> dict:
    out = np.zeros(4)
    lib().orc3_cell_props(ctypes.byref(p), int(n), _ptr(out))
    return dict(eps_s=out[0], eps_g=out[1], gamma=out[2], omega=out[3])


def stencil3(p: Orc3Params, P):
    P = np.ascontiguousarray(P, np.float64)
    idx, wt = np.zeros(8, np.int64), np.zeros(8)
    lib().orc3_stencil(ctypes.byref(p), _ptr(P), _ptr(idx), _ptr(wt))
    return idx, wt


def interp3(p: Orc3Params, q, P):
    q = np.ascontiguousarray(q, np.float64).reshape(-1)
    return lib().orc3_interp(ctypes.byref(p), _ptr(q), _ptr(np.ascontiguousarray(P, np.float64)))


def contacts3(p: Orc3Params, pos, brute=False, cap=None):
    pos = np.ascontiguousarray(pos, np.float64).reshape(-1, 3)
    n = len(pos)
    cap = cap if cap is not None else max(16, 32 * n)
    pairs = np.zeros((cap, 2), np.int32)
    m = ctypes.c_int64(0)
    fn = lib().orc3_contacts_brute if brute else lib().orc3_contacts_cells
    rc = fn(ctypes.byref(p), n, _ptr(pos), _ptr(pairs), cap, ctypes.byref(m))
    if rc != 0:
        raise RuntimeError(f"oracle contacts3 failed rc={rc}")
    return pairs[: m.value].copy()


def resolve3(p: Orc3Params, pos, vel, pairs):
    pos = np.ascontiguousarray(pos, np.float64).reshape(-1, 3)
    vel = np.array(vel, np.float64, copy=True).reshape(-1, 3)
    pairs = np.ascontiguousarray(pairs, np.int32)
    nc = ctypes.c_int64(0)
    lib().orc3_resolve(ctypes.byref(p), _ptr(pos), _ptr(vel), _ptr(pairs), len(pairs), ctypes.byref(nc))
    return vel, nc.value


def conservation3(p: Orc3Params, f, vel):
    f = np.ascontiguousarray(f, np.float64)
    vel = np.ascontiguousarray(vel, np.float64).reshape(-1, 3)
    out = np.zeros(7)
    lib().orc3_conservation(ctypes.byref(p), _ptr(f), len(vel), _ptr(vel), _ptr(out))
    return out


def equilibrium_state3(nx, ny, nz, rho=1.0, u=(0.0, 0.0, 0.0)):
    f = np.empty((19, nz, ny, nx))
    for i in range(19):
        f[i] = feq3(i, rho, *u)
    return f


@dataclass
class Step3Out:
    ncell: np.ndarray
    vs: np.ndarray
    rho: np.ndarray
    ugas: np.ndarray
    fpg: np.ndarray
    beta: np.ndarray
    fd: np.ndarray
    acc: np.ndarray
    pairs: np.ndarray
    ncollisions: int


class Sim3:
    """An oracle state of the 3-D coupled step (f [19][nz][ny][nx], pos and
    vel [N][3]) advanced with orc3_step."""

    def __init__(self, cfg: dict, f=None, pos=None, vel=None, omp: bool = False):
        self.cfg, self.omp = cfg, omp
        self.p = make_params3(cfg)
        nx, ny, nz = self.p.nx, self.p.ny, self.p.nz
        self.f = equilibrium_state3(nx, ny, nz) if f is None else np.array(f, np.float64, copy=True)
        self.pos = np.array(cfg["pos"] if pos is None else pos, np.float64, copy=True).reshape(-1, 3)
        self.vel = np.array(cfg["vel"] if vel is None else vel, np.float64, copy=True).reshape(-1, 3)

    def step(self, record=False, pair_cap=None):
        nx, ny, nz = self.p.nx, self.p.ny, self.p.nz
        C, n = nx * ny * nz, len(self.pos)
        o = Orc3Out()
        bufs = {}
        if record:
            bufs = dict(ncell=np.zeros(C, np.int32), vs=np.zeros((C, 3)), rho=np.zeros(C), ugas=np.zeros((C, 3)),
                        fpg=np.zeros((C, 3)), beta=np.zeros(C), fd=np.zeros((max(n, 1), 3)),
                        acc=np.zeros((max(n, 1), 3)))
            cap = pair_cap if pair_cap is not None else max(16, 32 * n)
            bufs["pairs"] = np.zeros((cap, 2), np.int32)
            for k, v in bufs.items():
                setattr(o, k, v.ctypes.data)
            o.pair_cap = cap
        rc = lib(self.omp).orc3_step(ctypes.byref(self.p), _ptr(self.f), n, _ptr(self.pos), _ptr(self.vel),
                                     ctypes.byref(o))
        if rc != 0:
            raise RuntimeError(f"oracle 3-D step failed rc={rc}")
        if not record:
            return None
        sh = (nz, ny, nx)
        return Step3Out(ncell=bufs["ncell"].reshape(sh), vs=bufs["vs"].reshape(*sh, 3), rho=bufs["rho"].reshape(sh),
                        ugas=bufs["ugas"].reshape(*sh, 3), fpg=bufs["fpg"].reshape(*sh, 3),
                        beta=bufs["beta"].reshape(sh), fd=bufs["fd"][:n].copy(), acc=bufs["acc"][:n].copy(),
                        pairs=bufs["pairs"][: o.npairs].copy(), ncollisions=o.ncollisions)

    def conservation(self):
        return conservation3(self.p, self.f, self.vel)
