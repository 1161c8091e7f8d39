"""Python binding of the lbdps C ABI (include/lbdps.h).

Argument marshalling only: every step of the simulation runs in the HIP
library ``liblbdps.so`` built next to this file.  PyTorch supplies device
memory (the workspace and the canonical FP64 in/out buffers) and the stream.
If the library has not been built, importing the binding raises ImportError:
there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
# torch first: the library's HIP runtime dependency then binds to the runtime
# torch has already loaded, so the process holds one HIP (and HSA) runtime.
# Loaded the other way round, the process holds two, and the library's finds
# no device.
import torch  # noqa: F401

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbdps.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "lbdps.h")

LBDPS_OK, LBDPS_E_INVALID, LBDPS_E_SHAPE, LBDPS_E_DEVICE = 0, -1, -2, -3
LBDPS_E_UNSUPPORTED, LBDPS_E_NONFINITE, LBDPS_E_CAPACITY, LBDPS_E_STALL = -4, -5, -6, -7
LBDPS_FP64, LBDPS_FP32, LBDPS_FP32_STORE_FP16, LBDPS_FP32_STORE_BF16 = 0, 1, 2, 3
LBDPS_BC_PERIODIC, LBDPS_BC_WALL, LBDPS_BC_INLET, LBDPS_BC_OUTLET = 0, 1, 2, 3
LBDPS_MAX_CONTACTS = 32
LBDPS_MAX_SUBSTEPS = 64
KERNELS = ["collide", "drag", "scan", "scatter", "contacts", "resolve"]

PRECISIONS = {"fp64": LBDPS_FP64, "fp32": LBDPS_FP32, "fp16": LBDPS_FP32_STORE_FP16, "bf16": LBDPS_FP32_STORE_BF16}
BCS = {"periodic": LBDPS_BC_PERIODIC, "wall": LBDPS_BC_WALL, "inlet": LBDPS_BC_INLET, "outlet": LBDPS_BC_OUTLET}

c_i32, c_i64, c_dbl, c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p


class lbdps_params(ctypes.Structure):
    _fields_ = [
        ("nx", c_i32), ("ny", c_i32), ("bc", c_i32 * 4),
        ("tau", c_dbl), ("rho_g", c_dbl), ("rho_s", c_dbl), ("d_p", c_dbl),
        ("e_pp", c_dbl), ("e_pw", c_dbl), ("g", c_dbl * 2), ("body_force", c_dbl * 2),
        ("drag_ratio_mode", c_i32), ("u_gas_porosity", c_i32), ("omega_mode", c_i32),
        ("pressure_force_sign", c_i32), ("omega_dense", c_dbl), ("cs_smag", c_dbl),
        ("precision", c_i32), ("diagnostics", c_i32), ("n_sub", c_i32), ("particles_periodic_y", c_i32),
        ("diag_every", c_i32),
    ]


class lbdps3_params(ctypes.Structure):
    _fields_ = [
        ("nx", c_i32), ("ny", c_i32), ("nz", c_i32), ("tau", c_dbl), ("rho_g", c_dbl), ("rho_s", c_dbl),
        ("d_p", c_dbl), ("e_pp", c_dbl), ("g", c_dbl * 3), ("body_force", c_dbl * 3), ("omega_dense", c_dbl),
        ("pressure_force_sign", c_i32), ("precision", c_i32), ("diagnostics", c_i32),
    ]


class lbdps_tuning(ctypes.Structure):
    _fields_ = [("cluster_lists", c_i32), ("cluster_groups_max", c_i32), ("drag_tile", c_i32), ("sphere_tile", c_i32)]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")

_lib = ctypes.CDLL(LIB_PATH)
_P = ctypes.POINTER(lbdps_params)
_SIGS = {
    "lbdps_validate_params": (c_i32, [_P, c_i64]),
    "lbdps_workspace_bytes": (c_i32, [_P, c_i64, ctypes.POINTER(ctypes.c_size_t)]),
    "lbdps_create": (c_i32, [_P, c_i64, c_vp, ctypes.c_size_t, c_vp, c_vp, ctypes.POINTER(c_vp)]),
    "lbdps_set_state": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_i64]),
    "lbdps_step": (c_i32, [c_vp, c_i32]),
    "lbdps_collide_particles": (c_i32, [c_vp]),
    "lbdps_set_inlet": (c_i32, [c_vp, c_vp]),
    "lbdps3_conservation": (c_i32, [c_vp, ctypes.POINTER(c_dbl)]),
    "lbdps3_bgk_step": (c_i32, [c_vp, c_vp, c_i32, c_i32, c_i32, c_dbl, c_i32, c_vp]),
    "lbdps3_psm_step": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp, c_i32, c_i32, c_i32, c_dbl, c_dbl, c_i32, c_vp]),
    "lbdps_voidage": (c_i32, [c_vp, c_i32, c_i32, c_dbl, c_vp, c_vp, c_vp]),
    "lbdps_get_fields": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "lbdps_get_particles": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp]),
    "lbdps_get_pairs": (c_i32, [c_vp, c_vp, c_i64, ctypes.POINTER(c_i64)]),
    "lbdps_get_accel": (c_i32, [c_vp, c_vp]),
    "lbdps_get_state": (c_i32, [c_vp, c_vp, c_vp, c_vp, ctypes.POINTER(c_i64)]),
    "lbdps_conservation": (c_i32, [c_vp, ctypes.POINTER(c_dbl)]),
    "lbdps_count_histogram": (c_i32, [c_vp, ctypes.POINTER(c_i64), c_i32]),
    "lbdps_conservation_noalloc": (c_i32, [c_vp, ctypes.POINTER(c_dbl)]),
    "lbdps_diag_last": (c_i32, [c_vp, ctypes.POINTER(c_dbl), ctypes.POINTER(c_i64)]),
    "lbdps_counters": (c_i32, [c_vp, ctypes.POINTER(c_i64)]),
    "lbdps_outlet_crossings": (c_i32, [c_vp, ctypes.POINTER(c_i64), ctypes.POINTER(c_i64)]),
    "lbdps_tile_stats": (c_i32, [c_vp, ctypes.POINTER(c_i64)]),
    "lbdps_time_kernels": (c_i32, [c_vp, ctypes.c_uint32]),
    "lbdps_kernel_times": (c_i32, [c_vp, ctypes.POINTER(c_dbl), ctypes.POINTER(c_i64)]),
    "lbdps_set_tuning": (c_i32, [c_vp, ctypes.POINTER(lbdps_tuning)]),
    "lbdps_get_tuning": (c_i32, [c_vp, ctypes.POINTER(lbdps_tuning)]),
    "lbdps_autotune": (c_i32, [c_vp, c_i32, ctypes.POINTER(lbdps_tuning)]),
    "lbdps_batch_autotune": (c_i32, [c_vp, c_i32, ctypes.c_char_p]),
    "lbdps_destroy": (c_i32, [c_vp]),
    "lbdps_batch_workspace_bytes": (c_i32, [_P, c_i32, ctypes.POINTER(c_i64), ctypes.POINTER(ctypes.c_size_t)]),
    "lbdps_batch_create": (c_i32, [_P, c_i32, ctypes.POINTER(c_i64), c_vp, c_vp, ctypes.c_size_t, c_vp,
                                   ctypes.POINTER(c_vp)]),
    "lbdps_batch_bed": (c_i32, [c_vp, c_i32, ctypes.POINTER(c_vp)]),
    "lbdps_batch_step": (c_i32, [c_vp, c_i32]),
    "lbdps_batch_capture": (c_i32, [c_vp, c_i32]),
    "lbdps_batch_launch": (c_i32, [c_vp]),
    "lbdps_batch_sync": (c_i32, [c_vp]),
    "lbdps_batch_time_kernels": (c_i32, [c_vp, ctypes.c_uint32]),
    "lbdps_batch_kernel_times": (c_i32, [c_vp, ctypes.POINTER(c_dbl), ctypes.POINTER(c_i64)]),
    "lbdps_batch_destroy": (c_i32, [c_vp]),
    "lbdps3_validate_params": (c_i32, [ctypes.POINTER(lbdps3_params), c_i64]),
    "lbdps3_workspace_bytes": (c_i32, [ctypes.POINTER(lbdps3_params), c_i64, ctypes.POINTER(ctypes.c_size_t)]),
    "lbdps3_create": (c_i32, [ctypes.POINTER(lbdps3_params), c_i64, c_vp, ctypes.c_size_t, c_vp,
                              ctypes.POINTER(c_vp)]),
    "lbdps3_set_state": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_i64]),
    "lbdps3_step": (c_i32, [c_vp, c_i32]),
    "lbdps3_get_state": (c_i32, [c_vp, c_vp, c_vp, c_vp]),
    "lbdps3_get_fields": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "lbdps3_get_drag": (c_i32, [c_vp, c_vp, c_vp]),
    "lbdps3_get_pairs": (c_i32, [c_vp, c_vp, c_i64, ctypes.POINTER(c_i64)]),
    "lbdps3_counters": (c_i32, [c_vp, ctypes.POINTER(c_i64)]),
    "lbdps3_destroy": (c_i32, [c_vp]),
    "lbdps_status_str": (ctypes.c_char_p, [c_i32]),
    "lbdps_last_error": (ctypes.c_char_p, []),
}
for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.restype, _fn.argtypes = _res, _args
    globals()[_name] = _fn


def header_functions(path: str = HEADER) -> list:
    """Names of the functions declared in include/lbdps.h."""
    text = open(path).read()
    decl = r"^\s*(?:lbdps_status|const\s+char\s*\*)\s*(lbdps[0-9]*_[a-z0-9_]+)\s*\("
    return sorted(set(re.findall(decl, text, flags=re.M)))


class LbdpsError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = lbdps_last_error().decode() or lbdps_status_str(status).decode()
        super().__init__(f"{where}: {lbdps_status_str(status).decode()} ({status}): {msg}")
        self.status = status


def check(status: int, where: str = "lbdps"):
    if status != LBDPS_OK:
        raise LbdpsError(status, where)


def make_params(cfg: dict, precision=None, diagnostics: bool = False) -> lbdps_params:
    """Parameter struct from a workload dict (keys as produced by ``synth``)."""
    p = lbdps_params()
    p.nx, p.ny = int(cfg["nx"]), int(cfg["ny"])
    for k, v in enumerate(cfg["bc"]):
        p.bc[k] = BCS[v] if isinstance(v, str) else int(v)
    p.tau = float(cfg.get("tau", 0.6))
    p.rho_g = float(cfg.get("rho_g", 1.0))
    p.rho_s = float(cfg.get("rho_s", 788.5))
    p.d_p = float(cfg.get("d", 0.5))
    p.e_pp = float(cfg.get("e_pp", 0.9))
    p.e_pw = float(cfg.get("e_pw", cfg.get("e_pp", 0.9)))
    g, G = cfg.get("g", (0.0, 0.0)), cfg.get("G", (0.0, 0.0))
    p.g[0], p.g[1] = float(g[0]), float(g[1])
    p.body_force[0], p.body_force[1] = float(G[0]), float(G[1])
    p.drag_ratio_mode = int(cfg.get("drag_ratio_mode", 0))
    p.u_gas_porosity = int(cfg.get("u_gas_porosity", 0))
    p.omega_mode = int(cfg.get("omega_mode", 0))
    p.pressure_force_sign = int(cfg.get("pressure_sign", -1))
    p.omega_dense = float(cfg.get("omega_dense", 1.0))
    p.cs_smag = float(cfg.get("cs_smag", 0.0))
    prec = precision if precision is not None else cfg.get("precision", "fp32")
    p.precision = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
    p.diagnostics = int(bool(diagnostics))
    p.n_sub = int(cfg.get("n_sub", 1))
    p.particles_periodic_y = int(cfg.get("particles_periodic_y", 0))
    p.diag_every = int(cfg.get("diag_every", 0))
    return p


def workspace_bytes(params: lbdps_params, max_particles: int) -> int:
    out = ctypes.c_size_t(0)
    check(lbdps_workspace_bytes(ctypes.byref(params), int(max_particles), ctypes.byref(out)), "workspace_bytes")
    return out.value


class Sim:
    """One context on the current HIP device (torch "cuda" device)."""

    def __init__(self, cfg: dict, precision=None, diagnostics: bool = False, max_particles=None, stream=None):
        import torch
        self.torch = torch
        self.cfg = cfg
        self.params = make_params(cfg, precision, diagnostics)
        pos = np.asarray(cfg["pos"], np.float64).reshape(-1, 2)
        self.n = len(pos)
        self.nmax = int(max_particles if max_particles is not None else self.n)
        self.nx, self.ny = self.params.nx, self.params.ny
        nbytes = workspace_bytes(self.params, self.nmax)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        inlet = cfg.get("inlet_uy")
        inlet_arr = None if inlet is None else np.ascontiguousarray(inlet, np.float64)
        ctx = c_vp()
        check(lbdps_create(ctypes.byref(self.params), self.nmax, self.ws.data_ptr(), nbytes,
                           None if inlet_arr is None else inlet_arr.ctypes.data_as(c_vp),
                           self.stream.cuda_stream, ctypes.byref(ctx)), "lbdps_create")
        self.ctx = ctx
        self._owner = None
        self.set_state(None, pos, cfg.get("vel", np.zeros_like(pos)))

    @classmethod
    def attach(cls, ctx, cfg: dict, params: lbdps_params, stream, owner):
        """View of a context that ``owner`` (a Batch) created and releases."""
        import torch
        self = cls.__new__(cls)
        self.torch = torch
        self.cfg, self.params, self.stream, self.ctx, self._owner = cfg, params, stream, ctx, owner
        self.nx, self.ny = params.nx, params.ny
        self.n = self.nmax = len(np.asarray(cfg["pos"]).reshape(-1, 2))
        return self

    def _dev(self, a, dtype=None):
        t = self.torch
        return t.as_tensor(np.ascontiguousarray(a), dtype=dtype or t.float64).to("cuda").contiguous()

    def set_state(self, f, pos, vel):
        t = self.torch
        with t.cuda.stream(self.stream):  # the uploads are ordered before the library's launches
            pos = self._dev(np.asarray(pos, np.float64).reshape(-1, 2))
            vel = self._dev(np.asarray(vel, np.float64).reshape(-1, 2))
            fd = None if f is None else self._dev(np.asarray(f, np.float64).reshape(9, self.ny, self.nx))
            self.n = pos.shape[0]
            check(lbdps_set_state(self.ctx, None if fd is None else fd.data_ptr(), pos.data_ptr(),
                                  vel.data_ptr(), self.n), "lbdps_set_state")
        self.stream.synchronize()

    def step(self, nsteps: int = 1):
        check(lbdps_step(self.ctx, int(nsteps)), "lbdps_step")

    def collide_particles(self):
        check(lbdps_collide_particles(self.ctx), "lbdps_collide_particles")

    def set_inlet(self, inlet_uy):
        a = np.ascontiguousarray(inlet_uy, np.float64)
        if a.shape != (self.nx,):
            raise ValueError(f"inlet profile must have {self.nx} entries")
        check(lbdps_set_inlet(self.ctx, a.ctypes.data), "lbdps_set_inlet")

    def voidage(self, y0: int = 0, y1=None, threshold: float = 0.85):
        """(row sums [ny], column sums over rows y0..y1-1 [nx], cells of those rows
        with eps_g > threshold) of the current positions (lbdps_voidage)."""
        t = self.torch
        y1 = self.ny if y1 is None else y1
        with t.cuda.stream(self.stream):  # zeroed before the library's launches
            rows = t.zeros(self.ny, dtype=t.float64, device="cuda")
            cols = t.zeros(self.nx, dtype=t.float64, device="cuda")
            cnt = t.zeros(1, dtype=t.int64, device="cuda")
            check(lbdps_voidage(self.ctx, int(y0), int(y1), float(threshold), rows.data_ptr(), cols.data_ptr(),
                                cnt.data_ptr()), "lbdps_voidage")
        self.stream.synchronize()
        return rows.cpu().numpy(), cols.cpu().numpy(), int(cnt.item())

    def fields(self):
        t = self.torch
        C = self.nx * self.ny
        rho = t.empty(C, dtype=t.float64, device="cuda")
        ug = t.empty(C, 2, dtype=t.float64, device="cuda")
        fpg = t.empty(C, 2, dtype=t.float64, device="cuda")
        beta = t.empty(C, dtype=t.float64, device="cuda")
        diag = bool(self.params.diagnostics)
        ncell = t.empty(C, dtype=t.int32, device="cuda") if diag else None
        vs = t.empty(C, 2, dtype=t.float64, device="cuda") if diag else None
        check(lbdps_get_fields(self.ctx, rho.data_ptr(), ug.data_ptr(), fpg.data_ptr(), beta.data_ptr(),
                               ncell.data_ptr() if diag else None, vs.data_ptr() if diag else None),
              "lbdps_get_fields")
        sh = (self.ny, self.nx)
        out = dict(rho=rho.cpu().numpy().reshape(sh), ugas=ug.cpu().numpy().reshape(*sh, 2),
                   fpg=fpg.cpu().numpy().reshape(*sh, 2), beta=beta.cpu().numpy().reshape(sh))
        if diag:
            out["ncell"] = ncell.cpu().numpy().reshape(sh)
            out["vs"] = vs.cpu().numpy().reshape(*sh, 2)
        return out

    def particles(self):
        t = self.torch
        n = max(self.n, 1)
        pos = t.empty(n, 2, dtype=t.float64, device="cuda")
        vel = t.empty(n, 2, dtype=t.float64, device="cuda")
        cell = t.empty(n, 2, dtype=t.int32, device="cuda")
        diag = bool(self.params.diagnostics)
        fd = t.empty(n, 2, dtype=t.float64, device="cuda") if diag else None
        check(lbdps_get_particles(self.ctx, pos.data_ptr(), vel.data_ptr(), fd.data_ptr() if diag else None,
                                  cell.data_ptr()), "lbdps_get_particles")
        out = dict(pos=pos.cpu().numpy()[: self.n], vel=vel.cpu().numpy()[: self.n],
                   cell=cell.cpu().numpy()[: self.n])
        if diag:
            out["fd"] = fd.cpu().numpy()[: self.n]
        return out

    def accel(self):
        """Acceleration of Eq. 16 of the most recent step by particle index
        [n][2] (lbdps_get_accel; diagnostics on or n_sub > 1)."""
        t = self.torch
        a = t.empty(max(self.n, 1), 2, dtype=t.float64, device="cuda")
        check(lbdps_get_accel(self.ctx, a.data_ptr()), "lbdps_get_accel")
        return a.cpu().numpy()[: self.n]

    def pairs(self, cap=None):
        t = self.torch
        cap = int(cap if cap is not None else max(16, LBDPS_MAX_CONTACTS * self.n // 2 + 16))
        buf = t.empty(cap, 2, dtype=t.int32, device="cuda")
        m = c_i64(0)
        check(lbdps_get_pairs(self.ctx, buf.data_ptr(), cap, ctypes.byref(m)), "lbdps_get_pairs")
        return buf[: min(m.value, cap)].cpu().numpy(), m.value

    def state(self):
        t = self.torch
        n = max(self.n, 1)
        f = t.empty(9, self.ny, self.nx, dtype=t.float64, device="cuda")
        pos = t.empty(n, 2, dtype=t.float64, device="cuda")
        vel = t.empty(n, 2, dtype=t.float64, device="cuda")
        st = c_i64(0)
        check(lbdps_get_state(self.ctx, f.data_ptr(), pos.data_ptr(), vel.data_ptr(), ctypes.byref(st)),
              "lbdps_get_state")
        return f.cpu().numpy(), pos.cpu().numpy()[: self.n], vel.cpu().numpy()[: self.n], st.value

    def conservation(self):
        out = (c_dbl * 6)()
        check(lbdps_conservation(self.ctx, out), "lbdps_conservation")
        return np.array(out[:])

    def conservation_noalloc(self):
        """lbdps_conservation_noalloc: the same sums, scratch in the library's
        static device array."""
        out = (c_dbl * 6)()
        check(lbdps_conservation_noalloc(self.ctx, out), "lbdps_conservation_noalloc")
        return np.array(out[:])

    def count_histogram(self, nbins: int = 16):
        """lbdps_count_histogram: cells holding 0, 1, ... nbins - 2 particles,
        and nbins - 1 or more."""
        out = (c_i64 * nbins)()
        check(lbdps_count_histogram(self.ctx, out, int(nbins)), "lbdps_count_histogram")
        return np.array(out[:])

    def diag_last(self):
        """lbdps_diag_last: the latest periodic check's sums and the step after
        which it ran (-1 if none has)."""
        out, step = (c_dbl * 6)(), c_i64(0)
        check(lbdps_diag_last(self.ctx, out, ctypes.byref(step)), "lbdps_diag_last")
        return np.array(out[:]), step.value

    def counters(self):
        out = (c_i64 * 4)()
        check(lbdps_counters(self.ctx, out), "lbdps_counters")
        return dict(pairs=out[0], collisions=out[1], walls=out[2], zero_den=out[3])

    def tile_stats(self):
        """(particles resolved in LDS tiles, particles left to the neighbour
        rows) of the most recent collision stage (lbdps_tile_stats)."""
        out = (c_i64 * 2)()
        check(lbdps_tile_stats(self.ctx, out), "lbdps_tile_stats")
        return out[0], out[1]

    def outlet_crossings(self):
        """(net particles across the outlet plane y = ny upward, steps) since
        the previous call (lbdps_outlet_crossings)."""
        net, steps = c_i64(0), c_i64(0)
        check(lbdps_outlet_crossings(self.ctx, ctypes.byref(net), ctypes.byref(steps)), "lbdps_outlet_crossings")
        return net.value, steps.value

    def tuning(self) -> dict:
        t = lbdps_tuning()
        check(lbdps_get_tuning(self.ctx, ctypes.byref(t)), "lbdps_get_tuning")
        return {n: getattr(t, n) for n, _ in lbdps_tuning._fields_}

    def set_tuning(self, **kw):
        t = lbdps_tuning(**{**self.tuning(), **kw})
        check(lbdps_set_tuning(self.ctx, ctypes.byref(t)), "lbdps_set_tuning")

    def autotune(self, steps: int = 4) -> dict:
        t = lbdps_tuning()
        check(lbdps_autotune(self.ctx, int(steps), ctypes.byref(t)), "lbdps_autotune")
        return {n: getattr(t, n) for n, _ in lbdps_tuning._fields_}

    def time_kernels(self, names):
        mask = 0
        for n in names:
            mask |= 1 << KERNELS.index(n)
        check(lbdps_time_kernels(self.ctx, mask), "lbdps_time_kernels")

    def kernel_times(self):
        ms = (c_dbl * len(KERNELS))()
        cnt = (c_i64 * len(KERNELS))()
        check(lbdps_kernel_times(self.ctx, ms, cnt), "lbdps_kernel_times")
        return {k: (ms[i], cnt[i]) for i, k in enumerate(KERNELS)}

    def close(self):
        if getattr(self, "_owner", None) is not None:
            return  # released with its batch
        if getattr(self, "ctx", None):
            self.stream.synchronize()
            lbdps_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_workspace_bytes(params, nmax) -> int:
    out = ctypes.c_size_t(0)
    check(lbdps_batch_workspace_bytes(params, len(params), nmax, ctypes.byref(out)), "batch_workspace_bytes")
    return out.value


class Batch:
    """Independent beds stepped together: one launch per phase of the step for
    all beds, optionally replayed from a captured hipGraph.  ``beds[i]`` is a
    Sim view of bed i (set_state, fields, particles, state, counters ...)."""

    def __init__(self, cfgs: list, precision=None, stream=None):
        import torch
        self.torch = torch
        nb = len(cfgs)
        self.params = (lbdps_params * nb)(*[make_params(c, precision) for c in cfgs])
        self.nmax = (c_i64 * nb)(*[len(np.asarray(c["pos"]).reshape(-1, 2)) for c in cfgs])
        nbytes = batch_workspace_bytes(self.params, self.nmax)
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self._inlets = [None if c.get("inlet_uy") is None else np.ascontiguousarray(c["inlet_uy"], np.float64)
                        for c in cfgs]
        ptrs = (c_vp * nb)(*[None if a is None else a.ctypes.data for a in self._inlets])
        torch.cuda.synchronize()
        b = c_vp()
        check(lbdps_batch_create(self.params, nb, self.nmax, ctypes.cast(ptrs, c_vp), self.ws.data_ptr(), nbytes,
                                 self.stream.cuda_stream, ctypes.byref(b)), "lbdps_batch_create")
        self.batch = b
        self.beds = []
        for i, c in enumerate(cfgs):
            ctx = c_vp()
            check(lbdps_batch_bed(b, i, ctypes.byref(ctx)), "lbdps_batch_bed")
            sim = Sim.attach(ctx, c, self.params[i], self.stream, self)
            pos = np.asarray(c["pos"], np.float64).reshape(-1, 2)
            sim.set_state(None, pos, c.get("vel", np.zeros_like(pos)))
            self.beds.append(sim)

    def reset(self):
        """Every bed back to its configuration's initial state."""
        for sim in self.beds:
            pos = np.asarray(sim.cfg["pos"], np.float64).reshape(-1, 2)
            sim.set_state(None, pos, sim.cfg.get("vel", np.zeros_like(pos)))

    def step(self, nsteps: int = 1):
        check(lbdps_batch_step(self.batch, int(nsteps)), "lbdps_batch_step")

    def autotune(self, steps: int = 4, cache_path=None) -> list:
        """Choose launch shapes per bed size class (see lbdps_batch_autotune);
        returns each bed's tuning."""
        path = None if cache_path is None else os.fsencode(cache_path)
        check(lbdps_batch_autotune(self.batch, int(steps), path), "lbdps_batch_autotune")
        return [b.tuning() for b in self.beds]

    def capture(self, nsteps: int):
        check(lbdps_batch_capture(self.batch, int(nsteps)), "lbdps_batch_capture")

    def launch(self):
        check(lbdps_batch_launch(self.batch), "lbdps_batch_launch")

    def sync(self):
        check(lbdps_batch_sync(self.batch), "lbdps_batch_sync")

    def time_kernels(self, names):
        mask = 0
        for n in names:
            mask |= 1 << KERNELS.index(n)
        check(lbdps_batch_time_kernels(self.batch, mask), "lbdps_batch_time_kernels")

    def kernel_times(self):
        ms = (c_dbl * len(KERNELS))()
        cnt = (c_i64 * len(KERNELS))()
        check(lbdps_batch_kernel_times(self.batch, ms, cnt), "lbdps_batch_kernel_times")
        return {k: (ms[i], cnt[i]) for i, k in enumerate(KERNELS)}

    def close(self):
        if getattr(self, "batch", None):
            self.stream.synchronize()
            lbdps_batch_destroy(self.batch)
            self.batch = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_params3(cfg: dict, precision=None, diagnostics: bool = False) -> lbdps3_params:
    """3-D parameters from a workload dict (nx, ny, nz, tau, rho_g, rho_s, d,
    e_pp, g[3], G[3], omega_dense, pressure_sign)."""
    p = lbdps3_params()
    p.nx, p.ny, p.nz = int(cfg["nx"]), int(cfg["ny"]), int(cfg["nz"])
    p.tau, p.rho_g, p.rho_s, p.d_p, p.e_pp = (float(cfg[k]) for k in ("tau", "rho_g", "rho_s", "d", "e_pp"))
    for a in range(3):
        p.g[a] = float(cfg["g"][a])
        p.body_force[a] = float(cfg["G"][a])
    p.omega_dense = float(cfg.get("omega_dense", 1.0))
    p.pressure_force_sign = int(cfg.get("pressure_sign", -1))
    prec = precision if precision is not None else cfg.get("precision", "fp64")
    p.precision = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
    p.diagnostics = int(bool(diagnostics))
    return p


class Sim3:
    """One 3-D coupled context (lbdps3_*) on the current HIP device."""

    def __init__(self, cfg: dict, precision=None, diagnostics: bool = False, stream=None):
        import torch
        self.torch = torch
        self.cfg = cfg
        self.params = make_params3(cfg, precision, diagnostics)
        pos = np.asarray(cfg["pos"], np.float64).reshape(-1, 3)
        self.n = len(pos)
        self.nx, self.ny, self.nz = self.params.nx, self.params.ny, self.params.nz
        nbytes = ctypes.c_size_t(0)
        check(lbdps3_workspace_bytes(ctypes.byref(self.params), self.n, ctypes.byref(nbytes)), "lbdps3_workspace_bytes")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.ws = torch.empty(nbytes.value, dtype=torch.uint8, device="cuda")
        ctx = c_vp()
        check(lbdps3_create(ctypes.byref(self.params), self.n, self.ws.data_ptr(), nbytes.value,
                            self.stream.cuda_stream, ctypes.byref(ctx)), "lbdps3_create")
        self.ctx = ctx
        self.set_state(None, pos, cfg.get("vel", np.zeros_like(pos)))

    def _dev(self, a):
        return self.torch.as_tensor(np.ascontiguousarray(a, np.float64)).to("cuda").contiguous()

    def set_state(self, f, pos, vel):
        t = self.torch
        with t.cuda.stream(self.stream):
            pos = self._dev(np.asarray(pos, np.float64).reshape(-1, 3))
            vel = self._dev(np.asarray(vel, np.float64).reshape(-1, 3))
            fd = None if f is None else self._dev(np.asarray(f, np.float64).reshape(19, self.nz, self.ny, self.nx))
            self.n = pos.shape[0]
            check(lbdps3_set_state(self.ctx, None if fd is None else fd.data_ptr(), pos.data_ptr(), vel.data_ptr(),
                                   self.n), "lbdps3_set_state")
        self.stream.synchronize()

    def step(self, nsteps: int = 1):
        check(lbdps3_step(self.ctx, int(nsteps)), "lbdps3_step")

    def state(self):
        t = self.torch
        n = max(self.n, 1)
        f = t.empty(19, self.nz, self.ny, self.nx, dtype=t.float64, device="cuda")
        pos = t.empty(n, 3, dtype=t.float64, device="cuda")
        vel = t.empty(n, 3, dtype=t.float64, device="cuda")
        check(lbdps3_get_state(self.ctx, f.data_ptr(), pos.data_ptr(), vel.data_ptr()), "lbdps3_get_state")
        return f.cpu().numpy(), pos.cpu().numpy()[: self.n], vel.cpu().numpy()[: self.n]

    def fields(self):
        t = self.torch
        C = self.nx * self.ny * self.nz
        rho = t.empty(C, dtype=t.float64, device="cuda")
        ug = t.empty(C, 3, dtype=t.float64, device="cuda")
        fpg = t.empty(C, 3, dtype=t.float64, device="cuda")
        beta = t.empty(C, dtype=t.float64, device="cuda")
        diag = bool(self.params.diagnostics)
        ncell = t.empty(C, dtype=t.int32, device="cuda") if diag else None
        check(lbdps3_get_fields(self.ctx, rho.data_ptr(), ug.data_ptr(), fpg.data_ptr(), beta.data_ptr(),
                                ncell.data_ptr() if diag else None), "lbdps3_get_fields")
        sh = (self.nz, self.ny, self.nx)
        out = dict(rho=rho.cpu().numpy().reshape(sh), ugas=ug.cpu().numpy().reshape(*sh, 3),
                   fpg=fpg.cpu().numpy().reshape(*sh, 3), beta=beta.cpu().numpy().reshape(sh))
        if diag:
            out["ncell"] = ncell.cpu().numpy().reshape(sh)
        return out

    def drag(self):
        t = self.torch
        n = max(self.n, 1)
        fd = t.empty(n, 3, dtype=t.float64, device="cuda")
        acc = t.empty(n, 3, dtype=t.float64, device="cuda")
        check(lbdps3_get_drag(self.ctx, fd.data_ptr(), acc.data_ptr()), "lbdps3_get_drag")
        return fd.cpu().numpy()[: self.n], acc.cpu().numpy()[: self.n]

    def pairs(self, cap=None):
        t = self.torch
        cap = int(cap if cap is not None else max(16, LBDPS_MAX_CONTACTS * self.n // 2 + 16))
        buf = t.empty(cap, 2, dtype=t.int32, device="cuda")
        m = c_i64(0)
        check(lbdps3_get_pairs(self.ctx, buf.data_ptr(), cap, ctypes.byref(m)), "lbdps3_get_pairs")
        return buf[: min(m.value, cap)].cpu().numpy(), m.value

    def counters(self):
        out = (c_i64 * 2)()
        check(lbdps3_counters(self.ctx, out), "lbdps3_counters")
        return dict(pairs=out[0], collisions=out[1])

    def conservation(self):
        """lbdps3_conservation: mass, gas momentum (3), particle momentum (3),
        non-finite flag."""
        out = (c_dbl * 8)()
        check(lbdps3_conservation(self.ctx, out), "lbdps3_conservation")
        return np.array(out[:])

    def close(self):
        if getattr(self, "ctx", None):
            self.stream.synchronize()
            lbdps3_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
