"""C ABI contract checks that need no GPU: the library loads, exports every
function include/lbdps.h declares, and validates parameters and sizes the
workspace without touching a device."""
import ctypes

import pytest

import synth

L = pytest.importorskip("paper_1303_2653_amd.lbdps", reason="HIP library not built")


def test_exports_every_declared_symbol():
    names = L.header_functions()
    assert len(names) >= 15
    lib = ctypes.CDLL(L.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n


def test_struct_layout_matches_header():
    # offsets of the C struct on x86-64 / LP64 (natural alignment)
    assert L.lbdps_params.tau.offset == 24
    assert L.lbdps_params.g.offset == 72
    assert L.lbdps_params.drag_ratio_mode.offset == 104
    assert L.lbdps_params.omega_dense.offset == 120
    assert L.lbdps_params.precision.offset == 136
    assert L.lbdps_params.n_sub.offset == 144
    assert L.lbdps_params.particles_periodic_y.offset == 148
    assert L.lbdps_params.diag_every.offset == 152
    assert ctypes.sizeof(L.lbdps_params) == 160


def _status(p, nmax=10):
    return L.lbdps_validate_params(ctypes.byref(p), nmax)


def test_validation_accepts_workloads():
    for cfg in (synth.bubble_small(), synth.bubble(), synth.riser_crop()):
        p = L.make_params(cfg)
        assert _status(p, len(cfg["pos"])) == L.LBDPS_OK, L.lbdps_last_error()


@pytest.mark.parametrize("field,value,code", [
    ("nx", 2, L.LBDPS_E_SHAPE), ("ny", 0, L.LBDPS_E_SHAPE), ("tau", 0.5, L.LBDPS_E_INVALID),
    ("tau", float("nan"), L.LBDPS_E_INVALID), ("d_p", 1.0, L.LBDPS_E_INVALID), ("d_p", 0.0, L.LBDPS_E_INVALID),
    ("e_pp", 1.5, L.LBDPS_E_INVALID), ("e_pw", -0.1, L.LBDPS_E_INVALID), ("rho_s", 0.0, L.LBDPS_E_INVALID),
    ("precision", 7, L.LBDPS_E_INVALID), ("pressure_force_sign", 2, L.LBDPS_E_INVALID),
    ("cs_smag", -0.1, L.LBDPS_E_INVALID), ("cs_smag", float("inf"), L.LBDPS_E_INVALID),
    ("drag_ratio_mode", 3, L.LBDPS_E_INVALID), ("n_sub", -1, L.LBDPS_E_INVALID),
    ("n_sub", L.LBDPS_MAX_SUBSTEPS + 1, L.LBDPS_E_INVALID), ("particles_periodic_y", 2, L.LBDPS_E_INVALID),
    ("diag_every", -1, L.LBDPS_E_INVALID),
])
def test_validation_rejects(field, value, code):
    p = L.make_params(synth.bubble_small())
    setattr(p, field, value)
    assert _status(p) == code
    assert L.lbdps_last_error()


def test_validation_rejects_bad_faces():
    p = L.make_params(synth.bubble_small())
    p.bc[0] = L.LBDPS_BC_INLET
    assert _status(p) == L.LBDPS_E_INVALID
    p = L.make_params(synth.bubble_small())
    p.bc[2] = L.LBDPS_BC_PERIODIC  # y- periodic with y+ outlet
    assert _status(p) == L.LBDPS_E_INVALID
    p = L.make_params(synth.bubble_small())
    assert _status(p, -1) == L.LBDPS_E_SHAPE
    assert L.lbdps_validate_params(None, 0) == L.LBDPS_E_INVALID


def test_substeps_accepted_and_sized():
    """n_sub 0 and 1 mean one sub-step; more keep two accelerations per particle."""
    p = L.make_params(synth.bubble_small())
    for v in (0, 1, 4, L.LBDPS_MAX_SUBSTEPS):
        p.n_sub = v
        assert _status(p) == L.LBDPS_OK
    p.n_sub = 1
    b1 = L.workspace_bytes(p, 2000)
    p.n_sub = 0
    assert L.workspace_bytes(p, 2000) == b1
    p.n_sub = 3
    assert L.workspace_bytes(p, 2000) >= b1 + 2 * 2000 * 4


def test_workspace_bytes_scale():
    p = L.make_params(synth.bubble())
    b0 = L.workspace_bytes(p, 0)
    b1 = L.workspace_bytes(p, 200_000)
    C = 256 * 1024
    assert b0 > 2 * 9 * C * 4  # two population buffers
    # per particle: 2 x 24-byte records, 5 int32 work arrays, 32 contact slots of 8 bytes
    assert b1 - b0 >= 200_000 * (48 + 20 + 256)
    p.precision = L.LBDPS_FP32_STORE_FP16
    assert L.workspace_bytes(p, 0) < b0
    p.diagnostics = 1
    assert L.workspace_bytes(p, 0) > L.workspace_bytes(L.make_params(synth.bubble(), "fp16"), 0)


def test_create_rejects_small_workspace_before_device():
    p = L.make_params(synth.bubble_small())
    ctx = ctypes.c_void_p()
    st = L.lbdps_create(ctypes.byref(p), 10, ctypes.c_void_p(256), 16, None, None, ctypes.byref(ctx))
    assert st == L.LBDPS_E_SHAPE and not ctx.value
    st = L.lbdps_create(ctypes.byref(p), 10, None, 1 << 30, None, None, ctypes.byref(ctx))
    assert st == L.LBDPS_E_INVALID


def test_status_strings():
    for s in range(-7, 1):
        assert L.lbdps_status_str(s)


def _batch(cfgs, prec=None):
    params = (L.lbdps_params * len(cfgs))(*[L.make_params(c, prec) for c in cfgs])
    nmax = (ctypes.c_int64 * len(cfgs))(*[len(c["pos"]) for c in cfgs])
    return params, nmax


def test_batch_workspace_covers_every_bed():
    cfgs = [synth.tiny(nx=16, ny=24, n=60), synth.tiny(nx=40, ny=20, n=10), synth.bubble_small()]
    params, nmax = _batch(cfgs, "fp32")
    total = L.batch_workspace_bytes(params, nmax)
    assert total >= sum(L.workspace_bytes(params[i], nmax[i]) for i in range(len(cfgs)))


def test_batch_rejects_mixed_precision_and_diagnostics():
    cfgs = [synth.tiny(nx=16, ny=24, n=60), synth.tiny(nx=40, ny=20, n=10)]
    params, nmax = _batch(cfgs, "fp32")
    params[1].precision = L.LBDPS_FP64
    out = ctypes.c_size_t(0)
    assert L.lbdps_batch_workspace_bytes(params, 2, nmax, ctypes.byref(out)) == L.LBDPS_E_INVALID
    params, nmax = _batch(cfgs, "fp32")
    params[0].diagnostics = 1
    assert L.lbdps_batch_workspace_bytes(params, 2, nmax, ctypes.byref(out)) == L.LBDPS_E_UNSUPPORTED
    params, nmax = _batch(cfgs, "fp32")
    params[1].n_sub = 2  # batched beds take one particle sub-step
    assert L.lbdps_batch_workspace_bytes(params, 2, nmax, ctypes.byref(out)) == L.LBDPS_E_UNSUPPORTED
    params[1].n_sub = 1
    assert L.lbdps_batch_workspace_bytes(params, 2, nmax, ctypes.byref(out)) == L.LBDPS_OK
    params[0].diag_every = 10  # batched beds take no periodic check
    assert L.lbdps_batch_workspace_bytes(params, 2, nmax, ctypes.byref(out)) == L.LBDPS_E_UNSUPPORTED
    params[0].diag_every = 0
    params, nmax = _batch(cfgs, "fp32")
    assert L.lbdps_batch_workspace_bytes(params, 0, nmax, ctypes.byref(out)) == L.LBDPS_E_SHAPE
    params[1].tau = 0.4
    assert L.lbdps_batch_workspace_bytes(params, 2, nmax, ctypes.byref(out)) == L.LBDPS_E_INVALID
    assert b"bed 1" in L.lbdps_last_error()


def test_batch_create_rejects_small_workspace_before_device():
    cfgs = [synth.tiny(nx=16, ny=24, n=60), synth.tiny(nx=40, ny=20, n=10)]
    params, nmax = _batch(cfgs, "fp32")
    b = ctypes.c_void_p()
    st = L.lbdps_batch_create(params, 2, nmax, None, ctypes.c_void_p(256), 16, None, ctypes.byref(b))
    assert st == L.LBDPS_E_SHAPE and not b.value
    assert L.lbdps_batch_step(None, 1) == L.LBDPS_E_INVALID
    assert L.lbdps_batch_capture(None, 2) == L.LBDPS_E_INVALID


def test_tuning_struct_layout():
    assert ctypes.sizeof(L.lbdps_tuning) == 16 and L.lbdps_tuning.sphere_tile.offset == 12
    assert L.lbdps_set_tuning(None, None) == L.LBDPS_E_INVALID
    assert L.lbdps_autotune(None, 1, None) == L.LBDPS_E_INVALID
    assert L.lbdps_batch_autotune(None, 1, None) == L.LBDPS_E_INVALID


def test_cell_row_by_multiplication_is_exact():
    """The library computes key // nx as (key * m) >> s with s = 31 +
    ceil(log2 nx), m = ceil(2^s / nx): exact for every key < 2^31 (the error
    term stays below 1 / nx).  Checked here on widths 1..4096, powers of two
    and their neighbours, at the keys where a floor changes."""
    import random
    rng = random.Random(3)
    widths = list(range(1, 4097)) + [2 ** k + d for k in range(12, 31) for d in (-1, 0, 1)]
    for nx in widths:
        if nx < 1:
            continue
        s = 31 + max(0, (nx - 1).bit_length())
        m = -(-(1 << s) // nx)
        top = (2 ** 31 - 1) // nx * nx
        keys = [0, 1, nx - 1, nx, nx + 1, top - 1, top, 2 ** 31 - 1] + [rng.randrange(2 ** 31) for _ in range(8)]
        for key in keys:
            if 0 <= key < 2 ** 31:
                assert (key * m) >> s == key // nx, (nx, key)


def test_size_limits_for_32_bit_offsets():
    """Arrays are addressed by 32-bit byte offsets: fewer than 2^29 particles and cells."""
    p = L.make_params(synth.bubble_small())
    assert _status(p, (1 << 29) - 1) == L.LBDPS_OK
    assert _status(p, 1 << 29) == L.LBDPS_E_SHAPE
    p.nx, p.ny = 1 << 15, 1 << 14  # exactly 2^29 cells
    assert _status(p) == L.LBDPS_E_SHAPE
    p.ny = (1 << 14) - 1
    assert _status(p) == L.LBDPS_OK, L.lbdps_last_error()


def test_one_hip_runtime_in_the_process():
    """Importing the binding first (as the test collection does) must leave a
    single HIP runtime mapped: the library binds to the one torch loads.  With
    two runtimes in one process the library's finds no device."""
    import os
    import subprocess
    import sys

    code = ("import paper_1303_2653_amd.lbdps\n"
            "maps = open('/proc/self/maps').read().splitlines()\n"
            "print(len({l.split()[-1] for l in maps if 'libamdhip64' in l}))\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == "1"
