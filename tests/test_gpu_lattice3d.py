"""The 3-D gas lattice (D3Q19 BGK on a periodic box, the first piece of the
3-D extension) through the C ABI against the oracle's step on the same
state: FP64 bit for bit; the deviation storages within their rounding."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
L = pytest.importorskip("paper_1303_2653_amd.lbdps")
import oracle  # noqa: E402

DT = {"fp64": (L.LBDPS_FP64, torch.float64), "fp32": (L.LBDPS_FP32, torch.float32),
      "fp16": (L.LBDPS_FP32_STORE_FP16, torch.float16), "bf16": (L.LBDPS_FP32_STORE_BF16, torch.bfloat16)}


def state(nx, ny, nz, seed=4):
    """A flow of u ~ 0.02 with a 1e-3 perturbation, [19][nz][ny][nx]."""
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ux = 0.02 * np.sin(2 * np.pi * z / nz)
    uy = 0.01 * np.cos(2 * np.pi * x / nx)
    f = np.empty((19, nz, ny, nx))
    for i in range(19):
        f[i] = np.vectorize(lambda a, b: oracle.feq3(i, 1.0, a, b, 0.0))(ux, uy)
    return f + (rng.random(f.shape) - 0.5) * 1e-3


def to_storage(f, prec):
    code, dt = DT[prec]
    if prec == "fp64":
        return torch.tensor(f, dtype=dt, device="cuda")
    _, w = oracle.lattice3()
    return torch.tensor(f - w[:, None, None, None], dtype=torch.float64, device="cuda").to(dt)


def from_storage(t, prec):
    a = t.to(torch.float64).cpu().numpy()
    if prec == "fp64":
        return a
    _, w = oracle.lattice3()
    return a + w[:, None, None, None]


# about three times the errors measured on these states (FP32 1.7e-9, FP16
# 2.7e-6, BF16 1.7e-5 after 5 steps)
@pytest.mark.parametrize("prec,tol,nx", [("fp64", 0.0, 12), ("fp32", 5e-9, 12), ("fp16", 8e-6, 12), ("bf16", 5e-5, 12),
                                         ("fp16", 8e-6, 13), ("bf16", 5e-5, 13)])
def test_d3q19_steps_match_oracle(prec, tol, nx):
    """An even nx runs the 16-bit storages two cells per thread, an odd one
    cell per thread."""
    ny, nz, steps, tau = 10, 9, 5, 0.7
    f0 = state(nx, ny, nz)
    a = to_storage(f0, prec)
    ref = from_storage(a, prec)  # the oracle starts from the stored state
    b = torch.empty_like(a)
    code = DT[prec][0]
    for _ in range(steps):
        L.check(L.lbdps3_bgk_step(a.data_ptr(), b.data_ptr(), nx, ny, nz, tau, code, None), "lbdps3_bgk_step")
        a, b = b, a
        ref = oracle.bgk3_step(ref, tau)
    torch.cuda.synchronize()
    got = from_storage(a, prec)
    err = float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1.0))
    print(prec, "D3Q19 after", steps, "steps: error", err, flush=True)
    assert err <= tol


def test_d3q19_rejects_bad_arguments():
    a = torch.zeros(19 * 8, dtype=torch.float32, device="cuda")
    b = torch.zeros_like(a)
    assert L.lbdps3_bgk_step(a.data_ptr(), a.data_ptr(), 2, 2, 2, 0.7, L.LBDPS_FP32, None) == L.LBDPS_E_INVALID
    assert L.lbdps3_bgk_step(a.data_ptr(), b.data_ptr(), 0, 2, 2, 0.7, L.LBDPS_FP32, None) == L.LBDPS_E_SHAPE
    assert L.lbdps3_bgk_step(a.data_ptr(), b.data_ptr(), 2, 2, 2, 0.5, L.LBDPS_FP32, None) == L.LBDPS_E_INVALID
    assert L.lbdps3_bgk_step(a.data_ptr(), b.data_ptr(), 2, 2, 2, 0.7, 9, None) == L.LBDPS_E_INVALID


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("nx", [2, 12, 130, 160, 256])
def test_d3q19_pairs_match_single_cells(prec, nx):
    """The two-cells-per-thread form (even nx, 4-byte aligned planes) against
    the one-cell form on the same state, bit for bit: both do the same
    arithmetic, so any difference is a misplaced store. A buffer offset by
    one element takes the one-cell form. The state is the rest weights plus
    deviations of 1e-2 drawn per population, so that a value written to a
    neighbour's slot is far from the right one; nx of 130 and 160 put row
    ends inside a wavefront and wavefront ends inside a row."""
    ny, nz, steps, tau = 5, 3, 3, 0.8
    code, dt = DT[prec]
    C = nx * ny * nz
    rng = np.random.default_rng(nx)
    g = torch.tensor((rng.random(19 * C) - 0.5) * 2e-2, dtype=torch.float64).to(dt).cuda()
    outs = []
    for off in (0, 1):
        a = torch.zeros(19 * C + 2, dtype=dt, device="cuda")
        b = torch.zeros_like(a)
        a[off:off + 19 * C] = g
        pa, pb = a[off:].data_ptr(), b[off:].data_ptr()
        assert (pa % 4 == 0) == (off == 0)
        for _ in range(steps):
            L.check(L.lbdps3_bgk_step(pa, pb, nx, ny, nz, tau, code, None), "lbdps3_bgk_step")
            pa, pb = pb, pa
        torch.cuda.synchronize()
        res = a if steps % 2 == 0 else b
        outs.append(res[off:off + 19 * C].view(torch.int16).cpu().numpy())
    bad = np.flatnonzero(outs[0] != outs[1])
    assert bad.size == 0, f"{bad.size} values differ, first at plane {bad[0] // C} cell {bad[0] % C}"


# (f tolerance against max(|f|, 1), force tolerance against max |F|): about
# three times the errors measured after 4 steps (f: FP32 1.2e-9, FP16 2.1e-6,
# BF16 1.6e-5; force: 2.4e-7, 7.2e-5, 5.3e-4)
PSM_TOL = {"fp64": (0.0, 0.0), "fp32": (4e-9, 7e-7), "fp16": (6e-6, 2.2e-4), "bf16": (5e-5, 1.6e-3)}


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16", "bf16"])
@pytest.mark.parametrize("nx", [12, 13])
def test_d3q19_psm_steps_match_oracle(prec, nx):
    """Partially saturated cells (Eqs. 6-7, 9, 25 on D3Q19) through the C ABI
    against the oracle, 4 steps with fixed solids: 0-3 spheres per cell, one
    cell far beyond the densest packing, velocities up to 0.03. FP64 bit for
    bit, populations and force; the other storages within their rounding."""
    ny, nz, steps, tau, d = 10, 9, 4, 0.7, 0.9
    C = nx * ny * nz
    rng = np.random.default_rng(nx)
    n = rng.integers(0, 4, (nz, ny, nx)).astype(np.int32)
    n[1, 2, 3] = 50
    vs = (rng.random((3, nz, ny, nx)) - 0.5) * 0.06
    f0 = state(nx, ny, nz)
    a = to_storage(f0, prec)
    ref = from_storage(a, prec)
    b = torch.empty_like(a)
    code, dt = DT[prec]
    vdt = torch.float64 if prec == "fp64" else torch.float32
    dn = torch.tensor(n, device="cuda")
    dvs = torch.tensor(vs, dtype=vdt, device="cuda")
    vs_ref = dvs.to(torch.float64).cpu().numpy()  # the oracle sees the velocities the kernel reads
    dF = torch.full((3, C), float("nan"), dtype=vdt, device="cuda")
    for _ in range(steps):
        L.check(L.lbdps3_psm_step(a.data_ptr(), b.data_ptr(), dn.data_ptr(), dvs.data_ptr(), dF.data_ptr(),
                                  nx, ny, nz, tau, d, code, None), "lbdps3_psm_step")
        a, b = b, a
        ref, F_ref = oracle.psm3_step(ref, tau, d, n, vs_ref)
    torch.cuda.synchronize()
    got = from_storage(a, prec)
    F = dF.to(torch.float64).cpu().numpy().reshape(3, nz, ny, nx)
    err = float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1.0))
    ferr = float(np.abs(F - F_ref).max() / np.abs(F_ref).max())
    print(prec, nx, "PSM after", steps, "steps: f error", err, "force error", ferr, flush=True)
    tol, ftol = PSM_TOL[prec]
    assert np.isfinite(F).all()
    assert err <= tol and ferr <= ftol


def test_d3q19_psm_rejects_bad_arguments():
    a = torch.zeros(19 * 8, dtype=torch.float32, device="cuda")
    b = torch.zeros_like(a)
    n = torch.zeros(8, dtype=torch.int32, device="cuda")
    v = torch.zeros(24, dtype=torch.float32, device="cuda")
    F = torch.zeros_like(v)
    ok = (a.data_ptr(), b.data_ptr(), n.data_ptr(), v.data_ptr(), F.data_ptr(), 2, 2, 2, 0.7, 0.5, L.LBDPS_FP32, None)
    assert L.lbdps3_psm_step(*ok) == L.LBDPS_OK
    torch.cuda.synchronize()
    bad = [(1, a.data_ptr(), L.LBDPS_E_INVALID), (2, 0, L.LBDPS_E_INVALID), (4, 0, L.LBDPS_E_INVALID),
           (5, 0, L.LBDPS_E_SHAPE), (8, 0.5, L.LBDPS_E_INVALID), (9, 0.0, L.LBDPS_E_INVALID),
           (9, float("nan"), L.LBDPS_E_INVALID), (10, 7, L.LBDPS_E_INVALID)]
    for k, val, want in bad:
        args = list(ok)
        args[k] = val
        assert L.lbdps3_psm_step(*args) == want, (k, val)


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("nx", [2, 130, 160])
def test_d3q19_psm_pairs_match_single_cells(prec, nx):
    """As test_d3q19_pairs_match_single_cells, with solids in the cells: the
    paired form (populations, counts, v_s and F two cells at a time) against
    the one-cell form, populations and force bit for bit."""
    ny, nz, steps, tau, d = 5, 3, 3, 0.8, 0.9
    code, dt = DT[prec]
    C = nx * ny * nz
    rng = np.random.default_rng(nx + 1)
    g = torch.tensor((rng.random(19 * C) - 0.5) * 2e-2, dtype=torch.float64).to(dt).cuda()
    n = torch.tensor(rng.integers(0, 5, C).astype(np.int32), device="cuda")
    vs = torch.tensor((rng.random(3 * C) - 0.5) * 0.06, dtype=torch.float32, device="cuda")
    outs, forces = [], []
    for off in (0, 1):
        a = torch.zeros(19 * C + 2, dtype=dt, device="cuda")
        b = torch.zeros_like(a)
        a[off:off + 19 * C] = g
        F = torch.full((3 * C,), float("nan"), dtype=torch.float32, device="cuda")
        pa, pb = a[off:].data_ptr(), b[off:].data_ptr()
        for _ in range(steps):
            L.check(L.lbdps3_psm_step(pa, pb, n.data_ptr(), vs.data_ptr(), F.data_ptr(), nx, ny, nz, tau, d, code,
                                      None), "lbdps3_psm_step")
            pa, pb = pb, pa
        torch.cuda.synchronize()
        res = a if steps % 2 == 0 else b
        outs.append(res[off:off + 19 * C].view(torch.int16).cpu().numpy())
        forces.append(F.view(torch.int32).cpu().numpy())
    bad = np.flatnonzero(outs[0] != outs[1])
    assert bad.size == 0, f"{bad.size} values differ, first at plane {bad[0] // C} cell {bad[0] % C}"
    assert np.array_equal(forces[0], forces[1])
