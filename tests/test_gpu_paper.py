"""The paper's own workloads (Tables 1 and 2) and the voidage observables of
Sec. 3 through the C ABI, against the FP64 oracle on the same inputs.

FP64 mode: states, fields and voidage sums within 1e-12 (norm-wise; the sums
run in a different order on each side), contact pairs and the counts of cells
above the bubble threshold bit for bit."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
L = pytest.importorskip("paper_1303_2653_amd.lbdps")
import oracle  # noqa: E402


def rel(a, b, floor=0.0):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    scale = max(np.abs(b).max() if b.size else 0.0, floor)
    return float(np.abs(a - b).max() / scale) if scale > 0 else float(np.abs(a).max())


def say(*a):
    print(*a, flush=True)


def check_state(gpu, ref, o, what, tol=1e-12):
    f, pos, vel, _ = gpu.state()
    fl = gpu.fields()
    errs = dict(f=rel(f, ref.f, 1.0), pos=rel(pos, ref.pos, 1.0), vel=rel(vel, ref.vel, 1e-300),
                rho=rel(fl["rho"], o.rho, 1.0), ugas=rel(fl["ugas"], o.ugas), beta=rel(fl["beta"], o.beta))
    say(what, {k: f"{v:.2e}" for k, v in errs.items()})
    assert (fl["ncell"] == o.ncell).all(), what
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, f"{what}: {bad}"
    pairs, m = gpu.pairs()
    assert m == len(o.pairs) and (pairs == o.pairs).all(), f"{what}: pairs differ"


def check_voidage(gpu, ref, y0, y1, what):
    rows, cols, count = gpu.voidage(y0, y1, 0.85)
    r_rows, r_cols, r_count = oracle.voidage(ref.p, ref.pos, y0, y1, 0.85)
    say(what, "voidage rows", f"{rel(rows, r_rows):.1e}", "cols", f"{rel(cols, r_cols):.1e}", "count", count,
        r_count)
    assert count == r_count
    assert rel(rows, r_rows) < 1e-13 and rel(cols, r_cols) < 1e-13
    return count


def test_paper_bubble_pulse_fp64():
    """Table 1 bed with the Smagorinsky model on: the jet runs for the first 12
    steps, then lbdps_set_inlet switches the orifice back to v_mf (the end of
    the 0.006 s pulse, brought forward), on both sides."""
    cfg = synth.paper_bubble()
    pulse = 12
    say("workload", cfg["name"], "tau", cfg["tau"], "C_s", cfg["cs_smag"], "pulse", pulse)
    gpu = L.Sim(cfg, precision="fp64", diagnostics=True)
    ref = oracle.Sim(cfg)
    for k in range(1, 2 * pulse + 1):
        if k == pulse + 1:
            gpu.set_inlet(cfg["inlet_after"])
            ref.inlet_uy = np.ascontiguousarray(cfg["inlet_after"], np.float64)
        gpu.step(1)
        o = ref.step(record=True)
        if k in (1, pulse, pulse + 1, 2 * pulse):
            check_state(gpu, ref, o, f"paper bubble step {k}")
            check_voidage(gpu, ref, 0, cfg["ny"], f"paper bubble step {k}")
    c = gpu.counters()
    assert c["collisions"] == o.ncollisions and c["walls"] == o.nwall


def test_paper_riser_fp64():
    """Table 2 riser (123 921 spheres of d = 0.2, LES on), gas started at the
    inlet velocity: three steps, and the voidage profiles of the lower and upper
    halves."""
    cfg = synth.paper_riser()
    say("workload", cfg["name"], "tau", cfg["tau"], "C_s", cfg["cs_smag"])
    f0 = oracle.equilibrium_state(cfg["nx"], cfg["ny"], 1.0, *cfg["u0"])
    gpu = L.Sim(cfg, precision="fp64", diagnostics=True)
    gpu.set_state(f0, cfg["pos"], cfg["vel"])
    ref = oracle.Sim(cfg, f=f0)
    for k in range(1, 4):
        gpu.step(1)
        o = ref.step(record=True)
    check_state(gpu, ref, o, "paper riser step 3")
    half = cfg["ny"] // 2
    check_voidage(gpu, ref, 0, half, "paper riser lower half")
    check_voidage(gpu, ref, half, cfg["ny"], "paper riser upper half")


def test_voidage_full_size_fp32():
    """The 256 x 1024 bubble bed in FP32 after 5 steps: the library's voidage
    statistics equal the oracle's definition evaluated at the library's own
    positions (cell + offset, exact in FP64), counts bit for bit."""
    cfg = synth.bubble()
    gpu = L.Sim(cfg, precision="fp32")
    gpu.step(5)
    _, pos, _, _ = gpu.state()
    p = oracle.make_params(cfg)
    for y0, y1, thr in ((0, cfg["ny"], 0.85), (100, 300, 0.95), (0, 0, 0.5)):
        rows, cols, count = gpu.voidage(y0, y1, thr)
        r_rows, r_cols, r_count = oracle.voidage(p, pos, y0, y1, thr)
        say("window", y0, y1, thr, "count", count, r_count, "rows", f"{rel(rows, r_rows):.1e}")
        assert count == r_count
        assert rel(rows, r_rows) < 1e-13 and rel(cols, r_cols, 1.0) < 1e-13


def test_observable_arguments_rejected():
    cfg = synth.tiny()
    gpu = L.Sim(cfg, precision="fp32")
    for y0, y1 in ((-1, 3), (5, 4), (0, cfg["ny"] + 1)):
        with pytest.raises(L.LbdpsError) as e:
            gpu.voidage(y0, y1)
        assert e.value.status == L.LBDPS_E_INVALID
    bad = np.full(cfg["nx"], 0.01)
    bad[3] = np.nan
    with pytest.raises(L.LbdpsError) as e:
        gpu.set_inlet(bad)
    assert e.value.status == L.LBDPS_E_INVALID
    gpu.set_inlet(np.full(cfg["nx"], 0.02))  # accepted; the next steps use it
    gpu.step(2)
