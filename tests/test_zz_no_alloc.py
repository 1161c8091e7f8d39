"""The allocation-free conservation entry point (lbdps_conservation_noalloc)
against lbdps_conservation, through the C ABI: the same sums bit for bit on
two calls in a row, the second on a smaller bed, and the same non-finite
report.  Its scratch is one library-static device array per GPU."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
L = pytest.importorskip("paper_1303_2653_amd.lbdps")


def test_noalloc_conservation_equals_the_workspace_form():
    big = L.Sim(synth.riser_crop(), precision="fp32")
    big.step(3)
    a = big.conservation_noalloc()
    b = big.conservation()
    print("riser crop", a, flush=True)
    assert np.array_equal(a, b) and a[5] == 0.0 and a[0] > 0
    small = L.Sim(synth.tiny(nx=16, ny=24, n=60, seed=7, vel_scale=1e-3, bc=("periodic",) * 4), precision="fp64")
    small.step(2)
    c = small.conservation_noalloc()  # second call, smaller bed: the scratch holds the first call's values
    d = small.conservation()
    print("tiny", c, flush=True)
    assert np.array_equal(c, d) and abs(c[0] - 16 * 24) < 1e-9
    assert np.array_equal(big.conservation_noalloc(), b)  # and back on the first bed


def test_noalloc_conservation_reports_non_finite():
    cfg = synth.tiny(nx=16, ny=24, n=60, seed=7)
    vel = np.zeros((60, 2))
    vel[5, 1] = np.nan
    sim = L.Sim(dict(cfg, vel=vel), precision="fp64")
    for fn in (sim.conservation_noalloc, sim.conservation):
        with pytest.raises(L.LbdpsError) as e:
            fn()
        assert e.value.status == L.LBDPS_E_NONFINITE
    sim.set_state(None, cfg["pos"], np.zeros((60, 2)))
    assert sim.conservation_noalloc()[5] == 0.0
