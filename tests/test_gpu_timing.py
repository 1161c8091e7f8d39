"""Per-kernel timing through the C ABI: every step phase is timed once per step
with events stamped by its own dispatch, for a single bed and for a batch."""
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
L = pytest.importorskip("paper_1303_2653_amd.lbdps")


@pytest.mark.parametrize("nsub", [1, 3])
def test_kernel_times_single_bed(nsub):
    """With particle sub-steps every phase still counts one launch per step
    (the later sub-steps' launches add their time)."""
    cfg = synth.tiny(nx=64, ny=48, n=600, seed=21, band=24.0, vel_scale=1e-3, n_sub=nsub)
    sim = L.Sim(cfg, precision="fp32")
    sim.step(2)
    sim.time_kernels(L.KERNELS)
    sim.step(3)
    kt = sim.kernel_times()
    sim.time_kernels([])
    assert set(kt) == set(L.KERNELS)
    for name, (ms, n) in kt.items():
        assert n == 3, (name, n)  # one timed launch per step (the two resolution launches count once)
        assert 0.0 < ms < 1e3, (name, ms)
    sim.step(1)  # no longer timed
    assert all(n == 0 for _, n in sim.kernel_times().values())
    sim.close()


def test_kernel_times_batch():
    cfgs = [synth.tiny(nx=32, ny=24, n=150, seed=22), synth.tiny(nx=40, ny=30, n=300, seed=23, band=15.0)]
    batch = L.Batch(cfgs, precision="fp32")
    batch.step(2)
    batch.time_kernels(L.KERNELS)
    batch.step(2)
    kt = batch.kernel_times()
    batch.time_kernels([])
    for name, (ms, n) in kt.items():
        assert n == 2, (name, n)
        assert 0.0 < ms < 1e3, (name, ms)
    batch.close()
