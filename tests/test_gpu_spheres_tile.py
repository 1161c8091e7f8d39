"""The collision stage's LDS tile kernel (k_spheres_tile) against the FP64
oracle and against the row path, on beds built to reach each of its branches:
tiny periodic lattices whose ring of cells wraps onto the tile itself, walls,
tiles holding more particles than LDS, clusters of more than ST_CMAX members
inside one tile, particles with more than ST_KL contacts, and clusters that
cross tile edges.  Every tile shape must give the row path's state, pair list
and counters bit for bit, and FP64 must stay within 1e-12 of the oracle."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
L = pytest.importorskip("paper_1303_2653_amd.lbdps")
import oracle  # noqa: E402
from test_gpu_parity import compare_step, say  # noqa: E402

SHAPES = (1, 2, 3)  # 32 x 8, 16 x 16, 64 x 4 cells


def blob(x0, y0, k, spacing):
    """A k x k grid of centres `spacing` apart from (x0, y0)."""
    g = np.arange(k) * spacing
    return np.stack(np.meshgrid(x0 + g, y0 + g), axis=-1).reshape(-1, 2)


def case(name):
    if name == "tiny-periodic":  # nx, ny below the tile: the ring wraps onto the tile's own cells
        return synth.tiny(nx=3, ny=5, n=14, seed=4, bc=("periodic",) * 4, vel_scale=2e-2, g=(0.0, 0.0))
    if name == "narrow-periodic":
        return synth.tiny(nx=5, ny=40, n=160, seed=5, bc=("periodic",) * 4, vel_scale=2e-2, g=(0.0, -1e-5))
    if name == "walls":
        return synth.tiny(nx=70, ny=37, n=2400, seed=6, bc=("wall",) * 4, vel_scale=2e-2, g=(1e-5, -2e-5))
    if name == "riser-walls":
        return synth.tiny(nx=33, ny=50, n=1500, seed=8, bc=("wall", "wall", "periodic", "periodic"),
                          vel_scale=2e-2, G=(0.0, 2e-5), g=(0.0, -3e-5))
    if name == "inlet":
        return synth.tiny(nx=40, ny=30, n=1000, seed=9, bc=("periodic", "periodic", "inlet", "outlet"),
                          band=20.0, vel_scale=1e-2)
    if name == "dense-patch":  # 4 spheres per cell on 40 x 20 cells: tiles beyond the LDS capacity
        cfg = synth.tiny(nx=80, ny=48, n=1200, seed=10, bc=("periodic",) * 4, vel_scale=1e-2, g=(0.0, 0.0))
        u = synth.uniform(12, 2 * 3200).reshape(-1, 2)
        patch = np.stack([20.0 + 40.0 * u[:, 0], 12.0 + 20.0 * u[:, 1]], axis=1)
        cfg["pos"] = np.concatenate([cfg["pos"], patch])
        cfg["vel"] = (np.random.default_rng(1).random(cfg["pos"].shape) - 0.5) * 1e-2
        return cfg
    if name == "big-clusters":
        # inside one 32 x 8 tile: a 10 x 10 grid 0.45 apart (one cluster of 100
        # members, 4 contacts each) and a 5 x 5 grid 0.3 apart (8 contacts each)
        cfg = synth.tiny(nx=64, ny=32, n=300, seed=11, bc=("periodic",) * 4, vel_scale=1e-2, g=(0.0, 0.0))
        extra = np.concatenate([blob(40.3, 2.2, 10, 0.45), blob(8.3, 18.4, 5, 0.3)])
        keep = np.min(np.hypot(*(cfg["pos"][:, None, :] - extra[None, :, :]).transpose(2, 0, 1)), axis=1) > 0.6
        cfg["pos"] = np.concatenate([cfg["pos"][keep], extra])
        cfg["vel"] = (np.random.default_rng(2).random(cfg["pos"].shape) - 0.5) * 2e-2
        return cfg
    raise KeyError(name)


CASES = ("tiny-periodic", "narrow-periodic", "walls", "riser-walls", "inlet", "dense-patch", "big-clusters")


@pytest.mark.parametrize("name", CASES)
def test_tile_shapes_match_oracle_and_rows(name):
    """FP64, 4 steps under each tile shape: within 1e-12 of the oracle each
    step, and state, drag, pair list and counters identical to the row path."""
    cfg = case(name)
    say("case", name, "particles", len(cfg["pos"]))
    runs = {}
    for shape in (0,) + SHAPES:
        gpu = L.Sim(cfg, precision="fp64", diagnostics=True)
        gpu.set_tuning(sphere_tile=shape)
        ref = oracle.Sim(cfg) if shape == 1 else None
        for k in range(4):
            gpu.step(1)
            if ref is not None:
                o = ref.step(record=True)
                compare_step(gpu, o, ref, 1e-12, what=f"{name} tile {shape} step {k + 1}")
                pairs, m = gpu.pairs()
                assert m == len(o.pairs) and (pairs == o.pairs).all(), f"{name}: pair lists differ"
                c = gpu.counters()
                assert (c["pairs"], c["collisions"], c["walls"]) == (len(o.pairs), o.ncollisions, o.nwall), \
                    (name, k, c, len(o.pairs), o.ncollisions, o.nwall)
        runs[shape] = gpu.state()[:3] + (gpu.particles()["fd"], gpu.pairs()[0], gpu.counters())
        gpu.close()
    for shape in SHAPES:
        for a, b in zip(runs[shape][:5], runs[0][:5]):
            assert np.array_equal(a, b), (name, shape)
        assert runs[shape][5] == runs[0][5], (name, shape, runs[shape][5], runs[0][5])


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_tile_shapes_identical_in_reduced_precision(prec):
    """The reduced precisions under every tile shape and the row path: the same
    state bit for bit after 5 steps of a walled bed with clusters of every
    size class (cell + offset positions; the collision arithmetic in FP32)."""
    cfg = case("walls")
    ref = None
    for shape in (0,) + SHAPES:
        gpu = L.Sim(cfg, precision=prec)
        gpu.set_tuning(sphere_tile=shape)
        gpu.step(5)
        st = gpu.state()[:3] + (gpu.counters(),)
        gpu.close()
        if ref is None:
            ref = st
            continue
        for a, b in zip(st[:3], ref[:3]):
            assert np.array_equal(a, b), (prec, shape)
        assert st[3] == ref[3], (prec, shape)


def test_collision_stage_alone_with_tiles():
    """lbdps_collide_particles on a crowded walled state (clusters that cross
    tile edges and clusters inside tiles): velocities, pair list and counters
    of every tile shape equal the oracle's sequential lexicographic sweep
    followed by the wall pass, bit for bit."""
    cfg = synth.tiny(nx=96, ny=40, n=5000, seed=21, bc=("wall", "wall", "periodic", "periodic"), vel_scale=3e-2,
                     g=(0.0, 0.0))
    p = oracle.make_params(cfg)
    ref_pairs = oracle.contacts(p, cfg["pos"])
    v1, nc = oracle.resolve(p, cfg["pos"], cfg["vel"], ref_pairs)
    v1, nw = oracle.walls(p, cfg["pos"], v1)
    for shape in (0,) + SHAPES:
        gpu = L.Sim(cfg, precision="fp64")
        gpu.set_tuning(sphere_tile=shape)
        gpu.collide_particles()
        st = gpu.particles()
        pairs, m = gpu.pairs()
        c = gpu.counters()
        gpu.close()
        assert m == len(ref_pairs) and (pairs == ref_pairs).all(), shape
        assert (st["vel"] == v1).all(), shape
        assert (c["pairs"], c["collisions"], c["walls"]) == (len(ref_pairs), nc, nw), (shape, c)
