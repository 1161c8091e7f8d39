"""MI355X-native LBM discrete particle simulation step (HIP library + binding).

The simulation runs in ``liblbdps.so`` (HIP, gfx950) behind the C ABI of
``include/lbdps.h``; ``paper_1303_2653_amd.lbdps`` is its Python binding.
"""
__all__ = ["lbdps"]
