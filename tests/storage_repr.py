"""The GPU library's storage formats written out on the host, so that a test
can give the FP64 oracle exactly the state the library holds in a reduced
precision.  Representation only: none of the method's arithmetic.

- populations: FP64 as is; otherwise the deviation f_i - w_i (computed in FP64)
  rounded to float32, then for FP16 / BF16 storage to that 16-bit format
  (round to nearest even);
- positions: FP64 as is; otherwise the cell floor(P) and the offset P - cell
  rounded to float32, carried into the next cell when it rounds to 1 (kept just
  below 1 at a wall);
- velocities: rounded to float32 (FP64 mode: as is).
"""
import numpy as np

W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def to_bf16(x: np.ndarray) -> np.ndarray:
    """float32 -> nearest bfloat16 (ties to even), returned as float32."""
    u = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def populations(f: np.ndarray, precision: str) -> np.ndarray:
    f = np.asarray(f, np.float64).reshape(9, -1)
    if precision == "fp64":
        return f.copy()
    g = (f - W[:, None]).astype(np.float32)
    if precision == "fp16":
        g = g.astype(np.float16).astype(np.float32)
    elif precision == "bf16":
        g = to_bf16(g)
    return W[:, None] + g.astype(np.float64)


def positions(pos: np.ndarray, nx: int, ny: int, per_x: bool, per_y: bool, precision: str) -> np.ndarray:
    pos = np.asarray(pos, np.float64).reshape(-1, 2)
    if precision == "fp64":
        return pos.copy()
    out = np.empty_like(pos)
    for ax, (n, per) in enumerate(((nx, per_x), (ny, per_y))):
        c = np.floor(pos[:, ax])
        o = (pos[:, ax] - c).astype(np.float32).astype(np.float64)
        carry = o >= 1.0
        c = np.where(carry, c + 1, c)
        o = np.where(carry, 0.0, o)
        over = c >= n
        if per:
            c = np.where(over, 0.0, c)
        else:
            c = np.where(over, n - 1, c)
            o = np.where(over, float(np.float32(0.99999994)), o)
        out[:, ax] = c + o
    return out


def velocities(vel: np.ndarray, precision: str) -> np.ndarray:
    vel = np.asarray(vel, np.float64).reshape(-1, 2)
    return vel.copy() if precision == "fp64" else vel.astype(np.float32).astype(np.float64)


def state(cfg: dict, f, pos, vel, precision: str):
    """(f, pos, vel) in FP64 as the library holds them in ``precision``."""
    per_x, per_y = cfg["bc"][0] == "periodic", cfg["bc"][2] == "periodic"
    fr = populations(f, precision).reshape(9, cfg["ny"], cfg["nx"])
    return fr, positions(pos, cfg["nx"], cfg["ny"], per_x, per_y, precision), velocities(vel, precision)


def cell_offset(pos: np.ndarray):
    """Split positions held as cell + float32 offset (see positions) into the
    int32 cell [N][2] and the float32 offset [N][2], exactly."""
    pos = np.asarray(pos, np.float64).reshape(-1, 2)
    cell = np.floor(pos)
    off = pos - cell
    assert (off.astype(np.float32).astype(np.float64) == off).all(), "not a cell + float32 offset state"
    return cell.astype(np.int32), off.astype(np.float32)
