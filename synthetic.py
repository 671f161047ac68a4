"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws random numbers and names workload sizes; it holds none of the
method's arithmetic, and neither the oracle nor the HIP library imports it.

The workloads are Gaussian random fields, as in the paper's own runs (Sec. 4): unit
white noise on the N_p^3 lattice (float64, C order [x][y][z]) which the simulation turns
into initial conditions through the Eisenstein-Hu spectrum.
"""
from dataclasses import dataclass, field

import numpy as np


def white_noise(N, seed=42):
    return np.random.default_rng(seed).standard_normal((N, N, N))


def loss_target(N, seed=43):
    """Target field of the density loss sum (delta_out - t)^2."""
    return 0.5 * np.random.default_rng(seed).standard_normal((N, N, N))


def uniform(shape, lo, hi, seed):
    return np.random.default_rng(seed).uniform(lo, hi, size=shape)


def normal(shape, scale, seed):
    return scale * np.random.default_rng(seed).standard_normal(shape)


@dataclass(frozen=True)
class Workload:
    name: str
    L: float                  # box side, Mpc/h
    Np: int                   # particles per side
    tiles_per_side: int       # 0 = explicit tile list (mixed sizes)
    buffer: int
    n_steps: int
    precision: str            # "fp32" or "fp64"
    a_i: float = 0.05
    a_f: float = 1.0
    note: str = ""
    mixed: tuple = field(default=())   # ((lo_x, lo_y, lo_z, core, buffer), ...)


def mixed_tiling_256():
    """Deterministic cubic tiling of the 256^3 lattice with cores 48, 64 and 32:
    [0,192)^3 as 4^3 tiles of 48^3 (buffer 16 -> 80^3 boxes); the rest as 64^3 blocks in
    lexicographic order, the first 8 of which are split into 8 tiles of 32^3 each (buffer
    8 -> 48^3 boxes) and the others kept whole (buffer 24 -> 112^3 boxes)."""
    tiles = []
    for ix in range(4):
        for iy in range(4):
            for iz in range(4):
                tiles.append((48 * ix, 48 * iy, 48 * iz, 48, 16))
    blocks = []
    for ix in range(4):
        for iy in range(4):
            for iz in range(4):
                lo = (64 * ix, 64 * iy, 64 * iz)
                if all(c < 192 for c in (64 * ix + 63, 64 * iy + 63, 64 * iz + 63)):
                    continue            # fully inside [0,192)^3, covered by 48^3 tiles
                blocks.append(lo)
    # blocks straddling 192 would overlap the 48-tiles: 192 is a multiple of 64, so none do
    for b, lo in enumerate(blocks):
        if b < 8:
            for dx in (0, 32):
                for dy in (0, 32):
                    for dz in (0, 32):
                        tiles.append((lo[0] + dx, lo[1] + dy, lo[2] + dz, 32, 8))
        else:
            tiles.append((lo[0], lo[1], lo[2], 64, 24))
    return tuple(tiles)


WORKLOADS = {
    "c1": Workload("c1", 200.0, 64, 2, 8, 10, "fp64",
                   note="plain FP64, 2^3 tiles of 32^3 + 8 buffer (48^3 boxes)"),
    "c2": Workload("c2", 500.0, 128, 4, 16, 20, "fp32",
                   note="batched FP32, 4^3 tiles of 32^3 + 16 buffer (64^3 boxes)"),
    "c3": Workload("c3", 1000.0, 256, 0, 0, 20, "fp32", mixed=mixed_tiling_256(),
                   note="uneven batch: 48^3/80^3/112^3 boxes"),
    "c4": Workload("c4", 500.0, 128, 4, 16, 20, "fp32",
                   note="adjoint of the c2 forward, checkpoint every 5 steps"),
    "c5": Workload("c5", 1000.0, 512, 8, 16, 30, "fp32",
                   note="8^3 tiles of 64^3 + 16 buffer (96^3 boxes)"),
}
