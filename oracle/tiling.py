"""Tiling of the Lagrangian lattice and per-box initial operations (FP64).

Test infrastructure only (see oracle/__init__.py).

Paper passages followed:
  * Sec. 3.2 step B.1: the N_p^3 lattice is split into N_tiles^3 cubic tiles of
    N_p,tile = N_p / N_tiles particles per side, each surrounded by N_p,buffer buffer
    particles, so a box holds N_p,sCOLA = N_p,tile + 2 N_p,buffer particles per side;
    over-simulation factor r and parallelisation potential p.
  * Sec. 3.3 steps C.1-C.2: Psi1 and Psi2 inside a box equal the full-box values
    (exact boundary conditions in the LPT step), so they are gathered from the full box.
  * Sec. 3.3 step C.3 and Sec. 3.4.2 eq. (LEP): Phi_BCs(x, a_K) = D1(a_K) phi1~(x),
    interpolated from the LPT grid to the PM grid, on a padding around the box (N_ghost
    layers deep beyond the faces, N_ghost = 1, 2, 3 at FDA order 2, 4, 6).

Box layout (the reading used everywhere, "convention Y"): a box of M particles per side
starts at Lagrangian index s (mod N_p); its particles sit at local positions i + 1/2,
i in [0, M).  PM nodes sit at integer local positions j: the Dirichlet problem has
N_g = M - 1 unknowns j in [1, M-1], Dirichlet nodes on the box faces j = 0 and j = M,
and one more ghost layer j = -1 and j = M + 1 for the gradient (N_ghost = 1, FDA-2).
PM spacing equals the lattice spacing.  Because PM nodes are half a cell away from LPT
nodes (which sit on the particles), the interpolation of phi1 to a PM node is the mean
of its 8 neighbouring LPT nodes (trilinear interpolation at the cell centre).
"""
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Tile:
    core_lo: tuple   # first core particle index (3 ints)
    core_n: int      # core particles per side
    buffer: int      # buffer particles per side

    @property
    def M(self):
        return self.core_n + 2 * self.buffer

    @property
    def origin(self):
        return tuple(c - self.buffer for c in self.core_lo)


def uniform_tiling(Np, tiles_per_side, buffer):
    if Np % tiles_per_side:
        raise ValueError("N_p must be a multiple of N_tiles (Sec. 3.2, B.1)")
    n = Np // tiles_per_side
    return [Tile((ix * n, iy * n, iz * n), n, buffer)
            for ix in range(tiles_per_side) for iy in range(tiles_per_side)
            for iz in range(tiles_per_side)]


def oversimulation_factor(Np, tiles_per_side, buffer):
    """Sec. 3.2: r = N_tiles^3 N_p,sCOLA^3 / N_p^3."""
    n = Np // tiles_per_side
    return tiles_per_side ** 3 * (n + 2 * buffer) ** 3 / Np ** 3


def parallelisation_potential(Np, tiles_per_side, buffer):
    """Sec. 3.2: p = N_tiles^3 / r = N_p^3 / N_p,sCOLA^3."""
    n = Np // tiles_per_side
    return Np ** 3 / (n + 2 * buffer) ** 3


def box_indices(tile, Np):
    """Global lattice indices of the box's particles along each axis (periodic wrap)."""
    return [np.mod(o + np.arange(tile.M), Np) for o in tile.origin]


def extract_box_field(field, tile):
    """field[..., N, N, N] restricted to the box's particles, local order [x][y][z]."""
    ix, iy, iz = box_indices(tile, field.shape[-1])
    return field[..., ix[:, None, None], iy[None, :, None], iz[None, None, :]]


def boundary_potential0(phi1, tile, ghosts=1):
    """Phi_BC^0 on the padded PM grid j in [-g, M+g]^3 (index j + g, g = N_ghost of the FDA
    order): the mean of phi1 over the 8 LPT nodes around each PM node.  Only the shell
    outside [1, M-1]^3 is used; interior values are left at zero."""
    N = phi1.shape[0]
    M = tile.M
    g = ghosts
    j = np.arange(-g, M + g + 1)
    out = np.zeros((M + 1 + 2 * g,) * 3)
    idx = [[np.mod(o + j - 1 + d, N) for d in (0, 1)] for o in tile.origin]
    for dx in (0, 1):
        for dy in (0, 1):
            for dz in (0, 1):
                out += phi1[idx[0][dx][:, None, None], idx[1][dy][None, :, None],
                            idx[2][dz][None, None, :]]
    out *= 0.125
    interior = (slice(g + 1, g + M),) * 3
    out[interior] = 0.0
    return out


def core_mask(tile):
    """Boolean (M, M, M) mask of the tile's core particles inside its box."""
    M = tile.M
    c = np.zeros(M, dtype=bool)
    c[tile.buffer:tile.buffer + tile.core_n] = True
    return c[:, None, None] & c[None, :, None] & c[None, None, :]
