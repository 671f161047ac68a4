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


def boundary_potential0(phi1, tile, ghosts=1, Np=None):
    """Phi_BC^0 on the padded PM grid j in [-g, M+g]^3 (index j + g, g = N_ghost of the FDA
    order): the mean of phi1 over the 8 LPT nodes around each PM node.  Only the shell
    outside [1, M-1]^3 is used; interior values are left at zero.  With an LPT grid coarser
    than the lattice (Np given and larger than phi1's N), see boundary_potential0_coarse."""
    N = phi1.shape[0]
    if Np is not None and Np != N:
        return boundary_potential0_coarse(phi1, tile, Np, ghosts)
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


# --- LPT grid coarser than the lattice (Sec. 3.3 C.2, Sec. 4: N = N_p / 2) ---------------
def lpt_coordinate(x_cells, Np, N):
    """Coordinate on the LPT grid of a lattice-cell position x: LPT node m sits at the centre
    (m + 1/2) (N_p / N) of its coarse cell, so u = x N / N_p - 1/2 (N = N_p: u = x - 1/2)."""
    return np.asarray(x_cells, dtype=np.float64) * (N / Np) - 0.5


def cic_periodic_1d(u, N):
    """(indices (2, n), weights (2, n)) of 1-D CiC on a periodic grid at coordinates u."""
    j0 = np.floor(u).astype(np.int64)
    f = u - j0
    return np.stack([np.mod(j0, N), np.mod(j0 + 1, N)]), np.stack([1.0 - f, f])


def interpolate_lpt_grid(field, points, Np):
    """CiC (B-bar) of field [..., N, N, N] on the periodic LPT grid at lattice-cell positions
    points (3, n); returns [..., n]."""
    N = field.shape[-1]
    idx = []
    wts = []
    for a in range(3):
        i, w = cic_periodic_1d(lpt_coordinate(points[a], Np, N), N)
        idx.append(i)
        wts.append(w)
    out = 0.0
    for dx in (0, 1):
        for dy in (0, 1):
            for dz in (0, 1):
                w = wts[0][dx] * wts[1][dy] * wts[2][dz]
                out = out + w * field[..., idx[0][dx], idx[1][dy], idx[2][dz]]
    return out


def psi_at_particles(psi_grid, Np):
    """Sec. 3.3 C.2: Psi = grad phi on the LPT grid (coarse-cell units, as
    lpt.displacement_vectors returns it) interpolated by CiC to the Lagrangian lattice sites
    q = i + 1/2 and converted to lattice cells (x N_p / N).  Shape (3, Np, Np, Np)."""
    N = psi_grid.shape[-1]
    i = np.arange(Np) + 0.5
    q = np.stack(np.meshgrid(i, i, i, indexing="ij")).reshape(3, -1)
    return (Np / N) * interpolate_lpt_grid(psi_grid, q, Np).reshape(psi_grid.shape[:-3] +
                                                                     (Np, Np, Np))


def boundary_potential0_coarse(phi1, tile, Np, ghosts=1):
    """Phi_BC^0 with an LPT grid of N < N_p nodes: phi1 (coarse-cell^2 units) interpolated by
    CiC to the padded PM nodes [-g, M+g]^3 at lattice-cell positions origin + j, converted
    to lattice cells^2 (x (N_p / N)^2); interior values zero."""
    N = phi1.shape[0]
    M = tile.M
    g = ghosts
    j = np.arange(-g, M + g + 1)
    X = [o + j for o in tile.origin]
    pts = np.stack(np.meshgrid(X[0], X[1], X[2], indexing="ij")).reshape(3, -1).astype(float)
    out = ((Np / N) ** 2 * interpolate_lpt_grid(phi1, pts, Np)).reshape((M + 1 + 2 * g,) * 3)
    out[(slice(g + 1, g + M),) * 3] = 0.0
    return out
