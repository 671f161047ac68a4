"""End-to-end tiled sCOLA run and its outputs (FP64).

Test infrastructure only (see oracle/__init__.py).

Paper passages followed:
  * Fig. 1 and Sec. 3: A.1-A.2 (full-box ICs and Lagrangian potentials), B.1 (tiling),
    C.1-C.3 (per-box Psi and Phi_BCs), D (evolution), B.2 (untiling: the core particles'
    final positions and momenta are gathered, buffer particles are dropped).
  * Sec. 4.1: the final density is the CiC assignment of all particles to a grid.
  * Sec. 4.2: P(k) and R(k) estimators with 100 log bins from 2 pi / L to 1 h/Mpc.

  * Sec. 3.3 C.2 and Sec. 4: with an LPT grid of N = N_p / 2 nodes per side, Psi is
    differenced on the LPT grid and interpolated (CiC) to the particles.

Readings: the output density grid has N_out nodes per side at integer multiples of
L / N_out (N_out = N_p by default), assigned with periodic CiC from the core particles
only; delta_out = count * (N_out/N_p)^3 - 1.
"""
import numpy as np

from .cosmology import Cosmology, cola_schedule
from .lpt import lagrangian_potentials, displacement_vectors
from .scola import cic_corners, evolve_box
from .tiling import (boundary_potential0, box_indices, core_mask, extract_box_field,
                     psi_at_particles, uniform_tiling)


def setup_full_box(white_noise, L, cosmo, a_i, fda_order=2):
    """Steps A.1-A.2: phi1, phi2 and Psi1, Psi2 on the LPT grid (cells)."""
    D1 = cosmo.growth(np.array([1.0]), a_i)[0][0]          # D1(1) / D1(a_i)
    phi1, phi2 = lagrangian_potentials(white_noise, L, cosmo, 1.0 / D1, fda_order)
    return (phi1, phi2, displacement_vectors(phi1, fda_order),
            displacement_vectors(phi2, fda_order))


def box_inputs(psi1, psi2, phi1, tile, fda_order=2, Np=None):
    """Steps C.1-C.3 for one box: its Psi1, Psi2 and Phi_BC^0.  psi1, psi2 are at the
    lattice sites (N_p^3); phi1 is on the LPT grid (of N_p, or fewer nodes when Np says so)."""
    return (extract_box_field(psi1, tile), extract_box_field(psi2, tile),
            boundary_potential0(phi1, tile, fda_order // 2, Np))


def untile(tile, Np, box_out, key="u"):
    """Step B.2 for one tile: (global lattice indices (3, n), values (3, n)) of its core."""
    mask = core_mask(tile)
    ix, iy, iz = box_indices(tile, Np)
    gi = np.stack(np.meshgrid(ix, iy, iz, indexing="ij"))[:, mask]
    return gi, box_out[key][:, mask]


def output_density(x_cells, Np, N_out):
    """Periodic CiC of positions (cells of the N_p lattice, any range) onto N_out^3
    nodes at integer multiples of N_p/N_out cells; returns delta."""
    u = np.asarray(x_cells, dtype=np.float64) * (N_out / Np)
    rho = np.zeros((N_out,) * 3)
    for _, idx, w in cic_corners(u):
        np.add.at(rho, tuple(np.mod(idx, N_out)), w)
    return rho * (N_out / Np) ** 3 - 1.0


def run_scola(white_noise, L, tiles, cosmo=None, a_i=0.05, a_f=1.0, n_steps=10,
              want_momenta=False, N_out=None, tile_subset=None, discretisation="modified",
              n_lpt=-2.5, tile_a_f=None, fda_order=2, Np=None):
    """Full tiled sCOLA run.  Returns dict with positions (3, Np, Np, Np) in Mpc/h in
    [0, L), momenta (or None) in Mpc/h (H0 = 1 units), the output density and the per-box
    raw results.  Entries of tiles outside tile_subset are left NaN in the outputs.
    discretisation, n_lpt: the time factors of App. B (see cola_schedule).
    tile_a_f: optional final scale factor per tile (Sec. 5.1: tiles need not share one final
    time; 0 or None entries mean a_f); each tile takes n_steps steps from a_i to its own.
    fda_order: 2, 4 or 6, the order of every Laplacian and gradient (Sec. 3).
    Np: particles per side when the white noise lives on a coarser LPT grid (N = its side,
    N_p / N an integer; Sec. 3.3 C.2 and Sec. 4): Psi is then interpolated to the particles
    and Phi_BC^0 to the PM nodes (tiling.psi_at_particles, boundary_potential0_coarse)."""
    cosmo = cosmo or Cosmology()
    N_lpt = white_noise.shape[0]
    Np = Np or N_lpt
    N_out = N_out or Np
    phi1, phi2, psi1, psi2 = setup_full_box(white_noise, L, cosmo, a_i, fda_order)
    if N_lpt != Np:
        psi1, psi2 = psi_at_particles(psi1, Np), psi_at_particles(psi2, Np)
    steps, final = cola_schedule(cosmo, a_i, a_f, n_steps, want_final_kick=want_momenta,
                                 discretisation=discretisation, n_lpt=n_lpt)
    pos = np.full((3, Np, Np, Np), np.nan)
    mom = np.full((3, Np, Np, Np), np.nan) if want_momenta else None
    boxes = {}
    subset = range(len(tiles)) if tile_subset is None else tile_subset
    for t in subset:
        tile = tiles[t]
        s1, s2, bc0 = box_inputs(psi1, psi2, phi1, tile, fda_order, Np)
        st, fin = steps, final
        if tile_a_f is not None and tile_a_f[t] and tile_a_f[t] != a_f:
            st, fin = cola_schedule(cosmo, a_i, tile_a_f[t], n_steps,
                                    want_final_kick=want_momenta,
                                    discretisation=discretisation, n_lpt=n_lpt)
        out = evolve_box(s1, s2, bc0, st, fin, fda_order=fda_order)
        boxes[t] = out
        gi, u = untile(tile, Np, out, "u")
        origin = np.array(tile.origin, dtype=np.float64)[:, None]
        pos[:, gi[0], gi[1], gi[2]] = u + origin
        if want_momenta:
            _, p = untile(tile, Np, out, "p")
            mom[:, gi[0], gi[1], gi[2]] = p
    dens = None
    if tile_subset is None:
        dens = output_density(pos.reshape(3, -1), Np, N_out)
    cell = L / Np
    return dict(pos=np.mod(pos * cell, L), pos_cells=pos,
                mom=None if mom is None else mom * cell,
                density=dens, boxes=boxes, psi1=psi1, psi2=psi2, phi1=phi1, phi2=phi2)


def power_spectrum(delta, L, n_bins=100, k_max=1.0, other=None):
    """Sec. 4.2 estimators: P(k) = L^3/N^6 <|delta_k|^2> in 100 log bins from 2 pi/L to
    k_max; with other given, also R(k) = <delta* other> / sqrt(<|delta|^2><|other|^2>)."""
    N = delta.shape[0]
    m = np.fft.fftfreq(N, d=1.0 / N)
    kmag = 2 * np.pi / L * np.sqrt(m[:, None, None] ** 2 + m[None, :, None] ** 2 +
                                   m[None, None, :] ** 2)
    edges = np.logspace(np.log10(2 * np.pi / L), np.log10(k_max), n_bins + 1)
    dk = np.fft.fftn(delta)
    which = np.digitize(kmag.ravel(), edges) - 1
    ok = (which >= 0) & (which < n_bins)
    cnt = np.bincount(which[ok], minlength=n_bins)
    pk = np.bincount(which[ok], weights=np.abs(dk.ravel()[ok]) ** 2, minlength=n_bins)
    with np.errstate(invalid="ignore", divide="ignore"):
        P = pk / cnt * L ** 3 / N ** 6
        res = dict(k_edges=edges, count=cnt, P=P)
        if other is not None:
            ok2 = np.fft.fftn(other)
            cross = np.bincount(which[ok], weights=(np.conj(dk) * ok2).real.ravel()[ok],
                                minlength=n_bins)
            po = np.bincount(which[ok], weights=np.abs(ok2.ravel()[ok]) ** 2,
                             minlength=n_bins)
            res["R"] = cross / np.sqrt(pk * po)
    return res


__all__ = ["run_scola", "setup_full_box", "box_inputs", "untile", "output_density",
           "power_spectrum", "uniform_tiling"]
