"""Pins of the oracle's coarse LPT grid (Sec. 3.3 C.2, Sec. 4: N = N_p / 2): Psi differenced
on the LPT grid and interpolated by CiC to the particles, Phi_BC^0 interpolated to the PM
nodes; LPT node m at the centre (m + 1/2) L / N of its cell."""
import numpy as np
import pytest

import synthetic
from oracle.tiling import (Tile, boundary_potential0, boundary_potential0_coarse,
                           interpolate_lpt_grid, psi_at_particles)


def test_full_resolution_grid_is_the_identity():
    rng = np.random.default_rng(1)
    N = 12
    psi = rng.normal(size=(3, N, N, N))
    np.testing.assert_array_equal(psi_at_particles(psi, N), psi)
    phi = rng.normal(size=(N, N, N))
    t = Tile((3, 5, 7), 4, 2)
    np.testing.assert_allclose(boundary_potential0_coarse(phi, t, N), boundary_potential0(phi, t),
                               atol=1e-15)


def test_cic_from_cell_centres_conserves_the_sum():
    # every coarse node hands out weights (1/4, 3/4, 3/4, 1/4) per axis to the lattice at
    # ratio 2: the particle sum is 2^3 times the node sum, for any field
    rng = np.random.default_rng(2)
    N = 8
    f = rng.normal(size=(2, N, N, N))
    out = psi_at_particles(f, 2 * N) / 2.0          # undo the unit conversion
    np.testing.assert_allclose(out.sum(axis=(1, 2, 3)), 8.0 * f.sum(axis=(1, 2, 3)), rtol=1e-12)


@pytest.mark.parametrize("p", [1, 3])
def test_interpolated_plane_wave_closed_form(p):
    # f(m) = cos(k m) on the LPT grid, k = 2 pi p / N; particle 2m sits at LPT coordinate
    # m - 1/4 (weights 1/4, 3/4 on nodes m - 1, m) and particle 2m + 1 at m + 1/4 (3/4, 1/4
    # on m, m + 1): the interpolated wave is Re[(3/4 + e^{-ik}/4) e^{ikm}] and
    # Re[(3/4 + e^{ik}/4) e^{ikm}]
    N = 16
    k = 2 * np.pi * p / N
    m = np.arange(N)
    f = np.cos(k * m)[:, None, None] * np.ones((1, N, N))
    i = np.arange(2 * N) + 0.5
    pts = np.stack([i, np.full_like(i, 0.5), np.full_like(i, 0.5)])
    got = interpolate_lpt_grid(f, pts, 2 * N)
    even = np.real((0.75 + 0.25 * np.exp(-1j * k)) * np.exp(1j * k * m))
    odd = np.real((0.75 + 0.25 * np.exp(1j * k)) * np.exp(1j * k * m))
    np.testing.assert_allclose(got[0::2], even, atol=1e-14)
    np.testing.assert_allclose(got[1::2], odd, atol=1e-14)


def test_interpolation_error_is_second_order():
    # against the continuous field at the particle position, CiC errs by O((k d)^2)
    errs = []
    for N in (16, 32):
        k = 2 * np.pi / N
        m = np.arange(N)
        f = np.cos(k * m)[:, None, None] * np.ones((1, N, N))
        i = np.arange(2 * N) + 0.5
        pts = np.stack([i, np.full_like(i, 0.5), np.full_like(i, 0.5)])
        u = i / 2 - 0.5
        errs.append(np.abs(interpolate_lpt_grid(f, pts, 2 * N) - np.cos(k * u)).max())
    assert errs[0] / errs[1] == pytest.approx(4.0, rel=0.02)


def test_boundary_potential_units_and_shell():
    # phi in coarse-cell^2 units becomes lattice-cell^2 units: a constant c gives 4 c on the
    # shell at ratio 2, zero inside
    N, c = 8, 0.3
    phi = np.full((N, N, N), c)
    t = Tile((4, 4, 4), 4, 2)
    bc = boundary_potential0_coarse(phi, t, 2 * N, ghosts=2)
    M = t.M
    assert bc.shape == (M + 5,) * 3
    shell = np.ones_like(bc, dtype=bool)
    shell[3:M + 2, 3:M + 2, 3:M + 2] = False
    np.testing.assert_allclose(bc[shell], 4 * c, rtol=1e-14)
    assert (bc[~shell] == 0).all()


def test_coarse_lpt_run_end_to_end_properties():
    # N = N_p / 2: the run uses the coarse white noise; the LPT displacement of the lattice is
    # the CiC interpolation of the coarse one, so the first deposit and the final positions
    # are finite and the output density has zero mean
    from oracle.run import run_scola
    from oracle.tiling import uniform_tiling
    Np, N = 16, 8
    w = synthetic.white_noise(N, 4)
    out = run_scola(w, 64.0, uniform_tiling(Np, 2, 4), n_steps=2, Np=Np)
    assert out["pos"].shape == (3, Np, Np, Np) and np.isfinite(out["pos"]).all()
    assert abs(out["density"].mean()) < 1e-12
    assert out["psi1"].shape == (3, Np, Np, Np)
