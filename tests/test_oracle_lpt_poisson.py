"""Pins of the oracle's ICs, 2LPT potentials (Sec. 2.1, 3.1) and Dirichlet Poisson
solver (App. C)."""
import numpy as np
import pytest
import scipy.fft as sfft

import synthetic
from oracle.cosmology import Cosmology
from oracle.lpt import (eh_nowiggle_transfer, fda2_laplacian_kernel,
                        initial_density_fourier, linear_power, mode_indices,
                        poisson_periodic, second_order_source, sigma_R_unnormalised)
from oracle.poisson import (bc_source_correction, dense_dirichlet_laplacian,
                            dirichlet_potential, dst1_3d, fda2_eigenvalues, idst1_3d,
                            sine_matrix, solve_zero_bc)


# --- initial power spectrum and ICs ---------------------------------------------------
def test_transfer_function_limits():
    c = Cosmology()
    assert eh_nowiggle_transfer(1e-6, c) == pytest.approx(1.0, abs=1e-5)
    k = np.logspace(-3, 1, 50)
    T = eh_nowiggle_transfer(k, c)
    assert np.all(np.diff(T) < 0)          # monotone suppression, no wiggles


def test_sigma8_normalisation():
    c = Cosmology(sigma8=0.81)
    amp = c.sigma8 ** 2 / sigma_R_unnormalised(c)
    # Independent quadrature of the normalised spectrum in linear k (trapezoid, dense grid).
    k = np.linspace(1e-5, 20.0, 2_000_001)
    x = 8.0 * k
    W = 3 * (np.sin(x) - x * np.cos(x)) / x ** 3
    integrand = k ** 2 * amp * k ** c.n_s * eh_nowiggle_transfer(k, c) ** 2 * W ** 2
    s2 = np.trapezoid(integrand, k) / (2 * np.pi ** 2)
    assert np.sqrt(s2) == pytest.approx(0.81, rel=2e-4)
    np.testing.assert_allclose(linear_power(k[1:5], c),
                               amp * k[1:5] ** c.n_s * eh_nowiggle_transfer(k[1:5], c) ** 2)


def test_ic_spectrum_matches_input_power():
    # The discrete estimator L^3/N^6 <|delta_k|^2> of the generated field must equal the
    # input P(k, a_i) mode by mode in expectation; averaged over all modes of one
    # realisation the ratio is 1 within ~1/sqrt(#modes).
    c = Cosmology()
    N, L, g = 32, 200.0, 1.0 / 15.699060481297867
    dk = initial_density_fourier(synthetic.white_noise(N, 7), L, c, g)
    m = mode_indices(N)
    kmag = 2 * np.pi / L * np.sqrt(m[:, None, None] ** 2 + m[None, :, None] ** 2 +
                                   m[None, None, :] ** 2)
    P = linear_power(kmag, c) * g ** 2
    ok = kmag > 0
    ratio = (np.abs(dk[ok]) ** 2 * L ** 3 / N ** 6) / P[ok]
    assert abs(ratio.mean() - 1.0) < 4.0 / np.sqrt(ok.sum())
    assert dk[0, 0, 0] == 0
    # Hermitian symmetry: the real-space field is real.
    assert np.abs(np.fft.ifftn(dk).imag).max() < 1e-12 * np.abs(np.fft.ifftn(dk).real).max()


# --- Lagrangian potentials ---------------------------------------------------------------
def test_periodic_poisson_plane_wave():
    N = 16
    x = np.arange(N)
    src = np.cos(2 * np.pi * 3 * x / N)[:, None, None] * np.ones((1, N, N))
    phi = poisson_periodic(src)
    np.testing.assert_allclose(phi, src / (-4 * np.sin(np.pi * 3 / N) ** 2), atol=1e-13)


def test_second_order_source_single_wave_vanishes():
    N = 16
    x = np.arange(N) + 0.5
    phi = np.cos(2 * np.pi * 2 * x / N)[:, None, None] * np.ones((1, N, N))
    assert np.abs(second_order_source(phi)).max() < 1e-14


def test_second_order_source_two_waves():
    # phi = A cos(k1 x) + B cos(k2 y): with wide central differences phi_,xx =
    # -A sin^2(k1) cos(k1 x), phi_,yy = -B sin^2(k2) cos(k2 y), phi_,xy = 0, so the source
    # is the product A B sin^2(k1) sin^2(k2) cos(k1 x) cos(k2 y).
    N = 16
    q = np.arange(N) + 0.5
    k1, k2, A, B = 2 * np.pi * 1 / N, 2 * np.pi * 3 / N, 0.7, -1.3
    phi = A * np.cos(k1 * q)[:, None, None] + B * np.cos(k2 * q)[None, :, None] + 0 * q[None, None, :]
    want = (A * B * np.sin(k1) ** 2 * np.sin(k2) ** 2 *
            np.cos(k1 * q)[:, None, None] * np.cos(k2 * q)[None, :, None] * np.ones((1, 1, N)))
    np.testing.assert_allclose(second_order_source(phi), want, atol=1e-13)


def test_fda_kernel_zero_mode_and_sign():
    K = fda2_laplacian_kernel(8)
    assert K[0, 0, 0] == 0 and np.all(K.ravel()[1:] < 0)


# --- DST-I and the Dirichlet solve (App. C) ----------------------------------------------
def test_dst_matches_library_type1():
    # scipy's DST-I is twice the paper's sum along each axis.
    f = synthetic.normal((5, 7, 6), 1.0, 3)
    np.testing.assert_allclose(dst1_3d(f), sfft.dstn(f, type=1) / 8.0, atol=1e-12)


@pytest.mark.parametrize("n", [1, 4, 7, 15])
def test_dst_orthogonality(n):
    S = sine_matrix(n)
    np.testing.assert_allclose(2.0 / (n + 1) * S @ S, np.eye(n), atol=1e-13)
    f = synthetic.normal((n, n, n), 1.0, n)
    np.testing.assert_allclose(idst1_3d(dst1_3d(f)), f, atol=1e-12)


def test_sine_basis_eigenvalues():
    # Each sine vector is an eigenvector of the 1-D second difference with zero ends.
    n = 9
    T = -2 * np.eye(n) + np.eye(n, k=1) + np.eye(n, k=-1)
    S = sine_matrix(n)
    lam = fda2_eigenvalues(n)
    np.testing.assert_allclose(T @ S, S * lam[None, :], atol=1e-13)
    # the paper's order-2 formula -(4/d^2) sin^2(k_l d/4 * N/(N+1)), k_l = 2 pi l / L_x,
    # d = L_x / N_x: with the node spacing d = 1 (L_x = N_x cells) it gives these values
    l = np.arange(1, n + 1)
    Lx, d = float(n), 1.0
    paper = -4.0 / d ** 2 * np.sin(2 * np.pi * l / Lx * d / 4 * n / (n + 1)) ** 2
    np.testing.assert_allclose(lam, paper, atol=1e-13)


@pytest.mark.parametrize("n", [2, 3, 5])
def test_zero_bc_solve_matches_direct_solve(n):
    src = synthetic.normal((n, n, n), 1.0, 11 + n)
    A = dense_dirichlet_laplacian(n)
    direct = np.linalg.solve(A, src.ravel()).reshape(n, n, n)
    np.testing.assert_allclose(solve_zero_bc(src), direct, atol=1e-12)


def test_dirichlet_solve_with_boundary_matches_direct_solve():
    # Non-zero Dirichlet values: brute force on the full (M+1)^3 node set with the
    # boundary nodes fixed, against the DST path with the corrected source.
    M = 5
    rng = np.random.default_rng(5)
    delta = rng.standard_normal((M - 1,) * 3)
    pad = rng.standard_normal((M + 3,) * 3)
    pad[2:M + 1, 2:M + 1, 2:M + 1] = 0.0
    phi = dirichlet_potential(delta, pad)
    n = M - 1
    A = dense_dirichlet_laplacian(n)
    rhs = bc_source_correction(delta, pad).ravel()
    np.testing.assert_allclose(phi[2:M + 1, 2:M + 1, 2:M + 1],
                               np.linalg.solve(A, rhs).reshape(n, n, n), atol=1e-12)
    # and the discrete Poisson equation holds at every interior node with the real BCs
    lap = (phi[3:M + 2, 2:M + 1, 2:M + 1] + phi[1:M, 2:M + 1, 2:M + 1] +
           phi[2:M + 1, 3:M + 2, 2:M + 1] + phi[2:M + 1, 1:M, 2:M + 1] +
           phi[2:M + 1, 2:M + 1, 3:M + 2] + phi[2:M + 1, 2:M + 1, 1:M] -
           6 * phi[2:M + 1, 2:M + 1, 2:M + 1])
    np.testing.assert_allclose(lap, delta, atol=1e-11)


def test_exact_boundary_reproduces_periodic_solution():
    # Sec. 4.3, eq. (test_setup4) at the level of one solve: the true density inside and
    # the true potential on the shell give back the periodic solution in the interior.
    N, M = 16, 10
    delta_full = synthetic.normal((N, N, N), 1.0, 21)
    delta_full -= delta_full.mean()
    phi_full = poisson_periodic(delta_full)
    o = np.array([11, 3, 7])                      # box origin, wraps around the box
    j = np.arange(-1, M + 2)
    idx = [np.mod(o[a] + j, N) for a in range(3)]
    pad = phi_full[idx[0][:, None, None], idx[1][None, :, None], idx[2][None, None, :]]
    shell = pad.copy()
    shell[2:M + 1, 2:M + 1, 2:M + 1] = 0.0
    inner = [np.mod(o[a] + np.arange(1, M), N) for a in range(3)]
    delta_box = delta_full[inner[0][:, None, None], inner[1][None, :, None],
                           inner[2][None, None, :]]
    phi = dirichlet_potential(delta_box, shell)
    np.testing.assert_allclose(phi, pad, atol=1e-12)
