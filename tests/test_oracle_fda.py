"""Pins of the oracle's finite-difference orders 4 and 6 (Sec. 3 operators; App. C.1-C.2).

The oracle derives its stencils from Taylor conditions and types the sine-space eigenvalues
from App. C.2; these tests tie the two together and to textbook facts that neither uses:
the standard central-difference coefficient tables, exactness on polynomials, the h^n
convergence of the error, and a dense direct solve of the wide stencil.
"""
import numpy as np
import pytest

from oracle.lpt import (central_diff, fda_laplacian_kernel, first_derivative_weights,
                        poisson_periodic, second_derivative_weights)
from oracle.poisson import (bc_source_correction, bc_source_correction_wide,
                            dense_dirichlet_laplacian, dense_odd_laplacian, dirichlet_potential,
                            fda_eigenvalues, solve_zero_bc)
from oracle.scola import box_gradient, periodic_gradient

ORDERS = (2, 4, 6)

# textbook central-difference coefficients on offsets -g..g (spacing one)
FIRST = {2: [-1, 0, 1], 4: [1, -8, 0, 8, -1], 6: [-1, 9, -45, 0, 45, -9, 1]}
FIRST_DEN = {2: 2.0, 4: 12.0, 6: 60.0}
SECOND = {2: [1, -2, 1], 4: [-1, 16, -30, 16, -1], 6: [2, -27, 270, -490, 270, -27, 2]}
SECOND_DEN = {2: 1.0, 4: 12.0, 6: 180.0}


def full_first(order):
    c = first_derivative_weights(order)
    return np.concatenate([-c[::-1], [0.0], c])


def full_second(order):
    a = second_derivative_weights(order)
    return np.concatenate([a[::-1], [-2.0 * a.sum()], a])


@pytest.mark.parametrize("order", ORDERS)
def test_stencils_match_the_coefficient_tables(order):
    np.testing.assert_allclose(full_first(order), np.array(FIRST[order]) / FIRST_DEN[order],
                               atol=1e-15)
    np.testing.assert_allclose(full_second(order), np.array(SECOND[order]) / SECOND_DEN[order],
                               atol=1e-14)


@pytest.mark.parametrize("order", ORDERS)
def test_stencils_are_exact_on_polynomials_up_to_their_order(order):
    g = order // 2
    k = np.arange(-g, g + 1, dtype=np.float64)
    d1, d2 = full_first(order), full_second(order)
    for p in range(order + 1):
        # derivative of x^p at 0: 1 for p = 1 (first), 2 for p = 2 (second), else 0
        assert d1 @ k ** p == pytest.approx(1.0 if p == 1 else 0.0, abs=1e-12)
        assert d2 @ k ** p == pytest.approx(2.0 if p == 2 else 0.0, abs=1e-12)
    # the next even/odd power is not exact: the truncation error of an order-n stencil
    assert abs(d1 @ k ** (order + 1)) > 1e-3
    assert abs(d2 @ k ** (order + 2)) > 1e-3


@pytest.mark.parametrize("order", (4, 6))
def test_sine_eigenvalues_are_the_stencil_symbol(order):
    # App. C.2's closed forms equal sum_k a_k (2 cos(k theta) - 2) at theta = pi l / (n+1)
    for n in (7, 15, 63):
        th = np.pi * np.arange(1, n + 1) / (n + 1)
        sym = sum(a * (2 * np.cos(k * th) - 2)
                  for k, a in enumerate(second_derivative_weights(order), start=1))
        np.testing.assert_allclose(fda_eigenvalues(n, 1.0, order), sym, atol=1e-12)
        # negative definite and, at small l, -(pi l/(n+1))^2 to O(theta^(order+2))
        assert (fda_eigenvalues(n, 1.0, order) < 0).all()
    lam = fda_eigenvalues(255, 1.0, order)[0]
    th = np.pi / 256
    assert abs(lam + th ** 2) < th ** (order + 2)


@pytest.mark.parametrize("order", ORDERS)
def test_dst_solve_equals_dense_odd_continued_solve(order):
    rng = np.random.default_rng(order)
    for n in (3, 6, 7):
        src = rng.normal(size=(n, n, n))
        got = solve_zero_bc(src, 1.0, order)
        want = np.linalg.solve(dense_odd_laplacian(n, order), src.ravel()).reshape(n, n, n)
        np.testing.assert_allclose(got, want, atol=1e-12 * np.abs(want).max())


def test_odd_continuation_is_zero_outside_at_order_2():
    for n in (3, 5):
        np.testing.assert_array_equal(dense_odd_laplacian(n, 2), dense_dirichlet_laplacian(n))


@pytest.mark.parametrize("order", (4, 6))
def test_periodic_kernel_matches_closed_forms_and_configuration_stencil(order):
    N = 16
    th = 2 * np.pi * np.fft.fftfreq(N, d=1.0 / N) / N
    s2 = lambda x: np.sin(x) ** 2
    if order == 4:
        one = (s2(th) - 16 * s2(th / 2)) / 3.0
    else:
        one = -(2 * s2(3 * th / 2) - 27 * s2(th) + 270 * s2(th / 2)) / 45.0
    K = fda_laplacian_kernel(N, order)
    np.testing.assert_allclose(K, one[:, None, None] + one[None, :, None] + one[None, None, :],
                               atol=1e-12)
    # the Fourier solve inverts the configuration-space stencil (up to the zero mode)
    rng = np.random.default_rng(3)
    src = rng.normal(size=(N, N, N))
    src -= src.mean()
    phi = poisson_periodic(src, order)
    c = np.array(SECOND[order]) / SECOND_DEN[order]
    g = order // 2
    lap = sum(c[i + g] * (np.roll(phi, -i, 0) + np.roll(phi, -i, 1) + np.roll(phi, -i, 2))
              for i in range(-g, g + 1))
    np.testing.assert_allclose(lap, src, atol=1e-11)


@pytest.mark.parametrize("order", ORDERS)
def test_gradient_converges_at_its_order(order):
    errs = []
    for N in (32, 64):
        x = np.arange(N)
        f = np.sin(2 * np.pi * 3 * x / N)[:, None, None] * np.ones((1, 2, 2))
        exact = 2 * np.pi * 3 / N * np.cos(2 * np.pi * 3 * x / N)
        d = periodic_gradient(f, order)[0][:, 0, 0]
        assert np.allclose(central_diff(f, 0, order)[:, 0, 0], d)
        # relative to the derivative's amplitude, the error scales as h^order
        errs.append(np.abs(d - exact).max() / (2 * np.pi * 3 / N))
    assert errs[0] / errs[1] == pytest.approx(2.0 ** order, rel=0.05)


@pytest.mark.parametrize("order", (4, 6))
def test_box_gradient_matches_periodic_gradient_inside(order):
    # with the padded grid cut from a periodic field, the box gradient is the periodic one
    rng = np.random.default_rng(order)
    N, M, g = 24, 10, order // 2
    phi = rng.normal(size=(N, N, N))
    o = 5
    pad = phi[o - g:o + M + g + 1, o - g:o + M + g + 1, o - g:o + M + g + 1]
    want = periodic_gradient(phi, order)[:, o:o + M + 1, o:o + M + 1, o:o + M + 1]
    np.testing.assert_allclose(box_gradient(pad, order), want, atol=1e-13)


@pytest.mark.parametrize("order", (4, 6))
def test_bc_correction_of_a_constant_boundary_potential(order):
    # Phi_BCs = c on every layer outside the interior: Delta Phi_BCs at an interior node at
    # distance t <= g from one face (and farther than g from the others) is c times the
    # sum of the stencil weights that reach past the face, sum_{k >= t} a_k
    M, g, c = 12, order // 2, 0.7
    pad = np.full((M + 1 + 2 * g,) * 3, c)
    delta = np.zeros((M - 1,) * 3)
    out = bc_source_correction_wide(delta, pad, order)
    w = np.array(SECOND[order]) / SECOND_DEN[order]      # offsets -g..g
    mid = (M - 1) // 2
    for t in range(1, g + 1):
        want = -c * w[:g - t + 1].sum()                   # offsets -g..-t reach past j = 0
        assert out[t - 1, mid, mid] == pytest.approx(want, abs=1e-14)
        assert out[M - 1 - t, mid, mid] == pytest.approx(want, abs=1e-14)
    assert out[g, mid, mid] == 0.0 and out[mid, mid, mid] == 0.0
    # an edge node sums the two faces' terms
    assert out[0, 0, mid] == pytest.approx(2 * out[0, mid, mid], abs=1e-14)


def test_wide_correction_reduces_to_the_order_2_one():
    # the general code with the order-2 weights (N_ghost = 1) agrees with the order-2 one
    rng = np.random.default_rng(9)
    M = 9
    pad = rng.normal(size=(M + 3,) * 3)
    delta = rng.normal(size=(M - 1,) * 3)
    np.testing.assert_allclose(bc_source_correction_wide(delta, pad, 2),
                               bc_source_correction(delta, pad), atol=1e-14)


@pytest.mark.parametrize("order", (4, 6))
def test_dirichlet_solve_of_an_odd_mode(order):
    # a product of sines vanishing on the faces is an eigenmode of the odd-continued stencil:
    # with zero Phi_BCs the solve returns it exactly from delta = lambda Phi
    M = 16
    n = M - 1
    j = np.arange(1, M)
    a, b, cc = 2, 3, 5
    mode = (np.sin(np.pi * a * j / M)[:, None, None] * np.sin(np.pi * b * j / M)[None, :, None] *
            np.sin(np.pi * cc * j / M)[None, None, :])
    lam = fda_eigenvalues(n, 1.0, order)
    delta = (lam[a - 1] + lam[b - 1] + lam[cc - 1]) * mode
    g = order // 2
    phi = dirichlet_potential(delta, np.zeros((M + 1 + 2 * g,) * 3), order=order)
    np.testing.assert_allclose(phi[g + 1:g + M, g + 1:g + M, g + 1:g + M], mode, atol=1e-12)


@pytest.mark.parametrize("order", (2, 4, 6))
def test_periodic_force_transfer_closed_form(order):
    # A tiny plane wave of lattice displacements s = -D1 Psi1: the chain CiC deposit ->
    # FDA-n Poisson -> order-n gradient -> CiC interpolation gives, per Fourier mode,
    # g = -sin(k) S_n(k) / K_n(k) * D1 Psi1 with S_n the gradient's and K_n the Laplacian's
    # symbol (the deposit differences s at the two half-cell neighbours, 2 i sin(k/2); the
    # interpolation averages them, cos(k/2)).  S_n, K_n from the coefficient tables above.
    from oracle.lpt import displacement_vectors
    from oracle.scola import (lattice_positions, periodic_deposit, periodic_interpolate,
                              periodic_potential)
    N, amp, D1, m = 32, 1e-6, 3.0, 2
    q = np.arange(N) + 0.5
    delta = amp * np.cos(2 * np.pi * m * q / N)[:, None, None] * np.ones((N, N, N))
    psi1 = displacement_vectors(poisson_periodic(delta, order), order)
    k = 2 * np.pi * m / N
    g = order // 2
    offs = np.arange(-g, g + 1)
    S = (np.array(FIRST[order]) / FIRST_DEN[order] * np.sin(offs * k)).sum()
    K = (np.array(SECOND[order]) / SECOND_DEN[order] * np.cos(offs * k)).sum()
    T = -np.sin(k) * S / K
    u = lattice_positions(N).reshape(3, -1) - D1 * psi1.reshape(3, -1)
    got = periodic_interpolate(periodic_gradient(periodic_potential(periodic_deposit(u, N),
                                                                    order), order), u)
    want = T * D1 * psi1.reshape(3, -1)
    assert np.abs(got - want).max() < 1e-5 * np.abs(want).max()
    if order == 2:
        assert T == pytest.approx(np.cos(k / 2) ** 2)


@pytest.mark.parametrize("order,lo,hi", [(2, 0.0, 1e-13), (4, 1e-3, 0.1), (6, 1e-3, 0.1)])
def test_exact_boundary_consistency_by_order(order, lo, hi):
    # The full-box periodic potential on the Dirichlet layers and the full-box density inside
    # reproduce the periodic solution exactly at order 2; at orders 4 and 6 the DST-I solve
    # continues the zero-boundary unknown antisymmetrically past the faces, not by zeros, so
    # the stated method departs from the periodic solution by a few per cent of max |Phi|.
    from oracle.poisson import dirichlet_potential
    rng = np.random.default_rng(0)
    N, M, o, g = 24, 12, 4, order // 2
    delta = rng.normal(size=(N, N, N))
    delta -= delta.mean()
    phi = poisson_periodic(delta, order)
    pad = phi[o - g:o + M + g + 1, o - g:o + M + g + 1, o - g:o + M + g + 1]
    bc = pad.copy()
    bc[g + 1:g + M, g + 1:g + M, g + 1:g + M] = 0.0
    sol = dirichlet_potential(delta[o + 1:o + M, o + 1:o + M, o + 1:o + M], bc, order=order)
    err = np.abs(sol - pad).max() / np.abs(pad).max()
    assert lo <= err < hi
