"""Pins of the oracle's time integrator in the Zel'dovich limit and of its power-spectrum
estimator against closed forms, each shown to fail for a mistake planted in a copy of the
oracle function (the copy is compiled from the oracle's own source with one edit)."""
import inspect
import textwrap

import numpy as np
import pytest

import synthetic
from oracle import run as oracle_run
from oracle import scola as oracle_scola
from oracle.cosmology import Cosmology, cola_schedule
from oracle.lpt import displacement_vectors, poisson_periodic, second_order_source
from oracle.run import power_spectrum
from oracle.scola import (box_force, evolve_box, evolve_periodic, lattice_positions,
                          periodic_deposit, periodic_gradient, periodic_interpolate,
                          periodic_potential)
from oracle.tiling import Tile, boundary_potential0, extract_box_field


def planted(func, old, new):
    """A copy of oracle function `func` with the source text `old` replaced by `new`."""
    src = textwrap.dedent(inspect.getsource(func))
    assert src.count(old) >= 1, old
    ns = dict(vars(inspect.getmodule(func)))
    exec(compile(src.replace(old, new), "<planted>", "exec"), ns)
    return ns[func.__name__]


# --- Zel'dovich limit of one KDK step (App. A-B) ---------------------------------------
# Over a short interval [a_i, a_i + eps] the residual displacement of COLA obeys
# dx_res/da = Dr(a) p_res and dp_res/da = K(a) F_res with p_res(a_i) = 0 (operator L-), where
# Dr = 1/(a^3 E) and K = -3/2 Omega_m/(a^2 E) are the drift and kick prefactors of App. A and
# F_res = g - D1 Psi1 + (D2 - D1^2) Psi2 is the residual force of eq. kick-scola.  Its Taylor
# expansion gives x_res = eps^2/2 Dr(a_i) K(a_i) F_res(a_i) + O(eps^3): one step must fall
# four times per halving of eps and reach that limit, whatever the modified time factors of
# the integrator are.
A_I = 0.05


def two_wave_fields(N, amp):
    """Psi1, Psi2 (cells) of two orthogonal small plane waves (the second-order source is
    then non-zero, so the Psi2 term of the kick is exercised)."""
    q = np.arange(N) + 0.5
    d = (amp * np.cos(2 * np.pi * q / N)[:, None, None] +
         0.7 * amp * np.sin(2 * np.pi * 2 * q / N)[None, :, None]) * np.ones((N,) * 3)
    phi1 = poisson_periodic(d)
    phi2 = poisson_periodic(second_order_source(phi1))
    return displacement_vectors(phi1), displacement_vectors(phi2), phi1


def residual_force_periodic(psi1, psi2, D1, D2):
    N = psi1.shape[1]
    u = (lattice_positions(N) - D1 * psi1 + D2 * psi2).reshape(3, -1)
    g = periodic_interpolate(periodic_gradient(periodic_potential(periodic_deposit(u, N))), u)
    return g - D1 * psi1.reshape(3, -1) + (D2 - D1 ** 2) * psi2.reshape(3, -1)


def limit_prediction(c, F):
    Dr = 1.0 / (A_I ** 3 * c.E(A_I))
    K = -1.5 * c.Omega_m / (A_I ** 2 * c.E(A_I))
    return 0.5 * Dr * K * F


def check_zeldovich_limit(evolve, F, c, eps_list=(4e-4, 2e-4, 1e-4)):
    """Returns (ratios of max|x_res| per halving of eps, relative deviation from the Taylor
    limit at the smallest eps)."""
    xs = []
    for eps in eps_list:
        steps, _ = cola_schedule(c, A_I, A_I + eps, 1)
        xs.append(evolve(steps).reshape(3, -1))
    ratios = [np.abs(xs[i]).max() / np.abs(xs[i + 1]).max() for i in range(len(xs) - 1)]
    pred = limit_prediction(c, F) * eps_list[-1] ** 2
    dev = np.abs(xs[-1] - pred).max() / np.abs(pred).max()
    return ratios, dev


def periodic_case():
    c = Cosmology()
    N = 16
    psi1, psi2, _ = two_wave_fields(N, 0.05)
    steps0, _ = cola_schedule(c, A_I, A_I + 1e-4, 1)
    F = residual_force_periodic(psi1, psi2, steps0[0]["D1"], steps0[0]["D2"])
    assert np.abs(F).max() > 1e-6 and np.abs(psi2).max() > 1e-6
    return c, psi1, psi2, F


def test_zeldovich_limit_periodic_step():
    c, psi1, psi2, F = periodic_case()
    ratios, dev = check_zeldovich_limit(
        lambda st: evolve_periodic(psi1, psi2, st)["x_res"], F, c)
    assert all(3.9 < r < 4.1 for r in ratios), ratios
    assert dev < 5e-3, dev


def test_zeldovich_limit_box_step():
    c = Cosmology()
    N = 16
    psi1, psi2, phi1 = two_wave_fields(N, 0.05)
    tile = Tile((2, 2, 2), 8, 4)
    s1, s2 = extract_box_field(psi1, tile), extract_box_field(psi2, tile)
    bc0 = boundary_potential0(phi1, tile)
    st0, _ = cola_schedule(c, A_I, A_I + 1e-4, 1)
    D1, D2 = st0[0]["D1"], st0[0]["D2"]
    M = tile.M
    u = (lattice_positions(M) - D1 * s1 + D2 * s2).reshape(3, -1)
    g, _, _ = box_force(u, M, D1 * bc0)
    F = g - D1 * s1.reshape(3, -1) + (D2 - D1 ** 2) * s2.reshape(3, -1)
    ratios, dev = check_zeldovich_limit(lambda st: evolve_box(s1, s2, bc0, st)["x_res"], F, c)
    assert all(3.9 < r < 4.1 for r in ratios), ratios
    assert dev < 5e-3, dev


@pytest.mark.parametrize("old,new", [
    # operator L- forgotten: the residual momentum starts from the LPT momentum instead of 0
    ("p_res = np.zeros((3, P)) if p_init is None else",
     "p_res = (-5.0 * s1) if p_init is None else"),
    # sign of the first-order LPT term of the kick
    ('(g - st["D1"] * s1 + (st["D2"]', '(g + st["D1"] * s1 + (st["D2"]'),
    # sign of the second-order term of the kick
    ('+ (st["D2"] - st["D1"] ** 2) * s2)', '- (st["D2"] - st["D1"] ** 2) * s2)'),
    # drift with the old momentum (kick and drift out of order)
    ('x_res = x_res + st["alpha"] * p_res\n            u = q', 
     'x_res = x_res + st["alpha"] * (p_res - st["beta"] * g)\n            u = q'),
])
def test_zeldovich_limit_catches_planted_integrator_mistakes(old, new):
    c, psi1, psi2, F = periodic_case()
    bad = planted(evolve_periodic, old, new)
    ratios, dev = check_zeldovich_limit(lambda st: bad(psi1, psi2, st)["x_res"], F, c)
    assert not (all(3.9 < r < 4.1 for r in ratios) and dev < 5e-3), (ratios, dev)


# --- P(k) and R(k) estimators (Sec. 4.2) ----------------------------------------------
def modes_with_norm2(N, n2):
    """Number of integer wave vectors of an N^3 FFT grid (components in [-N/2, N/2)) whose
    squared norm is n2, counted by brute force."""
    m = np.arange(-N // 2, N // 2)
    return int(np.sum((m[:, None, None] ** 2 + m[None, :, None] ** 2 +
                       m[None, None, :] ** 2) == n2))


def test_power_spectrum_of_one_cosine_mode():
    # delta = A cos(2 pi m x / N) has DFT amplitude A N^3 / 2 at the two wave vectors +-m
    # along x and zero elsewhere.  With P = L^3/N^6 <|delta_k|^2> over a bin, the bin of
    # |k| = 2 pi m / L holds (A N^3/2)^2 twice among its modes: P = A^2 L^3 / (2 n_modes);
    # every other bin is empty of power.
    N, L, A, m = 16, 100.0, 0.3, 3
    x = np.arange(N)
    delta = A * np.cos(2 * np.pi * m * x / N)[:, None, None] * np.ones((N, N, N))
    res = power_spectrum(delta, L)
    kc = 0.5 * (res["k_edges"][1:] + res["k_edges"][:-1])
    b = int(np.digitize([2 * np.pi * m / L], res["k_edges"])[0] - 1)
    n_modes = modes_with_norm2(N, m * m)          # |k| = 3: (3,0,0) and (2,2,1) families
    assert n_modes == 30 and res["count"][b] == n_modes
    assert res["P"][b] == pytest.approx(A ** 2 * L ** 3 / (2 * n_modes), rel=1e-12)
    others = np.delete(res["P"], b)[np.delete(res["count"], b) > 0]
    assert np.abs(others).max() < 1e-20 * res["P"][b]
    assert kc[b] == pytest.approx(2 * np.pi * m / L, rel=0.03)


def test_power_spectrum_of_white_noise_is_flat():
    # unit white noise on N^3 cells of volume (L/N)^3: E[P(k)] = (L/N)^3 in every bin.  |delta_k|^2
    # is exponential (relative spread 1) over cnt/2 independent modes per bin (conjugate
    # pairs), so the mean of 8 realisations has relative spread 1/sqrt(4 cnt): every bin
    # within 5 of those, the mode-weighted mean over all bins within 1 %.
    N, L = 32, 64.0
    ps = [power_spectrum(synthetic.normal((N, N, N), 1.0, s), L) for s in range(8)]
    cnt = ps[0]["count"]
    sel = cnt >= 8
    mean = np.mean([p["P"][sel] for p in ps], axis=0) / (L / N) ** 3
    assert np.all(np.abs(mean - 1) < 5.0 / np.sqrt(4 * cnt[sel]))
    assert abs(np.sum(mean * cnt[sel]) / np.sum(cnt[sel]) - 1) < 0.01


def test_cross_correlation_limits():
    d = synthetic.normal((16, 16, 16), 1.0, 7)
    for other, want in ((d, 1.0), (-d, -1.0), (3.0 * d, 1.0)):
        R = power_spectrum(d, 100.0, other=other)["R"]
        ok = power_spectrum(d, 100.0)["count"] > 0
        np.testing.assert_allclose(R[ok], want, atol=1e-12)


@pytest.mark.parametrize("old,new", [
    ("L ** 3 / N ** 6", "L ** 3 / N ** 3"),          # volume normalisation
    ("np.abs(dk.ravel()[ok]) ** 2", "np.abs(dk.ravel()[ok])"),  # amplitude, not power
    ("kmag = 2 * np.pi / L * np.sqrt(", "kmag = np.pi / L * np.sqrt("),   # wave number unit
])
def test_power_spectrum_pin_catches_planted_mistakes(old, new):
    bad = planted(oracle_run.power_spectrum, old, new)
    N, L, A, m = 16, 100.0, 0.3, 3
    x = np.arange(N)
    delta = A * np.cos(2 * np.pi * m * x / N)[:, None, None] * np.ones((N, N, N))
    res = bad(delta, L)
    b = int(np.digitize([2 * np.pi * m / L], res["k_edges"])[0] - 1)
    good = res["count"][b] == 30 and \
        abs(res["P"][b] / (A ** 2 * L ** 3 / 60) - 1) < 1e-12
    assert not good
