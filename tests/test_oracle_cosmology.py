"""Pins of the FP64 oracle's background, growth and time factors (App. A, App. B)."""
import numpy as np
import pytest

from oracle.cosmology import (Cosmology, N_LPT, cola_schedule, heath_growth,
                              lpt_momentum_factor, time_grid)


def test_eds_growth_closed_form():
    # Einstein-de Sitter: D1 = a / a_i exactly and D2 = -3/7 D1^2 (V[D2] = D2 - D1^2).
    eds = Cosmology(Omega_m=1.0)
    a = np.array([0.05, 0.1, 0.37, 1.0])
    D1, dD1, D2, dD2 = eds.growth(a, 0.05)
    np.testing.assert_allclose(D1, a / 0.05, rtol=1e-10)
    np.testing.assert_allclose(dD1, 1.0 / 0.05, rtol=1e-10)
    np.testing.assert_allclose(D2, -3.0 / 7.0 * (a / 0.05) ** 2, rtol=1e-9)
    np.testing.assert_allclose(dD2, -6.0 / 7.0 * a / 0.05 ** 2, rtol=1e-9)


def test_lcdm_growth_matches_heath_integral():
    c = Cosmology(Omega_m=0.31)
    a = np.array([0.05, 0.2, 0.5, 0.8, 1.0])
    D1 = c.growth(a, 0.05)[0]
    heath = np.array([heath_growth(c, x) for x in a])
    np.testing.assert_allclose(D1, heath / heath[0], rtol=1e-10)


def test_second_order_growth_ratio():
    # Early times: D2/D1^2 -> -3/7.  Late times: within 0.1% of the Bouchet et al. (1995)
    # fit -3/7 Omega_m(a)^(-1/143) (a published approximation, accurate to ~0.1%).
    c = Cosmology(Omega_m=0.31)
    a = np.array([0.001, 0.05, 0.5, 1.0])
    D1, _, D2, _ = c.growth(a, 0.001)
    ratio = D2 / D1 ** 2
    assert abs(ratio[0] + 3.0 / 7.0) < 1e-8
    om_a = c.Omega_m * a ** -3 / c.E(a) ** 2
    fit = -3.0 / 7.0 * om_a ** (-1.0 / 143.0)
    np.testing.assert_allclose(ratio, fit, rtol=1e-3)


def test_growth_derivatives_match_finite_differences():
    c = Cosmology()
    a = np.array([0.1, 0.6])
    h = 1e-5
    Dp = np.array(c.growth(a + h, 0.05))
    Dm = np.array(c.growth(a - h, 0.05))
    D = np.array(c.growth(a, 0.05))
    np.testing.assert_allclose(D[1], (Dp[0] - Dm[0]) / (2 * h), rtol=1e-8)
    np.testing.assert_allclose(D[3], (Dp[2] - Dm[2]) / (2 * h), rtol=1e-8)


def test_alpha_tilde_eds_closed_form():
    # EdS: H_conf = a^-1/2, so the integrand a^(n-2)/H_conf = a^(n-3/2).
    eds = Cosmology(Omega_m=1.0)
    n = N_LPT
    for ai, af, aK in [(0.1, 0.2, 0.15), (0.05, 0.145, 0.0975), (0.5, 1.0, 0.75)]:
        exact = (af ** (n - 0.5) - ai ** (n - 0.5)) / (n - 0.5) / aK ** n
        assert eds.alpha_tilde(ai, af, aK) == pytest.approx(exact, rel=1e-12)


def test_standard_factors_eds_closed_form():
    # App. B eq. alpha-beta-standard in EdS (E = a^-3/2): the drift prefactor 1/(a^3 E) =
    # a^-3/2 and the kick prefactor -3/2 / (a^2 E) = -3/2 a^-1/2 integrate in closed form.
    eds = Cosmology(Omega_m=1.0)
    for ai, af in [(0.1, 0.2), (0.05, 0.145), (0.5, 1.0)]:
        assert eds.alpha_standard(ai, af) == pytest.approx(
            2.0 * (ai ** -0.5 - af ** -0.5), rel=1e-12)
        assert eds.beta_standard(ai, af) == pytest.approx(
            -3.0 * (af ** 0.5 - ai ** 0.5), rel=1e-12)
    steps, _ = cola_schedule(eds, 0.1, 0.5, 4, discretisation="standard")
    assert steps[1]["alpha"] == pytest.approx(2.0 * (0.2 ** -0.5 - 0.3 ** -0.5), rel=1e-12)
    assert steps[1]["beta"] == pytest.approx(-3.0 * (0.25 ** 0.5 - 0.15 ** 0.5), rel=1e-12)


def test_modified_factors_converge_to_standard_ones():
    # App. B: the modified factors approximate int D dt and int K dt; as the step shrinks
    # their ratio to the standard discretisation tends to 1 at second order.
    c = Cosmology()
    a = 0.3
    errs = []
    for eps in (1e-2, 5e-3):
        al = c.alpha_tilde(a, a + eps, a + eps / 2) / c.alpha_standard(a, a + eps)
        be = c.beta_tilde(a, a + eps, a + eps / 2) / c.beta_standard(a, a + eps)
        errs.append((abs(al - 1), abs(be - 1)))
    assert errs[0][0] < 2e-3 and errs[0][1] < 2e-3
    assert errs[1][0] < errs[0][0] / 3 and errs[1][1] < errs[0][1] / 3


def test_schedule_structure():
    c = Cosmology()
    steps, final = cola_schedule(c, 0.05, 1.0, 10, want_final_kick=True)
    t = time_grid(0.05, 1.0, 10)
    assert len(steps) == 10
    assert steps[0]["a_D"] == 0.05 and steps[-1]["a_next"] == pytest.approx(1.0)
    # the first kick spans [t0, t_1/2], the others [t_{k-1/2}, t_{k+1/2}]
    assert steps[0]["beta"] == pytest.approx(c.beta_tilde(t[0], 0.5 * (t[0] + t[1]), t[0]))
    assert steps[3]["beta"] == pytest.approx(
        c.beta_tilde(0.5 * (t[2] + t[3]), 0.5 * (t[3] + t[4]), t[3]))
    assert final["beta"] == pytest.approx(c.beta_tilde(0.5 * (t[9] + t[10]), t[10], t[10]))
    D1 = np.array([s["D1"] for s in steps] + [steps[-1]["D1_next"]])
    assert D1[0] == pytest.approx(1.0)
    assert np.all(np.diff(D1) > 0)


def test_lpt_momentum_eds():
    # EdS: 1/D(a) = a^2 H_conf = a^(3/2); dD1/da = 1/a_i so p_LPT = -a^(3/2)/a_i Psi1.
    eds = Cosmology(Omega_m=1.0)
    c1, c2 = lpt_momentum_factor(eds, 0.4, 0.05)
    assert c1 == pytest.approx(-0.4 ** 1.5 / 0.05, rel=1e-9)
    assert c2 == pytest.approx(-6.0 / 7.0 * 0.4 / 0.05 ** 2 * 0.4 ** 1.5, rel=1e-8)
