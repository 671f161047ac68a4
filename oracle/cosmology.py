"""Background expansion, growth factors and COLA time factors (FP64).

Test infrastructure only (see oracle/__init__.py).

Paper passages followed:
  * App. A, eqs. (drift) and (kick): drift prefactor 1/(a^2 H_conf), kick prefactor
    -3/2 Omega_m H0^2 / (a H_conf), with H_conf = a'/a the conformal Hubble factor.
  * App. A, eqs. (VD1), (VD2): the operator V[.] = -(1/K) d/da((1/D) d./da) satisfies
    V[D1] = D1 and V[D2] = D2 - D1^2.  Written out, these are the growth ODEs below.
  * Sec. 3.3 (LEP paragraph): D1 is normalised to one at the initial scale factor.
  * App. B, modified discretisation: time factors alpha~ and beta~ with u(a) = a^n_LPT,
    n_LPT = -2.5, time variable t(a) = a.
  * Sec. 4: time steps linearly spaced in a.

Readings where the paper is silent: flat LambdaCDM without radiation (Omega_L =
1 - Omega_m), H0 = 1; the growth ODE starts on the growing mode deep in matter
domination (D1 = a, D2 = -3/7 a^2); D2 is scaled by the square of the D1 normalisation;
half-steps are midpoints in a.
"""
import numpy as np
from scipy.integrate import quad, solve_ivp

N_LPT = -2.5          # App. B, modified discretisation: the exponent adopted by the paper
A_START = 1e-6        # start of the growth integration (matter-dominated growing mode)


class Cosmology:
    """Flat LambdaCDM background; all rates in units of H0."""

    def __init__(self, Omega_m=0.31, Omega_b=0.0486, h=0.6774, n_s=0.9667,
                 sigma8=0.81, T_cmb=2.7255):
        self.Omega_m = float(Omega_m)
        self.Omega_b = float(Omega_b)
        self.h = float(h)
        self.n_s = float(n_s)
        self.sigma8 = float(sigma8)
        self.T_cmb = float(T_cmb)
        self._growth_cache = {}

    # --- background (App. A) ------------------------------------------------------
    def E(self, a):
        """H(a)/H0 for flat LambdaCDM."""
        return np.sqrt(self.Omega_m * np.asarray(a, dtype=np.float64) ** -3 + 1.0 - self.Omega_m)

    def H_conf(self, a):
        """Conformal Hubble factor a'/a = a H(a), in units of H0."""
        a = np.asarray(a, dtype=np.float64)
        return a * self.E(a)

    def drift_prefactor(self, a):
        """App. A eq. (drift): D(a) = 1 / (a^2 H_conf(a))."""
        a = np.asarray(a, dtype=np.float64)
        return 1.0 / (a * a * self.H_conf(a))

    def kick_prefactor(self, a):
        """App. A eq. (kick): K(a) = -3/2 Omega_m / (a H_conf(a))."""
        a = np.asarray(a, dtype=np.float64)
        return -1.5 * self.Omega_m / (a * self.H_conf(a))

    # --- growth factors (App. A, eqs. VD1 and VD2) ---------------------------------
    def _growth_rhs(self, a, y):
        # y = [D1, P1, D2, P2] with P = (1/drift_prefactor) dD/da = a^3 E dD/da.
        # V[D] = -(1/K) dP/da, so V[D1] = D1 gives dP1/da = -K D1, and
        # V[D2] = D2 - D1^2 gives dP2/da = -K (D2 - D1^2).
        D1, P1, D2, P2 = y
        inv_drift = a ** 3 * self.E(a)
        mK = -self.kick_prefactor(a)
        return [P1 / inv_drift, mK * D1, P2 / inv_drift, mK * (D2 - D1 * D1)]

    def growth_unnormalised(self, a):
        """(D1, dD1/da, D2, dD2/da) on the growing mode, D1 -> a as a -> 0."""
        a = np.atleast_1d(np.asarray(a, dtype=np.float64))
        grid, inverse = np.unique(a, return_inverse=True)
        a0 = A_START
        y0 = [a0, a0 ** 3 * self.E(a0) * 1.0,
              -3.0 / 7.0 * a0 * a0, a0 ** 3 * self.E(a0) * (-6.0 / 7.0 * a0)]
        sol = solve_ivp(self._growth_rhs, (a0, float(grid[-1])), y0, method="DOP853",
                        t_eval=grid, rtol=1e-13, atol=1e-30)
        if not sol.success:
            raise RuntimeError(sol.message)
        D1, P1, D2, P2 = sol.y
        inv_drift = grid ** 3 * self.E(grid)
        out = np.stack([D1, P1 / inv_drift, D2, P2 / inv_drift])
        return out[:, inverse.ravel()]

    def growth(self, a, a_norm):
        """Growth factors normalised so that D1(a_norm) = 1 (Sec. 3.3, LEP paragraph).

        Returns (D1, dD1/da, D2, dD2/da); D2 is divided by D1_unnorm(a_norm)^2 so that
        the second-order displacement keeps its amplitude relative to the first.
        """
        a = np.atleast_1d(np.asarray(a, dtype=np.float64))
        g = self.growth_unnormalised(np.concatenate([[a_norm], a]))
        n1 = g[0, 0]
        return g[0, 1:] / n1, g[1, 1:] / n1, g[2, 1:] / n1 ** 2, g[3, 1:] / n1 ** 2

    # --- COLA time factors (App. B, modified discretisation) -----------------------
    def alpha_tilde(self, a_i, a_f, a_K, n=N_LPT):
        """alpha~_p(a_i, a_f, a_K) = a_K^-n * integral_{a_i}^{a_f} a^(n-2) / H_conf(a) da."""
        val, _ = quad(lambda x: x ** (n - 2.0) / self.H_conf(x), a_i, a_f,
                      epsabs=0.0, epsrel=1e-13, limit=200)
        return val / a_K ** n

    def beta_tilde(self, a_i, a_f, a_D, n=N_LPT):
        """beta~_delta(a_i, a_f, a_D) = -3/2 Omega_m (a_f^n - a_i^n) / (n a_D^n H_conf(a_D))."""
        return -1.5 * self.Omega_m * (a_f ** n - a_i ** n) / (n * a_D ** n * self.H_conf(a_D))

    # --- standard discretisation (App. B, kept for tests of the modified one) -----
    def alpha_standard(self, a_i, a_f):
        val, _ = quad(lambda x: self.drift_prefactor(x), a_i, a_f, epsabs=0.0, epsrel=1e-13)
        return val

    def beta_standard(self, a_i, a_f):
        val, _ = quad(lambda x: self.kick_prefactor(x), a_i, a_f, epsabs=0.0, epsrel=1e-13)
        return val


def time_grid(a_i, a_f, n_steps):
    """Sec. 4: n_steps intervals linearly spaced in a; returns t_0..t_n."""
    return a_i + (a_f - a_i) * np.arange(n_steps + 1, dtype=np.float64) / n_steps


def cola_schedule(cosmo, a_i, a_f, n_steps, want_final_kick=False, discretisation="modified",
                  n_lpt=N_LPT):
    """Scalars of the KDK operator E~ of App. B (eq. operator_E with K~, D~).

    discretisation "modified" uses the time factors alpha~, beta~ with u(a) = a^n_lpt;
    "standard" uses eq. alpha-beta-standard (integrals of the drift and kick prefactors).

    Reading: the product in eq. (operator_E) runs over i = 0..n-1 so that the last drift
    ends at t_{n+1} = a_f; with n_steps = n+1 drifts there are n_steps kicks before the
    last drift ends, and one final half kick that only matters for momenta.

    Step k (k = 0..n_steps-1) is: kick with the force at t_k from t_{k-1/2} (t_0 when
    k = 0) to t_{k+1/2}; drift from t_k to t_{k+1} with the momentum at t_{k+1/2}.
    """
    t = time_grid(a_i, a_f, n_steps)
    half = 0.5 * (t[:-1] + t[1:])
    D1, dD1, D2, dD2 = cosmo.growth(t, a_i)
    if discretisation == "standard":
        beta = lambda ai, af, aD: cosmo.beta_standard(ai, af)
        alpha = lambda ai, af, aK: cosmo.alpha_standard(ai, af)
    else:
        beta = lambda ai, af, aD: cosmo.beta_tilde(ai, af, aD, n_lpt)
        alpha = lambda ai, af, aK: cosmo.alpha_tilde(ai, af, aK, n_lpt)
    steps = []
    for k in range(n_steps):
        aK_i = t[0] if k == 0 else half[k - 1]
        aK_f = half[k]
        steps.append(dict(
            a_D=t[k], a_next=t[k + 1],
            beta=beta(aK_i, aK_f, t[k]),
            alpha=alpha(t[k], t[k + 1], half[k]),
            D1=D1[k], D2=D2[k], D1_next=D1[k + 1], D2_next=D2[k + 1],
        ))
    final = None
    if want_final_kick:
        n = n_steps
        final = dict(a_D=t[n], beta=beta(half[n - 1], t[n], t[n]),
                     D1=D1[n], D2=D2[n], dD1=dD1[n], dD2=dD2[n],
                     inv_drift=1.0 / cosmo.drift_prefactor(t[n]))
    return steps, final


def heath_growth(cosmo, a):
    """Integral solution of the linear growth equation, valid when Omega_L is constant:
    D(a) proportional to E(a) * integral_0^a da' / (a' E(a'))^3.  Independent of the ODE
    above; used only to pin it."""
    val, _ = quad(lambda x: 1.0 / (x * cosmo.E(x)) ** 3, 0.0, a, epsabs=0.0, epsrel=1e-13,
                  limit=200)
    return 2.5 * cosmo.Omega_m * float(cosmo.E(a)) * val


def lpt_momentum_factor(cosmo, a, a_i):
    """L+ operator (App. B): p_LPT = (1/D(a)) (-dD1/da Psi1 + dD2/da Psi2).

    Returns the two coefficients (c1, c2) with p_LPT = c1 Psi1 + c2 Psi2."""
    _, dD1, _, dD2 = cosmo.growth(np.array([a]), a_i)
    inv_drift = 1.0 / float(cosmo.drift_prefactor(a))
    return -dD1[0] * inv_drift, dD2[0] * inv_drift


__all__ = ["Cosmology", "time_grid", "cola_schedule", "heath_growth",
           "lpt_momentum_factor", "N_LPT"]
