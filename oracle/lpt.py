"""Initial conditions and second-order LPT on the full-box LPT grid (FP64).

Test infrastructure only (see oracle/__init__.py).

Paper passages followed:
  * Sec. 3.1 step A.1: Gaussian initial density from the initial power spectrum by the
    standard convolution approach (white noise times the square root of P(k)).
  * Sec. 4 (first paragraph): Eisenstein-Hu fitting function for the initial spectrum,
    all operators approximated by finite differences at order 2.
  * Sec. 2.1, eqs. (LPTpotential1), (LPTpotential2): Delta phi1 = delta_i and
    Delta phi2 = sum_{i>j} [phi1_,ii phi1_,jj - (phi1_,ij)^2]; eqs. (LPT_Psi1),
    (LPT_Psi2) and App. A eq. (LPT-mapping): x = q - D1 Psi1 + D2 Psi2 with
    Psi1 = grad phi1 and Psi2 = grad phi2.
  * Sec. 3.1 step A.2: the second-order source by finite differencing costs nine
    one-dimensional gradient operations, i.e. phi_,ij = D_i (D_j phi) with the
    order-2 central difference D.

  * Sec. 3 (operators): Laplacians and gradients by finite differences at order 2, 4 or 6,
    N_ghost = 1, 2, 3 neighbours per side (fda_order arguments below; order 2 is the default
    and the order of every run of Sec. 4).

Readings where the paper is silent: the LPT grid has N = N_p nodes per side by default (or
N = N_p / 2, as in the paper's runs) and its node m sits at the centre (m + 1/2) L / N of
its cell, so with N = N_p the nodes coincide with the particles at q = (i + 1/2) cells; the
FDA-2 Laplacian kernel is used in every Fourier-space Poisson solve; the zero mode of
every potential is zero; the no-wiggle Eisenstein-Hu transfer function is used with
T_CMB = 2.7255 K; sigma_8 uses the top-hat window of radius 8 Mpc/h at a = 1.
"""
import numpy as np
from scipy.integrate import quad


# --- initial power spectrum (Sec. 4) ------------------------------------------------
def eh_nowiggle_transfer(k, cosmo):
    """Eisenstein & Hu (1998) zero-baryon-oscillation transfer function, k in h/Mpc."""
    k = np.asarray(k, dtype=np.float64)
    h = cosmo.h
    theta = cosmo.T_cmb / 2.7
    om_m = cosmo.Omega_m * h * h
    om_b = cosmo.Omega_b * h * h
    fb = cosmo.Omega_b / cosmo.Omega_m
    s = 44.5 * np.log(9.83 / om_m) / np.sqrt(1.0 + 10.0 * om_b ** 0.75)      # Mpc
    alpha_g = 1.0 - 0.328 * np.log(431.0 * om_m) * fb + 0.38 * np.log(22.3 * om_m) * fb * fb
    gamma_eff = cosmo.Omega_m * h * (alpha_g + (1.0 - alpha_g) / (1.0 + (0.43 * k * h * s) ** 4))
    q = k * theta * theta / gamma_eff
    L0 = np.log(2.0 * np.e + 1.8 * q)
    C0 = 14.2 + 731.0 / (1.0 + 62.5 * q)
    return L0 / (L0 + C0 * q * q)


def tophat_window(x):
    x = np.asarray(x, dtype=np.float64)
    return 3.0 * (np.sin(x) - x * np.cos(x)) / x ** 3


def sigma_R_unnormalised(cosmo, R=8.0):
    """sigma^2(R) = 1/(2 pi^2) int k^2 k^n_s T(k)^2 W(kR)^2 dk, for unit amplitude."""
    def integrand(lnk):
        k = np.exp(lnk)
        return k ** 3 * k ** cosmo.n_s * eh_nowiggle_transfer(k, cosmo) ** 2 * \
            tophat_window(k * R) ** 2 / (2.0 * np.pi ** 2)
    val, _ = quad(integrand, np.log(1e-6), np.log(1e3), epsabs=0.0, epsrel=1e-12, limit=2000)
    return val


def linear_power(k, cosmo):
    """P_lin(k, a = 1) in (Mpc/h)^3, normalised to cosmo.sigma8."""
    amp = cosmo.sigma8 ** 2 / sigma_R_unnormalised(cosmo)
    k = np.asarray(k, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        p = amp * k ** cosmo.n_s * eh_nowiggle_transfer(k, cosmo) ** 2
    return np.where(k > 0, p, 0.0)


# --- Fourier-space helpers -----------------------------------------------------------
def mode_indices(N):
    """Integer wave numbers m in [-N/2, N/2) along one axis, FFT order."""
    return np.fft.fftfreq(N, d=1.0 / N)


def ghosts(order):
    """N_ghost of an FDA order (Sec. 3): neighbours per side of the central stencils."""
    if order not in (2, 4, 6):
        raise ValueError("FDA order must be 2, 4 or 6")
    return order // 2


def first_derivative_weights(order):
    """Weights c_k (k = 1..g) of D f(i) = sum_k c_k (f(i+k) - f(i-k)), spacing one cell,
    from the Taylor conditions: f(i+k) - f(i-k) = 2 sum_{m odd} f^(m) k^m / m!, so the
    derivative needs 2 sum_k c_k k = 1 and sum_k c_k k^m = 0 for m = 3, 5, .., 2g - 1."""
    g = ghosts(order)
    k = np.arange(1, g + 1, dtype=np.float64)
    A = np.array([k ** m for m in range(1, 2 * g, 2)])
    rhs = np.zeros(g)
    rhs[0] = 0.5
    return np.linalg.solve(A, rhs)


def second_derivative_weights(order):
    """Weights a_k (k = 1..g) of D2 f(i) = sum_k a_k (f(i+k) + f(i-k) - 2 f(i)), from
    f(i+k) + f(i-k) - 2 f(i) = 2 sum_{m even >= 2} f^(m) k^m / m!: sum_k a_k k^2 = 1 and
    sum_k a_k k^m = 0 for m = 4, 6, .., 2g."""
    g = ghosts(order)
    k = np.arange(1, g + 1, dtype=np.float64)
    A = np.array([k ** m for m in range(2, 2 * g + 1, 2)])
    rhs = np.zeros(g)
    rhs[0] = 1.0
    return np.linalg.solve(A, rhs)


def fda_laplacian_kernel(N, order=2):
    """Fourier symbol of the order-`order` finite-difference Laplacian on a periodic N^3
    grid, spacing one cell: sum over axes of sum_k a_k (2 cos(k theta) - 2), theta =
    2 pi m / N.  Order 2 is fda2_laplacian_kernel."""
    if order == 2:
        return fda2_laplacian_kernel(N)
    a = second_derivative_weights(order)
    th = 2.0 * np.pi * mode_indices(N) / N
    s = sum(ak * (2.0 * np.cos((k + 1) * th) - 2.0) for k, ak in enumerate(a))
    return s[:, None, None] + s[None, :, None] + s[None, None, :]


def fda2_laplacian_kernel(N):
    """Fourier symbol of the order-2 finite-difference Laplacian, spacing one cell:
    -4 sum_i sin^2(pi m_i / N)."""
    s = np.sin(np.pi * mode_indices(N) / N) ** 2
    return -4.0 * (s[:, None, None] + s[None, :, None] + s[None, None, :])


def poisson_periodic(src, order=2):
    """Solve Delta phi = src on a periodic grid with the FDA Laplacian; zero mode 0."""
    K = fda_laplacian_kernel(src.shape[0], order)
    sk = np.fft.fftn(src)
    with np.errstate(divide="ignore", invalid="ignore"):
        pk = np.where(K != 0.0, sk / K, 0.0)
    return np.fft.ifftn(pk).real


# --- Step A.1: initial density --------------------------------------------------------
def initial_density_fourier(white_noise, L, cosmo, growth_ratio):
    """delta_i(k) = FFT(w)(k) * sqrt(P_lin(k, a_i) N^3 / L^3), zero mode removed.

    growth_ratio = D1(a_i) / D1(1), which scales P_lin(k, 1) to the initial time.
    With this normalisation the discrete estimator (L^3/N^6) <|delta_k|^2> equals P."""
    N = white_noise.shape[0]
    m = mode_indices(N)
    kf = 2.0 * np.pi / L
    kmag = kf * np.sqrt(m[:, None, None] ** 2 + m[None, :, None] ** 2 + m[None, None, :] ** 2)
    filt = np.sqrt(linear_power(kmag, cosmo) * growth_ratio ** 2 * N ** 3 / L ** 3)
    dk = np.fft.fftn(white_noise) * filt
    dk[0, 0, 0] = 0.0
    return dk


def initial_density(white_noise, L, cosmo, growth_ratio):
    return np.fft.ifftn(initial_density_fourier(white_noise, L, cosmo, growth_ratio)).real


# --- Step A.2: Lagrangian potentials ---------------------------------------------------
def central_diff(f, axis, order=2):
    """Central difference at the given FDA order, spacing one cell, periodic."""
    if order == 2:
        return 0.5 * (np.roll(f, -1, axis=axis) - np.roll(f, 1, axis=axis))
    out = np.zeros_like(f)
    for k, c in enumerate(first_derivative_weights(order), start=1):
        out += c * (np.roll(f, -k, axis=axis) - np.roll(f, k, axis=axis))
    return out


def second_order_source(phi1, order=2):
    """sum_{i>j} [phi_,ii phi_,jj - phi_,ij^2] with phi_,ij = D_i D_j phi (wide stencils)."""
    d = [central_diff(phi1, a, order) for a in range(3)]
    dd = [[central_diff(d[j], i, order) for j in range(3)] for i in range(3)]
    src = np.zeros_like(phi1)
    for i in range(3):
        for j in range(i):
            src += dd[i][i] * dd[j][j] - dd[i][j] ** 2
    return src


def lagrangian_potentials(white_noise, L, cosmo, growth_ratio, order=2):
    """phi1 = Delta^-1 delta_i and phi2 = Delta^-1 S[phi1] on the N^3 LPT grid."""
    dk = initial_density_fourier(white_noise, L, cosmo, growth_ratio)
    K = fda_laplacian_kernel(white_noise.shape[0], order)
    with np.errstate(divide="ignore", invalid="ignore"):
        phi1 = np.fft.ifftn(np.where(K != 0.0, dk / K, 0.0)).real
    phi2 = poisson_periodic(second_order_source(phi1, order), order)
    return phi1, phi2


def displacement_vectors(phi, order=2):
    """Psi = grad_q phi by central differences; shape (3, N, N, N)."""
    return np.stack([central_diff(phi, a, order) for a in range(3)])
