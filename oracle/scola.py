"""sCOLA evolution of one box and monolithic periodic tCOLA (FP64).

Test infrastructure only (see oracle/__init__.py).

Paper passages followed:
  * Sec. 3.4.1: density assignment B^sCOLA = CiC of the box's particles onto the PM grid
    of the box; fractional masses that would land outside the box are ignored.
  * Sec. 3.4.2 and App. C: Dirichlet Poisson solve with Phi_BCs = D1(a_K) Phi_BC^0 (LEP),
    Phi padded with Phi_BCs; gradient by finite differences (order 2, 4 or 6, Sec. 3) on
    the nodes padded by N_ghost; CiC interpolation to the particles.
  * App. A eq. (drift-cola) and eq. (kick-scola): the kick uses
    grad(Delta^-1 delta) - D1 Psi1 + (D2 - D1^2) Psi2; the drift is unmodified.
  * App. B eqs. (D_COLA), (K_COLA) with the modified time factors, the operator E~ of
    eq. (operator_E), and the L-/L+ operators: p_res = 0 at the start, p = p_res + p_LPT
    at the end.
  * Sec. 2.2 (tCOLA) and App. A eq. (kick-tcola): the same operators on the periodic full
    box, with an FFT Poisson solve (FDA kernel of the same order), used as the monolithic
    comparison.

Readings where the paper is silent: the mean density in delta is the global one (one
particle per cell); interpolation corners outside the gradient grid [0, M]^3 contribute
nothing (symmetric with the dropped deposit).  The last force evaluation is done only
when final momenta are requested, since positions do not depend on it.
"""
from itertools import product

import numpy as np

from .lpt import fda_laplacian_kernel, first_derivative_weights, ghosts
from .poisson import dirichlet_potential


# --- cloud-in-cell weights -------------------------------------------------------------
def cic_corners(u):
    """Yield (offset, node index array (3, P), weight (P,)) for the 8 CiC corners of
    positions u (3, P); nodes sit at integer coordinates."""
    j0 = np.floor(u).astype(np.int64)
    f = u - j0
    for off in product((0, 1), repeat=3):
        w = np.ones(u.shape[1])
        for a in range(3):
            w = w * (f[a] if off[a] else 1.0 - f[a])
        yield off, j0 + np.array(off)[:, None], w


def lattice_positions(M):
    """Local positions i + 1/2 of an M^3 box (3, M, M, M)."""
    i = np.arange(M, dtype=np.float64) + 0.5
    return np.stack(np.meshgrid(i, i, i, indexing="ij"))


# --- box operators (Sec. 3.4) ------------------------------------------------------------
def box_deposit(u, M):
    """B^sCOLA: CiC onto interior nodes [1, M-1]^3; returns (delta, deposited mass).
    u: (3, P) local positions."""
    rho = np.zeros((M - 1,) * 3)
    for _, idx, w in cic_corners(u):
        ok = np.all((idx >= 1) & (idx <= M - 1), axis=0)
        np.add.at(rho, tuple(idx[:, ok] - 1), w[ok])
    return rho - 1.0, rho.sum()


def box_gradient(phi_pad, order=2):
    """Central gradient of the padded potential [-g, M+g]^3 on nodes [0, M]^3 (g = N_ghost
    of the FDA order)."""
    if order == 2:
        M = phi_pad.shape[0] - 3
        c = slice(1, M + 2)
        return np.stack([
            0.5 * (phi_pad[2:M + 3, c, c] - phi_pad[0:M + 1, c, c]),
            0.5 * (phi_pad[c, 2:M + 3, c] - phi_pad[c, 0:M + 1, c]),
            0.5 * (phi_pad[c, c, 2:M + 3] - phi_pad[c, c, 0:M + 1]),
        ])
    g = ghosts(order)
    M = phi_pad.shape[0] - 1 - 2 * g
    c = slice(g, g + M + 1)
    out = np.zeros((3,) + (M + 1,) * 3)
    for k, w in enumerate(first_derivative_weights(order), start=1):
        up, dn = slice(g + k, g + k + M + 1), slice(g - k, g - k + M + 1)
        out[0] += w * (phi_pad[up, c, c] - phi_pad[dn, c, c])
        out[1] += w * (phi_pad[c, up, c] - phi_pad[c, dn, c])
        out[2] += w * (phi_pad[c, c, up] - phi_pad[c, c, dn])
    return out


def box_interpolate(g, u):
    """B-bar^sCOLA: CiC interpolation of g (3, M+1, M+1, M+1) on nodes [0, M]^3 to u (3, P);
    corners outside the node range contribute zero."""
    M = g.shape[1] - 1
    out = np.zeros_like(u)
    for _, idx, w in cic_corners(u):
        ok = np.all((idx >= 0) & (idx <= M), axis=0)
        vals = g[:, idx[0, ok], idx[1, ok], idx[2, ok]]
        out[:, ok] += w[ok] * vals
    return out


def box_force(u, M, phi_bc_pad, delta=None, order=2):
    """grad^sCOLA (Delta^sCOLA)^-1 delta^sCOLA at the particles."""
    if delta is None:
        delta, _ = box_deposit(u, M)
    phi = dirichlet_potential(delta, phi_bc_pad, order=order)
    return box_interpolate(box_gradient(phi, order), u), delta, phi


def evolve_box(psi1, psi2, phi_bc0, steps, final=None, overrides=None, record=None,
               fda_order=2):
    """Evolve one sCOLA box through the KDK operator E~ (App. B).

    psi1, psi2: (3, M, M, M) displacement vectors of the box's particles (cells).
    phi_bc0: (M+1+2g)^3 padded boundary potential at D1 = 1 (g = N_ghost of fda_order).
    steps, final: from oracle.cosmology.cola_schedule.
    overrides: optional callable(k, u) -> (delta or None, phi_bc_pad or None) replacing
      delta^sCOLA and/or Phi_BCs at the k-th force evaluation (consistency tests of
      Sec. 4.3, eqs. test_setup2-4).
    Returns dict(x_res, p_res, u, p) with arrays of shape (3, M, M, M)."""
    M = psi1.shape[1]
    P = M ** 3
    q = lattice_positions(M).reshape(3, P)
    s1 = psi1.reshape(3, P)
    s2 = psi2.reshape(3, P)
    x_res = np.zeros((3, P))
    p_res = np.zeros((3, P))

    def force(k, u, D1):
        delta, bc = (None, None) if overrides is None else overrides(k, u)
        if bc is None:
            bc = D1 * phi_bc0
        g, delta, phi = box_force(u, M, bc, delta, fda_order)
        if record is not None:
            record.append(dict(u=u.copy(), delta=delta, phi=phi, g=g))
        return g

    u = q - steps[0]["D1"] * s1 + steps[0]["D2"] * s2
    g = force(0, u, steps[0]["D1"])
    n = len(steps)
    for k, st in enumerate(steps):
        p_res = p_res + st["beta"] * (g - st["D1"] * s1 + (st["D2"] - st["D1"] ** 2) * s2)
        x_res = x_res + st["alpha"] * p_res
        u = q - st["D1_next"] * s1 + st["D2_next"] * s2 + x_res
        if k < n - 1 or final is not None:
            g = force(k + 1, u, st["D1_next"])
    out = dict(x_res=x_res.reshape(3, M, M, M), u=u.reshape(3, M, M, M))
    p = None
    if final is not None:
        p_res = p_res + final["beta"] * (g - final["D1"] * s1 +
                                         (final["D2"] - final["D1"] ** 2) * s2)
        # L+ : p = p_res + (1/D(a)) (-dD1/da Psi1 + dD2/da Psi2)
        p = p_res + final["inv_drift"] * (-final["dD1"] * s1 + final["dD2"] * s2)
        p = p.reshape(3, M, M, M)
    out["p_res"] = p_res.reshape(3, M, M, M)
    out["p"] = p
    return out


# --- periodic full box (tCOLA, Sec. 2.2) ------------------------------------------------
def periodic_deposit(u, N):
    rho = np.zeros((N,) * 3)
    for _, idx, w in cic_corners(u):
        np.add.at(rho, tuple(np.mod(idx, N)), w)
    return rho - 1.0


def periodic_potential(delta, order=2):
    K = fda_laplacian_kernel(delta.shape[0], order)
    dk = np.fft.fftn(delta)
    with np.errstate(divide="ignore", invalid="ignore"):
        pk = np.where(K != 0.0, dk / K, 0.0)
    return np.fft.ifftn(pk).real


def periodic_gradient(phi, order=2):
    if order == 2:
        return np.stack([0.5 * (np.roll(phi, -1, a) - np.roll(phi, 1, a)) for a in range(3)])
    out = np.zeros((3,) + phi.shape)
    for k, w in enumerate(first_derivative_weights(order), start=1):
        for a in range(3):
            out[a] += w * (np.roll(phi, -k, a) - np.roll(phi, k, a))
    return out


def periodic_interpolate(g, u):
    N = g.shape[1]
    out = np.zeros_like(u)
    for _, idx, w in cic_corners(u):
        idx = np.mod(idx, N)
        out += w * g[:, idx[0], idx[1], idx[2]]
    return out


def evolve_periodic(psi1, psi2, steps, final=None, record=None, pm_only=False, p_init=None,
                    fda_order=2):
    """Monolithic tCOLA on the periodic N^3 box (same KDK operator as evolve_box).

    pm_only=True switches the COLA split off (plain PM, App. A eqs. drift/kick): the kick
    has no LPT terms, the drift moves x by alpha p, and p starts from p_init."""
    N = psi1.shape[1]
    P = N ** 3
    q = lattice_positions(N).reshape(3, P)
    s1 = psi1.reshape(3, P)
    s2 = psi2.reshape(3, P)
    x_res = np.zeros((3, P))
    p_res = np.zeros((3, P)) if p_init is None else p_init.reshape(3, P).copy()

    def force(u):
        delta = periodic_deposit(u, N)
        phi = periodic_potential(delta, fda_order)
        g = periodic_interpolate(periodic_gradient(phi, fda_order), u)
        if record is not None:
            record.append(dict(u=u.copy(), delta=delta, phi=phi, g=g))
        return g

    D1_0, D2_0 = steps[0]["D1"], steps[0]["D2"]
    if pm_only:
        x0 = q - D1_0 * s1 + D2_0 * s2
        u = x0.copy()
    else:
        u = q - D1_0 * s1 + D2_0 * s2
    g = force(u)
    n = len(steps)
    for k, st in enumerate(steps):
        if pm_only:
            p_res = p_res + st["beta"] * g
            x_res = x_res + st["alpha"] * p_res
            u = x0 + x_res
        else:
            p_res = p_res + st["beta"] * (g - st["D1"] * s1 + (st["D2"] - st["D1"] ** 2) * s2)
            x_res = x_res + st["alpha"] * p_res
            u = q - st["D1_next"] * s1 + st["D2_next"] * s2 + x_res
        if k < n - 1 or final is not None:
            g = force(u)
    out = dict(x_res=x_res.reshape(3, N, N, N), u=u.reshape(3, N, N, N), p_res=p_res)
    if final is not None and not pm_only:
        p_res = p_res + final["beta"] * (g - final["D1"] * s1 +
                                         (final["D2"] - final["D1"] ** 2) * s2)
        out["p_res"] = p_res
        out["p"] = (p_res + final["inv_drift"] * (-final["dD1"] * s1 + final["dD2"] * s2)
                    ).reshape(3, N, N, N)
    return out
