"""Poisson solver with Dirichlet boundary conditions by type-I discrete sine transform.

Test infrastructure only (see oracle/__init__.py).

Paper passages followed (App. C):
  * C.1: Phi = Phi~ + Phi_BCs with Phi_BCs non-zero only on the layer just outside the
    active domain; delta' = delta - Delta Phi_BCs differs from delta only on the layer
    of active nodes next to the faces; Phi~ solves Delta Phi~ = delta' with zero
    boundary values.
  * C.2, eq. (DST_delta): 3-D DST-I with basis sin(pi l i / (N+1)), written here as a
    dense sine matrix per axis (the definition itself, no fast transform).
  * C.2, eqs. (IDST_delta), (IDST_Phi): inverse = DST-I times 8 / prod(N+1).
  * C.2, the order-2, -4 and -6 eigenvalue formulas and eq. (Poisson_sine_space):
    Phi^{lmn} = delta^{lmn} / (lambda_l + lambda_m + lambda_n).
  * Sec. 3.4.2: the Dirichlet layers are N_ghost cells thick (1, 2, 3 at FDA order 2, 4,
    6) and Phi is padded with Phi_BCs.

Reading: the eigenvalue uses the true PM node spacing d (one lattice cell), so that
lambda_l = -(4/d^2) sin^2(pi l / (2 (N_g + 1))); the paper's own parenthetical value of
L_x is a slip (see the design notes).  Inverse sums in eqs. (IDST_*) run over l, m, n.
At orders 4 and 6 the sine basis is an eigenbasis of the wide stencil only when the zero-
boundary unknown is continued antisymmetrically past each face (node -k = -node k); the
method as stated (DST-I with the App. C.2 eigenvalues) solves that problem, and so does this
oracle.  delta' = delta - Delta Phi_BCs takes Phi_BCs on the N_ghost layers outside the
interior, zero inside, with the same order-n stencil.
"""
import numpy as np


def sine_matrix(n):
    """S[i-1, l-1] = sin(pi l i / (n + 1)), i, l in [1, n]."""
    i = np.arange(1, n + 1)
    return np.sin(np.pi * np.outer(i, i) / (n + 1))


def dst1_3d(f):
    """Eq. (DST_delta): sum_ijk f_ijk X_i^l Y_j^m Z_k^n (unnormalised)."""
    Sx, Sy, Sz = (sine_matrix(n) for n in f.shape)
    return np.einsum("ijk,il,jm,kn->lmn", f, Sx, Sy, Sz, optimize=True)


def idst1_3d(F):
    """Eqs. (IDST_delta)/(IDST_Phi): DST-I times 8 / ((Nx+1)(Ny+1)(Nz+1))."""
    nx, ny, nz = F.shape
    return dst1_3d(F) * 8.0 / ((nx + 1) * (ny + 1) * (nz + 1))


def fda2_eigenvalues(n, d=1.0):
    """Order-2 eigenvalues of the 1-D second difference on the DST-I basis."""
    l = np.arange(1, n + 1)
    return -4.0 / d ** 2 * np.sin(np.pi * l / (2.0 * (n + 1))) ** 2


def fda_eigenvalues(n, d=1.0, order=2):
    """App. C.2: eigenvalues of the order-2, -4, -6 one-dimensional second difference on
    the DST-I basis of n unknowns, written with k_l d N/(N+1) = 2 pi l / (n + 1)."""
    if order == 2:
        return fda2_eigenvalues(n, d)
    l = np.arange(1, n + 1)
    kd = 2.0 * np.pi * l / (n + 1)          # k_l d_x N_x / (N_x + 1)
    s2 = lambda x: np.sin(x) ** 2
    if order == 4:
        return (s2(kd / 2) - 16.0 * s2(kd / 4)) / (3.0 * d ** 2)
    if order == 6:
        return -(2.0 * s2(3.0 * kd / 4) - 27.0 * s2(kd / 2) + 270.0 * s2(kd / 4)) / (45.0 * d ** 2)
    raise ValueError("FDA order must be 2, 4 or 6")


def solve_zero_bc(src, d=1.0, order=2):
    """Delta phi = src with phi = 0 on the nodes just outside the array (App. C.2)."""
    lx, ly, lz = (fda_eigenvalues(n, d, order) for n in src.shape)
    F = dst1_3d(src)
    F = F / (lx[:, None, None] + ly[None, :, None] + lz[None, None, :])
    return idst1_3d(F)


def bc_source_correction(delta, phi_pad, d=1.0):
    """App. C.1: delta' = delta - Delta Phi_BCs.

    delta: interior nodes [1, M-1]^3 (array index j-1).  phi_pad: potential on the padded
    grid [-1, M+1]^3 (index j+1) whose face layer j in {0, M} holds Phi_BCs.  Phi_BCs
    vanishes inside, so Delta Phi_BCs at an interior node is the sum of the Phi_BCs values
    at its face-layer neighbours, divided by d^2."""
    M = delta.shape[0] + 1
    out = delta.copy()
    # face j = 0 neighbours interior j = 1; face j = M neighbours interior j = M-1
    out[0, :, :] -= phi_pad[1, 2:M + 1, 2:M + 1] / d ** 2
    out[-1, :, :] -= phi_pad[M + 1, 2:M + 1, 2:M + 1] / d ** 2
    out[:, 0, :] -= phi_pad[2:M + 1, 1, 2:M + 1] / d ** 2
    out[:, -1, :] -= phi_pad[2:M + 1, M + 1, 2:M + 1] / d ** 2
    out[:, :, 0] -= phi_pad[2:M + 1, 2:M + 1, 1] / d ** 2
    out[:, :, -1] -= phi_pad[2:M + 1, 2:M + 1, M + 1] / d ** 2
    return out


def bc_source_correction_wide(delta, phi_pad, order, d=1.0):
    """App. C.1 at FDA order 4 or 6: delta' = delta - Delta Phi_BCs with the order-n
    Laplacian.  phi_pad: the potential on [-g, M+g]^3 (index j + g, g = N_ghost) whose
    layers outside [1, M-1] hold Phi_BCs; Phi_BCs is zero on the interior, so the stencil of
    an interior node picks up only the (at most g) outside nodes along each axis."""
    from .lpt import ghosts, second_derivative_weights
    g = ghosts(order)
    M = delta.shape[0] + 1
    bc = phi_pad.copy()
    bc[g + 1:g + M, g + 1:g + M, g + 1:g + M] = 0.0
    inner = slice(g + 1, g + M)
    lap = np.zeros_like(delta)
    for k, a in enumerate(second_derivative_weights(order), start=1):
        lo, hi = slice(g + 1 - k, g + M - k), slice(g + 1 + k, g + M + k)
        lap += a * (bc[lo, inner, inner] + bc[hi, inner, inner] +
                    bc[inner, lo, inner] + bc[inner, hi, inner] +
                    bc[inner, inner, lo] + bc[inner, inner, hi])
    return delta - lap / d ** 2


def dirichlet_potential(delta, phi_bc_pad, d=1.0, order=2):
    """Potential on the padded grid [-g, M+g]^3 (g = N_ghost): the interior from the
    zero-BC solve of delta' (App. C), the shell from Phi_BCs (Sec. 3.4.2, padding of Phi
    with Phi_BCs)."""
    M = delta.shape[0] + 1
    phi = phi_bc_pad.copy()
    if order == 2:
        phi[2:M + 1, 2:M + 1, 2:M + 1] = solve_zero_bc(bc_source_correction(delta, phi_bc_pad, d), d)
        return phi
    g = order // 2
    src = bc_source_correction_wide(delta, phi_bc_pad, order, d)
    phi[g + 1:g + M, g + 1:g + M, g + 1:g + M] = solve_zero_bc(src, d, order)
    return phi


def dense_dirichlet_laplacian(n, d=1.0):
    """Brute-force matrix of the FDA-2 Laplacian on n^3 unknowns with zero Dirichlet
    values outside (for the direct-solve pin on tiny meshes)."""
    N = n ** 3
    A = np.zeros((N, N))
    idx = np.arange(N).reshape(n, n, n)
    for i in range(n):
        for j in range(n):
            for k in range(n):
                r = idx[i, j, k]
                A[r, r] = -6.0 / d ** 2
                for di, dj, dk in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0),
                                   (0, 0, 1), (0, 0, -1)):
                    a, b, c = i + di, j + dj, k + dk
                    if 0 <= a < n and 0 <= b < n and 0 <= c < n:
                        A[r, idx[a, b, c]] = 1.0 / d ** 2
    return A


def dense_odd_laplacian(n, order, d=1.0):
    """Brute-force matrix of the order-n Laplacian on n^3 unknowns (nodes 1..n per axis)
    with the unknown continued antisymmetrically past each face: node 0 and node n + 1 are
    zero and, with period 2 (n + 1), node -k is minus node k (the continuation on which the
    DST-I basis diagonalises the wide stencil), for the direct-solve pin at orders 4, 6."""
    from .lpt import second_derivative_weights
    a = second_derivative_weights(order)
    per = 2 * (n + 1)

    def image(i):
        """(unknown index 0..n-1 or -1, sign) of node i under the odd continuation."""
        r = i % per
        if r == 0 or r == n + 1:
            return -1, 0.0
        return (r - 1, 1.0) if r <= n else (per - r - 1, -1.0)

    D2 = np.zeros((n, n))
    for i in range(1, n + 1):
        D2[i - 1, i - 1] -= 2.0 * a.sum()
        for k, ak in enumerate(a, start=1):
            for j in (i - k, i + k):
                col, sgn = image(j)
                if col >= 0:
                    D2[i - 1, col] += sgn * ak
    I = np.eye(n)
    return (np.kron(np.kron(D2, I), I) + np.kron(np.kron(I, D2), I) +
            np.kron(np.kron(I, I), D2)) / d ** 2
