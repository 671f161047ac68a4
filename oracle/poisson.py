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
  * C.2, order-2 eigenvalue formula and eq. (Poisson_sine_space):
    Phi^{lmn} = delta^{lmn} / (lambda_l + lambda_m + lambda_n).

Reading: the eigenvalue uses the true PM node spacing d (one lattice cell), so that
lambda_l = -(4/d^2) sin^2(pi l / (2 (N_g + 1))); the paper's own parenthetical value of
L_x is a slip (see the design notes).  Inverse sums in eqs. (IDST_*) run over l, m, n.
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


def solve_zero_bc(src, d=1.0):
    """Delta phi = src with phi = 0 on the nodes just outside the array (App. C.2)."""
    lx, ly, lz = (fda2_eigenvalues(n, d) for n in src.shape)
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


def dirichlet_potential(delta, phi_bc_pad, d=1.0):
    """Potential on the padded grid [-1, M+1]^3: the interior from the zero-BC solve of
    delta' (App. C), the shell from Phi_BCs (Sec. 3.4.2, padding of Phi with Phi_BCs)."""
    M = delta.shape[0] + 1
    phi = phi_bc_pad.copy()
    phi[2:M + 1, 2:M + 1, 2:M + 1] = solve_zero_bc(bc_source_correction(delta, phi_bc_pad, d), d)
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
