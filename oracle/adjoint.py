"""Reverse-mode reference of the whole tiled-sCOLA chain: d loss / d white noise (FP64).

Test infrastructure only (see oracle/__init__.py).

This is an operation-for-operation twin of the NumPy oracle (oracle.lpt, oracle.tiling,
oracle.poisson, oracle.scola, oracle.run) written with torch float64 tensors on the CPU, so
that torch's automatic differentiation supplies the adjoint of every step; it is pinned
against the NumPy forward (identical loss to round-off) and against central finite
differences.  The loss is the sum of squared residuals of the output CiC density against a
target field (the paper has no loss; this is the differentiation workload of the build).

Piecewise-linear CiC weights are differentiated with the cell index held fixed (the index
is floor(u) of the same positions), which is the derivative almost everywhere.
"""
import numpy as np
import torch

from .cosmology import Cosmology, cola_schedule
from .lpt import fda2_laplacian_kernel, linear_power, mode_indices
from .poisson import fda2_eigenvalues, sine_matrix
from .tiling import box_indices

T64 = torch.float64


def _roll_diff(f, axis):
    return 0.5 * (torch.roll(f, -1, axis) - torch.roll(f, 1, axis))


def potentials(w, L, cosmo, a_i):
    """Steps A.1-A.2 (Sec. 3.1) on torch tensors: phi1, phi2."""
    N = w.shape[0]
    D1_1 = cosmo.growth(np.array([1.0]), a_i)[0][0]
    m = mode_indices(N)
    kf = 2.0 * np.pi / L
    kmag = kf * np.sqrt(m[:, None, None] ** 2 + m[None, :, None] ** 2 + m[None, None, :] ** 2)
    filt = np.sqrt(linear_power(kmag, cosmo) / D1_1 ** 2 * N ** 3 / L ** 3)
    K = fda2_laplacian_kernel(N)
    with np.errstate(divide="ignore", invalid="ignore"):
        g1 = np.where(K != 0, filt / K, 0.0)
        invK = np.where(K != 0, 1.0 / K, 0.0)
    g1 = torch.from_numpy(g1)
    invK = torch.from_numpy(invK)
    phi1 = torch.fft.ifftn(torch.fft.fftn(w) * g1).real
    d = [_roll_diff(phi1, a) for a in range(3)]
    dd = [[_roll_diff(d[j], i) for j in range(3)] for i in range(3)]
    src = torch.zeros_like(phi1)
    for i in range(3):
        for j in range(i):
            src = src + dd[i][i] * dd[j][j] - dd[i][j] ** 2
    phi2 = torch.fft.ifftn(torch.fft.fftn(src) * invK).real
    return phi1, phi2


def _box(field, tile):
    ix, iy, iz = (torch.from_numpy(a) for a in box_indices(tile, field.shape[-1]))
    return field[..., ix[:, None, None], iy[None, :, None], iz[None, None, :]]


def _boundary_potential0(phi1, tile):
    N = phi1.shape[0]
    M = tile.M
    j = np.arange(-1, M + 2)
    out = 0.0
    for dx in (0, 1):
        for dy in (0, 1):
            for dz in (0, 1):
                ix = torch.from_numpy(np.mod(tile.origin[0] + j - 1 + dx, N))
                iy = torch.from_numpy(np.mod(tile.origin[1] + j - 1 + dy, N))
                iz = torch.from_numpy(np.mod(tile.origin[2] + j - 1 + dz, N))
                out = out + phi1[ix[:, None, None], iy[None, :, None], iz[None, None, :]]
    out = 0.125 * out
    mask = torch.ones((M + 3,) * 3, dtype=T64)
    mask[2:M + 1, 2:M + 1, 2:M + 1] = 0.0
    return out * mask


def _corners(u):
    j0 = torch.floor(u.detach()).to(torch.int64)
    f = u - j0.to(T64)
    for ox in (0, 1):
        for oy in (0, 1):
            for oz in (0, 1):
                off = torch.tensor([ox, oy, oz])[:, None]
                w = ((f[0] if ox else 1 - f[0]) * (f[1] if oy else 1 - f[1]) *
                     (f[2] if oz else 1 - f[2]))
                yield j0 + off, w


def _deposit(u, M):
    rho = torch.zeros((M - 1) ** 3, dtype=T64)
    for idx, w in _corners(u):
        ok = torch.all((idx >= 1) & (idx <= M - 1), dim=0)
        lin = ((idx[0] - 1) * (M - 1) + (idx[1] - 1)) * (M - 1) + (idx[2] - 1)
        rho = rho.index_add(0, lin[ok], w[ok])
    return rho.reshape((M - 1,) * 3) - 1.0


def _dst3(f, S):
    return torch.einsum("ijk,il,jm,kn->lmn", f, S, S, S)


def _potential(delta, bc, M):
    n = M - 1
    S = torch.from_numpy(sine_matrix(n))
    lam = torch.from_numpy(fda2_eigenvalues(n))
    src = delta.clone()
    src = src - torch.nn.functional.pad(bc[1:2, 2:M + 1, 2:M + 1], (0, 0, 0, 0, 0, n - 1))
    src = src - torch.nn.functional.pad(bc[M + 1:M + 2, 2:M + 1, 2:M + 1], (0, 0, 0, 0, n - 1, 0))
    src = src - torch.nn.functional.pad(bc[2:M + 1, 1:2, 2:M + 1], (0, 0, 0, n - 1, 0, 0))
    src = src - torch.nn.functional.pad(bc[2:M + 1, M + 1:M + 2, 2:M + 1], (0, 0, n - 1, 0, 0, 0))
    src = src - torch.nn.functional.pad(bc[2:M + 1, 2:M + 1, 1:2], (0, n - 1, 0, 0, 0, 0))
    src = src - torch.nn.functional.pad(bc[2:M + 1, 2:M + 1, M + 1:M + 2], (n - 1, 0, 0, 0, 0, 0))
    F = _dst3(src, S) / (lam[:, None, None] + lam[None, :, None] + lam[None, None, :])
    inner = _dst3(F, S) * 8.0 / M ** 3
    return bc + torch.nn.functional.pad(inner, (2, 2, 2, 2, 2, 2))


def _force(u, M, bc):
    phi = _potential(_deposit(u, M), bc, M)
    c = slice(1, M + 2)
    g = torch.stack([
        0.5 * (phi[2:M + 3, c, c] - phi[0:M + 1, c, c]),
        0.5 * (phi[c, 2:M + 3, c] - phi[c, 0:M + 1, c]),
        0.5 * (phi[c, c, 2:M + 3] - phi[c, c, 0:M + 1]),
    ])
    out = torch.zeros_like(u)
    for idx, w in _corners(u):
        ok = torch.all((idx >= 0) & (idx <= M), dim=0).to(T64)
        cl = idx.clamp(0, M)
        out = out + (w * ok) * g[:, cl[0], cl[1], cl[2]]
    return out


def evolve_box(s1, s2, bc0, steps):
    """Positions (3, M^3) of one box after the KDK operator (App. B), torch."""
    M = s1.shape[1]
    i = torch.arange(M, dtype=T64) + 0.5
    q = torch.stack(torch.meshgrid(i, i, i, indexing="ij")).reshape(3, -1)
    s1 = s1.reshape(3, -1)
    s2 = s2.reshape(3, -1)
    x = torch.zeros_like(q)
    p = torch.zeros_like(q)
    u = q - steps[0]["D1"] * s1 + steps[0]["D2"] * s2
    g = _force(u, M, steps[0]["D1"] * bc0)
    for k, st in enumerate(steps):
        p = p + st["beta"] * (g - st["D1"] * s1 + (st["D2"] - st["D1"] ** 2) * s2)
        x = x + st["alpha"] * p
        u = q - st["D1_next"] * s1 + st["D2_next"] * s2 + x
        if k < len(steps) - 1:
            g = _force(u, M, st["D1_next"] * bc0)
    return u


def output_density(positions, Np, N_out):
    u = positions * (N_out / Np)
    rho = torch.zeros(N_out ** 3, dtype=T64)
    for idx, w in _corners(u):
        idx = torch.remainder(idx, N_out)
        lin = (idx[0] * N_out + idx[1]) * N_out + idx[2]
        rho = rho.index_add(0, lin, w)
    return rho.reshape((N_out,) * 3) * (N_out / Np) ** 3 - 1.0


def density_loss(w, L, tiles, target, cosmo=None, a_i=0.05, a_f=1.0, n_steps=4, N_out=None):
    """L = sum (delta_out - target)^2 of the tiled-sCOLA run, as a torch scalar."""
    cosmo = cosmo or Cosmology()
    Np = w.shape[0]
    N_out = N_out or Np
    phi1, phi2 = potentials(w, L, cosmo, a_i)
    psi1 = torch.stack([_roll_diff(phi1, a) for a in range(3)])
    psi2 = torch.stack([_roll_diff(phi2, a) for a in range(3)])
    steps, _ = cola_schedule(cosmo, a_i, a_f, n_steps)
    parts = []
    for tile in tiles:
        u = evolve_box(_box(psi1, tile), _box(psi2, tile), _boundary_potential0(phi1, tile),
                       steps)
        M = tile.M
        c = torch.zeros(M, dtype=torch.bool)
        c[tile.buffer:tile.buffer + tile.core_n] = True
        core = (c[:, None, None] & c[None, :, None] & c[None, None, :]).reshape(-1)
        parts.append(u[:, core] + torch.tensor(tile.origin, dtype=T64)[:, None])
    dens = output_density(torch.cat(parts, dim=1), Np, N_out)
    return ((dens - torch.as_tensor(target)) ** 2).sum(), dens


def loss_and_gradient(white_noise, L, tiles, target, **kw):
    """(loss, d loss / d white noise, output density) by reverse mode."""
    w = torch.tensor(np.asarray(white_noise, dtype=np.float64), requires_grad=True)
    loss, dens = density_loss(w, L, tiles, target, **kw)
    loss.backward()
    return float(loss.detach()), w.grad.numpy().copy(), dens.detach().numpy()
