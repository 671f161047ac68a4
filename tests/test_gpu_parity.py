"""GPU parity of the HIP path against the FP64 oracle, operator by operator and end to end.

Every GPU call goes through the C ABI (libscola.so via the ctypes binding).  Inputs are
seeded and synthetic; the oracle gets the same inputs.  Tolerances:
  * integer work (fixed-point mass, conservation): exact;
  * FP64 path: 1e-9 relative (the fixed-point deposit quantises weights to 2^-40);
  * FP32 path: potential 3e-6 of its maximum (the matrix-core DST carries operands of 22
    significant bits and accumulates in FP32; measured 3e-7 to 9e-7 for M = 16 ... 128);
    one step from an identical state moves positions by less than 1e-5 cell away from the
    oracle (the bar is 1e-4 cell).
"""
import sys

import numpy as np
import pytest

import synthetic

pytestmark = pytest.mark.gpu



def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def make_sim(torch, precision="fp32", Np=32, L=128.0, tps=2, buffer=8, n_steps=4,
             schedule="batched", want_momenta=False):
    import paper_2003_04925_amd as S
    tiles = S.uniform_tiling(Np, tps, buffer)
    return S.Simulation(L, Np, tiles, n_steps, precision=precision, schedule=schedule,
                        want_momenta=want_momenta)


def oracle_setup(Np, L, seed):
    from oracle.cosmology import Cosmology
    from oracle.run import setup_full_box
    c = Cosmology()
    return setup_full_box(synthetic.white_noise(Np, seed), L, c, 0.05)


def oracle_tile(sim, t):
    from oracle.tiling import Tile
    lo, n, b = sim.tiles[t]
    return Tile(tuple(lo), n, b)


def dep_tol(precision):
    """Deposit tolerance per node: FP64 plans form CiC weights in FP64 and quantise them to
    2^-40; FP32 plans form them in FP32 (rounding up to 2^-24 per weight) and quantise to
    2^-21 (error up to 2^-22 = 2.4e-7 per weight); a node collects up to ~40 weights."""
    return 1e-9 if precision == "fp64" else 1e-5


def box(arr, off, M):
    """Box particles of a workspace array, in lattice order (3, M, M, M)."""
    from paper_2003_04925_amd import particle_order
    return arr[:, off + particle_order(M)].reshape(3, M, M, M)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_setup_matches_oracle(torch, precision):
    from oracle.tiling import boundary_potential0, extract_box_field
    say("setup parity", precision)
    sim = make_sim(torch, precision)
    w = synthetic.white_noise(32, 11)
    sim.setup(torch.from_numpy(w).cuda())
    torch.cuda.synchronize()
    phi1, phi2, psi1, psi2 = oracle_setup(32, 128.0, 11)
    np.testing.assert_allclose(sim.view("phi1").cpu().numpy(), phi1, atol=1e-12 * np.abs(phi1).max())
    np.testing.assert_allclose(sim.view("phi2").cpu().numpy(), phi2, atol=1e-11 * np.abs(phi2).max())
    g1 = sim.view("psi1").cpu().numpy()
    g2 = sim.view("psi2").cpu().numpy()
    bc = sim.view("bc0").cpu().numpy()
    for t, (po, M, go, ho) in enumerate(sim.box_slices()):
        tile = oracle_tile(sim, t)
        for g, ref, rel in ((g1, psi1, 1e-12), (g2, psi2, 1e-11)):
            want = extract_box_field(ref, tile)
            got = box(g, po, M)
            if precision == "fp64":
                np.testing.assert_allclose(got, want, atol=rel * np.abs(ref).max())
            else:
                # Psi is differenced in FP64 and stored rounded to FP32: within one unit in
                # the last place of the oracle's value rounded the same way
                w32 = want.astype(np.float32)
                assert (np.abs(got.astype(np.float64) - w32) <=
                        np.spacing(np.abs(w32)).astype(np.float64)).all()
        np.testing.assert_allclose(bc[ho:ho + (M + 3) ** 3].reshape((M + 3,) * 3),
                                   boundary_potential0(phi1, tile), atol=1e-12 * np.abs(phi1).max())
    assert float(sim.view("x_res").abs().max()) == 0.0


def seeded_state(sim, torch, seed, spread=2.0, pscale=1.0):
    P = sim.layout.n_particles
    xr = synthetic.uniform((3, P), -spread, spread, seed)
    pr = synthetic.normal((3, P), pscale, seed + 1)
    sim.view("x_res").copy_(torch.from_numpy(xr).to(sim.real))
    sim.view("p_res").copy_(torch.from_numpy(pr).to(sim.real))
    torch.cuda.synchronize()
    # the oracle sees exactly the values the GPU holds
    return (sim.view("x_res").double().cpu().numpy(), sim.view("p_res").double().cpu().numpy())


def box_positions(sim, psi1, psi2, xr, t, D1, D2):
    """Oracle positions of box t in lattice order (3, M^3), from workspace arrays."""
    from oracle.scola import lattice_positions
    po, M, _, _ = sim.box_slices()[t]
    q = lattice_positions(M).reshape(3, -1)
    b = lambda a: box(a, po, M).reshape(3, -1)
    return q - D1 * b(psi1) + D2 * b(psi2) + b(xr)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_deposit_matches_oracle_and_conserves_mass(torch, precision):
    from oracle.scola import box_deposit
    say("deposit parity", precision)
    sim = make_sim(torch, precision)
    sim.setup(torch.from_numpy(synthetic.white_noise(32, 12)).cuda())
    xr, _ = seeded_state(sim, torch, 5, spread=3.0)
    D1, D2 = 4.0, -7.0
    sim.op_deposit(D1, D2)
    torch.cuda.synchronize()
    rho = sim.view("rho").cpu().numpy()
    dropped = sim.view("dropped").cpu().numpy()
    g1 = sim.view("psi1").cpu().numpy()
    g2 = sim.view("psi2").cpu().numpy()
    for t, (po, M, go, ho) in enumerate(sim.box_slices()):
        r = rho[go:go + (M - 1) ** 3]
        # every particle carries exactly 2^fixed_bits units, deposited or dropped (integer
        # identity)
        bits = sim.layout.fixed_bits
        assert int(r.sum()) + int(dropped[t]) == M ** 3 * (1 << bits)
        u = box_positions(sim, g1, g2, xr, t, D1, D2)
        want, _ = box_deposit(u, M)
        got = r.reshape((M - 1,) * 3).astype(np.float64) / 2.0 ** bits - 1.0
        np.testing.assert_allclose(got, want, atol=dep_tol(precision))


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_poisson_matches_oracle(torch, precision):
    from oracle.poisson import dirichlet_potential
    say("poisson parity", precision)
    sim = make_sim(torch, precision)
    sim.setup(torch.from_numpy(synthetic.white_noise(32, 13)).cuda())
    xr, _ = seeded_state(sim, torch, 6, spread=2.0)
    sim.op_deposit(3.0, -4.0)
    torch.cuda.synchronize()
    rho = sim.view("rho").cpu().numpy().copy()
    D1 = 3.0
    sim.op_poisson(D1)
    torch.cuda.synchronize()
    phi = sim.view("phi").double().cpu().numpy()
    bc = sim.view("bc0").cpu().numpy()
    assert int(np.abs(sim.view("rho").cpu().numpy()).max()) == 0     # left zeroed
    tol = 1e-10 if precision == "fp64" else 3e-6
    for t, (po, M, go, ho) in enumerate(sim.box_slices()):
        delta = rho[go:go + (M - 1) ** 3].reshape((M - 1,) * 3) / 2.0 ** sim.layout.fixed_bits - 1.0
        want = dirichlet_potential(delta, D1 * bc[ho:ho + (M + 3) ** 3].reshape((M + 3,) * 3))
        got = phi[ho:ho + (M + 3) ** 3].reshape((M + 3,) * 3)
        err = np.abs(got - want).max() / np.abs(want).max()
        say("  tile", t, "rel err", err)
        assert err < tol


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("Np,buffer", [(16, 0), (32, 8), (32, 24), (32, 32), (32, 40), (32, 48)])
def test_poisson_every_fft_radix(torch, precision, Np, buffer):
    """One box of M = Np + 2 buffer = 16, 48, 80, 96, 112, 128 nodes per side: the DST-I runs
    an FFT of length 2M = 32 R with an R-point register DFT, R = 1, 3, 5, 6, 7, 8 (R = 2, 4
    are covered above).  Boxes larger than the lattice hold periodic images, as the oracle's
    box extraction does."""
    from oracle.poisson import dirichlet_potential
    sim = make_sim(torch, precision, Np=Np, L=4.0 * Np, tps=1, buffer=buffer)
    M = Np + 2 * buffer
    say("poisson M", M, precision)
    sim.setup(torch.from_numpy(synthetic.white_noise(Np, 17)).cuda())
    seeded_state(sim, torch, 8, spread=2.0)
    sim.op_deposit(2.0, -2.0)
    torch.cuda.synchronize()
    rho = sim.view("rho").cpu().numpy().copy()
    D1 = 2.0
    sim.op_poisson(D1)
    torch.cuda.synchronize()
    phi = sim.view("phi").double().cpu().numpy()
    bc = sim.view("bc0").cpu().numpy()
    delta = rho[:(M - 1) ** 3].reshape((M - 1,) * 3) / 2.0 ** sim.layout.fixed_bits - 1.0
    want = dirichlet_potential(delta, D1 * bc[:(M + 3) ** 3].reshape((M + 3,) * 3))
    got = phi[:(M + 3) ** 3].reshape((M + 3,) * 3)
    err = np.abs(got - want).max() / np.abs(want).max()
    say("  rel err", err)
    assert err < (1e-10 if precision == "fp64" else 3e-6)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("M_buffer", [(2, 8, 32), (1, 24, 32), (1, 32, 64)])
def test_one_step_from_identical_state(torch, precision, M_buffer):
    """Boxes of 32^3, 80^3 and 128^3 (the largest admitted size)."""
    from oracle.scola import box_deposit, box_gradient, box_interpolate
    tps, buf, Np = M_buffer
    say("one-step parity", precision, "Np", Np, "tiles/side", tps, "buffer", buf)
    sim = make_sim(torch, precision, Np=Np, tps=tps, buffer=buf)
    sim.setup(torch.from_numpy(synthetic.white_noise(Np, 14)).cuda())
    xr, pr = seeded_state(sim, torch, 7, spread=2.0, pscale=0.5)
    D1, D2, D1n, D2n = 3.0, -4.0, 3.5, -5.3
    beta, alpha = -0.05, 1.7
    sim.op_deposit(D1, D2)
    sim.op_poisson(D1)
    torch.cuda.synchronize()
    phi = sim.view("phi").double().cpu().numpy()
    g1 = sim.view("psi1").cpu().numpy()
    g2 = sim.view("psi2").cpu().numpy()
    sim.op_step(beta, alpha, D1, D2, D1n, D2n, deposit=True)
    torch.cuda.synchronize()
    xr2 = sim.view("x_res").double().cpu().numpy()
    pr2 = sim.view("p_res").double().cpu().numpy()
    rho = sim.view("rho").cpu().numpy()
    xtol = 1e-10 if precision == "fp64" else 1e-5
    for t, (po, M, go, ho) in enumerate(sim.box_slices()):
        b = lambda a: box(a, po, M).reshape(3, -1)
        u = box_positions(sim, g1, g2, xr, t, D1, D2)
        g = box_interpolate(box_gradient(phi[ho:ho + (M + 3) ** 3].reshape((M + 3,) * 3)), u)
        p_want = b(pr) + beta * (g - D1 * b(g1) + (D2 - D1 ** 2) * b(g2))
        x_want = b(xr) + alpha * p_want
        perr = np.abs(b(pr2) - p_want).max()
        xerr = np.abs(b(xr2) - x_want).max()
        say("  tile", t, "max |dx| cells", xerr, "max |dp|", perr)
        assert xerr < xtol
        assert perr < xtol / alpha * 2
        u2 = box_positions(sim, g1, g2, xr2, t, D1n, D2n)
        want, _ = box_deposit(u2, M)
        got = rho[go:go + (M - 1) ** 3].reshape((M - 1,) * 3) / 2.0 ** sim.layout.fixed_bits - 1.0
        np.testing.assert_allclose(got, want, atol=dep_tol(precision))


def window_forms(u, M, clamped=False):
    """Which LDS window form each 4 x 8 x 8 brick of a box takes for its force stencils, from
    positions u (3, M^3) in lattice order: 0 = fixed 16^3 window, 1 = window sized to the
    block's stencil extent (at most 4096 nodes), 2 = global memory; -1 = no particle inside.
    The forward step sizes its window to the whole extent; the reverse pass (`clamped`) to
    the part of it inside the padded grid [-1, M + 1]."""
    M4, M8 = M // 4, M // 8
    j0 = np.floor(u).reshape(3, M4, 4, M8, 8, M8, 8).transpose(0, 1, 3, 5, 2, 4, 6)
    j0 = j0.reshape(3, -1, 256)
    uu = u.reshape(3, M4, 4, M8, 8, M8, 8).transpose(0, 1, 3, 5, 2, 4, 6).reshape(3, -1, 256)
    inside = ((uu >= -1) & (uu < M + 1)).all(axis=0)
    forms = []
    for b in range(j0.shape[1]):
        if not inside[b].any():
            forms.append(-1)
            continue
        lo = j0[:, b, inside[b]].min(axis=1)
        hi = j0[:, b, inside[b]].max(axis=1)
        if (hi - lo + 4 <= 16).all():
            forms.append(0)
            continue
        if clamped:
            vol = np.prod(np.minimum(hi + 2, M + 1) - np.maximum(lo - 1, -1) + 1)
        else:
            vol = np.prod(hi - lo + 4)
        forms.append(1 if vol <= 4096 else 2)
    return np.array(forms)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_one_step_every_window_form(torch, precision):
    """Bricks given small, elongated and wide residual displacements take the fixed, the
    sized and the global-memory window forms; every form must match the oracle."""
    from oracle.scola import box_deposit, box_gradient, box_interpolate
    say("one-step parity over the window forms", precision)
    Np = 32
    sim = make_sim(torch, precision, Np=Np, tps=2, buffer=8)
    sim.setup(torch.from_numpy(synthetic.white_noise(Np, 21)).cuda())
    P = sim.layout.n_particles
    xr = synthetic.uniform((3, P), -0.5, 0.5, 31)
    wide = synthetic.uniform((3, P), -8.0, 8.0, 32)
    for po, M, _, _ in sim.box_slices():
        for b in range(M ** 3 // 256):
            sl = slice(po + 256 * b, po + 256 * (b + 1))
            if b % 3 == 1:
                xr[0, sl] = 0.9 * wide[0, sl]          # elongated along x: sized window
            elif b % 3 == 2:
                xr[:, sl] = wide[:, sl]                # wide: global memory
    sim.view("x_res").copy_(torch.from_numpy(xr).to(sim.real))
    sim.view("p_res").copy_(torch.from_numpy(synthetic.normal((3, P), 0.5, 33)).to(sim.real))
    torch.cuda.synchronize()
    xr = sim.view("x_res").double().cpu().numpy()
    pr = sim.view("p_res").double().cpu().numpy()
    D1, D2, D1n, D2n = 3.0, -4.0, 3.5, -5.3
    beta, alpha = -0.05, 1.7
    sim.op_deposit(D1, D2)
    sim.op_poisson(D1)
    torch.cuda.synchronize()
    phi = sim.view("phi").double().cpu().numpy()
    g1 = sim.view("psi1").cpu().numpy()
    g2 = sim.view("psi2").cpu().numpy()
    seen = set()
    for t in range(len(sim.tiles)):
        M = sim.box_slices()[t][1]
        seen |= set(window_forms(box_positions(sim, g1, g2, xr, t, D1, D2), M).tolist())
    say("  window forms present", sorted(seen))
    assert {0, 1, 2} <= seen
    sim.op_step(beta, alpha, D1, D2, D1n, D2n, deposit=True)
    torch.cuda.synchronize()
    xr2 = sim.view("x_res").double().cpu().numpy()
    pr2 = sim.view("p_res").double().cpu().numpy()
    rho = sim.view("rho").cpu().numpy()
    xtol = 1e-10 if precision == "fp64" else 1e-5
    for t, (po, M, go, ho) in enumerate(sim.box_slices()):
        b = lambda a: box(a, po, M).reshape(3, -1)
        u = box_positions(sim, g1, g2, xr, t, D1, D2)
        g = box_interpolate(box_gradient(phi[ho:ho + (M + 3) ** 3].reshape((M + 3,) * 3)), u)
        p_want = b(pr) + beta * (g - D1 * b(g1) + (D2 - D1 ** 2) * b(g2))
        x_want = b(xr) + alpha * p_want
        xerr = np.abs(b(xr2) - x_want).max()
        say("  tile", t, "max |dx| cells", xerr)
        assert xerr < xtol
        u2 = box_positions(sim, g1, g2, xr2, t, D1n, D2n)
        want, _ = box_deposit(u2, M)
        got = rho[go:go + (M - 1) ** 3].reshape((M - 1,) * 3) / 2.0 ** sim.layout.fixed_bits - 1.0
        np.testing.assert_allclose(got, want, atol=dep_tol(precision))


def decode_cells(h):
    """Packed block cell extents (rows of uint32 words, as int64) -> lo, hi (n, 3): words 0
    and 1 hold 2^14 + min j0 for x, y, z in 16-bit halves, words 1 (high half) and 2 hold
    2^14 - max j0."""
    off = 1 << 14
    lo = np.stack([(h[:, 0] & 0xffff) - off, (h[:, 0] >> 16) - off, (h[:, 1] & 0xffff) - off], 1)
    hi = np.stack([off - (h[:, 1] >> 16), off - (h[:, 2] & 0xffff), off - (h[:, 2] >> 16)], 1)
    return lo, hi


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_cell_hints_exact_and_step_independent_of_them(torch, precision):
    """Each deposit keeps the cell extent of every block of 256 particles for the force pass
    of the next step, which checks it against its particles and uses it in place of its own
    reduction.  The kept extents equal min / max of floor(u) over the block's particles
    inside [-1, M+1)^3, exactly; and valid, widened (other window origins and forms),
    narrowed (fails the check), zeroed and random hints give bitwise the same step."""
    from paper_2003_04925_amd import particle_order
    say("cell hints", precision)
    sim = make_sim(torch, precision)
    sim.setup(torch.from_numpy(synthetic.white_noise(32, 23)).cuda())
    xr, _ = seeded_state(sim, torch, 24, spread=1.0, pscale=0.5)
    x0, p0 = sim.view("x_res").clone(), sim.view("p_res").clone()
    D1, D2, D1n, D2n = 3.0, -4.0, 3.5, -5.3
    beta, alpha = -0.05, 1.7
    g1 = sim.view("psi1").cpu().numpy()
    g2 = sim.view("psi2").cpu().numpy()
    cells = sim.view("cells")
    rng = np.random.default_rng(25)
    names = ("x_res", "p_res", "rho", "dropped", "cells")
    ref = None
    for kind in ("valid", "widened", "narrowed", "zero", "random"):
        sim.view("x_res").copy_(x0)
        sim.view("p_res").copy_(p0)
        sim.op_deposit(D1, D2)
        sim.op_poisson(D1)
        torch.cuda.synchronize()
        h = cells.cpu().numpy().astype(np.int64) & 0xffffffff
        if kind == "valid":
            lo, hi = decode_cells(h)
            n_checked = 0
            for t, (po, M, go, ho) in enumerate(sim.box_slices()):
                u = box_positions(sim, g1, g2, xr, t, D1, D2)
                order = particle_order(M)
                j0 = np.empty((3, M ** 3), dtype=np.int64)
                j0[:, order] = np.floor(u).astype(np.int64)
                inside = np.empty(M ** 3, dtype=bool)
                inside[order] = ((u >= -1) & (u < M + 1)).all(axis=0)
                j0 = j0.reshape(3, -1, 256)
                inside = inside.reshape(-1, 256)
                b0, nb = po // 256, M ** 3 // 256
                for b in range(nb):
                    if inside[b].any():
                        np.testing.assert_array_equal(lo[b0 + b], j0[:, b, inside[b]].min(axis=1))
                        np.testing.assert_array_equal(hi[b0 + b], j0[:, b, inside[b]].max(axis=1))
                        n_checked += 1
                    else:
                        assert (h[b0 + b, :3] == 0xffffffff).all()
            say("  extents of", n_checked, "blocks exact")
        elif kind == "widened":
            h[:, :3] -= 0x00010001    # lo - 1 and hi + 1 along every axis
        elif kind == "narrowed":
            h[:, :3] += 0x00010001    # lo + 1 and hi - 1: some particle falls outside
        elif kind == "zero":
            h[:] = 0
        else:
            h = rng.integers(0, 1 << 32, size=h.shape, dtype=np.int64)
        h &= 0xffffffff
        cells.copy_(torch.from_numpy(h.astype(np.uint32).view(np.int32)))
        sim.op_step(beta, alpha, D1, D2, D1n, D2n, deposit=True)
        torch.cuda.synchronize()
        out = [sim.view(n).cpu().clone() for n in names]
        if ref is None:
            ref = out
        for n, a, b in zip(names, ref, out):
            assert torch.equal(a, b), (kind, n)
        say("  hints", kind, "bitwise equal")


def test_fp64_run_matches_oracle_end_to_end(torch):
    from oracle.run import run_scola
    from oracle.tiling import uniform_tiling as otiling
    say("end-to-end fp64 per-tile vs oracle")
    Np, L, n = 32, 128.0, 4
    sim = make_sim(torch, "fp64", Np=Np, L=L, n_steps=n, schedule="per_tile", want_momenta=True)
    w = synthetic.white_noise(Np, 15)
    out = sim.forward(torch.from_numpy(w).cuda())
    torch.cuda.synchronize()
    ora = run_scola(w, L, otiling(Np, 2, 8), n_steps=n, want_momenta=True)
    cell = L / Np
    d = (out["pos"].cpu().numpy() - ora["pos"]) / cell
    d = (d + Np / 2) % Np - Np / 2
    say("  max |dx| cells", np.abs(d).max())
    assert np.abs(d).max() < 1e-8
    np.testing.assert_allclose(out["mom"].cpu().numpy(), ora["mom"],
                               atol=1e-8 * np.abs(ora["mom"]).max())
    np.testing.assert_allclose(out["density"].cpu().numpy(), ora["density"], atol=1e-9)


def test_fp32_batched_run_close_to_oracle(torch):
    from oracle.run import run_scola
    from oracle.tiling import uniform_tiling as otiling
    say("end-to-end fp32 batched vs oracle")
    Np, L, n = 32, 128.0, 4
    sim = make_sim(torch, "fp32", Np=Np, L=L, n_steps=n)
    w = synthetic.white_noise(Np, 15)
    out = sim.forward(torch.from_numpy(w).cuda())
    torch.cuda.synchronize()
    ora = run_scola(w, L, otiling(Np, 2, 8), n_steps=n)
    cell = L / Np
    d = (out["pos"].double().cpu().numpy() - ora["pos"]) / cell
    d = (d + Np / 2) % Np - Np / 2
    say("  max |dx| cells", np.abs(d).max(), "p99.9", np.quantile(np.abs(d), 0.999))
    assert np.abs(d).max() < 1e-4
    u_o = ora["pos"] / cell
    u_g = out["pos"].double().cpu().numpy() / cell
    frac = u_o - np.floor(u_o)
    far = (np.minimum(frac, 1 - frac) > 1e-4).all(axis=0)
    assert ((np.floor(u_g) == np.floor(u_o)).all(axis=0) | ~far).all()
    assert np.abs(out["density"].double().cpu().numpy() - ora["density"]).max() < 1e-3


def test_determinism_and_tile_recompute(torch):
    say("determinism / tile subset")
    Np = 32
    sim = make_sim(torch, "fp32", Np=Np, n_steps=3)
    w = torch.from_numpy(synthetic.white_noise(Np, 16)).cuda()
    a = sim.forward(w)["pos"].clone()
    b = sim.forward(w)["pos"].clone()
    assert torch.equal(a, b)
    sub = sim.forward(w, tile_subset=[5])["pos"]
    lo, n, _ = sim.tiles[5]
    sl = (slice(None),) + tuple(slice(c, c + n) for c in lo)
    assert torch.equal(sub[sl], a[sl])
    per = make_sim(torch, "fp32", Np=Np, n_steps=3, schedule="per_tile")
    c = per.forward(w)["pos"]
    assert torch.equal(c, a)


def test_tile_subset_refusals_and_order(torch):
    """An empty subset, tile indices out of range and a repeated tile are refused with
    SCOLA_EINVAL; a valid subset gives bitwise the same boxes in any order, also right after
    a refused call."""
    import paper_2003_04925_amd as S
    say("tile subset refusals and order")
    Np = 32
    sim = make_sim(torch, "fp32", Np=Np, n_steps=3)
    w = torch.from_numpy(synthetic.white_noise(Np, 16)).cuda()
    a = sim.forward(w, tile_subset=[2, 5])["pos"].clone()
    nt = len(sim.tiles)
    for bad in ([], [-1], [nt], [5, 5]):
        with pytest.raises(S.ScolaError) as e:
            sim.forward(w, tile_subset=bad)
        assert e.value.status == -1, bad
    b = sim.forward(w, tile_subset=[5, 2])["pos"]
    for t in (2, 5):
        lo, n, _ = sim.tiles[t]
        sl = (slice(None),) + tuple(slice(c, c + n) for c in lo)
        assert torch.equal(a[sl], b[sl]), t
