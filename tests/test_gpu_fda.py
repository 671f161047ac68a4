"""Finite differences of order 4 and 6 (Sec. 3; App. C.1-C.2) on the GPU against the oracle.

The same tolerances as the order-2 parity tests: FP64 set-up fields to 1e-11 of their
maximum, the potential to 1e-10 (FP64) / 3e-5 (FP32) of its maximum, one step from an
identical state within 1e-10 / 1e-5 cell, end to end within 1e-8 / 1e-4 cell.  Order 2
is covered by test_gpu_parity; here every test runs at orders 4 and 6.
"""
import sys

import numpy as np
import pytest

import synthetic

pytestmark = pytest.mark.gpu

ORDERS = (4, 6)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def make_sim(order, precision="fp32", Np=32, L=128.0, tps=2, buffer=8, n_steps=4,
             want_momenta=False, checkpoint_every=0):
    import paper_2003_04925_amd as S
    return S.Simulation(L, Np, S.uniform_tiling(Np, tps, buffer), n_steps, precision=precision,
                        want_momenta=want_momenta, fda_order=order,
                        checkpoint_every=checkpoint_every)


def box(arr, off, M):
    from paper_2003_04925_amd import particle_order
    return arr[:, off + particle_order(M)].reshape(3, M, M, M)


def oracle_tile(sim, t):
    from oracle.tiling import Tile
    lo, n, b = sim.tiles[t]
    return Tile(tuple(lo), n, b)


def padded(arr, ho, M, g):
    Mp = M + 1 + 2 * g
    return arr[ho:ho + Mp ** 3].reshape((Mp,) * 3)


def seeded_state(sim, torch, seed, spread=2.0, pscale=1.0, wide_every=0):
    P = sim.layout.n_particles
    xr = synthetic.uniform((3, P), -spread, spread, seed)
    if wide_every:
        # every wide_every-th brick of 256 particles spreads over +-8 cells: its force
        # stencils exceed the LDS window and are gathered from global memory
        wide = synthetic.uniform((3, P), -8.0, 8.0, seed + 7)
        for b in range(0, P // 256, wide_every):
            xr[:, 256 * b:256 * (b + 1)] = wide[:, 256 * b:256 * (b + 1)]
    pr = synthetic.normal((3, P), pscale, seed + 1)
    sim.view("x_res").copy_(torch.from_numpy(xr).to(sim.real))
    sim.view("p_res").copy_(torch.from_numpy(pr).to(sim.real))
    torch.cuda.synchronize()
    return (sim.view("x_res").double().cpu().numpy(), sim.view("p_res").double().cpu().numpy())


def box_positions(sim, psi1, psi2, xr, t, D1, D2):
    from oracle.scola import lattice_positions
    po, M, _, _ = sim.box_slices()[t]
    q = lattice_positions(M).reshape(3, -1)
    b = lambda a: box(a, po, M).reshape(3, -1)
    return q - D1 * b(psi1) + D2 * b(psi2) + b(xr)


@pytest.mark.parametrize("order", ORDERS)
def test_setup_matches_oracle(torch, order):
    from oracle.cosmology import Cosmology
    from oracle.run import setup_full_box
    from oracle.tiling import boundary_potential0, extract_box_field
    say("setup parity, order", order)
    sim = make_sim(order, "fp64")
    w = synthetic.white_noise(32, 11)
    sim.setup(torch.from_numpy(w).cuda())
    torch.cuda.synchronize()
    phi1, phi2, psi1, psi2 = setup_full_box(w, 128.0, Cosmology(), 0.05, order)
    np.testing.assert_allclose(sim.view("phi1").cpu().numpy(), phi1, atol=1e-12 * np.abs(phi1).max())
    np.testing.assert_allclose(sim.view("phi2").cpu().numpy(), phi2, atol=1e-11 * np.abs(phi2).max())
    g1 = sim.view("psi1").cpu().numpy()
    g2 = sim.view("psi2").cpu().numpy()
    bc = sim.view("bc0").cpu().numpy()
    g = order // 2
    for t, (po, M, go, ho) in enumerate(sim.box_slices()):
        tile = oracle_tile(sim, t)
        np.testing.assert_allclose(box(g1, po, M), extract_box_field(psi1, tile),
                                   atol=1e-12 * np.abs(psi1).max())
        np.testing.assert_allclose(box(g2, po, M), extract_box_field(psi2, tile),
                                   atol=1e-11 * np.abs(psi2).max())
        np.testing.assert_allclose(padded(bc, ho, M, g), boundary_potential0(phi1, tile, g),
                                   atol=1e-12 * np.abs(phi1).max())


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("order", ORDERS)
@pytest.mark.parametrize("Np,tps,buffer", [(32, 2, 8), (16, 1, 16)])
def test_poisson_matches_oracle(torch, order, precision, Np, tps, buffer):
    """Boxes of M = 32 (two per side) and M = 48 (one box larger than the lattice)."""
    from oracle.poisson import dirichlet_potential
    say("poisson parity, order", order, precision, "M", Np // tps + 2 * buffer)
    sim = make_sim(order, precision, Np=Np, L=4.0 * Np, tps=tps, buffer=buffer)
    sim.setup(torch.from_numpy(synthetic.white_noise(Np, 13)).cuda())
    seeded_state(sim, torch, 6, spread=2.0)
    sim.op_deposit(3.0, -4.0)
    torch.cuda.synchronize()
    rho = sim.view("rho").cpu().numpy().copy()
    D1 = 3.0
    sim.op_poisson(D1)
    torch.cuda.synchronize()
    phi = sim.view("phi").double().cpu().numpy()
    bc = sim.view("bc0").cpu().numpy()
    g = order // 2
    tol = 1e-10 if precision == "fp64" else 3e-5
    for t, (po, M, go, ho) in enumerate(sim.box_slices()):
        delta = rho[go:go + (M - 1) ** 3].reshape((M - 1,) * 3) / 2.0 ** sim.layout.fixed_bits - 1.0
        want = dirichlet_potential(delta, D1 * padded(bc, ho, M, g), order=order)
        got = padded(phi, ho, M, g)
        err = np.abs(got - want).max() / np.abs(want).max()
        say("  tile", t, "rel err", err)
        assert err < tol


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("order", ORDERS)
def test_one_step_from_identical_state(torch, order, precision):
    """Fused force + kick + drift + deposit; every third brick is spread over +-8 cells so
    that both the LDS-window and the global-memory gathers run."""
    from oracle.scola import box_deposit, box_gradient, box_interpolate
    say("one-step parity, order", order, precision)
    Np = 32
    sim = make_sim(order, precision, Np=Np)
    sim.setup(torch.from_numpy(synthetic.white_noise(Np, 14)).cuda())
    xr, pr = seeded_state(sim, torch, 7, spread=2.0, pscale=0.5, wide_every=3)
    D1, D2, D1n, D2n = 3.0, -4.0, 3.5, -5.3
    beta, alpha = -0.05, 1.7
    sim.op_deposit(D1, D2)
    sim.op_poisson(D1)
    torch.cuda.synchronize()
    phi = sim.view("phi").double().cpu().numpy()
    g1 = sim.view("psi1").double().cpu().numpy()
    g2 = sim.view("psi2").double().cpu().numpy()
    sim.op_step(beta, alpha, D1, D2, D1n, D2n, deposit=True)
    torch.cuda.synchronize()
    xr2 = sim.view("x_res").double().cpu().numpy()
    pr2 = sim.view("p_res").double().cpu().numpy()
    rho = sim.view("rho").cpu().numpy()
    xtol = 1e-10 if precision == "fp64" else 1e-5
    dtol = 1e-9 if precision == "fp64" else 1e-5     # fixed-point weights: 2^-40 / 2^-21
    gpad = order // 2
    for t, (po, M, go, ho) in enumerate(sim.box_slices()):
        b = lambda a: box(a, po, M).reshape(3, -1)
        u = box_positions(sim, g1, g2, xr, t, D1, D2)
        g = box_interpolate(box_gradient(padded(phi, ho, M, gpad), order), u)
        p_want = b(pr) + beta * (g - D1 * b(g1) + (D2 - D1 ** 2) * b(g2))
        x_want = b(xr) + alpha * p_want
        xerr = np.abs(b(xr2) - x_want).max()
        perr = np.abs(b(pr2) - p_want).max()
        say("  tile", t, "max |dx| cells", xerr, "max |dp|", perr)
        assert xerr < xtol
        assert perr < xtol / alpha * 2
        u2 = box_positions(sim, g1, g2, xr2, t, D1n, D2n)
        want, _ = box_deposit(u2, M)
        got = rho[go:go + (M - 1) ** 3].reshape((M - 1,) * 3) / 2.0 ** sim.layout.fixed_bits - 1.0
        np.testing.assert_allclose(got, want, atol=dtol)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-8), ("fp32", 1e-4)])
@pytest.mark.parametrize("order", ORDERS)
def test_end_to_end_matches_oracle(torch, order, precision, tol):
    from oracle.run import run_scola
    from oracle.tiling import uniform_tiling as otiling
    Np, L, n = 32, 128.0, 4
    w = synthetic.white_noise(Np, 19)
    ora = run_scola(w, L, otiling(Np, 2, 8), n_steps=n, fda_order=order)
    sim = make_sim(order, precision, Np=Np, L=L, n_steps=n)
    out = sim.forward(torch.from_numpy(w).cuda())
    torch.cuda.synchronize()
    cell = L / Np
    d = (out["pos"].double().cpu().numpy() - ora["pos"]) / cell
    d = np.abs((d + Np / 2) % Np - Np / 2).max()
    dd = np.abs(out["density"].double().cpu().numpy() - ora["density"]).max()
    say("end to end, order", order, precision, "max |dx| cells", d, "max |d delta|", dd)
    assert d < tol
    assert dd < (1e-8 if precision == "fp64" else 1e-3)
    # the order matters: the order-2 run differs by far more than the tolerance
    ref2 = run_scola(w, L, otiling(Np, 2, 8), n_steps=n)
    d2 = (ref2["pos"] - ora["pos"]) / cell
    assert np.abs((d2 + Np / 2) % Np - Np / 2).max() > 100 * tol


@pytest.mark.parametrize("order", ORDERS)
def test_tcola_matches_oracle(torch, order):
    from oracle.cosmology import Cosmology, cola_schedule
    from oracle.run import setup_full_box
    from oracle.scola import evolve_periodic
    Np, L, n = 32, 128.0, 4
    c = Cosmology()
    w = synthetic.white_noise(Np, 23)
    _, _, psi1, psi2 = setup_full_box(w, L, c, 0.05, order)
    steps, _ = cola_schedule(c, 0.05, 1.0, n)
    ora = evolve_periodic(psi1, psi2, steps, fda_order=order)
    sim = make_sim(order, "fp64", Np=Np, L=L, n_steps=n)
    out = sim.tcola_forward(torch.from_numpy(w).cuda())
    torch.cuda.synchronize()
    u = ora["u"].reshape(3, -1)
    cell = L / Np
    got = out["pos"].double().cpu().numpy().reshape(3, -1) / cell
    d = got - np.mod(u, Np)
    d = np.abs((d + Np / 2) % Np - Np / 2).max()
    say("tCOLA, order", order, "max |dx| cells", d)
    assert d < 1e-8


@pytest.mark.parametrize("order", ORDERS)
def test_reverse_mode_and_persistent_step_refuse_wide_orders(torch, order):
    import paper_2003_04925_amd as S
    sim = make_sim(order, "fp32", checkpoint_every=2)
    dens = sim.forward(torch.from_numpy(synthetic.white_noise(32, 5)).cuda())["density"]
    with pytest.raises(S.ScolaError) as e:
        sim.backward(dens)
    assert e.value.status == -5 and "order 2" in str(e.value)
    with pytest.raises(S.ScolaError) as e:
        sim.set_persistent(True)
    assert e.value.status == -5
