"""GPU reverse mode (scola_backward, through the C ABI) against the oracle's reverse-mode
reference and against finite differences of the GPU forward.

Loss: L = sum (delta_out - t)^2 with a seeded target t, so dL/ddelta = 2 (delta_out - t).
Tolerances: the FP64 plan matches the FP64 reference to 1e-7 of the largest gradient entry
(measured ~1e-11: the forward differs from the oracle by ~1e-12 and the adjoint is linear
in it).  The FP32 plan is held to a relative L2 error below 5e-5 and a cosine similarity
above 1 - 1e-9 (measured 2e-6 and 1 - 1e-12): its trajectories differ from the FP64 ones by
~1e-6 cell, which can put a particle on the other side of a cell face, where the CiC weight
derivative jumps (the map is only piecewise differentiable); with 2 steps the FP32 error is
~1e-5 plus a bounded share for each particle that ends in another output cell than the
oracle's.  Finite differences of the GPU FP64 forward use eps = 1e-3 because the loss carries
fixed-point quantisation noise of ~1e-10 (2^-40 per CiC weight over all nodes).
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


def gpu_gradient(torch, precision, Np, L, tps, buffer, n_steps, ckpt, seed=3):
    import paper_2003_04925_amd as S
    sim = S.Simulation(L, Np, S.uniform_tiling(Np, tps, buffer), n_steps, precision=precision,
                       checkpoint_every=ckpt)
    w = torch.from_numpy(synthetic.white_noise(Np, seed)).cuda()
    t = torch.from_numpy(synthetic.loss_target(Np, 43)).cuda().to(sim.real)
    dens = sim.forward(w)["density"]
    loss = float(((dens.double() - t.double()) ** 2).sum())
    grad = sim.backward(2.0 * (dens - t))
    torch.cuda.synchronize()
    return sim, loss, grad.cpu().numpy(), dens


def oracle_gradient(Np, L, tps, buffer, n_steps, seed=3):
    from oracle.adjoint import loss_and_gradient
    from oracle.tiling import uniform_tiling
    return loss_and_gradient(synthetic.white_noise(Np, seed), L, uniform_tiling(Np, tps, buffer),
                             synthetic.loss_target(Np, 43), n_steps=n_steps)


@pytest.mark.parametrize("ckpt", [1, 2, 3])
def test_fp64_gradient_matches_oracle_reference(torch, ckpt):
    Np, L, tps, buf, n = 16, 150.0, 2, 4, 3
    say("fp64 adjoint vs oracle, checkpoint every", ckpt)
    _, loss, g, _ = gpu_gradient(torch, "fp64", Np, L, tps, buf, n, ckpt)
    oloss, og, _ = oracle_gradient(Np, L, tps, buf, n)
    assert loss == pytest.approx(oloss, rel=1e-9)
    err = np.abs(g - og).max() / np.abs(og).max()
    say("  max rel err", err)
    assert err < 1e-7


def test_fp64_gradient_with_wide_windows_and_coarse_output(torch):
    """A small, strongly clustered volume (L = 16 Mpc/h, sigma_8 = 2) sends most blocks of
    the late steps to the sized and global-memory window forms of the reverse pass, and the
    loss is taken on an output grid coarser than the lattice (N_out = 8 for N_p = 16); the
    gradient must still match the oracle's reverse-mode reference."""
    import paper_2003_04925_amd as S
    from oracle.adjoint import _box, _boundary_potential0, _roll_diff, evolve_box, potentials
    from oracle.adjoint import loss_and_gradient
    from oracle.cosmology import Cosmology, cola_schedule
    from oracle.tiling import uniform_tiling
    from test_gpu_parity import window_forms
    Np, L, tps, buf, n, N_out, s8 = 16, 16.0, 2, 4, 3, 8, 2.0
    say("fp64 adjoint, wide windows, N_out", N_out)
    cosmo = Cosmology(sigma8=s8)
    wn = synthetic.white_noise(Np, 3)
    otiles = uniform_tiling(Np, tps, buf)
    # premise: the final positions put blocks in every window form
    w64 = torch.tensor(wn)
    phi1, phi2 = potentials(w64, L, cosmo, 0.05)
    psi1 = torch.stack([_roll_diff(phi1, a) for a in range(3)])
    psi2 = torch.stack([_roll_diff(phi2, a) for a in range(3)])
    steps, _ = cola_schedule(cosmo, 0.05, 1.0, n)
    forms = set()
    for t in otiles:
        u = evolve_box(_box(psi1, t), _box(psi2, t), _boundary_potential0(phi1, t), steps)
        forms |= set(window_forms(u.detach().numpy().reshape(3, -1), t.M, clamped=True).tolist())
    say("  window forms at the final step", sorted(forms))
    assert {0, 1, 2} <= forms
    target = 0.5 * synthetic.normal((N_out,) * 3, 1.0, 43)
    sim = S.Simulation(L, Np, S.uniform_tiling(Np, tps, buf), n, precision="fp64",
                       N_out=N_out, cosmology=S.CosmologyParams(sigma8=s8), checkpoint_every=2)
    w = torch.from_numpy(wn).cuda()
    t = torch.from_numpy(target).cuda()
    dens = sim.forward(w)["density"]
    loss = float(((dens - t) ** 2).sum())
    g = sim.backward(2.0 * (dens - t)).cpu().numpy()
    torch.cuda.synchronize()
    oloss, og, odens = loss_and_gradient(wn, L, otiles, target, cosmo=cosmo, n_steps=n,
                                         N_out=N_out)
    derr = np.abs(dens.cpu().numpy() - odens).max()
    say("  output density max err", derr, "loss", loss, oloss)
    assert derr < 1e-9
    assert loss == pytest.approx(oloss, rel=1e-9)
    err = np.abs(g - og).max() / np.abs(og).max()
    say("  max rel err", err)
    assert err < 1e-7


def test_fp32_gradient_close_to_oracle_reference(torch):
    Np, L, tps, buf, n = 32, 200.0, 2, 8, 6
    say("fp32 adjoint vs oracle")
    _, loss, g, _ = gpu_gradient(torch, "fp32", Np, L, tps, buf, n, 4)
    oloss, og, _ = oracle_gradient(Np, L, tps, buf, n)
    cos = float((g * og).sum() / np.sqrt((g * g).sum() * (og * og).sum()))
    rel = float(np.sqrt(((g - og) ** 2).sum() / (og * og).sum()))
    say("  loss", loss, oloss, "cosine", cos, "rel L2", rel)
    assert loss == pytest.approx(oloss, rel=1e-4)
    # measured: relative L2 2.1e-6, cosine 1 - 1e-12 (six steps)
    assert cos > 1 - 1e-9 and rel < 5e-5
    # over two steps the FP32 trajectory stays within ~1e-5 cell of the FP64 one, and the
    # gradient agrees to ~1e-5 except through particles that end in a different output cell
    # than the oracle's (within ~1e-5 cell of a face): there the piecewise-linear CiC weight
    # has a kink and the one-sided derivatives differ.  Each such particle is allowed 2e-3
    # of relative L2 (one measured at ~6e-4).
    from oracle.run import run_scola
    from oracle.tiling import uniform_tiling
    sim2, loss2, g2, _ = gpu_gradient(torch, "fp32", Np, L, tps, buf, 2, 4)
    _, og2, _ = oracle_gradient(Np, L, tps, buf, 2)
    pos = sim2.forward(torch.from_numpy(synthetic.white_noise(Np, 3)).cuda())["pos"]
    cell = L / Np
    u_gpu = pos.double().cpu().numpy() / cell
    u_ora = run_scola(synthetic.white_noise(Np, 3), L, uniform_tiling(Np, tps, buf),
                      n_steps=2)["pos"] / cell
    flips = int((np.floor(u_gpu) != np.floor(u_ora)).any(axis=0).sum())
    rel2 = float(np.sqrt(((g2 - og2) ** 2).sum() / (og2 * og2).sum()))
    say("  two steps: rel L2", rel2, "particles in another output cell", flips)
    assert rel2 < 1e-4 + 2e-3 * flips


def test_fp64_gradient_matches_gpu_finite_differences(torch):
    import paper_2003_04925_amd as S
    Np, L, tps, buf, n = 16, 150.0, 2, 4, 3
    say("fp64 adjoint vs GPU finite differences")
    sim, loss, g, _ = gpu_gradient(torch, "fp64", Np, L, tps, buf, n, 2)
    w0 = synthetic.white_noise(Np, 3)
    t = torch.from_numpy(synthetic.loss_target(Np, 43)).cuda()
    fwd = S.Simulation(L, Np, S.uniform_tiling(Np, tps, buf), n, precision="fp64")

    def lossf(w):
        d = fwd.forward(torch.from_numpy(w).cuda())["density"]
        return float(((d - t) ** 2).sum())

    rng = np.random.default_rng(1)
    eps = 1e-3
    for _ in range(3):
        i = tuple(int(v) for v in rng.integers(0, Np, 3))
        wp, wm = w0.copy(), w0.copy()
        wp[i] += eps
        wm[i] -= eps
        fd = (lossf(wp) - lossf(wm)) / (2 * eps)
        say("  ", i, g[i], fd)
        assert g[i] == pytest.approx(fd, rel=2e-3, abs=1e-4 * np.abs(g).max())


def test_autograd_function_uses_library_backward(torch):
    import paper_2003_04925_amd as S
    Np, L = 16, 150.0
    say("autograd.Function")
    sim = S.Simulation(L, Np, S.uniform_tiling(Np, 2, 4), 3, precision="fp64",
                       checkpoint_every=2)
    w = torch.from_numpy(synthetic.white_noise(Np, 3)).cuda().requires_grad_(True)
    t = torch.from_numpy(synthetic.loss_target(Np, 43)).cuda()
    dens = S.DensityFunction.apply(sim, w)
    loss = ((dens - t) ** 2).sum()
    loss.backward()
    _, _, g, _ = gpu_gradient(torch, "fp64", Np, L, 2, 4, 3, 2)
    np.testing.assert_allclose(w.grad.cpu().numpy(), g, rtol=1e-12, atol=1e-12 * np.abs(g).max())


def test_autograd_refuses_a_graph_of_an_earlier_forward(torch):
    """Two forwards through one Simulation: the library holds the second trajectory, so the
    first output's backward must raise instead of returning the second one's gradient."""
    import paper_2003_04925_amd as S
    Np, L = 16, 150.0
    sim = S.Simulation(L, Np, S.uniform_tiling(Np, 2, 4), 3, precision="fp64",
                       checkpoint_every=2)
    w1 = torch.from_numpy(synthetic.white_noise(Np, 3)).cuda().requires_grad_(True)
    w2 = torch.from_numpy(synthetic.white_noise(Np, 4)).cuda().requires_grad_(True)
    d1 = S.DensityFunction.apply(sim, w1)
    d2 = S.DensityFunction.apply(sim, w2)
    with pytest.raises(RuntimeError, match="another forward"):
        (d1 ** 2).sum().backward()
    (d2 ** 2).sum().backward()
    # the latest forward still differentiates: d sum d^2 / dw from a fresh Simulation
    sim2 = S.Simulation(L, Np, S.uniform_tiling(Np, 2, 4), 3, precision="fp64",
                        checkpoint_every=2)
    d = sim2.forward(w2.detach())["density"]
    g2 = sim2.backward(2.0 * d).cpu().numpy()
    np.testing.assert_allclose(w2.grad.cpu().numpy(), g2, rtol=1e-12, atol=1e-12 * np.abs(g2).max())


@pytest.mark.parametrize("disc,nl", [("standard", 0.0), ("modified", -1.5)])
def test_time_factor_variants_match_oracle(torch, disc, nl):
    """The standard discretisation of App. B and a non-default n_LPT of the modified one,
    end to end (FP64 plan) against the oracle run with the same time factors."""
    import paper_2003_04925_amd as S
    from oracle.run import run_scola
    from oracle.tiling import uniform_tiling
    Np, L, n = 16, 150.0, 3
    say("time factors", disc, "n_lpt", nl)
    sim = S.Simulation(L, Np, S.uniform_tiling(Np, 2, 4), n, precision="fp64",
                       want_momenta=True, discretisation=disc, n_lpt=nl)
    w = synthetic.white_noise(Np, 6)
    out = sim.forward(torch.from_numpy(w).cuda())
    torch.cuda.synchronize()
    ora = run_scola(w, L, uniform_tiling(Np, 2, 4), n_steps=n, want_momenta=True,
                    discretisation=disc, n_lpt=nl if nl else -2.5)
    ref = run_scola(w, L, uniform_tiling(Np, 2, 4), n_steps=n, want_momenta=True)
    cell = L / Np
    d = (out["pos"].cpu().numpy() - ora["pos"]) / cell
    d = (d + Np / 2) % Np - Np / 2
    dref = (ora["pos"] - ref["pos"]) / cell
    dref = (dref + Np / 2) % Np - Np / 2
    say("  max |dx| cells", np.abs(d).max(), "differs from the default by", np.abs(dref).max())
    assert np.abs(d).max() < 1e-8 and np.abs(dref).max() > 1e-4
    np.testing.assert_allclose(out["mom"].cpu().numpy(), ora["mom"],
                               atol=1e-8 * np.abs(ora["mom"]).max())


def test_backward_requires_forward_state(torch):
    import paper_2003_04925_amd as S
    sim = S.Simulation(150.0, 16, S.uniform_tiling(16, 2, 4), 3, precision="fp32",
                       checkpoint_every=2)
    with pytest.raises(S.ScolaError) as e:
        sim.backward(torch.zeros((16,) * 3, device="cuda"))
    assert e.value.status == -4
    nock = S.Simulation(150.0, 16, S.uniform_tiling(16, 2, 4), 3, precision="fp32")
    nock.forward(torch.from_numpy(synthetic.white_noise(16, 3)).cuda())
    with pytest.raises(S.ScolaError):
        nock.backward(torch.zeros((16,) * 3, device="cuda"))
