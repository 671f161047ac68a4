"""Monolithic periodic tCOLA on the GPU (scola_tcola_forward, Sec. 2.2, App. A eq.
kick-tcola) against the oracle's evolve_periodic, and the sCOLA-versus-tCOLA accuracy
measures of Sec. 4.2 (P(k) ratio and cross-correlation R(k) of the final densities).

Bars: one KDK step from the LPT state (identical inputs on both sides) within 1e-5 cell in
FP32 and 1e-10 in FP64; several steps end to end within 1e-4 cell (FP32, equal cell indices
away from faces) and 1e-8 (FP64); the total residual momentum stays zero to round-off (CiC
deposit and interpolation are transposes and the central gradient is antisymmetric, so the
mesh force sums to zero, and the LPT momentum sums to zero on the periodic lattice)."""
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


def oracle_tcola(w, L, n, want_momenta=False, record=None):
    from oracle.cosmology import Cosmology, cola_schedule
    from oracle.run import setup_full_box
    from oracle.scola import evolve_periodic
    c = Cosmology()
    _, _, psi1, psi2 = setup_full_box(w, L, c, 0.05)
    steps, final = cola_schedule(c, 0.05, 1.0, n, want_final_kick=want_momenta)
    return evolve_periodic(psi1, psi2, steps, final, record=record)


def cell_errors(pos_gpu, u_ora, Np, cell):
    u_gpu = pos_gpu.double().cpu().numpy() / cell
    d = np.abs((u_gpu - np.mod(u_ora, Np) + Np / 2) % Np - Np / 2).max(axis=0)
    uo = np.mod(u_ora, Np)
    frac = uo - np.floor(uo)
    far = (np.minimum(frac, 1 - frac) > 1e-4).all(axis=0)
    same = (np.floor(np.mod(u_gpu, Np)) == np.floor(uo)).all(axis=0)
    return float(d.max()), int((far & ~same).sum())


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_tcola_matches_oracle(torch, precision):
    import paper_2003_04925_amd as S
    Np, L = 32, 128.0
    cell = L / Np
    w = synthetic.white_noise(Np, 21)
    for n, tol in ((1, 1e-5 if precision == "fp32" else 1e-10),
                   (4, 1e-4 if precision == "fp32" else 1e-8)):
        sim = S.Simulation(L, Np, S.uniform_tiling(Np, 2, 8), n, precision=precision,
                           want_momenta=True)
        out = sim.tcola_forward(torch.from_numpy(w).cuda(), record=True)
        torch.cuda.synchronize()
        rec = []
        ora = oracle_tcola(w, L, n, want_momenta=True, record=rec)
        dmax, mism = cell_errors(out["pos"], ora["u"], Np, cell)
        mom = out["mom"].double().cpu().numpy() / cell
        merr = float(np.abs(mom - ora["p"]).max() / np.abs(ora["p"]).max())
        # total momentum: the LPT part sums to zero, so the sum is the residual momentum's
        tot = np.abs(mom.reshape(3, -1).sum(axis=1)).max() / np.abs(mom).sum(axis=(1, 2, 3)).max()
        say(f"tcola {precision} {n} steps: max {dmax:.3e} cell, index mismatches {mism}, "
            f"momenta {merr:.3e}, total momentum / sum |p| {tot:.3e}")
        assert dmax < tol and mism == 0
        assert merr < (1e-4 if precision == "fp32" else 1e-8)
        assert tot < (1e-6 if precision == "fp32" else 1e-12)
        # the recorded density contrast and potential of every force evaluation
        assert out["record_delta"].shape[0] == len(rec) == n + 1
        for k in (0, n):
            dd = out["record_delta"][k].double().cpu().numpy()
            pp = out["record_phi"][k].double().cpu().numpy()
            ed = np.abs(dd - rec[k]["delta"]).max() / np.abs(rec[k]["delta"]).max()
            ep = np.abs(pp - rec[k]["phi"]).max() / np.abs(rec[k]["phi"]).max()
            say(f"  force {k}: delta {ed:.3e}, phi {ep:.3e} (relative)")
            assert ed < (1e-3 if precision == "fp32" else 1e-9)
            assert ep < (1e-4 if precision == "fp32" else 1e-9)


def test_scola_versus_tcola_accuracy_study(torch):
    """Sec. 4.2 measures on the c2 shape (128^3 particles, 4^3 tiles of 32^3 + 16 buffer):
    P_sCOLA / P_tCOLA and R(k) of the final densities, both runs on the GPU (FP32).  The
    paper finds ~1-3 % for tiles and buffers of this physical size (62.5 Mpc/h buffers);
    the measured figures are printed and held to 5 % (P) and 0.97 (R) up to half the
    Nyquist wave number."""
    import paper_2003_04925_amd as S
    from oracle.run import power_spectrum
    wl = synthetic.WORKLOADS["c2"]
    sim = S.Simulation(wl.L, wl.Np, S.uniform_tiling(wl.Np, wl.tiles_per_side, wl.buffer),
                       wl.n_steps, precision="fp32")
    w = torch.from_numpy(synthetic.white_noise(wl.Np, 42)).cuda()
    ds = sim.forward(w)["density"].double().cpu().numpy()
    dt = sim.tcola_forward(w)["density"].double().cpu().numpy()
    kny = np.pi * wl.Np / wl.L
    ps = power_spectrum(ds, wl.L, n_bins=40, k_max=kny, other=dt)
    pt = power_spectrum(dt, wl.L, n_bins=40, k_max=kny)
    ok = ps["count"] > 0
    kc = np.sqrt(ps["k_edges"][1:] * ps["k_edges"][:-1])
    ratio = ps["P"][ok] / pt["P"][ok]
    R = ps["R"][ok]
    for k, r, c in zip(kc[ok], ratio, R):
        say(f"  k {k:.4f} h/Mpc: P_sCOLA/P_tCOLA {r:.4f}, R {c:.4f}")
    half = kc[ok] <= kny / 2
    say("  max |P ratio - 1| (k <= k_Ny/2)", float(np.abs(ratio[half] - 1).max()),
        "min R", float(R[half].min()))
    assert np.abs(ratio[half] - 1).max() < 0.05
    assert R[half].min() > 0.97
