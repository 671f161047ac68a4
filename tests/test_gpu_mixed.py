"""Uneven batches: boxes of three sizes (mixed cores and buffers) in one plan, each size
class with its own launches, against the FP64 oracle on the same tiling.

The tiling of the 64^3 lattice: core 32 + buffer 8 (48^3 box) at the origin, core 32 +
buffer 16 (64^3 box) next to it along x, and the remaining six 32^3 blocks split into
cores of 16 + buffer 8 (32^3 boxes): 50 tiles, every lattice site in exactly one core.
Tolerances as in test_gpu_parity: FP64 positions within 1e-8 cell of the oracle, FP32
within 1e-3 cell after the run.
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


def mixed_tiles():
    tiles = [((0, 0, 0), 32, 8), ((32, 0, 0), 32, 16)]
    for bx, by, bz in ((0, 32, 0), (32, 32, 0), (0, 0, 32), (32, 0, 32), (0, 32, 32),
                       (32, 32, 32)):
        for dx in (0, 16):
            for dy in (0, 16):
                for dz in (0, 16):
                    tiles.append(((bx + dx, by + dy, bz + dz), 16, 8))
    return tiles


def test_mixed_tiling_covers_lattice_once():
    Np = 64
    cover = np.zeros((Np,) * 3, dtype=np.int32)
    for (x, y, z), n, _ in mixed_tiles():
        cover[x:x + n, y:y + n, z:z + n] += 1
    assert (cover == 1).all()


@pytest.fixture(scope="module")
def oracle_run():
    from oracle.run import run_scola
    from oracle.tiling import Tile
    Np, L, n = 64, 256.0, 3
    w = synthetic.white_noise(Np, 31)
    tiles = [Tile(lo, c, b) for lo, c, b in mixed_tiles()]
    return w, run_scola(w, L, tiles, n_steps=n)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-8), ("fp32", 1e-4)])
def test_mixed_batch_matches_oracle(torch, oracle_run, precision, tol):
    import paper_2003_04925_amd as S
    w, ora = oracle_run
    Np, L, n = 64, 256.0, 3
    sim = S.Simulation(L, Np, mixed_tiles(), n, precision=precision, schedule="batched")
    sched = sim.schedule()
    say("mixed batch", precision, "size classes", sorted(sched))
    assert sorted(sched) == [32, 48, 64]
    out = sim.forward(torch.from_numpy(w).cuda())
    torch.cuda.synchronize()
    cell = L / Np
    d = (out["pos"].double().cpu().numpy() - ora["pos"]) / cell
    d = (d + Np / 2) % Np - Np / 2
    dd = np.abs(out["density"].double().cpu().numpy() - ora["density"]).max()
    say("  max |dx| cells", np.abs(d).max(), "p99.9", np.quantile(np.abs(d), 0.999),
        "max |d delta|", dd)
    assert np.abs(d).max() < tol
    u_o = ora["pos"] / cell
    u_g = out["pos"].double().cpu().numpy() / cell
    frac = u_o - np.floor(u_o)
    far = (np.minimum(frac, 1 - frac) > 1e-4).all(axis=0)
    assert ((np.floor(u_g) == np.floor(u_o)).all(axis=0) | ~far).all()
    assert dd < (1e-8 if precision == "fp64" else 1e-3)


def test_mixed_batch_tuned_and_replayed_is_bitwise_stable(torch, oracle_run):
    import paper_2003_04925_amd as S
    w, _ = oracle_run
    Np, L, n = 64, 256.0, 3
    ref = S.Simulation(L, Np, mixed_tiles(), n, precision="fp32").forward(
        torch.from_numpy(w).cuda())
    sim = S.Simulation(L, Np, mixed_tiles(), n, precision="fp32")
    sim.setup(torch.from_numpy(w).cuda())
    say("tuned", sim.tune(reps=2))
    pos = torch.empty_like(ref["pos"])
    dens = torch.empty_like(ref["density"])
    for _ in range(3):                    # eager, recorded + replayed, replayed
        sim.evolve()
        sim.output(pos=pos, density=dens)
        torch.cuda.synchronize()
        assert torch.equal(pos, ref["pos"]) and torch.equal(dens, ref["density"])
    # per-tile schedule (one launch per box) gives bitwise the same result
    per = S.Simulation(L, Np, mixed_tiles(), n, precision="fp32", schedule="per_tile").forward(
        torch.from_numpy(w).cuda())
    assert torch.equal(per["pos"], ref["pos"]) and torch.equal(per["density"], ref["density"])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_per_tile_final_scale_factor_matches_oracle(torch, precision):
    """Sec. 5.1 (light cones): tiles evolved to different final scale factors, each with the
    run's number of steps from a_i to its own a_f; batched launches group the tiles by box
    size and final time.  Against the oracle's per-tile schedules; the per-tile launch
    schedule gives bitwise the same result; the reverse mode refuses mixed final times."""
    import paper_2003_04925_amd as S
    from oracle.run import run_scola
    from oracle.tiling import uniform_tiling as otiling
    Np, L, n = 32, 128.0, 4
    a_f = [1.0, 0.5, 0.7, 0.0, 0.3, 0.9, 1.0, 0.6]        # 0: the run's a_f (1.0)
    tiles = [t + (af,) for t, af in zip(S.uniform_tiling(Np, 2, 8), a_f)]
    w = synthetic.white_noise(Np, 17)
    sim = S.Simulation(L, Np, tiles, n, precision=precision)
    say("per-tile a_f", precision, "classes", len(sim.schedule()), sorted(sim.schedule()))
    out = sim.forward(torch.from_numpy(w).cuda())
    torch.cuda.synchronize()
    ora = run_scola(w, L, otiling(Np, 2, 8), n_steps=n, tile_a_f=a_f)
    cell = L / Np
    d = (out["pos"].double().cpu().numpy() - ora["pos"]) / cell
    d = np.abs((d + Np / 2) % Np - Np / 2).max()
    dd = np.abs(out["density"].double().cpu().numpy() - ora["density"]).max()
    say("  max |dx| cells", d, "max |d delta|", dd)
    assert d < (1e-8 if precision == "fp64" else 1e-4)
    assert dd < (1e-8 if precision == "fp64" else 1e-3)
    # tiles at earlier times moved less than the same tiles evolved to a = 1
    ref = run_scola(w, L, otiling(Np, 2, 8), n_steps=n)
    assert np.abs(ora["pos"] - ref["pos"]).max() > 1e-3
    per = S.Simulation(L, Np, tiles, n, precision=precision, schedule="per_tile").forward(
        torch.from_numpy(w).cuda())
    assert torch.equal(per["pos"], out["pos"]) and torch.equal(per["density"], out["density"])
    bw = S.Simulation(L, Np, tiles, n, precision=precision, checkpoint_every=2)
    dens = bw.forward(torch.from_numpy(w).cuda())["density"]
    with pytest.raises(S.ScolaError) as e:
        bw.backward(dens)
    assert e.value.status == -5
