"""GPU edge cases of the particle kernels, through the C ABI.

Blocks whose particles all lie outside their box: the block-wide LDS window is empty (no
thread contributes a node range) and must be treated as empty, not formed from the
reduction's sentinels.  Such a block deposits nothing (every particle's unit of mass is
counted as dropped, exactly) and its particles feel no mesh force (every interpolation
corner lies outside [0, M]^3), so the kick reduces to its LPT terms.
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


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_blocks_entirely_outside_their_box(torch, precision):
    import paper_2003_04925_amd as S
    Np, L = 32, 128.0
    tiles = S.uniform_tiling(Np, 2, 8)
    sim = S.Simulation(L, Np, tiles, 4, precision=precision)
    say("all-outside blocks", precision)
    sim.setup(torch.from_numpy(synthetic.white_noise(Np, 5)).cuda())
    po, M, _, _ = sim.box_slices()[0]
    n0 = M ** 3
    x = sim.view("x_res")
    x[:, po:po + n0] = 10.0 * M        # every particle of box 0 far outside its box
    row = sim.step_table()[2]
    beta, alpha, D1, D2, D1n, D2n = row[1], row[2], row[3], row[4], row[5], row[6]
    sim.op_deposit(D1, D2)
    torch.cuda.synchronize()
    bits = sim.layout.fixed_bits
    dropped = sim.view("dropped").cpu().numpy()
    assert int(dropped[0]) == n0 * (1 << bits)            # exact: all of box 0's mass
    assert all(0 <= int(d) < n0 * (1 << bits) for d in dropped[1:len(tiles)])
    assert int(dropped[len(tiles)]) == 0                   # no mass alarm
    sim.op_poisson(D1)
    p_before = sim.view("p_res").clone()
    sim.op_step(beta, alpha, D1, D2, D1n, D2n, True)
    torch.cuda.synchronize()
    p = sim.view("p_res")[:, po:po + n0].double().cpu().numpy()
    s1 = sim.view("psi1")[:, po:po + n0].double().cpu().numpy()
    s2 = sim.view("psi2")[:, po:po + n0].double().cpu().numpy()
    p0 = p_before[:, po:po + n0].double().cpu().numpy()
    expect = p0 + beta * (-D1 * s1 + (D2 - D1 * D1) * s2)
    tol = 1e-12 if precision == "fp64" else 1e-5
    err = np.abs(p - expect).max() / max(np.abs(expect).max(), 1e-30)
    say("  zero-force kick error", err)
    assert np.isfinite(sim.view("p_res").double().cpu().numpy()).all()
    assert err < tol


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_launch_schedule_does_not_change_results(torch, precision):
    """Occupancy variants and block numberings change only the launch; the fixed-point
    deposit makes every schedule bitwise identical."""
    import paper_2003_04925_amd as S
    Np, L = 32, 128.0
    w = torch.from_numpy(synthetic.white_noise(Np, 9)).cuda()
    outs = []
    for occ, rp, rm in ((6, 1, 1), (8, 0, 1), (6, 0, 0), (8, 1, 0)):
        sim = S.Simulation(L, Np, S.uniform_tiling(Np, 2, 8), 4, precision=precision)
        sim.set_schedule({M: {"waves_per_simd": occ, "xcd_remap_particles": rp,
                              "xcd_remap_mesh": rm} for M in sim.schedule()})
        say("schedule", precision, sim.schedule())
        r = sim.forward(w)
        outs.append((r["pos"].cpu().numpy(), r["density"].cpu().numpy()))
    for pos, dens in outs[1:]:
        assert np.array_equal(pos, outs[0][0])
        assert np.array_equal(dens, outs[0][1])


def test_tuner_picks_a_valid_schedule_and_keeps_the_state(torch):
    import paper_2003_04925_amd as S
    Np, L = 32, 128.0
    w = torch.from_numpy(synthetic.white_noise(Np, 9)).cuda()
    ref = S.Simulation(L, Np, S.uniform_tiling(Np, 2, 8), 4, precision="fp32").forward(w)
    sim = S.Simulation(L, Np, S.uniform_tiling(Np, 2, 8), 4, precision="fp32")
    with pytest.raises(S.ScolaError):
        sim.tune()                                   # needs the set-up first
    sim.setup(w)
    sched = sim.tune(reps=2)
    say("tuned schedule", sched)
    assert list(sched) == [32]
    assert sched[32]["waves_per_simd"] in (6, 8)
    assert sched[32]["xcd_remap_particles"] in (0, 1) and sched[32]["xcd_remap_mesh"] in (0, 1)
    sim.evolve()
    pos = torch.empty_like(ref["pos"])
    dens = torch.empty_like(ref["density"])
    sim.output(pos=pos, density=dens)
    assert torch.equal(pos, ref["pos"]) and torch.equal(dens, ref["density"])


def test_graph_replay_matches_eager_runs(torch):
    """The batched evolution replayed as a captured hipGraph gives bitwise the eager result on
    every replay, with other eager GPU work (torch reductions, another plan) in between."""
    import paper_2003_04925_amd as S
    Np, L = 32, 128.0
    w = torch.from_numpy(synthetic.white_noise(Np, 21)).cuda()
    tiles = S.uniform_tiling(Np, 2, 8)
    eager = S.Simulation(L, Np, tiles, 5, precision="fp32")
    eager.set_graph(False)
    ref = eager.forward(w)
    sim = S.Simulation(L, Np, tiles, 5, precision="fp32")
    sim.setup(w)
    pos = torch.empty_like(ref["pos"])
    dens = torch.empty_like(ref["density"])
    for r in range(4):             # call 1 eager, call 2 records the graph, calls 2-4 replay it
        sim.evolve()
        sim.output(pos=pos, density=dens)
        noise = float(torch.rand(1 << 20, device="cuda").sum())    # unrelated eager work
        eager.evolve()
        torch.cuda.synchronize()
        say("replay", r, "extra work", round(noise))
        assert torch.equal(pos, ref["pos"]) and torch.equal(dens, ref["density"])


def test_backward_after_a_graph_replayed_forward(torch):
    import paper_2003_04925_amd as S
    Np, L = 16, 150.0
    w = torch.from_numpy(synthetic.white_noise(Np, 3)).cuda()
    t = torch.from_numpy(synthetic.loss_target(Np, 43)).cuda()
    grads = []
    for n_forward in (1, 3):
        sim = S.Simulation(L, Np, S.uniform_tiling(Np, 2, 4), 3, precision="fp64",
                           checkpoint_every=2)
        for _ in range(n_forward):
            dens = sim.forward(w)["density"]
        grads.append(sim.backward(2.0 * (dens - t)).cpu().numpy())
    # the reverse pass sums with floating-point atomics, so two runs agree to round-off only
    err = np.abs(grads[0] - grads[1]).max() / np.abs(grads[0]).max()
    say("graph-forward gradient max rel diff", err)
    assert err < 1e-12


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_concurrent_box_groups_match_one(torch, precision):
    """Two or four shares of the boxes advanced on as many streams (eager and
    graph-replayed, with checkpoints) give bitwise the single-stream result; the reverse pass
    after them agrees to round-off."""
    import paper_2003_04925_amd as S
    Np, L = 32, 128.0
    w = torch.from_numpy(synthetic.white_noise(Np, 23)).cuda()
    t = torch.from_numpy(synthetic.loss_target(Np, 43)).cuda()
    outs, grads = [], []
    for groups in (1, 2, 4):
        sim = S.Simulation(L, Np, S.uniform_tiling(Np, 2, 8), 4, precision=precision,
                           checkpoint_every=2)
        sim.groups = groups
        assert sim.groups == groups
        for _ in range(3):                  # eager, recorded + replayed, replayed
            r = sim.forward(w)
        outs.append((r["pos"].cpu().numpy(), r["density"].cpu().numpy()))
        grads.append(sim.backward(2.0 * (r["density"] - t.to(sim.real))).cpu().numpy())
    for (pos, dens), g in zip(outs[1:], grads[1:]):
        assert np.array_equal(outs[0][0], pos) and np.array_equal(outs[0][1], dens)
        err = np.abs(grads[0] - g).max() / np.abs(grads[0]).max()
        say("groups", precision, "gradient rel diff", err)
        assert err < (1e-12 if precision == "fp64" else 1e-5)


def test_fp32_mass_alarm_flags_crowded_nodes(torch):
    """FP32 plans hold node masses in 32-bit integers (2^21 units per particle): the Poisson
    pass counts nodes that reach 2^31 units (1024 particles), within a factor 2 of wrapping,
    and every deposit addition checks the value it returns, so a node pushed past 2^32
    units (2048 particles; after the wrap it reads as 52 particles, below the first alarm)
    is counted too and scola_mass_alarm reports SCOLA_EOVERFLOW."""
    import paper_2003_04925_amd as S
    Np, L = 32, 128.0
    tiles = S.uniform_tiling(Np, 2, 8)
    sim = S.Simulation(L, Np, tiles, 4, precision="fp32")
    sim.setup(torch.from_numpy(synthetic.white_noise(Np, 5)).cuda())
    po, M, _, _ = sim.box_slices()[0]
    order = torch.from_numpy(S.particle_order(M)).cuda()
    i = torch.arange(M ** 3, device="cuda")
    site = torch.stack([i // (M * M), (i // M) % M, i % M]).double()     # lattice order
    x = sim.view("x_res")
    for crowd, near, wrapped in ((1000, 0, 0), (1500, 1, 0), (2100, 0, 1)):
        x.zero_()
        # the first `crowd` sites of box 0 moved exactly onto node (10, 10, 10): u = q + x_res
        # with D1 = D2 = 0, and 10 - (i + 1/2) is exact in FP32
        x[:, po + order[:crowd]] = (10.0 - (site[:, :crowd] + 0.5)).float()
        sim.op_deposit(0.0, 0.0)
        sim.op_poisson(1.0)
        torch.cuda.synchronize()
        counts = sim.view("dropped").cpu().tolist()
        nt = len(tiles)
        say("crowd", crowd, "near-limit", counts[nt], "deposits", counts[2 * nt + 1:])
        assert counts[nt] == near and counts[2 * nt + 1:] == [1] * nt
        # mass identity per box: found + dropped = M^3 units, short by 2^32 per wrap
        for t in range(nt):
            assert M ** 3 * (1 << 21) - counts[t] - counts[nt + 1 + t] == \
                (wrapped << 32 if t == 0 else 0)
        if wrapped:
            with pytest.raises(S.ScolaError) as e:
                sim.mass_alarm()
            assert e.value.status == -6 and "2048" in str(e.value)
        else:
            assert sim.mass_alarm() == (near, 0)


def _eighth_corner_remainder(f, precision):
    """Remainder unit - sum of the seven other rounded CiC weights of a particle at
    fractional offsets f, computed as the deposit rounds them (FP32 plans: FP32 products,
    2^21 units; FP64 plans: FP64 products, 2^40 units)."""
    if precision == "fp32":
        one = np.float32(1 << 21)
        a = [(np.float32(1) - np.float32(v), np.float32(v)) for v in f]
        s = sum(int(np.rint(np.float32(np.float32(np.float32(a[0][(c >> 2) & 1] * a[1][(c >> 1) & 1])
                                                   * a[2][c & 1]) * one))) for c in range(7))
        return (1 << 21) - s
    one = float(1 << 40)
    a = [(1.0 - v, v) for v in f]
    s = sum(int(np.rint(a[0][(c >> 2) & 1] * a[1][(c >> 1) & 1] * a[2][c & 1] * one))
            for c in range(7))
    return (1 << 40) - s


# residual displacements (cells) of a particle at lattice site (0, 0, 0), found by search:
# its eighth corner weight is far below one unit and the other seven round up past it
_LONE_XR = {"fp32": [-0.4999984, -0.44526124, 0.28910556],
            "fp64": [-0.3513036516968437, -0.4999999999985568, 0.01860954926463826]}


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_rounding_remainder_leaves_no_node_below_zero(torch, precision):
    """A lone particle whose seven rounded CiC weights overshoot one unit: if the eighth
    corner took the remainder, its node would hold a negative total (which a 32-bit
    unsigned mass word reads as 2048 particles).  Every node total must stay >= 0, mass must
    be conserved exactly, and the Poisson pass must match the oracle's solve."""
    import paper_2003_04925_amd as S
    from oracle.poisson import dirichlet_potential
    from paper_2003_04925_amd import particle_order
    Np = 32
    sim = S.Simulation(128.0, Np, S.uniform_tiling(Np, 2, 8), 4, precision=precision)
    say("rounding remainder, lone particle", precision)
    sim.setup(torch.from_numpy(synthetic.white_noise(Np, 8)).cuda())
    po, M, go, ho = sim.box_slices()[0]
    x = sim.view("x_res")
    x[:, po:po + M ** 3] = 10.0 * M                    # box 0 empty but for one particle
    slot = po + int(particle_order(M)[0])             # lattice site (0, 0, 0): q = 0.5
    x[:, slot] = torch.tensor(_LONE_XR[precision], dtype=sim.real, device=x.device)
    torch.cuda.synchronize()
    f = 0.5 + sim.view("x_res")[:, slot].double().cpu().numpy()   # D1 = D2 = 0 below
    assert ((f > 0) & (f < 1)).all()
    assert _eighth_corner_remainder(f, precision) < 0              # the premise
    sim.op_deposit(0.0, 0.0)
    torch.cuda.synchronize()
    bits = sim.layout.fixed_bits
    rho = sim.view("rho").cpu().numpy()[go:go + (M - 1) ** 3].astype(np.int64)
    assert rho.min() >= 0
    dropped = int(sim.view("dropped").cpu().numpy()[0])
    assert int(rho.sum()) + dropped == M ** 3 * (1 << bits)
    # the one interior corner, node (1, 1, 1), holds the particle's weight fx fy fz to within
    # three fixed-point units
    exact = float(np.prod(f)) * 2.0 ** bits
    got = int(rho.reshape((M - 1,) * 3)[0, 0, 0])
    say("  node (1, 1, 1)", got, "units, exact", exact)
    assert abs(got - exact) <= 3
    sim.op_poisson(0.0)
    torch.cuda.synchronize()
    phi = sim.view("phi").double().cpu().numpy()[ho:ho + (M + 3) ** 3].reshape((M + 3,) * 3)
    delta = rho.reshape((M - 1,) * 3) / 2.0 ** bits - 1.0
    want = dirichlet_potential(delta, np.zeros((M + 3,) * 3))
    err = np.abs(phi - want).max() / np.abs(want).max()
    say("  min node total", int(rho.min()), "potential rel err", err)
    assert err < (1e-10 if precision == "fp64" else 3e-5)


def test_persistent_step_matches_the_default_schedule(torch):
    """One persistent cooperative launch per KDK step (particle step + Poisson passes of
    the next force, grid-wide barriers between them) gives bitwise the results of the
    default four-launch step, on uniform and mixed box sizes, with no barrier wait giving
    up; FP64 plans refuse it."""
    import paper_2003_04925_amd as S
    from test_gpu_mixed import mixed_tiles
    for Np, L, tiles in ((32, 128.0, S.uniform_tiling(32, 2, 8)), (64, 256.0, mixed_tiles())):
        w = torch.from_numpy(synthetic.white_noise(Np, 23)).cuda()
        ref = S.Simulation(L, Np, tiles, 4, precision="fp32", want_momenta=True).forward(w)
        sim = S.Simulation(L, Np, tiles, 4, precision="fp32", want_momenta=True)
        sim.set_persistent(True)
        for _ in range(2):
            out = sim.forward(w)
            torch.cuda.synchronize()
            st = sim.persistent()
            say("persistent", Np, st)
            assert st["enabled"] and st["grid"] >= 8 and st["barrier_failures"] == 0
            for k in ("pos", "mom", "density"):
                assert torch.equal(out[k], ref[k]), k
    sim64 = S.Simulation(128.0, 32, S.uniform_tiling(32, 2, 8), 2, precision="fp64")
    with pytest.raises(S.ScolaError) as e:
        sim64.set_persistent(True)
    assert e.value.status == -5
