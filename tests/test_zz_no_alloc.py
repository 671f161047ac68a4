"""scola_forward_noalloc (static device workspace) against scola_forward (caller's workspace):
two calls in a row on one GPU, the second on a smaller problem, every output bitwise equal
(the same kernels on the same inputs; fixed-point deposits make runs reproducible)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    t = pytest.importorskip("torch")
    if not t.cuda.is_available():
        pytest.skip("needs a GPU")
    return t


def _run(torch, S, synthetic, Np, L, tiles, n_steps, precision, seed):
    sim = S.Simulation(L, Np, tiles, n_steps, precision=precision, want_momenta=True)
    w = torch.from_numpy(synthetic.white_noise(Np, seed)).cuda()
    a = sim.forward_noalloc(w)
    torch.cuda.synchronize()
    a = {k: v.cpu().numpy() for k, v in a.items()}
    b = sim.forward(w)
    torch.cuda.synchronize()
    b = {k: v.cpu().numpy() for k, v in b.items()}
    return sim, a, b


def test_noalloc_matches_forward_twice_second_smaller(torch):
    import paper_2003_04925_amd as S
    import synthetic
    # first call: 2^3 boxes of 32^3 (FP32); second: one 16^3 box (FP64), a smaller input
    cases = [(32, 128.0, S.uniform_tiling(32, 2, 8), 3, "fp32", 3),
             (16, 64.0, [((0, 0, 0), 16, 0)], 2, "fp64", 4)]
    for Np, L, tiles, n, prec, seed in cases:
        say(f"noalloc case Np={Np} tiles={len(tiles)} steps={n} {prec}")
        sim, a, b = _run(torch, S, synthetic, Np, L, tiles, n, prec, seed)
        assert sim.layout.total <= S.STATIC_WORKSPACE_BYTES
        for k in ("pos", "mom", "density"):
            assert np.all(np.isfinite(a[k])), k
            assert np.array_equal(a[k], b[k]), (k, float(np.abs(a[k] - b[k]).max()))
        del sim


def test_noalloc_rejects_a_plan_beyond_the_static_size(torch):
    import paper_2003_04925_amd as S
    import synthetic
    Np = 128    # 2^3 boxes of 64^3: a workspace above 128 MiB
    sim = S.Simulation(500.0, Np, S.uniform_tiling(Np, 2, 0), 2, precision="fp32")
    assert sim.layout.total > S.STATIC_WORKSPACE_BYTES
    w = torch.from_numpy(synthetic.white_noise(Np, 5)).cuda()
    with pytest.raises(S.ScolaError) as e:
        sim.forward_noalloc(w)
    assert e.value.status == -1 and "static workspace" in str(e.value)
