"""Pins of the oracle's reverse-mode reference (oracle/adjoint.py): its forward equals the
NumPy oracle, and its gradient equals central finite differences of the loss."""
import numpy as np
import pytest
import torch

import synthetic
from oracle.adjoint import density_loss, loss_and_gradient
from oracle.run import run_scola
from oracle.tiling import uniform_tiling


@pytest.mark.slow
def test_adjoint_reference_matches_forward_and_finite_differences():
    Np, L, n = 16, 150.0, 3
    tiles = uniform_tiling(Np, 2, 4)
    w = synthetic.white_noise(Np, 3)
    t = synthetic.loss_target(Np, 43)
    loss, grad, dens = loss_and_gradient(w, L, tiles, t, n_steps=n)
    ora = run_scola(w, L, tiles, n_steps=n)
    np.testing.assert_allclose(dens, ora["density"], atol=1e-12)
    assert loss == pytest.approx(((ora["density"] - t) ** 2).sum(), rel=1e-12)
    rng = np.random.default_rng(0)
    eps = 1e-5
    for _ in range(3):
        i = tuple(int(v) for v in rng.integers(0, Np, 3))
        wp, wm = w.copy(), w.copy()
        wp[i] += eps
        wm[i] -= eps
        lp = float(density_loss(torch.tensor(wp), L, tiles, t, n_steps=n)[0])
        lm = float(density_loss(torch.tensor(wm), L, tiles, t, n_steps=n)[0])
        fd = (lp - lm) / (2 * eps)
        assert grad[i] == pytest.approx(fd, rel=1e-5, abs=1e-8)
