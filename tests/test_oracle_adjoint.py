"""Pins of the oracle's analytic (adjoint) gradient: central finite
differences of the oracle's own loss, with the relative step of the
adjoint workload (h = 1e-6)."""
import numpy as np
import pytest

from oracle import adjoint as adj
from paper_2307_13483_amd import inputs


def _setup(Ng, Nu, eps):
    p = inputs.base_params()
    target = inputs.draw_params(inputs.SEED + 1)
    finals = [(k, 0) for k in range(4)]
    sig_t, _ = adj.forward(target, Ng, Nu, eps, (0, 0), finals)
    return p, finals, sig_t


def _min_threshold_distance(p, Ng, Nu, eps):
    """Smallest |eps_nu| over the basis: the level shift has a sqrt(eps)
    branch point at threshold, where d/d(omega) diverges."""
    return min(abs(e - p["omega_g"] * g - p["omega_u"] * u) for e in eps
               for g in range(Ng) for u in range(Nu))


def test_gradient_matches_central_differences():
    """Energies chosen off the 0.05 eV lattice of the base frequencies, so no
    eps_nu = eps_i - w_g n_g - w_u n_u sits at the threshold singularity."""
    Ng, Nu = 9, 7
    eps = [0.57, 1.73, 2.61]
    p, finals, sig_t = _setup(Ng, Nu, eps)
    assert _min_threshold_distance(p, Ng, Nu, eps) > 0.01
    L, g, _ = adj.loss_and_grad(p, Ng, Nu, eps, (0, 0), finals, sig_t)
    fd = adj.finite_difference_grad(p, Ng, Nu, eps, (0, 0), finals, sig_t, h=1e-6)
    scale = np.max(np.abs(g))
    for k, name in enumerate(adj.PARAM_NAMES):
        assert abs(g[k] - fd[name]) <= 2e-5 * scale + 1e-6 * abs(fd[name]), (name, g[k], fd[name])


def test_dense_and_sparse_lu_gradients_agree():
    Ng, Nu = 6, 5
    eps = [1.1, 2.2]
    p, finals, sig_t = _setup(Ng, Nu, eps)
    _, g1, _ = adj.loss_and_grad(p, Ng, Nu, eps, (0, 0), finals, sig_t, dense=False)
    _, g2, _ = adj.loss_and_grad(p, Ng, Nu, eps, (0, 0), finals, sig_t, dense=True)
    assert np.max(np.abs(g1 - g2)) <= 1e-10 * np.max(np.abs(g1))


def test_gradient_vanishes_at_the_target():
    """sigma* computed with the same parameters: L = 0 and every
    component of the gradient is 0 (the adjoint weights vanish)."""
    Ng, Nu = 6, 5
    eps = [1.3]
    p = inputs.base_params()
    finals = [(0, 0), (1, 0)]
    sig, _ = adj.forward(p, Ng, Nu, eps, (0, 0), finals)
    L, g, _ = adj.loss_and_grad(p, Ng, Nu, eps, (0, 0), finals, sig)
    assert L == 0.0 and np.all(g == 0.0)
