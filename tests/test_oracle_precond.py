"""Pins of the oracle's block-diagonal preconditioners (Sec. III.B) against
exact special cases: where A itself has only the couplings a block keeps,
M = A and preconditioned GMRES must finish in one step at the LU solution."""
import numpy as np
import scipy.sparse as sp
import pytest

from oracle import model2d as m2
from oracle import precond as pc
from oracle import solvers
from paper_2307_13483_amd import inputs


def _model(p, Ng, Nu, eps=1.7):
    E = m2.total_energy(p, eps, (0, 0))
    mdl = m2.Model2D(p, Ng, Nu, E)
    return mdl, mdl.matrix()


def test_blocks_partition_the_basis():
    for Ng, Nu, s in ((7, 5, 3), (6, 4, 6), (5, 3, 1), (9, 2, 4)):
        idx = np.concatenate(pc.segmented_blocks(Ng, Nu, s))
        assert np.array_equal(np.sort(idx), np.arange(2 * Ng * Nu))


def test_segment_length_one_is_the_diagonal():
    mdl, A = _model(inputs.draw_params(11), 6, 5)
    v = np.random.default_rng(0).standard_normal(A.shape[0]) + 1j
    Minv = pc.BlockInverse(A, pc.segmented_blocks(6, 5, 1))
    np.testing.assert_allclose(Minv(v), v / np.asarray(A.diagonal()).ravel(), rtol=1e-14)


def test_blocks_are_symmetric():
    mdl, A = _model(inputs.draw_params(12), 8, 6)
    M = pc.block_matrix(A, pc.segmented_blocks(8, 6, 3)).toarray()
    assert np.max(np.abs(M - M.T)) <= 1e-15 * np.max(np.abs(M))


def _no_u_coupling(p):
    """lam = 0 and no width for the q_u-carrying functions (2, e) and (1, o):
    every term of A that changes n_u vanishes."""
    q = dict(p)
    q.update(lam=0.0, A2e=0.0, A1o=0.0)
    return q


@pytest.mark.parametrize("mu", m2.MU)
def test_full_columns_are_exact_without_u_couplings(mu):
    Ng, Nu = 9, 6
    mdl, A = _model(_no_u_coupling(inputs.draw_params(13)), Ng, Nu)
    b = mdl.phi((0, 0), mu)
    x_lu = solvers.lu_solve(A, b)
    Minv = pc.BlockInverse(A, pc.segmented_blocks(Ng, Nu, Ng))
    np.testing.assert_allclose(Minv(b), x_lu, rtol=1e-10, atol=1e-12 * np.max(np.abs(x_lu)))
    x, info = solvers.gmres(A, b, m=8, tol=1e-10, psolve=Minv)
    assert info["converged"] and info["iters"] == 1
    # shorter segments cut couplings along n_g, which A still has here
    x3, info3 = solvers.gmres(A, b, m=8, tol=1e-10, psolve=pc.BlockInverse(A, pc.segmented_blocks(Ng, Nu, 3)))
    assert info3["converged"] and info3["iters"] > 1


def test_every_segment_length_is_exact_for_a_diagonal_matrix():
    p = _no_u_coupling(inputs.draw_params(14))
    p.update(kappa1=0.0, kappa2=0.0, lam1=0.0, lam2=0.0)
    Ng, Nu = 7, 5
    mdl, A = _model(p, Ng, Nu)
    assert (A - sp.diags(A.diagonal())).count_nonzero() == 0
    b = mdl.phi((0, 0), "e")
    for s in (1, 2, 3, 7):
        x, info = solvers.gmres(A, b, m=4, tol=1e-12, psolve=pc.BlockInverse(A, pc.segmented_blocks(Ng, Nu, s)))
        assert info["iters"] == 1
        np.testing.assert_allclose(x, solvers.lu_solve(A, b), rtol=1e-12)


def test_block_preconditioned_gmres_reaches_the_lu_solution():
    Ng, Nu = 14, 12
    mdl, A = _model(inputs.draw_params(15), Ng, Nu, eps=2.4)
    b = mdl.phi((0, 0), "o")
    x_lu = solvers.lu_solve(A, b)
    x, info = solvers.gmres(A, b, m=6, tol=1e-11, psolve=pc.BlockInverse(A, pc.segmented_blocks(Ng, Nu, 4)))
    assert info["converged"]
    assert np.linalg.norm(x - x_lu) <= 1e-8 * np.linalg.norm(x_lu)
    xj, infoj = solvers.gmres(A, b, m=6, tol=1e-11, dinv=1.0 / m2.jacobi_diagonal(A))
    assert info["iters"] <= infoj["iters"]
