"""Pins of the oracle's COCG (Sec. III.A, preconditioned as in Sec. III.B):
the iterate is the Galerkin solution of the bilinear form on the Krylov
space (computed by dense linear algebra, independent of the recurrences),
the residuals are conjugate orthogonal (the defining property the paper
states), an exact preconditioner converges in one step, and on the
two-state model COCG reaches the LU solution."""
import numpy as np
import pytest

from oracle import model2d as m2
from oracle import precond as pc
from oracle import solvers
from paper_2307_13483_amd import inputs


def _complex_symmetric(n, seed, shift=6.0):
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return (B + B.T) / 2 + shift * np.eye(n) + 1j * np.diag(rng.uniform(0.1, 1.0, n))


def _galerkin(A, b, Kinv, k):
    """x in K_k(K^{-1} A, K^{-1} b) with X^T (b - A x) = 0 (bilinear, no
    conjugate): the COCG iterate after k steps in exact arithmetic."""
    cols = [Kinv @ b]
    for _ in range(k - 1):
        cols.append(Kinv @ (A @ cols[-1]))
    X, _ = np.linalg.qr(np.array(cols).T)       # any basis of the space
    c = np.linalg.solve(X.T @ A @ X, X.T @ b)
    return X @ c


@pytest.mark.parametrize("precond", ["none", "diag", "block"])
def test_iterates_are_the_bilinear_galerkin_solutions(precond):
    n = 14
    A = _complex_symmetric(n, 3)
    b = np.random.default_rng(4).standard_normal(n) + 0j
    if precond == "none":
        Kinv = np.eye(n)
    elif precond == "diag":
        Kinv = np.diag(1.0 / np.diag(A))
    else:   # a symmetric block-diagonal section of A
        Kb = np.zeros_like(A)
        for s in range(0, n, 4):
            Kb[s:s + 4, s:s + 4] = A[s:s + 4, s:s + 4]
        Kinv = np.linalg.inv(Kb)
    for k in range(1, 7):
        x, info = solvers.cocg(A, b, tol=1e-300, max_iter=k, psolve=lambda v: Kinv @ v)
        assert info["iters"] == k
        ref = _galerkin(A, b, Kinv, k)
        assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref), (precond, k)


def test_residuals_are_conjugate_orthogonal():
    n = 20
    A = _complex_symmetric(n, 5)
    b = np.random.default_rng(6).standard_normal(n) + 1j * np.random.default_rng(7).standard_normal(n)
    dinv = 1.0 / np.diag(A)
    _, info = solvers.cocg(A, b, tol=1e-12, psolve=lambda v: dinv * v, history=True)
    R = info["residuals"]
    assert len(R) >= 5
    for i in range(len(R)):
        for j in range(i):
            g = abs(solvers.bilinear(R[i], dinv * R[j]))
            assert g <= 1e-9 * np.linalg.norm(R[i]) * np.linalg.norm(np.sqrt(np.abs(dinv)) * R[j]) * 10


def test_exact_preconditioner_converges_in_one_step():
    A = _complex_symmetric(12, 8)
    b = np.arange(1.0, 13.0) + 0j
    Ainv = np.linalg.inv(A)
    x, info = solvers.cocg(A, b, tol=1e-12, psolve=lambda v: Ainv @ v)
    assert info["converged"] and info["iters"] == 1


@pytest.mark.parametrize("prec", ["diag", "block"])
def test_two_state_model_reaches_lu(prec):
    p = inputs.base_params()
    E = m2.total_energy(p, 1.3, (0, 0))
    M = m2.Model2D(p, 10, 9, E)
    A = M.matrix()
    b = M.phi((0, 0), "e")
    if prec == "diag":
        dinv = 1.0 / A.diagonal()
        ps = lambda v: dinv * v
    else:
        ps = pc.BlockInverse(A, pc.segmented_blocks(10, 9, 4))
    x, info = solvers.cocg(A, b, tol=1e-11, psolve=ps)
    assert info["converged"] and not info["breakdown"]
    ref = solvers.lu_solve(A, b)
    assert np.linalg.norm(x - ref) <= 1e-8 * np.linalg.norm(ref)
