"""Pins of the oracle's CO2-like polynomial model: an exact reduction to the
pinned two-state model, hand-computed matrix elements of the new operators,
the symmetries of the model class, and the optical theorem."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import model2d as m2
from oracle import poly
from oracle import precond as pc
from oracle import solvers
from paper_2307_13483_amd import inputs

P = inputs.co2like_params()


def _model(sizes, eps=1.9, p=None, v=(0, 0, 0, 0)):
    p = p or P
    M = poly.PolyModel(p, sizes, poly.total_energy(p, eps, v))
    return M, M.matrix()


def test_matrix_is_complex_symmetric():
    M, A = _model(dict(s=4, x=5, y=5, a=3))
    assert abs(A - A.T).max() <= 1e-15 * abs(A).max()


def test_reflections_split_the_basis_and_place_the_right_hand_sides():
    sizes = dict(s=3, x=5, y=4, a=2)
    M, A = _model(sizes)
    rx, ry = poly.reflection_labels(sizes)
    C = A.tocoo()
    assert np.all(rx[C.row] == rx[C.col]) and np.all(ry[C.row] == ry[C.col])
    want = {"s": (1, 1), "px": (-1, 1), "py": (1, -1)}
    for mu in poly.WAVES:
        nz = np.nonzero(M.phi((0, 0, 0, 0), mu))[0]
        assert set(rx[nz]) == {want[mu][0]} and set(ry[nz]) == {want[mu][1]}


def test_second_order_matrix_elements_by_hand():
    """<n|q^2|n> = n + 1/2 below the top state, <n|q^2|n+2> = sqrt((n+1)(n+2))/2,
    <n_x n_y|q_x q_y|n_x+1 n_y+1> = sqrt((n_x+1)(n_y+1))/2: the Renner-Teller
    pair and the quadratic terms assembled from truncated q matrices."""
    p = {k: 0.0 for k in P}
    p.update(omega_s=0.0, omega_b=0.0, omega_a=0.0, K=64, X=10.0,
             A_sigma_s=0.0, A_sigma_p=0.0, A_pi_s=0.0, A_pi_p=0.0,
             B_sigma_s=1.0, B_sigma_p=1.0, B_pi_s=1.0, B_pi_p=1.0)
    sizes = dict(s=1, x=5, y=5, a=1)
    p.update(c_rt=1.0)
    M, A = _model(sizes, eps=0.0, p=p)
    n = M.n
    idx = lambda x, y: x * 5 + y
    U = -A.toarray()            # E = 0, H_0 = 0, F = 0: A = -U
    xx = U[n:2 * n, n:2 * n]    # U_pix pix = c_rt (q_x^2 - q_y^2)
    assert np.isclose(xx[idx(2, 1), idx(2, 1)], (2 + 0.5) - (1 + 0.5))
    assert np.isclose(xx[idx(1, 3), idx(3, 3)], np.sqrt(2 * 3) / 2)
    assert np.isclose(xx[idx(4, 0), idx(4, 0)], 4 / 2 - 0.5)     # top state: only n/2
    xy = U[n:2 * n, 2 * n:]     # U_pix piy = 2 c_rt q_x q_y
    assert np.isclose(xy[idx(1, 2), idx(2, 3)], 2 * np.sqrt(2 * 3) / 2)
    assert np.isclose(xy[idx(1, 2), idx(1, 3)], 0.0)


def test_reduces_exactly_to_the_two_state_model():
    """One basis function in y and a, no second-order terms, c' = 0: the
    (sigma, Pi_x) part is the generalized two-state model with g = s, u = x,
    E_1 = E_sigma, gap = E_pi - E_sigma, lam = c, and the h factors folded
    into the widths (Gamma -> h^2 Gamma); the frozen modes add w_b/2 + w_a/2
    to every E_nu."""
    p = dict(P)
    for k in ("gs_sigma", "gb_sigma", "ga_sigma", "gs_pi", "gb_pi", "ga_pi", "c_rt", "c_sp2"):
        p[k] = 0.0
    Ns, Nx = 7, 6
    sizes = dict(s=Ns, x=Nx, y=1, a=1)
    q = dict(omega_g=p["omega_s"], omega_u=p["omega_b"], kappa1=p["k_sigma"], kappa2=p["k_pi"],
             lam=p["c_sp"], lam1=p["l_sigma"], lam2=p["l_pi"], E1=p["E_sigma"],
             gap=p["E_pi"] - p["E_sigma"],
             A1e=p["A_sigma_s"], B1e=p["B_sigma_s"], A2e=p["h_pi"] ** 2 * p["A_pi_s"], B2e=p["B_pi_s"],
             A1o=p["h_sigma"] ** 2 * p["A_sigma_p"], B1o=p["B_sigma_p"], A2o=p["A_pi_p"],
             B2o=p["B_pi_p"], l_e=0, l_o=1, K=p["K"], X=p["X"])
    for eps in (0.7, 2.3):
        E = poly.total_energy(p, eps, (0, 0, 0, 0))
        M = poly.PolyModel(p, sizes, E)
        A = M.matrix().tocsr()
        n = M.n
        keep = np.arange(2 * n)
        E2 = E - 0.5 * p["omega_b"] - 0.5 * p["omega_a"]
        ref = m2.Model2D(q, Ns, Nx, E2)
        A2 = ref.matrix()
        assert abs(A[keep][:, keep] - A2).max() <= 1e-13 * abs(A2).max()
        assert abs(A[keep][:, 2 * n:]).max() == 0.0
        for mu, mu2 in (("s", "e"), ("px", "o")):
            b = M.phi((0, 0, 0, 0), mu)
            np.testing.assert_allclose(b[:2 * n], ref.phi((0, 0), mu2), rtol=1e-14, atol=1e-16)
            assert np.all(b[2 * n:] == 0)


def test_optical_theorem():
    """-Im T_ii = pi sum over open final channels |T_fi|^2 (unitarity of the
    truncated problem; independent of Re F)."""
    sizes = dict(s=4, x=5, y=5, a=2)
    eps = 1.3
    M, A = _model(sizes, eps=eps)
    b = M.phi((0, 0, 0, 0), "s")
    psi = solvers.lu_solve(A, b)
    Tii = b @ psi
    tot = 0.0
    for s in range(4):
        for x in range(5):
            for y in range(5):
                for a in range(2):
                    for mu in poly.WAVES:
                        bf = M.phi((s, x, y, a), mu)
                        tot += abs(bf @ psi) ** 2
    assert np.isclose(-Tii.imag, np.pi * tot, rtol=1e-10)


def test_bend_block_preconditioner():
    """The paper's block choice for this class (every state and bend point
    per (n_s, n_a)): exact when nothing couples different (n_s, n_a), and far
    fewer iterations than the diagonal otherwise (3x at this small basis,
    two orders of magnitude at 8 x 12 x 12 x 4 near 2 eV)."""
    sizes = dict(s=3, x=6, y=6, a=2)
    p = dict(P)
    for k in ("k_sigma", "k_pi", "gs_sigma", "gs_pi", "ga_sigma", "ga_pi", "c_sp2", "l_sigma", "l_pi"):
        p[k] = 0.0
    M, A = _model(sizes, eps=2.0, p=p)
    b = M.phi((0, 0, 0, 0), "px")
    Minv = pc.BlockInverse(A, poly.bend_blocks(sizes))
    x, info = solvers.gmres(A, b, m=10, tol=1e-10, psolve=Minv)
    assert info["iters"] == 1
    M2, A2 = _model(dict(s=5, x=8, y=8, a=3), eps=2.0)
    b2 = M2.phi((0, 0, 0, 0), "s")
    _, i_blk = solvers.gmres(A2, b2, m=20, tol=1e-10, psolve=pc.BlockInverse(A2, poly.bend_blocks(M2.sizes)))
    _, i_dg = solvers.gmres(A2, b2, m=20, tol=1e-10, dinv=1.0 / m2.jacobi_diagonal(A2), max_iter=4000)
    assert i_blk["converged"] and i_blk["iters"] * 3 < i_dg["iters"]
