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


# ------------------------------------------------- the paper's six block choices

def test_paper_blocks_partition_and_sizes():
    Ng, Nu = 5, 4
    sizes = {"dg": Nu, "gu": 2, "du": Ng, "d": Ng * Nu, "g": 2 * Nu, "u": 2 * Ng}
    for fixed, size in sizes.items():
        blocks = pc.paper_blocks(Ng, Nu, fixed)
        idx = np.concatenate(blocks)
        assert np.array_equal(np.sort(idx), np.arange(2 * Ng * Nu))
        assert all(len(b) == size for b in blocks)


def _same(A, f1, f2, Ng, Nu):
    M1 = pc.block_matrix(A, pc.paper_blocks(Ng, Nu, f1))
    M2 = pc.block_matrix(A, pc.paper_blocks(Ng, Nu, f2))
    return abs(M1 - M2).max() == 0.0


def test_ecd86_block_choices_that_coincide():
    """Sec. III.C on the ECD86 model: M^{dg} and M^{gu} hold only the diagonal
    of A, and M^{du}, M^d and M^u hold the same elements (A has no term that
    the larger blocks would add)."""
    Ng, Nu = 7, 6
    mdl, A = _model(inputs.ecd86_params(), Ng, Nu, eps=3.1)
    D = sp.diags(A.diagonal())
    for f in ("dg", "gu"):
        assert abs(pc.block_matrix(A, pc.paper_blocks(Ng, Nu, f)) - D).max() == 0.0
    assert _same(A, "du", "d", Ng, Nu) and _same(A, "du", "u", Ng, Nu)
    # the large rows M^g do hold more: the lam q_u couplings
    assert not _same(A, "g", "dg", Ng, Nu)


def test_ecd86_rows_hold_exactly_the_lam_coupling():
    """Within a row (fixed n_g) the ECD86 matrix couples only through
    -lam q_u between the two states (Eq. (18)); q_u's matrix elements are
    sqrt(max(n, n')/2) for |n - n'| = 1."""
    Ng, Nu = 4, 7
    p = inputs.ecd86_params()
    mdl, A = _model(p, Ng, Nu, eps=2.2)
    A = A.toarray()
    n = Ng * Nu
    for g in range(Ng):
        for d in range(2):
            for u in range(Nu):
                for d2 in range(2):
                    for u2 in range(Nu):
                        if (d, u) == (d2, u2):
                            continue
                        a = A[d * n + g * Nu + u, d2 * n + g * Nu + u2]
                        want = -p["lam"] * np.sqrt(max(u, u2) / 2.0) if (d != d2 and abs(u - u2) == 1) else 0.0
                        assert a == pytest.approx(want, abs=1e-15)


def test_generalized_model_du_equals_u_and_dg_differs_from_gu():
    """Sec. III.C on the generalized model: M^{du} and M^u coincide (at fixed n_u
    the two states never meet), while the small blocks M^{dg} and M^{gu} are
    distinct (its q_u sandwiches put elements inside M^{dg})."""
    Ng, Nu = 6, 5
    mdl, A = _model(inputs.draw_params(16), Ng, Nu, eps=2.0)
    assert _same(A, "du", "u", Ng, Nu)
    assert not _same(A, "dg", "gu", Ng, Nu)


def test_rows_are_exact_without_g_couplings():
    """With kappa_d = lam_d = 0 nothing in A changes n_g, so M^g = A and
    preconditioned GMRES finishes in one step at the LU solution."""
    p = inputs.draw_params(17)
    p.update(kappa1=0.0, kappa2=0.0, lam1=0.0, lam2=0.0)
    Ng, Nu = 6, 7
    mdl, A = _model(p, Ng, Nu, eps=2.3)
    assert abs(pc.block_matrix(A, pc.paper_blocks(Ng, Nu, "g")) - A).max() == 0.0
    b = mdl.phi((0, 0), "o")
    x, info = solvers.gmres(A, b, m=4, tol=1e-12, psolve=pc.BlockInverse(A, pc.paper_blocks(Ng, Nu, "g")))
    assert info["iters"] == 1
    np.testing.assert_allclose(x, solvers.lu_solve(A, b), rtol=1e-11)


def test_ecd86_rows_cut_the_iterations_where_the_paper_finds():
    """Sec. III.C, ECD86: convergence is fast at low energy and slows above
    2 eV; M^g is the most effective block choice there, far ahead of the
    diagonal.  Small basis, GMRES(50) and COCG."""
    Ng = Nu = 30
    it = {}
    for eps in (1.0, 3.0):
        mdl, A = _model(inputs.ecd86_params(), Ng, Nu, eps=eps)
        b = mdl.phi((0, 0), "e")
        dinv = 1.0 / np.asarray(A.diagonal()).ravel()
        rows = pc.BlockInverse(A, pc.paper_blocks(Ng, Nu, "g"))
        it[eps] = dict(diag=solvers.gmres(A, b, m=50, dinv=dinv)[1]["iters"],
                       rows=solvers.gmres(A, b, m=50, psolve=rows)[1]["iters"],
                       cocg_diag=solvers.cocg(A, b, psolve=lambda v: dinv * v)[1]["iters"],
                       cocg_rows=solvers.cocg(A, b, psolve=rows)[1]["iters"])
    assert it[1.0]["diag"] <= 30 and it[1.0]["rows"] <= it[1.0]["diag"]
    assert it[3.0]["diag"] >= 3 * it[1.0]["diag"]
    assert 3 * it[3.0]["rows"] <= it[3.0]["diag"]
    assert 3 * it[3.0]["cocg_rows"] <= it[3.0]["cocg_diag"]
