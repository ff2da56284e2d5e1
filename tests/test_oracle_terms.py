"""Pins of the oracle's term-list model (oracle/terms.py): it must reduce
exactly to the separately pinned two-state and CO2-like assemblies when given
their term lists, its monomials must match hand-computed matrix elements of
products of truncated coordinates, and on a model with quartic and cross
terms it must keep A^T = A and the truncated-basis optical theorem."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import model2d as m2
from oracle import poly
from oracle import solvers
from oracle import terms
from paper_2307_13483_amd import inputs


def _maxdiff(A, B):
    d = (sp.csr_matrix(A) - sp.csr_matrix(B))
    return 0.0 if d.nnz == 0 else float(abs(d).max())


@pytest.mark.parametrize("seed,Ng,Nu", [(None, 6, 5), (3, 9, 4), (7, 1, 3)])
def test_two_state_model_as_terms(seed, Ng, Nu):
    """The generalized model written as terms gives the model2d matrix and
    right-hand sides (same layout: state, n_g, n_u fastest)."""
    p = inputs.base_params() if seed is None else inputs.draw_params(seed)
    desc = inputs.terms_from_2d(p, Ng, Nu)
    for eps_i, vi in ((1.3, (0, 0)), (2.2, (min(1, Ng - 1), 0))):
        E = m2.total_energy(p, eps_i, vi)
        assert abs(terms.total_energy(desc, eps_i, vi) - E) <= 1e-15
        A = m2.Model2D(p, Ng, Nu, E).matrix()
        At = terms.TermModel(desc, E).matrix()
        assert _maxdiff(A, At) <= 1e-15
        ref = m2.Model2D(p, Ng, Nu, E)
        tm = terms.TermModel(desc, E)
        for mu in (0, 1):
            assert np.max(np.abs(ref.phi(vi, m2.MU[mu]) - tm.phi(vi, mu))) <= 1e-16


@pytest.mark.parametrize("sizes,eps", [(dict(s=3, x=4, y=4, a=2), 1.7), (dict(s=2, x=5, y=3, a=3), 3.2)])
def test_co2_like_model_as_terms(sizes, eps):
    """The CO2-like model written as terms gives poly's matrix and
    right-hand sides (same layout: state, n_s, n_x, n_y, n_a fastest)."""
    p = inputs.co2like_params()
    desc = inputs.terms_from_co2(p, sizes)
    v = (0, 1, 0, 0)
    E = poly.total_energy(p, eps, v)
    A = poly.PolyModel(p, sizes, E).matrix()
    At = terms.TermModel(desc, E).matrix()
    assert _maxdiff(A, At) <= 1e-15
    ref, tm = poly.PolyModel(p, sizes, E), terms.TermModel(desc, E)
    for mu, w in enumerate(poly.WAVES):
        assert np.max(np.abs(ref.phi(v, w) - tm.phi(v, mu))) <= 1e-16


def test_monomials_by_hand():
    """Products of truncated coordinates, N = 3: P q P = [[0, 1/r2, 0],
    [1/r2, 0, 1], [0, 1, 0]]; (PqP)^2 = [[1/2, 0, 1/r2], [0, 3/2, 0],
    [1/r2, 0, 1]] (the last diagonal entry is 1, not the Galerkin 5/2);
    (PqP)^4 = [[3/4, 0, 3/(2 r2)], [0, 9/4, 0], [3/(2 r2), 0, 3/2]];
    a two-mode monomial is the Kronecker product."""
    r2 = math.sqrt(2.0)
    q2 = np.array([[0.5, 0, 1 / r2], [0, 1.5, 0], [1 / r2, 0, 1.0]])
    q4 = np.array([[0.75, 0, 3 / (2 * r2)], [0, 2.25, 0], [3 / (2 * r2), 0, 1.5]])
    assert np.max(np.abs(terms.monomial([3], [2]).toarray() - q2)) <= 1e-15
    assert np.max(np.abs(terms.monomial([3], [4]).toarray() - q4)) <= 1e-15
    q1 = np.array([[0, 1 / r2, 0], [1 / r2, 0, 1.0], [0, 1.0, 0]])
    got = terms.monomial([3, 2, 3], [1, 0, 2]).toarray()
    assert np.max(np.abs(got - np.kron(np.kron(q1, np.eye(2)), q2))) <= 1e-15
    # interior elements agree with the untruncated <n|q^4|n> = (6n^2 + 6n + 3)/4
    q4b = terms.monomial([12], [4]).toarray()
    for n in range(0, 8):
        assert abs(q4b[n, n] - (6 * n * n + 6 * n + 3) / 4.0) <= 1e-13


def test_quartic_model_symmetric_and_optical_theorem():
    """A^T = A (every monomial is symmetric, U is filled symmetrically, the
    level-shift sandwich keeps the operator order), and -Im T_ii = pi sum
    over open (v_f, mu_f) |T_fi|^2 in the truncated basis."""
    desc = inputs.quartic_model(nbasis=(8, 6, 4))
    for eps_i, vi in ((0.7, (0, 0, 0)), (1.9, (1, 0, 0))):
        E = terms.total_energy(desc, eps_i, vi)
        tm = terms.TermModel(desc, E)
        A = tm.matrix()
        assert _maxdiff(A, A.T) <= 1e-16
        grid = [(a, b, c) for a in range(8) for b in range(6) for c in range(4)]
        opened = [v for v in grid if E - terms.vib_energy(desc, v) > 0]
        for mu in (0, 1):
            b = tm.phi(vi, mu)
            psi = solvers.lu_solve(A, b)
            Tii = b @ psi
            tot = sum(abs(tm.phi(v, mf) @ psi) ** 2 for v in opened for mf in (0, 1))
            assert abs(-Tii.imag - math.pi * tot) <= 1e-12 * abs(Tii)


def test_frozen_mode_reduces_the_model():
    """A mode with one basis function that no term moves (mode freezing,
    Sec. III.C) only shifts E_nu by w/2: the model with it equals the model
    without it at a total energy higher by w/2."""
    desc = inputs.quartic_model(nbasis=(7, 5, 4))
    d3 = dict(desc, omega=desc["omega"] + [0.33], nbasis=list(desc["nbasis"]) + [1],
              uterms=[(d, e, c, list(pw) + [0]) for d, e, c, pw in desc["uterms"]],
              vterms=[(d, e, c, list(pw) + [0]) for d, e, c, pw in desc["vterms"]])
    E = 1.4
    A = terms.TermModel(desc, E).matrix()
    A3 = terms.TermModel(d3, E + 0.33 / 2).matrix()
    assert _maxdiff(A, A3) <= 1e-14
