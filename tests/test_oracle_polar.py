"""Pins of the polar bend basis (oracle/polar.py) for the CO2-like model:
the polar and Cartesian bases truncated to the same triangle n_x + n_y <= K
span the same space shell by shell, so every polynomial in the truncated
coordinates is the same operator in both and the spectra of H_0 + U agree;
in the polar basis the vibronic angular momentum K = l + Lambda is
conserved (the Hamiltonian is block diagonal in it); and the polar bend
operators obey the ladder algebra of the isotropic oscillator."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import polar
from paper_2307_13483_amd import inputs


def test_polar_basis_counts_and_ladder_algebra():
    K = 6
    st = polar.polar_states(K)
    assert len(st) == (K + 1) * (K + 2) // 2 == len(polar.cartesian_states(K))
    qx, qy, n, l = polar.polar_bend_operators(K)
    # Hermitian coordinates; q_x^2 + q_y^2 = 2 n + 2 + truncation at the top shell
    for q in (qx, qy):
        assert abs(q - q.conj().T).max() <= 1e-15
    r2 = (qx @ qx + qy @ qy).toarray()
    inner = n < K
    assert np.allclose(np.diag(r2)[inner], (n + 1.0)[inner], atol=1e-14)
    # q_+ raises l by one: every element links l' = l + 1
    qp = (qx + 1j * qy).tocoo()
    for i, j, v in zip(qp.row, qp.col, qp.data):
        if abs(v) > 1e-14:
            assert l[i] == l[j] + 1
    # angular momentum L = q_x p_y - q_y p_x is diagonal with eigenvalue l:
    # with a_+- it is n_+ - n_-, i.e. [L, q_+] = q_+ on the untruncated shells
    assert set(l) == set(range(-K, K + 1))


@pytest.mark.parametrize("Ns,K,Na", [(1, 5, 1), (2, 4, 2)])
def test_polar_and_cartesian_spectra_agree(Ns, K, Na):
    """H_0 + U (F = 0) of the CO2-like model: the polar basis with sigma and
    the circular Pi pair (Lambda = -1, +1) and the Cartesian triangle with (sigma, Pi_x, Pi_y) give the
    same eigenvalues (a unitary maps one to the other within each shell)."""
    p = inputs.co2like_params()
    # couplings large enough that every term moves the spectrum visibly
    p = dict(p, c_rt=0.03, c_sp=0.08, gb_sigma=0.02, gb_pi=-0.015)
    Hp, _ = polar.co2_hamiltonian(p, Ns, K, Na, "polar")
    Hc, _ = polar.co2_hamiltonian(p, Ns, K, Na, "cartesian")
    assert abs(Hp - Hp.conj().T).max() <= 1e-14
    assert abs(Hc - Hc.T).max() <= 1e-14 and abs(Hc.imag).max() == 0
    ep = np.linalg.eigvalsh(Hp.toarray())
    ec = np.linalg.eigvalsh(Hc.toarray().real)
    assert np.max(np.abs(ep - ec)) <= 1e-12


def test_a_wrong_bend_operator_changes_the_spectrum(monkeypatch):
    """The comparison has teeth: with q_y = (q_+ + q_-)/(2 i) (a sign slip)
    the polar spectrum no longer matches the Cartesian one."""
    p = dict(inputs.co2like_params(), c_rt=0.03, c_sp=0.08, gb_sigma=0.02)
    good = polar.polar_bend_operators

    def wrong(K):
        qx, qy, n, l = good(K)
        qp = qx + 1j * qy
        qm = qx - 1j * qy
        return qx, (qp + qm) / 2j, n, l
    monkeypatch.setattr(polar, "polar_bend_operators", wrong)
    Hp, _ = polar.co2_hamiltonian(p, 1, 5, 1, "polar")
    Hc, _ = polar.co2_hamiltonian(p, 1, 5, 1, "cartesian")
    ep = np.linalg.eigvalsh((0.5 * (Hp + Hp.conj().T)).toarray())
    ec = np.linalg.eigvalsh(Hc.toarray().real)
    assert np.max(np.abs(ep - ec)) > 1e-3


@pytest.mark.parametrize("Ns,K,Na", [(2, 5, 1), (1, 6, 2)])
def test_vibronic_angular_momentum_is_conserved(Ns, K, Na):
    """Every nonzero element of H_0 + U in the polar basis links functions
    with the same K = l + Lambda (Renner-Teller pair and sigma-Pi coupling
    included); the K blocks are therefore independent problems."""
    p = dict(inputs.co2like_params(), c_rt=0.03, c_sp=0.08)
    H, lab = polar.co2_hamiltonian(p, Ns, K, Na, "polar")
    Kv = np.array([lam + l for lam, l in lab])
    Hc = H.tocoo()
    big = np.abs(Hc.data) > 1e-14
    assert np.all(Kv[Hc.row[big]] == Kv[Hc.col[big]])
    # the coupling terms are really present (elements between different Lambda)
    lam = np.array([x for x, _ in lab])
    assert np.any(lam[Hc.row[big]] != lam[Hc.col[big]])
