"""The two-dimensional harmonic bend in polar form (oracle; test
infrastructure), for the CO2-like model of Sec. III.C.

The paper describes its CO2 bend (the doubly degenerate mode) in the basis
of the 2D isotropic oscillator with vibrational angular momentum l.  Here
that basis is built from circular quanta: with a_+- = (a_x -+ i a_y)/sqrt 2,
the states |n_+, n_-> have n = n_+ + n_- quanta and angular momentum
l = n_+ - n_- (l = -n, -n + 2, ..., n), and the basis keeps n <= K (a
triangle of the Cartesian grid, the same space as n_x + n_y <= K).  Then
    q_+ = q_x + i q_y = a_- + a_+^dagger   (raises l by 1),
    q_- = q_x - i q_y = a_+ + a_-^dagger   (lowers l by 1),
    q_x = (q_+ + q_-)/2,  q_y = (q_+ - q_-)/(2 i),
each truncated to the basis, and polynomials are products of the truncated
matrices (as for the Cartesian modes).

The electronic Pi pair in circular form, (Pi_x -+ i Pi_y)/sqrt 2 with
Lambda = -+1 (Pi_x and Pi_y transform like x and y, and x -+ i y like
exp(-+ i phi)), with sigma (Lambda = 0), makes the vibronic angular momentum
K = l + Lambda a good quantum number of H_0 + U: the Hamiltonian is block
diagonal in K.  Built here: the bend operators in both bases, and the
CO2-like model's H_0 + U (no level shift) in the polar basis.
"""
import numpy as np
import scipy.sparse as sp

from .model2d import position_matrix


def polar_states(K):
    """(n_+, n_-) with n_+ + n_- <= K, ordered by n, then by l descending."""
    out = []
    for n in range(K + 1):
        for n_plus in range(n, -1, -1):
            out.append((n_plus, n - n_plus))
    return out


def cartesian_states(K):
    """(n_x, n_y) with n_x + n_y <= K, ordered by n, then by n_x descending."""
    out = []
    for n in range(K + 1):
        for nx in range(n, -1, -1):
            out.append((nx, n - nx))
    return out


def _ladder(states, which, dagger):
    """Truncated a_which (or its adjoint) on a list of two-index states:
    which 0 lowers (or raises) the first index, 1 the second."""
    idx = {s: k for k, s in enumerate(states)}
    rows, cols, vals = [], [], []
    for k, s in enumerate(states):
        t = list(s)
        if dagger:
            t[which] += 1
            amp = np.sqrt(t[which])
        else:
            if t[which] == 0:
                continue
            amp = np.sqrt(t[which])
            t[which] -= 1
        j = idx.get(tuple(t))
        if j is None:
            continue
        rows.append(j)
        cols.append(k)
        vals.append(amp)
    n = len(states)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n), dtype=complex)


def polar_bend_operators(K):
    """(q_x, q_y, n_quanta, l) on the polar basis with n <= K."""
    st = polar_states(K)
    ap, am = _ladder(st, 0, False), _ladder(st, 1, False)
    apd, amd = _ladder(st, 0, True), _ladder(st, 1, True)
    q_plus = am + apd
    q_minus = ap + amd
    qx = 0.5 * (q_plus + q_minus)
    qy = (q_plus - q_minus) / 2j
    n = np.array([a + b for a, b in st])
    l = np.array([a - b for a, b in st])
    return qx, qy, n, l


def cartesian_bend_operators(K):
    """(q_x, q_y, n_quanta) on the Cartesian triangle n_x + n_y <= K."""
    st = cartesian_states(K)
    ax, ay = _ladder(st, 0, False), _ladder(st, 1, False)
    qx = (ax + ax.T) / np.sqrt(2.0)
    qy = (ay + ay.T) / np.sqrt(2.0)
    n = np.array([a + b for a, b in st])
    return qx, qy, n


def co2_hamiltonian(p, Ns, K, Na, basis="polar"):
    """H_0 + U of the CO2-like model (the same U as oracle.poly, no level
    shift) with the bend truncated to n_x + n_y <= K, in the polar basis with
    electronic states (sigma, Pi with Lambda = -1, Pi with Lambda = +1), or the
    Cartesian triangle with
    (sigma, Pi_x, Pi_y).  Basis order (state, n_s, bend state, n_a).
    Returns (H, labels) with labels the (Lambda, l) of every basis function
    (polar only; None for the Cartesian)."""
    if basis == "polar":
        qx, qy, nb, lb = polar_bend_operators(K)
    else:
        qx, qy, nb = cartesian_bend_operators(K)
        lb = None
    nbend = qx.shape[0]
    Is, Ib, Ia = (sp.identity(n, format="csr", dtype=complex) for n in (Ns, nbend, Na))
    Qs = sp.csr_matrix(position_matrix(Ns), dtype=complex)
    Qa = sp.csr_matrix(position_matrix(Na), dtype=complex)

    def op(s=None, b=None, a=None):
        return sp.kron(sp.kron(s if s is not None else Is, b if b is not None else Ib),
                       a if a is not None else Ia, format="csr")

    n = Ns * nbend * Na
    I = sp.identity(n, format="csr", dtype=complex)
    Xs, Xa = op(s=Qs), op(a=Qa)
    Xx, Xy = op(b=qx), op(b=qy)
    H0 = (p["omega_s"] * (op(s=sp.diags(np.arange(Ns) + 0.5).astype(complex)))
          + p["omega_b"] * op(b=sp.diags(nb + 1.0).astype(complex))
          + p["omega_a"] * op(a=sp.diags(np.arange(Na) + 0.5).astype(complex)))
    bend2 = Xx @ Xx + Xy @ Xy
    rt = Xx @ Xx - Xy @ Xy
    Uss = (p["E_sigma"] * I + p["k_sigma"] * Xs + p["gs_sigma"] * (Xs @ Xs) + p["gb_sigma"] * bend2
           + p["ga_sigma"] * (Xa @ Xa))
    Upi = (p["E_pi"] * I + p["k_pi"] * Xs + p["gs_pi"] * (Xs @ Xs) + p["gb_pi"] * bend2
           + p["ga_pi"] * (Xa @ Xa))
    cs = p["c_sp"] * (I + p["c_sp2"] * Xs)
    # Cartesian electronic blocks (sigma, Pi_x, Pi_y), as in oracle.poly; the
    # lower blocks are the adjoints of the upper ones (on the triangle the
    # truncated q_x and q_y do not commute, and in the polar basis they are
    # complex: U is Hermitian, and real symmetric in the Cartesian basis)
    Usx, Usy, Uxy = cs @ Xx, cs @ Xy, 2.0 * p["c_rt"] * (Xx @ Xy)
    Ucart = [[Uss, Usx, Usy],
             [Usx.conj().T, Upi + p["c_rt"] * rt, Uxy],
             [Usy.conj().T, Uxy.conj().T, Upi - p["c_rt"] * rt]]
    H = sp.bmat(Ucart, format="csr")
    H = H + sp.block_diag([H0, H0, H0], format="csr")
    if basis != "polar":
        return H, None
    # electronic rotation to (Pi_x -+ i Pi_y)/sqrt 2 (Lambda = -+1): H -> C^dagger H C
    c = 1.0 / np.sqrt(2.0)
    C = sp.bmat([[I, None, None], [None, c * I, c * I], [None, -1j * c * I, 1j * c * I]],
                format="csr")
    H = (C.conj().T @ H @ C).tocsr()
    ls = np.tile(np.repeat(lb, Na), Ns)
    labels = [(0, l) for l in ls] + [(-1, l) for l in ls] + [(1, l) for l in ls]
    return H, labels
