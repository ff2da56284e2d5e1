"""A vibronic model given by polynomial term lists, assembled as an explicit
sparse matrix (oracle; test infrastructure).

The model class of Sec. II.A-C in general form: D discrete states, M
vibrational modes with harmonic H_0 = sum_k w_k (n_k + 1/2) (Eq. (21)), P
partial waves, and
  * U_dd' (Eq. (18) generalised to polynomials): E_d delta_dd' plus a sum of
    terms c prod_k q_k^p_k, each listed once for a pair (d, d') and applied
    to both U_dd' and U_d'd (U is symmetric);
  * the discrete-continuum coupling V_d^mu = f_d^mu(eps) O_d^mu with
    O_d^mu a sum of terms c prod_k q_k^p_k, 2 pi (f_d^mu)^2 = Gamma_d^mu =
    A eps^(l_mu + 1/2) exp(-eps/B) (Eq. (22)), the exponent l_mu belonging to
    the partial wave;
  * F_dd' = sum_mu (O_d^mu)^T diag(F[f_d^mu f_d'^mu](eps_nu)) O_d'^mu with the
    level shift of Eq. (19) on the node grid (Eq. (23), operator order kept);
  * A = E - H_0 - U - F, Phi^{v mu}_d = f_d^mu(E - E_v) O_d^mu |v>   (Eqs. (25), (28)).
Every monomial is a Kronecker product over the modes of powers of the
truncated coordinate matrix P q P (products of truncated matrices).

Basis: index (d, n_0, ..., n_{M-1}), the last mode fastest.

desc is a dict: omega [M], nbasis [M], e_state [D], uterms and vterms as
lists of (d, d' or mu, coeff, powers [M]), width {(d, mu): (A, B)} (absent =
no coupling), l [P], K, X.
"""
import numpy as np
import scipy.sparse as sp

from . import levelshift as ls
from .model2d import position_matrix


def monomial(nbasis, powers):
    """prod_k (P q_k P)^p_k as a sparse matrix on the product basis."""
    out = None
    for n, p in zip(nbasis, powers):
        q = position_matrix(n)
        m = sp.identity(n, format="csr")
        for _ in range(int(p)):
            m = m @ q
        out = m if out is None else sp.kron(out, m, format="csr")
    return sp.csr_matrix(out)


def vib_energies(desc):
    grids = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in desc["nbasis"]], indexing="ij")
    E = np.zeros(grids[0].shape)
    for w, g in zip(desc["omega"], grids):
        E = E + w * (g + 0.5)
    return E.ravel()


def vib_energy(desc, v):
    return float(sum(w * (n + 0.5) for w, n in zip(desc["omega"], v)))


def total_energy(desc, eps_i, v_i):
    """E = eps_i + E_{v_i}  (Eq. (2))."""
    return float(eps_i) + vib_energy(desc, v_i)


def width_of(desc, d, mu):
    """(A, B, l) of Gamma_d^mu, or None without coupling."""
    w = desc["width"].get((d, mu))
    if w is None or w[0] == 0.0:
        return None
    return (w[0], w[1], desc["l"][mu])


def default_tables(desc, eps):
    """F[f_d^mu f_d'^mu](eps) for every wave mu and state pair d <= d' that
    both couple to mu (Eq. (19))."""
    D, P = len(desc["e_state"]), len(desc["l"])
    out = {}
    for mu in range(P):
        for d in range(D):
            for e in range(d, D):
                a, b = width_of(desc, d, mu), width_of(desc, e, mu)
                if a is None or b is None:
                    continue
                out[(mu, d, e)] = ls.level_shift(eps, a[0], a[1], b[0], b[1], desc["l"][mu],
                                                 desc["K"], desc["X"])
    return out


class TermModel:
    """Explicit operator pieces of the model at one total energy E."""

    def __init__(self, desc, E, tables=None):
        self.desc, self.E = desc, float(E)
        self.D, self.P = len(desc["e_state"]), len(desc["l"])
        self.n = int(np.prod(desc["nbasis"]))
        self.I = sp.identity(self.n, format="csr")
        self.Ev = vib_energies(desc)
        self.eps_nu = self.E - self.Ev
        self.tables = (tables or default_tables)(desc, self.eps_nu)
        self.U = {}
        for (d, e, c, pw) in desc["uterms"]:
            key = (min(d, e), max(d, e))
            self.U[key] = self.U.get(key, 0) + c * monomial(desc["nbasis"], pw)
        self.O = {}
        for (d, mu, c, pw) in desc["vterms"]:
            self.O[(d, mu)] = self.O.get((d, mu), 0) + c * monomial(desc["nbasis"], pw)

    def U_block(self, d, e):
        M = self.U.get((min(d, e), max(d, e)))
        M = sp.csr_matrix((self.n, self.n)) if M is None else M
        if d == e:
            M = M + self.desc["e_state"][d] * self.I
        return M

    def F_block(self, d, e):
        acc = sp.csr_matrix((self.n, self.n), dtype=complex)
        for mu in range(self.P):
            Od, Oe = self.O.get((d, mu)), self.O.get((e, mu))
            t = self.tables.get((mu, min(d, e), max(d, e)))
            if Od is None or Oe is None or t is None:
                continue
            acc = acc + Od.T @ sp.diags(t, 0, format="csr") @ Oe
        return acc

    def matrix(self):
        """A = E - H_0 - U - F as a sparse (D n) x (D n) complex matrix."""
        H0 = sp.diags(self.Ev, 0, format="csr")
        blocks = [[None] * self.D for _ in range(self.D)]
        for d in range(self.D):
            for e in range(self.D):
                b = -self.U_block(d, e) - self.F_block(d, e)
                if d == e:
                    b = b + self.E * self.I - H0
                blocks[d][e] = b
        return sp.bmat(blocks, format="csr").astype(np.complex128)

    def unit(self, v):
        e = np.zeros(self.n)
        idx = 0
        for n, vk in zip(self.desc["nbasis"], v):
            if not 0 <= vk < n:
                return e
            idx = idx * n + vk
        e[idx] = 1.0
        return e

    def f(self, d, mu, eps):
        w = width_of(self.desc, d, mu)
        if w is None:
            return 0.0
        return float(ls.coupling_f(np.array([eps]), w[0], w[1], w[2])[0])

    def phi(self, v, mu):
        """Phi^{v mu}_d = f_d^mu(E - E_v) O_d^mu |v>  (Eq. (25))."""
        eps = self.E - vib_energy(self.desc, v)
        ev = self.unit(v)
        parts = []
        for d in range(self.D):
            O = self.O.get((d, mu))
            parts.append(np.zeros(self.n) if O is None else self.f(d, mu, eps) * (O @ ev))
        return np.concatenate(parts)

