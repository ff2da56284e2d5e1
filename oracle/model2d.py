"""The generalized two-state, two-mode model assembled as an explicit matrix
(oracle; test infrastructure).

Paper, Sec. II.B-II.D:
  * H_0 harmonic in q_g, q_u, E_nu = w_g (n_g + 1/2) + w_u (n_u + 1/2)   (Eq. (21))
  * U = [[E_1 + k_1 q_g, lam q_u], [lam q_u, E_2 + k_2 q_g]]              (Eq. (18))
  * V_eps = [[f_1^e (1 + lam_1 q_g), f_1^o q_u],
             [f_2^e q_u,             f_2^o (1 + lam_2 q_g)]]             (Sec. II.C)
  * level-shift operator F with the operator order kept                  (Eq. (23))
  * A = <nu| (E - H_ef)_{dd'} |nu'>, H_ef = H_0 + U + F                  (Eqs. (13), (28))
  * right-hand side Phi^{v mu}_{d,nu} = <nu| V^mu_{d eps} |v>, eps = E - E_v
                                                                          (Eq. (25))
Basis: compound index alpha = (d, n_g, n_u), truncated n_g < N_g, n_u < N_u
(Sec. II.D); flat index d*N_g*N_u + n_g*N_u + n_u (n_u fastest).

Every operator is built as an explicit sparse matrix product of truncated
matrices (P q P), i.e. the sandwich P V P . diag(F) . P V P; nothing here is a
stencil.

Parameters are a dict with the keys of PARAM_NAMES plus E1, l_e, l_o and the
grid (K, X).  PARAM_NAMES is the order of the 16 model parameters used for
gradients: w_g, w_u, k_1, k_2, lam, lam_1, lam_2, gap (E_2 = E_1 + gap),
then A_d^mu and B_d^mu of the widths Gamma_d^mu = A eps^(l+1/2) exp(-eps/B).
"""
import numpy as np
import scipy.sparse as sp

from . import levelshift as ls

PARAM_NAMES = ("omega_g", "omega_u", "kappa1", "kappa2", "lam", "lam1", "lam2", "gap",
               "A1e", "A2e", "A1o", "A2o", "B1e", "B2e", "B1o", "B2o")
MU = ("e", "o")


def position_matrix(n):
    """Truncated q = (a + a^dagger)/sqrt 2 in the HO basis |0..n-1>:
    <m|q|m+1> = <m+1|q|m> = sqrt((m+1)/2)  (the ladder action of Sec. III)."""
    if n <= 1:
        return sp.csr_matrix((n, n), dtype=np.float64)
    off = np.sqrt(np.arange(1, n, dtype=np.float64) / 2.0)
    return sp.diags([off, off], [-1, 1], shape=(n, n), format="csr")


def vib_energies(p, Ng, Nu):
    """E_nu on the (n_g, n_u) grid, flattened with n_u fastest (Eq. (21))."""
    ng = np.arange(Ng, dtype=np.float64)[:, None]
    nu = np.arange(Nu, dtype=np.float64)[None, :]
    return (p["omega_g"] * (ng + 0.5) + p["omega_u"] * (nu + 0.5)).ravel()


def vib_energy(p, v):
    return p["omega_g"] * (v[0] + 0.5) + p["omega_u"] * (v[1] + 0.5)


def widths_of(p):
    """(A, B, l) for each (d, mu), d in {1, 2}, mu in {e, o}."""
    return {
        (1, "e"): (p["A1e"], p["B1e"], p["l_e"]),
        (2, "e"): (p["A2e"], p["B2e"], p["l_e"]),
        (1, "o"): (p["A1o"], p["B1o"], p["l_o"]),
        (2, "o"): (p["A2o"], p["B2o"], p["l_o"]),
    }


def default_tables(p, eps):
    """The six level-shift diagonals F[f_d^mu f_d'^mu](eps) for (dd') in
    {11, 12, 22} and mu in {e, o}, evaluated at the points eps (Eq. (19))."""
    w = widths_of(p)
    out = {}
    for mu in MU:
        A1, B1, l = w[(1, mu)]
        A2, B2, _ = w[(2, mu)]
        out[(mu, 1, 1)] = ls.level_shift(eps, A1, B1, A1, B1, l, p["K"], p["X"])
        out[(mu, 2, 2)] = ls.level_shift(eps, A2, B2, A2, B2, l, p["K"], p["X"])
        out[(mu, 1, 2)] = ls.level_shift(eps, A1, B1, A2, B2, l, p["K"], p["X"])
    return out


def default_f(p, d, mu, eps):
    A, B, l = widths_of(p)[(d, mu)]
    return float(ls.coupling_f(np.array([eps]), A, B, l)[0])


class Model2D:
    """Explicit operator pieces of the model at one total energy E.

    ``tables`` and ``fcoef`` may be replaced (test-only special cases, e.g. a
    constant width) by callables with the signatures of default_tables and
    default_f.
    """

    def __init__(self, p, Ng, Nu, E, tables=None, fcoef=None):
        self.p, self.Ng, self.Nu, self.E = p, Ng, Nu, float(E)
        n = Ng * Nu
        self.n = n
        I_g = sp.identity(Ng, format="csr")
        I_u = sp.identity(Nu, format="csr")
        self.Qg = sp.kron(position_matrix(Ng), I_u, format="csr")
        self.Qu = sp.kron(I_g, position_matrix(Nu), format="csr")
        self.I = sp.identity(n, format="csr")
        self.Ev = vib_energies(p, Ng, Nu)
        self.eps_nu = self.E - self.Ev
        self.tables = (tables or default_tables)(p, self.eps_nu)
        self.fcoef = fcoef or (lambda d, mu, eps: default_f(p, d, mu, eps))
        self.G = {1: self.I + p["lam1"] * self.Qg, 2: self.I + p["lam2"] * self.Qg}
        # O_d^mu: the coordinate-dependent factor of V^mu_{d eps} (Sec. II.C)
        self.O = {(1, "e"): self.G[1], (2, "e"): self.Qu,
                  (1, "o"): self.Qu, (2, "o"): self.G[2]}

    def Fdiag(self, mu, d, dp):
        key = (mu, min(d, dp), max(d, dp))
        return sp.diags(self.tables[key], 0, format="csr")

    def F_block(self, d, dp):
        """F_{dd'} = sum_mu O_d^mu F^mu_{dd'} O_d'^mu  (Eq. (23), order kept)."""
        out = sp.csr_matrix((self.n, self.n), dtype=np.complex128)
        for mu in MU:
            out = out + self.O[(d, mu)] @ self.Fdiag(mu, d, dp) @ self.O[(dp, mu)]
        return out

    def U_block(self, d, dp):
        p = self.p
        if d == dp:
            Ed = p["E1"] if d == 1 else p["E1"] + p["gap"]
            kap = p["kappa1"] if d == 1 else p["kappa2"]
            return Ed * self.I + kap * self.Qg
        return p["lam"] * self.Qu

    def matrix(self):
        """A = E - H_0 - U - F as a sparse 2n x 2n complex matrix (Eq. (28))."""
        blocks = [[None, None], [None, None]]
        H0 = sp.diags(self.Ev, 0, format="csr")
        for d in (1, 2):
            for dp in (1, 2):
                b = -self.U_block(d, dp) - self.F_block(d, dp)
                if d == dp:
                    b = b + self.E * self.I - H0
                blocks[d - 1][dp - 1] = b
        return sp.bmat(blocks, format="csr").astype(np.complex128)

    def unit(self, v):
        ng, nu = v
        e = np.zeros(self.n)
        if 0 <= ng < self.Ng and 0 <= nu < self.Nu:
            e[ng * self.Nu + nu] = 1.0
        return e

    def phi(self, v, mu):
        """Phi^{v mu}_{d, nu} = f_d^mu(E - E_v) <nu| O_d^mu |v>  (Eq. (25))."""
        eps = self.E - vib_energy(self.p, v)
        ev = self.unit(v)
        parts = [self.fcoef(d, mu, eps) * (self.O[(d, mu)] @ ev) for d in (1, 2)]
        return np.concatenate(parts).astype(np.float64)


def total_energy(p, eps_i, v_i):
    """E = eps_i + E_{v_i}  (Eq. (2))."""
    return float(eps_i) + vib_energy(p, v_i)


def jacobi_diagonal(A):
    """diag(A), the diagonal (M^{dg} = M^{gu}) preconditioner of Sec. III.B."""
    return np.asarray(A.diagonal()).ravel()


def parity_of(Ng, Nu):
    """Symmetry label s_d (-1)^{n_u} of every basis function, s_1 = +1, s_2 = -1
    (gerade/ungerade decomposition of Sec. IV)."""
    nu = np.tile(np.arange(Nu), Ng)
    par = (-1.0) ** nu
    return np.concatenate([par, -par])
