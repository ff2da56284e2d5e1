"""The CO2-like three-state, four-mode polynomial vibronic model (oracle;
test infrastructure).

Sec. III.C (the paragraph on e + CO2) describes the model class: three
discrete states (a virtual state sigma and the two components Pi_x, Pi_y of
a shape resonance) coupled to each other through the bending mode, four
vibrational degrees of freedom (symmetric stretch s, the two-dimensional bend
(x, y), asymmetric stretch a), polynomial couplings, and several electron
partial waves.  The paper's CO2 parameters are not given, so this is a
synthetic member of that class with couplings up to second order, built on
the same equations as the two-state model:
  * H_0 = sum_k w_k (n_k + 1/2), w_x = w_y = w_b                     (Eq. (21))
  * U (3 x 3, symmetric in the states):
      U_ss  = E_s  + k_s q_s + g_s^s q_s^2 + g_s^b (q_x^2 + q_y^2) + g_s^a q_a^2
      U_xx  = E_p  + k_p q_s + g_p^s q_s^2 + g_p^b (q_x^2 + q_y^2) + g_p^a q_a^2
              + c_rt (q_x^2 - q_y^2)
      U_yy  = the same with - c_rt (q_x^2 - q_y^2)
      U_xy  = 2 c_rt q_x q_y                        (Renner-Teller pair)
      U_sx  = c (1 + c' q_s) q_x,  U_sy = c (1 + c' q_s) q_y       (Eq. (18) generalised)
  * discrete-continuum couplings V_d^mu = f_d^mu(eps) O_d^mu, partial waves
    mu in (s, px, py):
      O_sigma^s = 1 + l_s q_s,  O_pix^s = h_p q_x,  O_piy^s = h_p q_y,
      O_sigma^px = h_s q_x,     O_pix^px = 1 + l_p q_s,  O_piy^px = 0,
      O_sigma^py = h_s q_y,     O_pix^py = 0,  O_piy^py = 1 + l_p q_s,
    widths Gamma = A eps^(l+1/2) exp(-eps/B) with l = 0 for the s wave and
    l = 1 for the p waves, f = sqrt(Gamma / 2 pi), one (A, B) per state class
    (sigma, pi) and wave class (s, p)                               (Eq. (22))
  * F_dd' = sum_mu (O_d^mu)^T diag(F[f_d^mu f_d'^mu](eps_nu)) O_d'^mu with the
    level shift of Eq. (19) on the same 4096-node grid                (Eq. (23))
  * A = E - H_0 - U - F, Phi^{v mu}_d = f_d^mu(E - E_v) O_d^mu |v>   (Eqs. (25), (28))
Every product uses truncated matrices (P q P), as in the two-state model.

Basis: index (d, n_s, n_x, n_y, n_a), n_a fastest; states d = 0 (sigma),
1 (Pi_x), 2 (Pi_y).
"""
import numpy as np
import scipy.sparse as sp

from . import levelshift as ls
from .model2d import position_matrix

STATES = ("sigma", "pix", "piy")
WAVES = ("s", "px", "py")
MODES = ("s", "x", "y", "a")


def wave_class(mu):
    return "s" if mu == "s" else "p"


def state_class(d):
    return "sigma" if d == 0 else "pi"


def width_params(p, d, mu):
    """(A, B, l) of Gamma_d^mu."""
    w, c = wave_class(mu), state_class(d)
    return p["A_%s_%s" % (c, w)], p["B_%s_%s" % (c, w)], (0 if w == "s" else 1)


def vib_energies(p, sizes):
    ns, nx, ny, na = [np.arange(sizes[k], dtype=np.float64) for k in MODES]
    E = (p["omega_s"] * (ns[:, None, None, None] + 0.5) + p["omega_b"] * (nx[None, :, None, None] + 0.5)
         + p["omega_b"] * (ny[None, None, :, None] + 0.5) + p["omega_a"] * (na[None, None, None, :] + 0.5))
    return E.ravel()


def vib_energy(p, v):
    return (p["omega_s"] * (v[0] + 0.5) + p["omega_b"] * (v[1] + 0.5) + p["omega_b"] * (v[2] + 0.5)
            + p["omega_a"] * (v[3] + 0.5))


def pair_tables(p, eps):
    """F[f_d f_d'](eps) for the wave classes (s, p) and the state-class pairs
    (sigma sigma), (sigma pi), (pi pi)."""
    out = {}
    for w in ("s", "p"):
        l = 0 if w == "s" else 1
        As, Bs = p["A_sigma_" + w], p["B_sigma_" + w]
        Ap, Bp = p["A_pi_" + w], p["B_pi_" + w]
        out[(w, "ss")] = ls.level_shift(eps, As, Bs, As, Bs, l, p["K"], p["X"])
        out[(w, "sp")] = ls.level_shift(eps, As, Bs, Ap, Bp, l, p["K"], p["X"])
        out[(w, "pp")] = ls.level_shift(eps, Ap, Bp, Ap, Bp, l, p["K"], p["X"])
    return out


def pair_key(d1, d2):
    c = sorted((state_class(d1), state_class(d2)))
    return {("sigma", "sigma"): "ss", ("pi", "sigma"): "sp", ("pi", "pi"): "pp"}[tuple(c)]


class PolyModel:
    """Explicit operator pieces of the model at one total energy E."""

    def __init__(self, p, sizes, E, tables=None):
        self.p, self.E = p, float(E)
        self.sizes = dict(sizes)
        dims = [self.sizes[k] for k in MODES]
        self.n = int(np.prod(dims))
        eye = [sp.identity(d, format="csr") for d in dims]

        def on_mode(k, M):
            mats = list(eye)
            mats[MODES.index(k)] = M
            out = mats[0]
            for m in mats[1:]:
                out = sp.kron(out, m, format="csr")
            return out

        self.Q = {k: on_mode(k, position_matrix(self.sizes[k])) for k in MODES}
        self.I = sp.identity(self.n, format="csr")
        self.Ev = vib_energies(p, self.sizes)
        self.eps_nu = self.E - self.Ev
        self.tables = (tables or pair_tables)(p, self.eps_nu)
        Qs, Qx, Qy, Qa = (self.Q[k] for k in MODES)
        I = self.I
        # O_d^mu as sparse matrices (None where zero)
        self.O = {
            (0, "s"): I + p["l_sigma"] * Qs, (1, "s"): p["h_pi"] * Qx, (2, "s"): p["h_pi"] * Qy,
            (0, "px"): p["h_sigma"] * Qx, (1, "px"): I + p["l_pi"] * Qs, (2, "px"): None,
            (0, "py"): p["h_sigma"] * Qy, (1, "py"): None, (2, "py"): I + p["l_pi"] * Qs,
        }
        self.U = self._U()

    def _U(self):
        p = self.p
        Qs, Qx, Qy, Qa = (self.Q[k] for k in MODES)
        I = self.I
        bend2 = Qx @ Qx + Qy @ Qy
        rt = Qx @ Qx - Qy @ Qy
        Uss = (p["E_sigma"] * I + p["k_sigma"] * Qs + p["gs_sigma"] * (Qs @ Qs)
               + p["gb_sigma"] * bend2 + p["ga_sigma"] * (Qa @ Qa))
        Upi = (p["E_pi"] * I + p["k_pi"] * Qs + p["gs_pi"] * (Qs @ Qs) + p["gb_pi"] * bend2
               + p["ga_pi"] * (Qa @ Qa))
        cs = p["c_sp"] * (I + p["c_sp2"] * Qs)
        return {
            (0, 0): Uss, (1, 1): Upi + p["c_rt"] * rt, (2, 2): Upi - p["c_rt"] * rt,
            (1, 2): 2.0 * p["c_rt"] * (Qx @ Qy), (0, 1): cs @ Qx, (0, 2): cs @ Qy,
        }

    def U_block(self, d1, d2):
        return self.U[(min(d1, d2), max(d1, d2))].T if d1 > d2 else self.U[(d1, d2)]

    def F_block(self, d1, d2):
        acc = sp.csr_matrix((self.n, self.n), dtype=complex)
        for mu in WAVES:
            O1, O2 = self.O[(d1, mu)], self.O[(d2, mu)]
            if O1 is None or O2 is None:
                continue
            t = self.tables[(wave_class(mu), pair_key(d1, d2))]
            acc = acc + O1.T @ sp.diags(t, 0, format="csr") @ O2
        return acc

    def matrix(self):
        """A = E - H_0 - U - F as a sparse 3n x 3n complex matrix."""
        H0 = sp.diags(self.Ev, 0, format="csr")
        blocks = [[None] * 3 for _ in range(3)]
        for d1 in range(3):
            for d2 in range(3):
                b = -self.U_block(d1, d2) - self.F_block(d1, d2)
                if d1 == d2:
                    b = b + self.E * self.I - H0
                blocks[d1][d2] = b
        return sp.bmat(blocks, format="csr")

    def unit(self, v):
        e = np.zeros(self.n)
        idx = 0
        for k, vk in zip(MODES, v):
            if not 0 <= vk < self.sizes[k]:
                return e
            idx = idx * self.sizes[k] + vk
        e[idx] = 1.0
        return e

    def phi(self, v, mu):
        """Phi^{v mu}_d = f_d^mu(E - E_v) O_d^mu |v>  (Eq. (25))."""
        eps = self.E - vib_energy(self.p, v)
        ev = self.unit(v)
        parts = []
        for d in range(3):
            O = self.O[(d, mu)]
            A, B, l = width_params(self.p, d, mu)
            f = float(ls.coupling_f(np.array([eps]), A, B, l)[0])
            parts.append(np.zeros(self.n) if O is None else f * (O @ ev))
        return np.concatenate(parts)


def total_energy(p, eps_i, v_i):
    return float(eps_i) + vib_energy(p, v_i)


def reflection_labels(sizes):
    """Eigenvalues of the reflections x -> -x and y -> -y on every basis
    function: (-1)^{n_x} and (-1)^{n_y}, times -1 for Pi_x (x) or Pi_y (y)."""
    ns, nx, ny, na = np.meshgrid(*[np.arange(sizes[k]) for k in MODES], indexing="ij")
    px0 = ((-1.0) ** nx).ravel()
    py0 = ((-1.0) ** ny).ravel()
    rx = np.concatenate([px0, -px0, px0])
    ry = np.concatenate([py0, py0, -py0])
    return rx, ry


def bend_blocks(sizes):
    """Index sets of the paper's preconditioner for this model class: one
    block per (n_s, n_a) holding every state and every bend point (n_x, n_y)."""
    dims = [sizes[k] for k in MODES]
    n = int(np.prod(dims))
    ns, nx, ny, na = np.meshgrid(*[np.arange(d) for d in dims], indexing="ij")
    flat = np.arange(n).reshape(dims)
    out = []
    for s in range(dims[0]):
        for a in range(dims[3]):
            pts = flat[s, :, :, a].ravel()
            out.append(np.concatenate([pts, pts + n, pts + 2 * n]))
    return out
